/*
 * bkwd.h -- block Krylov solves of the O(a)-improved Wilson-Dirac equation
 * with many right-hand sides on one AMD Instinct MI355X (gfx950).
 *
 * Method: T. Sakurai, H. Tadano, Y. Kuramashi, "Application of block Krylov
 * subspace algorithms to the Wilson-Dirac equation with multiple right-hand
 * sides in lattice QCD" (arXiv:0903.4936).
 *
 * ---------------------------------------------------------------- layouts
 * Lattice dims are {Lx, Ly, Lz, Lt}, every extent >= 2, periodic in all four
 * directions (Sec. 2).  Flat site index: site = x + Lx*(y + Ly*(z + Lz*t));
 * site 0 is the origin.  Direction mu = 0..3 is x, y, z, t (gamma_4 is the
 * temporal matrix of Sec. 2).
 *
 * Gauge links (host, input of bkwd_lattice_create): complex128 interleaved
 * (re, im) as doubles, layout [4][V][3][3]: links[((mu*V + site)*3 + a)*3 + b]
 * is U_mu(site, a, b) of Sec. 2.
 *
 * Spinor blocks (device): the N x L matrices X, B of Sec. 3 (Eq. (14)),
 * N = 12 V, stored row-major with the right-hand-side index innermost:
 * element (row, i) with row = 12*site + 3*spin + colour (spin, colour
 * 0-based: the paper's (alpha - 1, a - 1)) is at offset row*L + i, i.e. the
 * layout is [V][4][3][L].  Complex values are interleaved (re, im):
 * complex128 for BKWD_FP64 and for every block argument of bkwd_block_solve /
 * bkwd_true_residual, complex64 for BKWD_FP32 in bkwd_apply.
 *
 * ---------------------------------------------------------------- ownership
 * All device memory is owned by the caller (for example allocated with
 * PyTorch): the lattice buffer, spinor blocks and solver workspace are passed
 * in; the library never allocates or frees device memory.  It allocates
 * 64 KiB of pinned host memory per lattice (hipHostMalloc) for the solver's
 * status and column-norm read-back, freed by bkwd_lattice_destroy.
 * A handle is not thread-safe; distinct handles are independent.
 *
 * ---------------------------------------------------------------- errors
 * Every entry point returns a bkwd_status.  BKWD_EINVAL is returned for bad
 * arguments before any device work is queued; the reason is available from
 * bkwd_last_error() (thread-local).  No C++ exception crosses this ABI.
 * `stream` is a hipStream_t (NULL = the default stream).  bkwd_apply is
 * asynchronous on `stream`; bkwd_lattice_create, bkwd_lattice_set_params,
 * bkwd_block_solve and bkwd_true_residual synchronise `stream` before they
 * return.
 */
#ifndef BKWD_H
#define BKWD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BKWD_OK = 0,
  BKWD_EINVAL = -1,      /* invalid argument (nothing was queued)          */
  BKWD_ENOMEM = -2,      /* a caller buffer is too small                   */
  BKWD_EDEVICE = -3,     /* a HIP runtime call failed                      */
  BKWD_ENOCONV = -4,     /* not converged within the iteration/restart cap */
  BKWD_EBREAKDOWN = -5   /* singular L x L system or non-finite scalar     */
} bkwd_status;

/* arithmetic of an operator application or of a solve */
enum { BKWD_FP64 = 0, BKWD_FP32 = 1, BKWD_MIXED = 2 };

/* solvers of Sec. 3 */
enum {
  BKWD_BICGSTAB = 0,        /* BiCGSTAB, each column solved on its own      */
  BKWD_BLOCK_BICGSTAB = 1,  /* block BiCGSTAB                               */
  BKWD_BLOCK_BICGGR = 2     /* the paper's new block method (Block BiCGGR)  */
};

/* lattice flags */
#define BKWD_COMPRESS12 1u  /* FP32 links kept as two rows (12 reals); the
                               third row is rebuilt as conj(row0 x row1)    */

#define BKWD_MAX_RHS 64     /* largest L accepted by every entry point */

typedef struct bkwd_lattice bkwd_lattice;

/*
 * Device bytes the lattice buffer must hold for these dims and flags (gauge
 * links in FP64 and FP32, the site-local clover blocks in FP64 and FP32, and
 * a copy of the input links).  Returns 0 if dims are invalid.
 */
size_t bkwd_lattice_bytes(const int dims[4], unsigned flags);

/*
 * Build the operator D_W of Sec. 2, Eq. (1) for links U, hopping parameter
 * kappa and clover coefficient csw.  `links_host` is host memory in the
 * layout above (not retained).  `dev_buf` is caller device memory of at least
 * bkwd_lattice_bytes(dims, flags) bytes, 256-byte aligned, that must outlive
 * the handle.  The field strength F_{mu nu} is built from the four clover
 * leaves of Sec. 2 (the two leaves whose printed index does not close a loop
 * are read as the standard plaquettes) without trace removal.
 * On success *out is a new handle; on error *out is NULL.
 */
int bkwd_lattice_create(const int dims[4], const double *links_host, double kappa, double csw,
                        unsigned flags, void *dev_buf, size_t dev_buf_bytes, void *stream,
                        bkwd_lattice **out);

/* Change kappa and csw (rebuilds the clover blocks on the device). */
int bkwd_lattice_set_params(bkwd_lattice *lat, double kappa, double csw, void *stream);

/* Release the handle (host memory only; dev_buf stays the caller's). */
int bkwd_lattice_destroy(bkwd_lattice *lat);

/* Query the lattice: dims, volume, kappa, csw. */
int bkwd_lattice_info(const bkwd_lattice *lat, int dims_out[4], long long *volume,
                      double *kappa, double *csw);

/*
 * Y = D_W X (dagger = 0) or Y = D_W^dagger X = gamma_5 D_W gamma_5 X
 * (dagger = 1) for all L columns (Sec. 2, Eq. (1)).  X and Y are device
 * spinor blocks of L columns in `prec` (BKWD_FP64: complex128, BKWD_FP32:
 * complex64) and must not overlap.  1 <= L <= BKWD_MAX_RHS.
 */
int bkwd_apply(bkwd_lattice *lat, int dagger, int L, int prec, const void *X, void *Y, void *stream);

/* block layouts of bkwd_apply_layout */
enum {
  BKWD_SITE_MAJOR = 0,      /* [V][4][3][L], the layout of every other entry point  */
  BKWD_COMPONENT_MAJOR = 1  /* [4][3][V][L]: element (row = 12*site + 3*spin + colour,
                               i) at offset ((3*spin + colour)*V + site)*L + i; the
                               layout of the solver's FP32 Krylov blocks            */
};

/*
 * bkwd_apply with the spinor blocks in `layout` (Sec. 2, Eq. (1), as for
 * bkwd_apply).  With BKWD_COMPONENT_MAJOR and BKWD_FP32 it runs the operator
 * launches of the mixed solve's inner iteration.  BKWD_EINVAL for an unknown
 * layout; otherwise the same arguments and behaviour as bkwd_apply.
 */
int bkwd_apply_layout(bkwd_lattice *lat, int dagger, int L, int prec, int layout, const void *X, void *Y,
                      void *stream);

typedef struct {
  int method;         /* BKWD_BICGSTAB, BKWD_BLOCK_BICGSTAB, BKWD_BLOCK_BICGGR          */
  int prec;           /* BKWD_FP64, or BKWD_MIXED: FP32 inner iteration inside an FP64
                         defect-correction loop                                          */
  int max_iter;       /* cap on iterations of one Krylov cycle                           */
  int max_restarts;   /* cap on extra cycles (FP64: restarts from X when the true
                         residual misses tol; MIXED: defect-correction cycles)           */
  int use_x0;         /* 1: X holds the initial guess on entry; 0: X_0 = 0               */
  int shadow;         /* 0: R~_0 = R_0 of each cycle (default); 1: seeded complex Gaussian
                         R~_0; 2: R~_0 taken from shadow_block.  Whatever the choice, a
                         cycle that does not lower the true residual (for example a
                         breakdown of R~_0 = R_0 on point sources in a free field) is
                         undone and retried with a fresh seeded Gaussian R~_0            */
  int check_every;    /* host reads the device status every this many iterations (>=1) */
  int stagnation;     /* stop a cycle after this many iterations without a new minimum
                         of the max relative residual (0 = off)                          */
  double tol;         /* target for max_i ||b_i - D x_i|| / ||b_i|| (true residual)      */
  double inner_tol;   /* MIXED: relative reduction asked of each FP32 cycle, in (0, 1);
                         0 = by L: 1e-5 for L <= 16, 3e-2 for L > 16 (the FP32 block
                         iteration loses convergence speed above L = 16, so shorter
                         cycles with more FP64 restarts need fewer iterations)       */
  unsigned long long seed;  /* seed of the Gaussian shadow residual                      */
  double *history;    /* optional host array: max relative recursive residual per
                         iteration, iterations of all cycles concatenated               */
  int history_len;    /* its length (0 = no history)                                     */
  int profile;        /* 1: time every operator application with HIP events           */
  const void *shadow_block; /* shadow = 2: device complex128 block of L columns (same
                               layout as B), the caller's R~_0                            */
  int qr_frame;       /* BKWD_BLOCK_BICGGR only.  -1 (default): 0 for FP64 solves; for
                         MIXED 2, or 1 with reliable updates (FP32 cycles do not
                         converge without a frame; in FP64 the listing takes the same
                         iterations with fewer block passes).
                         1: carry the residual as
                         R_k = Q_k xi_k with orthonormal Q_k (FP64 Cholesky QR each
                         iteration) and the other blocks in that frame; the iterates
                         are those of the listing in exact arithmetic, and the blocks
                         the FP32 arithmetic sees stay well conditioned.  2: the
                         same frame with the normalisation and the blocks P, V
                         folded into the L x L coefficients (used for L <= 16, else
                         as 1): 16 instead of 20 block passes per iteration, and at
                         8-column FP32 blocks 12, the solution update riding in the
                         U pass and one Gram set in the operator launch.
                         0: the listing's recurrences as printed.                     */
  int dagger;         /* 0: solve D_W X = B; 1: solve D_W^dagger X = B (the adjoint system
                         of a gradient: D_W^dagger = gamma_5 D_W gamma_5, same kernels)     */
  double reliable;    /* MIXED with BLOCK_BICGGR and qr_frame 1 (or -1) only, else
                         BKWD_EINVAL.  0: each FP32 cycle
                         stops at inner_tol and the next one restarts the Krylov space.
                         delta in (0, 1): one FP32 cycle runs to tol with reliable updates:
                         whenever its residual has dropped by delta, the correction is
                         added in FP64, the FP64 true residual becomes the new frame and
                         the search blocks are carried over (no restart).                */
  int max_block;      /* block methods: most columns per block solve.  The L columns
                         are split into blocks of max_block columns and one with the
                         rest, solved one after another, each an independent block
                         solve of its own columns.  0 (default): 8 for MIXED (the FP32
                         block iteration needs far more iterations above 16 columns
                         and about as many per block from 4 to 16, and 8 columns fill
                         the operator and update kernels best); for FP64 one block up
                         to 16 columns, else 16 (wider FP64 blocks run VALU-bound
                         update kernels).                                             */
  int evenodd;        /* 1: even-odd preconditioning (every lattice extent even).  Each
                         Krylov cycle solves the Schur complement on the even sites,
                         S = A_ee - kappa^2 H_eo A_oo^{-1} H_oe (A: the site-local term,
                         H: the hopping sum of Sec. 2, Eq. (1)), for the right-hand side
                         r_e + kappa H_eo A_oo^{-1} r_o, and the odd sites follow as
                         A_oo^{-1} (r_o + kappa H_oe x_e); the FP64 outer loop and its
                         stop test are those of the unpreconditioned solve.  Half the
                         rows per Krylov block.  Not with reliable > 0 or shadow = 2.
                         0 (default): the operator of Eq. (1) as it stands.            */
  int deflate;        /* block methods: 1 = before each Krylov cycle leave out the columns
                         whose true residual already meets tol, and of the others solve
                         only an independent subset: a pivoted Cholesky factorisation of
                         their residual Gram matrix keeps the columns whose part
                         orthogonal to those kept before is at least max(drop ||r_i||,
                         tol ||b_i|| / 10), drop = 1e-6 (FP64) or 1e-4 (MIXED); every
                         other column's correction is the least-squares
                         combination of the kept ones' (exact for a column in their
                         span, e.g. duplicated right-hand sides, which break the block
                         iteration down without it).  0 (default): every column in every
                         cycle.                                                         */
} bkwd_solve_opts;

typedef struct {
  int iterations;               /* Krylov iterations, all cycles, summed over the column
                                   blocks (and over the columns for BKWD_BICGSTAB)         */
  int outer_cycles;             /* cycles run (1 = no restart), summed over the blocks      */
  int matvecs;                  /* applications of D_W (any precision)                      */
  int converged;                /* 1 if the true residual reached tol                      */
  int status_detail;            /* 0 ok, 1 max_iter, 2 breakdown, 3 stagnation              */
  int history_written;          /* entries written to opts.history                          */
  double true_residual_max;     /* max_i ||b_i - D x_i|| / ||b_i||, FP64, at return          */
  double recursive_residual_max;/* last recursive residual (relative to the cycle's rhs)    */
  double seconds;               /* wall time of the call                                   */
  double dslash_ms;             /* profile = 1: summed kernel time of operator applications*/
  int dslash_calls;             /* profile = 1: number of timed applications                */
  int dslash_calls_fp32;        /* profile = 1: how many of them were FP32                  */
  double dslash_ms_fp32;        /* profile = 1: summed time of the FP32 ones               */
  double update_ms[3];          /* profile = 1: summed time of the block update kernels of
                                   Block BiCGGR: [0] U, [1] X and R, [2] P and V (with
                                   their Gram products); in the fused frame [2] is the
                                   Gram pass, or the operator launch W' = A T that also
                                   forms those Grams when gram_operator is 1             */
  int update_calls[3];          /* profile = 1: their launch counts                         */
  int reliable_updates;         /* reliable updates performed (opts.reliable > 0)           */
  int main_width;               /* columns per column block of the solve (L if not split;
                                   the last block of a split solve may be narrower)         */
  double dslash_ms_fp32_main;   /* profile = 1: dslash_ms_fp32, dslash_calls_fp32,
                                   update_ms and update_calls counting only the launches
                                   of the blocks of main_width columns                      */
  int dslash_calls_fp32_main;
  double update_ms_main[3];
  int update_calls_main[3];
  int deflated_columns;         /* opts.deflate: columns left out, summed over the cycles  */
  int gram_operator;            /* 1: the fused frame's Grams of W' = A T were formed in the
                                   operator launch itself (8-column FP32 blocks; with
                                   evenodd, in the second launch of the Schur operator)   */
} bkwd_solve_info;

/* Fill opts with defaults: BLOCK_BICGGR, MIXED, tol 1e-12, inner_tol 0 (by L),
   max_iter 10000, max_restarts 20, shadow 0 (R~_0 = R_0), check_every 8,
   stagnation 200, qr_frame -1 (by precision), dagger 0, reliable 0, max_block 0,
   evenodd 0, deflate 0. */
void bkwd_solve_opts_default(bkwd_solve_opts *opts);

/* Device workspace bytes bkwd_block_solve needs for L columns and opts
   (also enough for bkwd_true_residual).  0 if the arguments are invalid. */
size_t bkwd_solve_workspace_bytes(const bkwd_lattice *lat, int L, const bkwd_solve_opts *opts);

/*
 * Solve D_W X = B (or D_W^dagger X = B with opts->dagger) for L right-hand
 * sides (Sec. 3, Eq. (14)) with the chosen method, stopping when
 * max_i ||b_i - D x_i||_2 / ||b_i||_2 <= opts->tol for the FP64 true residual
 * of Sec. 4.3 (D^dagger in place of D for the adjoint system).  B and X are complex128 device blocks.
 * Every column of B must be non-zero.  `workspace` is caller device memory
 * of at least bkwd_solve_workspace_bytes() bytes, 256-byte aligned.
 * Returns BKWD_OK, or BKWD_ENOCONV / BKWD_EBREAKDOWN with *info filled and X
 * holding the last iterate.  Synchronises `stream`.
 */
int bkwd_block_solve(bkwd_lattice *lat, int L, const void *B, void *X, const bkwd_solve_opts *opts,
                     void *workspace, size_t workspace_bytes, bkwd_solve_info *info, void *stream);

/*
 * per_col_host[i] = ||b_i - D_W x_i||_2 / ||b_i||_2 in FP64 (Sec. 4.3) for
 * complex128 device blocks B, X.  Needs a workspace of
 * bkwd_solve_workspace_bytes() bytes.  Synchronises `stream`.
 */
int bkwd_true_residual(bkwd_lattice *lat, int L, const void *B, const void *X, double *per_col_host,
                       void *workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * per_col_host[i] = ||b_i - D_W x_i||_2 / ||b_i||_2 as bkwd_true_residual, in
 * FP64, with no workspace argument.  The kernels' partial sums and their
 * reduction live in a static device array of BKWD_NOALLOC_SCRATCH_BYTES that
 * the library holds on each GPU it runs on until the process ends; the call
 * allocates nothing (per_col_host is filled through the lattice's pinned
 * host area).  1 <= L <= BKWD_MAX_RHS, else BKWD_EINVAL.  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (several threads
 * or streams) race.  Synchronises `stream`.
 */
#define BKWD_NOALLOC_SCRATCH_BYTES 1065984u
int bkwd_true_residual_noalloc(bkwd_lattice *lat, int L, const void *B, const void *X, double *per_col_host,
                               void *stream);

/*
 * Gradients of a solve (growth of the method; derived from Sec. 2, Eq. (1)).
 * For X = D_W^{-1} B and a real loss l with gradient G = dl/dRe X + i dl/dIm X,
 * the caller first solves the adjoint system D_W^dagger Lambda = G
 * (bkwd_block_solve with opts.dagger = 1); then grad_B = Lambda and this call
 * returns, with the same convention (dl = Re sum conj(g) dz for complex z):
 *   *grad_kappa = Re <Lambda, (c_SW C + H) X>  (= -Re <Lambda, dD/dkappa X>),
 *   *grad_csw   = kappa Re <Lambda, C X>        (= -Re <Lambda, dD/dc_SW X>),
 *   grad_links  = the gradient of -Re <Lambda, D_W(U) X> with respect to the
 *                 links (hopping term and the four clover leaves),
 * where <a, b> = sum conj(a) b, C = sum_{mu,nu} (i/2) sigma_{mu nu} F_{mu nu}
 * and H is the hopping sum, D_W = 1 - kappa c_SW C - kappa H.
 * X and Lambda are complex128 device blocks of L columns (layout of B).
 * grad_kappa and grad_csw are host pointers, grad_links a device complex128
 * array in the layout of the input links, [4][V][3][3]; any of the three may
 * be NULL to skip it.  `workspace` needs bkwd_gradients_workspace_bytes()
 * bytes, 256-byte aligned.  Synchronises `stream`.
 */
size_t bkwd_gradients_workspace_bytes(const bkwd_lattice *lat, int L);
int bkwd_gradients(bkwd_lattice *lat, int L, const void *X, const void *Lambda, double *grad_kappa,
                   double *grad_csw, void *grad_links, void *workspace, size_t workspace_bytes, void *stream);

/* Meson two-point functions from the 12 point-source solutions: the columns of
   X (device complex128 [V][4][3][12], the solution of D_W X = B with the point
   sources of Sec. 2 at the origin, column i = colour + 3*spin) form the quark
   propagator S(x) from the origin.  With gamma_5-hermiticity
   S(0, x) = gamma_5 S(x, 0)^dagger gamma_5, the Wick contraction of
   psibar G psi summed over the spatial sites of time slice t is
     C_G(t) = -sum_x Re Tr[G S(x) Gbar gamma_5 S(x)^dagger gamma_5],
     Gbar = gamma_4 G^dagger gamma_4,
   trace over spin and colour, gamma matrices of Sec. 2.  pion receives
   C_{gamma_5}(t) (= sum_x ||S(x)||^2), rho the average of C_{gamma_k}(t) over
   k = 1, 2, 3, for t = 0 .. Lt-1 (distance from the source slice t = 0).
   pion and rho: device arrays of Lt doubles owned by the caller.  Runs on
   `stream` without synchronising; allocates nothing.  Returns BKWD_EINVAL for
   NULL arguments, BKWD_EDEVICE if the launch fails. */
int bkwd_meson_correlators(bkwd_lattice *lat, const void *X, double *pion, double *rho, void *stream);

/* Text of the last error on this thread ("" if none). */
const char *bkwd_last_error(void);

/* Library version string. */
const char *bkwd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BKWD_H */
