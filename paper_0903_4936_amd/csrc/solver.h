// Host drivers of the block Krylov solves.
#pragma once

#include <string>

#include "../../include/bkwd.h"
#include "bkwd_internal.h"

struct WsLayout {
  int L;          // columns of the caller's blocks
  int Lc;         // columns of one Krylov cycle (1 for column-by-column BiCGSTAB)
  int method, prec;
  int nblocks;    // cycle blocks
  size_t elem;    // bytes per complex of the cycle precision
  size_t off_res64, off_col_b, off_col_x, off_col_s, off_res64c, off_blocks, block_bytes;
  size_t off_partials, n_partials, off_stage, stage_half;
  size_t off_red_a, off_red_b, off_red_c, off_red_r;
  size_t off_coef, off_weight, off_scale, off_unscale, off_ctl, off_hist, hist_cap;
  // even-odd solves: inverse site-local blocks (FP64, FP32), the FP64
  // whole-lattice block of the preparation / correction, the half block
  // between the Schur operator's two steps
  int evenodd;
  size_t off_cinv64, off_cinv32, off_eo64, off_eotmp;
  // deflation: the cycle's right-hand side columns, their indices, the map
  // of the correction back onto all columns
  int deflate;
  size_t off_defl_sub, off_defl_idx, off_defl_m;
  size_t total;
};

bool ws_layout(const LatticeImpl& lat, int L, const bkwd_solve_opts& o, WsLayout* out, std::string* err,
               bool residual_only = false);

int solve_driver(LatticeImpl& lat, int L, const cpx<double>* B, cpx<double>* X, const bkwd_solve_opts& o,
                 void* ws, size_t ws_bytes, bkwd_solve_info* info, hipStream_t s, std::string* err);

int true_residual_driver(LatticeImpl& lat, int L, const cpx<double>* B, const cpx<double>* X, double* per_col,
                         void* ws, size_t ws_bytes, hipStream_t s, std::string* err);
