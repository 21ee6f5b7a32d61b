// Truncation (density-matrix / SVD split) of the two-site wave function.
#pragma once
#include "hpsi.h"

namespace bsd {

struct TruncBlock {
  Q ql;            // left bond label of the new site tensor block
  int s = 0;
  int rows = 0, cols = 0;
  std::vector<double> data;   // row-major
};

struct TruncResult {
  double trunc_err = 0.0;     // discarded weight
  double norm2 = 0.0;         // total weight (psi norm squared)
  int D_kept = 0;
  std::vector<double> sv;     // kept singular values, descending
  std::vector<TruncBlock> blocks;  // new site tensor
};

// left_to_right: new left-canonical tensor of `site`; else new
// right-canonical tensor of site + 1.
TruncResult truncate_psi(Ctx& ctx, const HpsiPlan& plan, const double* psi, int D, bool left_to_right,
                         DevBuf& work, hipStream_t s);

}  // namespace bsd
