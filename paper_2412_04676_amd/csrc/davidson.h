// Davidson eigensolver on the two-site effective Hamiltonian.
#pragma once
#include "hpsi.h"

namespace bsd {

struct DavidsonOpts {
  int max_iter = 50;
  int max_sub = 24;
  int restart = 4;
  double tol = 1e-8;
  double precond_floor = 1e-4;
  int precision = 0;   // precision of the H.psi products
  int precond = 0;     // 0 diagonal, 1 none
};

struct DavidsonResult {
  double energy = 0.0, resid = 0.0;
  int iters = 0;
  int products = 0;           // H.psi products applied (both stages)
  std::vector<double> ritz;   // lowest Ritz value after every iteration
};

// psi: in guess, out normalized eigenvector (psi layout of the plan);
// diag: diagonal of H_eff in the same layout.
DavidsonResult davidson(HpsiPlan& plan, const double* diag, double* psi, const DavidsonOpts& o,
                        DevBuf& work, hipStream_t s);

}  // namespace bsd
