// Batched projected CG for exact corrections (training pairs).
#pragma once
#include <vector>

#include "solver.hpp"

namespace phs {

struct CgBufs {
  double *P, *AP, *Res, *T, *Y, *v;
  int *flags;
};

void carve_cg(Arena &ar, int64_t m, int64_t n, int bw, CgBufs &cb);
// Solves the projected equations (I - QQ^T)(C - rho theta_j I)(I - QQ^T) t
// = r_j for the nb columns of R (row-major, stride bw) with Q = [Xl | Xb],
// rho = shift_scale (the Jacobi-Davidson correction with the sign of a
// preconditioned residual, t = M r); the solutions are left in cb.T.
// Returns per column whether CG converged without non-positive curvature.
std::vector<int> projected_cg_block(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                                    const double *Xl, int nl, const double *Xb, int nb, int bw,
                                    const double *theta, double shift_scale, const double *R,
                                    double tol, int maxit,
                                    CgBufs &cb, SmallPool &sp);

}  // namespace phs
