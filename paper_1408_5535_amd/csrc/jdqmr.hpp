// JDQMR second stage: the inner symmetric QMR solve of the projected
// Jacobi-Davidson correction equation (Section 3.2), and the triplet
// residual of a stage-2 candidate (the stopping test of Section 5).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "solver.hpp"

namespace phs {

// Ten N-vectors of work space (N = m + n), contiguous.
constexpr int kJdVectors = 10;

struct JdInput {
  Tall<double> Q1, Q2;  // projector basis Q = [Q1 | Q2]: locked vectors, then x
  Tall<double> r;       // outer residual B x - theta x (one column)
  double theta = 0.0;   // Rayleigh quotient of x
  double eta = 0.0;     // shift of the correction equation (the target shift)
  double thr = 0.0;     // outer stopping threshold on ||B x - theta x||
  int max_inner = 50;
  const double *jacobi_d = nullptr;  // diag(C) for the B-form Jacobi preconditioner
  // or another preconditioner of B (Stage2Params::precB; called with one
  // contiguous N-vector, ld 1, and theta = eta)
  std::function<void(const double *, double *, int, int, const double *)> precB;
};

struct JdResult {
  int steps = 0;
  int reason = 0;  // 0 cap, 1 converged, 2 linear, 3 stagnation, 4 breakdown
};

// t (one column, any layout) = P u with u the sQMR approximation of
//   P (B - eta I) P u = -P r,   P = I - Q Q^T,
// stopped by the dynamic rules of the second stage.  Products with B count
// as stage-2 products, preconditioner products as mv_prec.
JdResult jd_correction(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                       const JdInput &in, double *work, const Tall<double> &t, SmallPool &sp);

// sqrt(||A^T u - theta v||^2 + ||A v - theta u||^2) for the normalised halves
// v = x_top / ||x_top||, u = x_bot / ||x_bot|| of x, from x and its residual
// R = B x - theta x (both one column, row stride ldx): B x = R + theta x.
// Infinite when a half is zero.  Synchronises the stream.
double triplet_residual(Ctx &c, const double *x, const double *R, int ldx, int64_t n, int64_t N,
                        double theta, SmallPool &sp);

}  // namespace phs
