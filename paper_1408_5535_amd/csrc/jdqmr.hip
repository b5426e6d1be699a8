// JDQMR correction of the second stage (Section 3.2): each outer step of
// the refined GD iteration on B = [0 A^T; A 0] expands the basis by an
// approximate solution of the projected correction equation
//
//     P (B - eta I) P t = -P r,   P = I - Q Q^T,   Q = [locked vectors, x],
//
// with eta the target shift from stage 1, found by symmetric QMR (quasi-
// minimal residual smoothing of the conjugate-gradient recurrences; it
// stays defined for the indefinite operator) and stopped dynamically:
//   1. the eigen-residual of the outer candidate x + t is below the outer
//      threshold;
//   2. the linear residual is below a tenth of that eigen-residual (the
//      shift, not the linear system, now limits it);
//   3. the eigen-residual has not fallen by 1% over the last 20 steps;
//   4. the step cap.
// The eigen-residual needs no extra product: with s the linear residual,
// (B - eta) (x + t) = -s + a x, a = theta - eta + r^T t, so for the best
// shift mu = eta + b, b = (a - s^T t) / (1 + t^T t),
//   ||(B - mu)(x + t)||^2 = s^T s + 2 b s^T t + b^2 t^T t + (a - b)^2.
//
// Vector kernels stream the N-vectors once per step and leave per-block
// partial dot products; a one-block kernel adds them in a fixed order and
// advances the scalar recurrence on the device, so a step needs no host
// round trip until its end, where the host reads the few status scalars it
// takes the stopping decision from.
#include "jdqmr.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

#include "wave.hpp"

namespace phs {
namespace {

constexpr int kJdThreads = 256;
constexpr int kJdMaxBlocks = 1024;
constexpr int kJdDots = 4;

// scalar block (device, float64)
enum {
  J_RHO, J_TAU, J_THP, J_ALPHA, J_C2, J_F, J_BETA, J_A1, J_GG, J_EST, J_SN, J_BREAK,
  J_THETA, J_ETA, J_PREC, J_COUNT
};

struct JdPtrs {
  double *y, *q, *g, *d, *e, *t, *s, *w, *z, *r;
};

enum JdOp { OP_NEG_R, OP_INIT, OP_SHIFT, OP_SIG, OP_G, OP_UPD, OP_RHO, OP_W, OP_TRIP };

// Block partials of nd dot products: part[blockIdx.x * kJdDots + j].
__device__ inline void block_dots(const double (&v)[kJdDots], int nd, double *part) {
  __shared__ double red[kJdThreads / 64][kJdDots];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = 0; j < nd; ++j) {
    const double s = wave_total(v[j]);
    if (lane == 0) red[w][j] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < nd) {
    const int j = threadIdx.x;
    double s = red[0][j];
    for (int q = 1; q < kJdThreads / 64; ++q) s += red[q][j];
    part[(int64_t)blockIdx.x * kJdDots + j] = s;
  }
}

template <int OP>
__global__ __launch_bounds__(kJdThreads) void k_jd_vec(int64_t N, JdPtrs p, const double *sc,
                                                       double *part) {
  if ((OP == OP_G || OP == OP_UPD || OP == OP_RHO || OP == OP_W) && sc[J_BREAK] != 0.0) return;
  double v[kJdDots] = {0.0, 0.0, 0.0, 0.0};
  const double alpha = (OP == OP_G) ? sc[J_ALPHA] : 0.0;
  const double f = (OP == OP_UPD) ? sc[J_F] : 0.0;
  const double a1 = (OP == OP_UPD) ? sc[J_A1] : 0.0;
  const double beta = (OP == OP_UPD || OP == OP_W) ? sc[J_BETA] : 0.0;
  const bool prec = sc[J_PREC] != 0.0;
  const double eta = (OP == OP_SHIFT) ? sc[J_ETA] : 0.0;
  const int64_t stride = (int64_t)gridDim.x * kJdThreads;
  for (int64_t i = (int64_t)blockIdx.x * kJdThreads + threadIdx.x; i < N; i += stride) {
    if (OP == OP_NEG_R) {
      p.g[i] = -p.r[i];
    } else if (OP == OP_INIT) {
      const double gi = p.g[i];
      p.s[i] = gi;
      if (!prec) p.w[i] = gi;
      p.d[i] = 0.0;
      p.e[i] = 0.0;
      p.t[i] = 0.0;
      v[0] = fma(gi, gi, v[0]);
    } else if (OP == OP_SHIFT) {
      p.q[i] = fma(-eta, p.w[i], p.y[i]);
    } else if (OP == OP_SIG) {
      v[0] = fma(p.w[i], p.q[i], v[0]);
    } else if (OP == OP_G) {
      const double gi = fma(-alpha, p.q[i], p.g[i]);
      p.g[i] = gi;
      v[0] = fma(gi, gi, v[0]);
    } else if (OP == OP_UPD) {
      const double wi = p.w[i], qi = p.q[i];
      const double di = fma(f, p.d[i], a1 * wi);
      const double ei = fma(f, p.e[i], a1 * qi);
      const double ti = p.t[i] + di;
      const double si = p.s[i] - ei;
      p.d[i] = di;
      p.e[i] = ei;
      p.t[i] = ti;
      p.s[i] = si;
      if (!prec) p.w[i] = fma(beta, wi, p.g[i]);
      v[0] = fma(p.r[i], ti, v[0]);
      v[1] = fma(ti, ti, v[1]);
      v[2] = fma(si, ti, v[2]);
      v[3] = fma(si, si, v[3]);
    } else if (OP == OP_RHO) {
      v[0] = fma(p.g[i], p.z[i], v[0]);
    } else if (OP == OP_W) {
      p.w[i] = fma(beta, p.w[i], p.z[i]);
    }
  }
  constexpr int nd = OP == OP_UPD ? 4 : (OP == OP_INIT || OP == OP_SIG || OP == OP_G ||
                                         OP == OP_RHO) ? 1 : 0;
  if (nd > 0) block_dots(v, nd, part);
}

// Sum of partial j over nblk blocks, fixed order (lane-strided, then the
// wavefront's fixed combination); every lane gets the total.
__device__ inline double sum_part(const double *part, int nblk, int j) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[(int64_t)b * kJdDots + j];
  return wave_total(s);
}

template <int OP>
__global__ __launch_bounds__(64) void k_jd_scalar(const double *part, int nblk, double *sc) {
  if ((OP == OP_G || OP == OP_UPD || OP == OP_RHO) && sc[J_BREAK] != 0.0) return;
  double v[kJdDots];
  constexpr int nd = OP == OP_UPD ? 4 : 1;
  for (int j = 0; j < nd; ++j) v[j] = sum_part(part, nblk, j);
  if (threadIdx.x != 0) return;
  const bool prec = sc[J_PREC] != 0.0;
  if (OP == OP_INIT) {
    sc[J_GG] = v[0];
    sc[J_TAU] = sqrt(v[0]);
    sc[J_THP] = 0.0;
    sc[J_BREAK] = v[0] > 0.0 ? 0.0 : 1.0;
    if (!prec) sc[J_RHO] = v[0];
  } else if (OP == OP_SIG) {
    const double sig = v[0], rho = sc[J_RHO];
    if (sig == 0.0 || rho == 0.0) {
      sc[J_BREAK] = 1.0;
      sc[J_ALPHA] = 0.0;
    } else {
      sc[J_ALPHA] = rho / sig;
    }
  } else if (OP == OP_G) {
    const double gg = v[0], tau = sc[J_TAU], thp = sc[J_THP], alpha = sc[J_ALPHA];
    const double th = sqrt(gg) / tau;
    const double c2 = 1.0 / (1.0 + th * th);
    sc[J_TAU] = tau * th * sqrt(c2);
    sc[J_C2] = c2;
    sc[J_F] = c2 * thp * thp;
    sc[J_A1] = c2 * alpha;
    sc[J_THP] = th;
    sc[J_GG] = gg;
    if (!prec) {
      sc[J_BETA] = gg / sc[J_RHO];
      sc[J_RHO] = gg;
    }
  } else if (OP == OP_UPD) {
    const double rt = v[0], tt = v[1], st = v[2], ss = v[3];
    const double a = sc[J_THETA] - sc[J_ETA] + rt;
    const double b = (a - st) / (1.0 + tt);
    const double f = ss + 2.0 * b * st + b * b * tt + (a - b) * (a - b);
    sc[J_EST] = sqrt((f > 0.0 ? f : 0.0) / (1.0 + tt));
    sc[J_SN] = sqrt(ss > 0.0 ? ss : 0.0);
  } else if (OP == OP_RHO) {
    const double rho = v[0], old = sc[J_RHO];
    sc[J_BETA] = old != 0.0 ? rho / old : 0.0;
    sc[J_RHO] = rho;
    if (rho == 0.0) sc[J_BREAK] = 1.0;
  }
}

// Triplet residual partials of a stage-2 candidate: rows below n belong to
// the top half v (r_u rows), the others to the bottom half u (r_v rows):
//   r_u = (R_top + theta x_top) / ||u|| - theta x_top / ||v||
//   r_v = (R_bot + theta x_bot) / ||v|| - theta x_bot / ||u||
__global__ __launch_bounds__(kJdThreads) void k_jd_trip(const double *x, const double *R, int ldx,
                                                        int64_t n, int64_t N, double theta,
                                                        const double *nrm, double *part) {
  const double nv = sqrt(nrm[0]), nu = sqrt(nrm[1]);
  double v[kJdDots] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kJdThreads;
  for (int64_t i = (int64_t)blockIdx.x * kJdThreads + threadIdx.x; i < N; i += stride) {
    const double xi = x[i * ldx], ri = R[i * ldx];
    const double bx = fma(theta, xi, ri);
    const double res = i < n ? bx / nu - theta * xi / nv : bx / nv - theta * xi / nu;
    v[0] = fma(res, res, v[0]);
  }
  block_dots(v, 1, part);
}

__global__ __launch_bounds__(64) void k_jd_total(const double *part, int nblk, double *out) {
  const double v = sum_part(part, nblk, 0);
  if (threadIdx.x == 0) out[0] = v;
}

int jd_blocks(int64_t N) { return (int)std::min<int64_t>(cdiv(N, kJdThreads), kJdMaxBlocks); }

Tall<double> col(double *p, int64_t N) { return cm(p, N, 1, N); }

// y <- P y = y - Q (Q^T y)
void project(Ctx &c, const JdInput &in, double *y, int64_t N, SmallPool &sp) {
  if (in.Q1.cols + in.Q2.cols == 0) return;
  double *G = sp.vec(18);
  tn(in.Q1, in.Q2, col(y, N), G, kSP, c.sc, c.s);
  nn(in.Q1, in.Q2, G, kSP, -1.0, col(y, N), 1.0, c.s);
}

template <int OP>
void vec_op(Ctx &c, int64_t N, const JdPtrs &p, double *sc, bool reduce) {
  const int nb = jd_blocks(N);
  k_jd_vec<OP><<<nb, kJdThreads, 0, c.s>>>(N, p, sc, c.sc.part);
  PHS_CHECK_LAUNCH();
  if (reduce) {
    k_jd_scalar<OP><<<1, 64, 0, c.s>>>(c.sc.part, nb, sc);
    PHS_CHECK_LAUNCH();
  }
}

}  // namespace

JdResult jd_correction(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                       const JdInput &in, double *work, const Tall<double> &tout, SmallPool &sp) {
  const int64_t n = A.n, N = A.m + A.n;
  JdPtrs p;
  double **slot[kJdVectors] = {&p.y, &p.q, &p.g, &p.d, &p.e, &p.t, &p.s, &p.w, &p.z, &p.r};
  for (int i = 0; i < kJdVectors; ++i) *slot[i] = work + (int64_t)i * N;
  double *sc = sp.vec(19);
  {
    double init[J_COUNT] = {};
    init[J_THETA] = in.theta;
    init[J_ETA] = in.eta;
    init[J_PREC] = (in.jacobi_d || in.precB) ? 1.0 : 0.0;
    c.h2d(sc, init, sizeof(init));
  }
  const bool prec = in.jacobi_d != nullptr || bool(in.precB);
  // z = P K g with K the preconditioner of B: the B-form [M A^T g; A M f]
  // of M = D^-1 (Jacobi), or the given one
  auto apply_prec = [&]() {
    if (in.precB) {
      const double eta = in.eta;
      in.precB(p.g, p.z, 1, 1, &eta);
    } else {
      row_scale(p.g, in.jacobi_d, n, 1, true, p.q, c.s);  // D^-1 g_top (q is free here)
      spmm(A, 1, p.q, p.z + n, false, c.s);
      spmm(At, 1, p.g + n, p.z, false, c.s);
      row_scale(p.z, in.jacobi_d, n, 1, true, p.z, c.s);
      c.st->mv_prec += 1;
    }
    project(c, in, p.z, N, sp);
  };
  // right-hand side -P r, then the sQMR start
  copy(in.r, col(p.r, N), c.s);
  vec_op<OP_NEG_R>(c, N, p, sc, false);
  project(c, in, p.g, N, sp);
  vec_op<OP_INIT>(c, N, p, sc, true);
  if (prec) {
    apply_prec();
    copy(col(p.z, N), col(p.w, N), c.s);
    vec_op<OP_RHO>(c, N, p, sc, true);
  }
  JdResult res;
  std::vector<double> hist;
  double hs[J_COUNT];
  c.d2h(hs, sc, sizeof(hs));
  c.sync();
  if (hs[J_BREAK] != 0.0) res.reason = 4;
  for (int k = 1; k <= in.max_inner && res.reason == 0; ++k) {
    spmm(At, 1, p.w + n, p.y, false, c.s);
    spmm(A, 1, p.w, p.y + n, false, c.s);
    c.st->mv_stage2 += 1;
    vec_op<OP_SHIFT>(c, N, p, sc, false);
    project(c, in, p.q, N, sp);
    vec_op<OP_SIG>(c, N, p, sc, true);
    vec_op<OP_G>(c, N, p, sc, true);
    vec_op<OP_UPD>(c, N, p, sc, true);
    c.d2h(hs, sc, sizeof(hs));
    c.sync();
    if (hs[J_BREAK] != 0.0) {
      res.steps = k - 1;
      res.reason = 4;
      break;
    }
    res.steps = k;
    const double est = hs[J_EST];
    hist.push_back(est);
    if (est < in.thr) {
      res.reason = 1;
    } else if (hs[J_SN] < 0.1 * est) {
      res.reason = 2;
    } else if (hist.size() > 20) {
      const double recent = *std::min_element(hist.end() - 20, hist.end());
      const double before = *std::min_element(hist.begin(), hist.end() - 20);
      if (recent > 0.99 * before) res.reason = 3;
    }
    if (res.reason == 0 && prec && k < in.max_inner) {
      apply_prec();
      vec_op<OP_RHO>(c, N, p, sc, true);
      vec_op<OP_W>(c, N, p, sc, false);
    }
  }
  c.st->inner2 += res.steps;
  project(c, in, p.t, N, sp);
  copy(col(p.t, N), tout, c.s);
  return res;
}

double triplet_residual(Ctx &c, const double *x, const double *R, int ldx, int64_t n, int64_t N,
                        double theta, SmallPool &sp) {
  double *nrm = sp.vec(18);
  Tall<double> xv;
  xv.p = const_cast<double *>(x);
  xv.rows = N;
  xv.cols = 1;
  xv.rs = ldx;
  xv.cs = 1;
  colnorm2(xv, 0, n, nrm, c.sc, c.s);
  colnorm2(xv, n, N, nrm + 1, c.sc, c.s);
  double h[2];
  c.d2h(h, nrm, sizeof(h));
  c.sync();
  if (!(h[0] > 0.0) || !(h[1] > 0.0)) return INFINITY;
  const int nb = jd_blocks(N);
  k_jd_trip<<<nb, kJdThreads, 0, c.s>>>(x, R, ldx, n, N, theta, nrm, c.sc.part);
  PHS_CHECK_LAUNCH();
  k_jd_total<<<1, 64, 0, c.s>>>(c.sc.part, nb, nrm + 2);
  PHS_CHECK_LAUNCH();
  double t2 = 0.0;
  c.d2h(&t2, nrm + 2, sizeof(double));
  c.sync();
  return std::sqrt(std::max(t2, 0.0));
}

}  // namespace phs
