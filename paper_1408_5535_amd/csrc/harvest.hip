// Harvest of training pairs for the learned preconditioner: stage-1 Ritz
// blocks are snapshotted and their exact corrections computed by a batched
// projected conjugate-gradient solve of
//   (I - Q Q^T)(C - rho theta_j I)(I - Q Q^T) t_j = r_j,  t_j orthogonal to Q,
// Q = [X_lock, X_block], one column per Ritz pair with its own theta_j.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "harvest.hpp"

namespace phs {

// alpha_j = rr_j / (p_j^T A p_j); non-positive curvature ends column j
__global__ void k_cg_alpha(int nb, const double *G, int ldg, const double *rr, double *alpha,
                           int *active, int *fail) {
  int j = threadIdx.x;
  if (j >= nb) return;
  double pap = G[j + (int64_t)j * ldg];
  if (!active[j]) {
    alpha[j] = 0.0;
  } else if (!(pap > 0.0)) {
    alpha[j] = 0.0;
    active[j] = 0;
    fail[j] = 1;
  } else {
    alpha[j] = rr[j] / pap;
  }
}

// beta_j = rr_new / rr; convergence at ||res|| <= tol ||b||
__global__ void k_cg_beta(int nb, const double *rrn, double *rr, const double *rr0, double tol,
                          double *beta, int *active, int *done) {
  int j = threadIdx.x;
  if (j >= nb) return;
  if (!active[j]) {
    beta[j] = 0.0;
    return;
  }
  beta[j] = rr[j] > 0 ? rrn[j] / rr[j] : 0.0;
  rr[j] = rrn[j];
  if (sqrt(rrn[j]) <= tol * sqrt(rr0[j])) {
    done[j] = 1;
    active[j] = 0;
  }
}

// T += alpha P ; Res -= alpha AP   (row-major, stride bw)
__global__ void k_cg_update(int64_t n, int nb, int bw, const double *alpha, const double *P,
                            const double *AP, double *T, double *Res) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nb;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / nb;
    int j = (int)(e % nb);
    int64_t q = i * bw + j;
    T[q] += alpha[j] * P[q];
    Res[q] -= alpha[j] * AP[q];
  }
}

// P = Res + beta P for active columns, 0 otherwise
__global__ void k_cg_dir(int64_t n, int nb, int bw, const double *beta, const int *active,
                         const double *Res, double *P) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nb;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / nb;
    int j = (int)(e % nb);
    int64_t q = i * bw + j;
    P[q] = active[j] ? Res[q] + beta[j] * P[q] : 0.0;
  }
}

static Tall<double> rmv_(double *p, int64_t rows, int cols, int bw) {
  Tall<double> t;
  t.p = p;
  t.rows = rows;
  t.cols = cols;
  t.rs = bw;
  t.cs = 1;
  return t;
}

void carve_cg(Arena &ar, int64_t m, int64_t n, int bw, CgBufs &cb) {
  cb.P = ar.take<double>(n * bw);
  cb.AP = ar.take<double>(n * bw);
  cb.Res = ar.take<double>(n * bw);
  cb.T = ar.take<double>(n * bw);
  cb.Y = ar.take<double>(m * bw);
  cb.v = ar.take<double>(1024);
  cb.flags = ar.take<int>(256);
}

std::vector<int> projected_cg_block(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                                    const double *Xl, int nl, const double *Xb, int nb, int bw,
                                    const double *theta, double shift_scale, const double *R,
                                    double tol, int maxit,
                                    CgBufs &cb, SmallPool &sp) {
  const int64_t n = A.n;
  const int ld = kSP;
  double *G = sp.mat(35), *Gp = sp.mat(36), *Dn = sp.mat(37);
  double *rr = cb.v, *rr0 = cb.v + 64, *rrn = cb.v + 128, *alpha = cb.v + 192,
         *beta = cb.v + 256, *ones = cb.v + 320;
  int *active = cb.flags, *fail = cb.flags + 64, *done = cb.flags + 128;
  const Tall<double> Q1 = cm(const_cast<double *>(Xl), n, nl, n);
  const Tall<double> Q2 = rmv_(const_cast<double *>(Xb), n, nb, bw);
  auto proj = [&](double *V) {
    Tall<double> Vv = rmv_(V, n, nb, bw);
    tn(Q1, Q2, Vv, G, ld, c.sc, c.s);
    nn(Q1, Q2, G, ld, -1.0, Vv, 1.0, c.s);
  };
  {
    // right-hand side +r: T = M r with M the inverse of the projected
    // operator (the sign of a preconditioned residual)
    std::vector<double> dn((size_t)kSP * nb, 0.0), mo(nb, 1.0);
    for (int j = 0; j < nb; ++j) dn[j + (size_t)j * kSP] = -shift_scale * theta[j];
    c.h2d(Dn, dn.data(), dn.size() * sizeof(double));
    c.h2d(ones, mo.data(), nb * sizeof(double));
    std::vector<int> a(64, 0);
    for (int j = 0; j < nb; ++j) a[j] = 1;
    c.h2d(active, a.data(), 64 * sizeof(int));
    std::vector<int> z(128, 0);
    c.h2d(fail, z.data(), 128 * sizeof(int));
  }
  // Res = proj(R), T = 0, P = Res
  copy(rmv_(const_cast<double *>(R), n, nb, bw), rmv_(cb.Res, n, nb, bw), c.s);
  proj(cb.Res);
  scale_cols(rmv_(cb.Res, n, nb, bw), ones, c.s);
  PHS_HIP(hipMemsetAsync(cb.T, 0, n * bw * sizeof(double), c.s));
  PHS_HIP(hipMemsetAsync(cb.P, 0, n * bw * sizeof(double), c.s));
  copy(rmv_(cb.Res, n, nb, bw), rmv_(cb.P, n, nb, bw), c.s);
  colnorm2(rmv_(cb.Res, n, nb, bw), 0, n, rr, c.sc, c.s);
  copy(cm(rr, nb, 1, nb), cm(rr0, nb, 1, nb), c.s);
  // no iterations asked: pairs without exact targets (T = 0), for training
  // objectives that need none
  if (maxit == 0) return std::vector<int>(nb, 1);
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(n * nb, 256), 4096);
  for (int it = 1; it <= maxit; ++it) {
    proj(cb.P);
    spmm(A, bw, cb.P, cb.Y, false, c.s);
    spmm(At, bw, cb.Y, cb.AP, false, c.s);
    nn(rmv_(cb.P, n, nb, bw), cm<double>(nullptr, n, 0, n), Dn, ld, 1.0, rmv_(cb.AP, n, nb, bw),
       1.0, c.s);
    proj(cb.AP);
    c.st->mv_prec += nb;
    tn(rmv_(cb.P, n, nb, bw), cm<double>(nullptr, n, 0, n), rmv_(cb.AP, n, nb, bw), Gp, ld, c.sc,
       c.s);
    k_cg_alpha<<<1, 64, 0, c.s>>>(nb, Gp, ld, rr, alpha, active, fail);
    k_cg_update<<<grid, 256, 0, c.s>>>(n, nb, bw, alpha, cb.P, cb.AP, cb.T, cb.Res);
    colnorm2(rmv_(cb.Res, n, nb, bw), 0, n, rrn, c.sc, c.s);
    k_cg_beta<<<1, 64, 0, c.s>>>(nb, rrn, rr, rr0, tol, beta, active, done);
    k_cg_dir<<<grid, 256, 0, c.s>>>(n, nb, bw, beta, active, cb.Res, cb.P);
    PHS_CHECK_LAUNCH();
    if (it % 10 == 0 || it == maxit) {
      int h[64];
      c.d2h(h, active, nb * sizeof(int));
      c.sync();
      bool any = false;
      for (int j = 0; j < nb; ++j) any = any || h[j];
      if (!any) break;
    }
  }
  proj(cb.T);
  int hd[64], hf[64];
  c.d2h(hd, done, nb * sizeof(int));
  c.d2h(hf, fail, nb * sizeof(int));
  c.sync();
  std::vector<int> ok(nb);
  for (int j = 0; j < nb; ++j) ok[j] = hd[j] && !hf[j];
  return ok;
}

}  // namespace phs
