// PHSVDS host orchestration: stage 1 (block GD+k on C = A^T A, Algorithm 1
// with the dynamic tolerance of Section 3.1), the post-processing
// Rayleigh-Ritz (Section 3.1), stage 2 (GD+k with the refined projection on
// B = [0 A^T; A 0], Algorithm 2) and the final float64 residual check
// (Section 5).  Every numerical step runs in the device kernels; the host
// only reads Ritz values, residual norms and dependency flags (a few
// hundred bytes per iteration) to take the method's control decisions.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "jdqmr.hpp"
#include "prof.hpp"

namespace phs {

constexpr size_t kPinBytes = 64 * 1024;

void Ctx::d2h(void *h, const void *d, size_t bytes) {
  if (!pin_) PHS_HIP(hipHostMalloc((void **)&pin_, kPinBytes, hipHostMallocDefault));
  const size_t off = (pin_used_ + 15) & ~(size_t)15;
  if (off + bytes > kPinBytes) {  // larger than the staging buffer: direct copy
    PHS_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
    PHS_HIP(hipStreamSynchronize(s));
    return;
  }
  PHS_HIP(hipMemcpyAsync(pin_ + off, d, bytes, hipMemcpyDeviceToHost, s));
  pending_.push_back({h, off, bytes});
  pin_used_ = off + bytes;
}
void Ctx::sync() {
  PHS_HIP(hipStreamSynchronize(s));
  for (const Pending &q : pending_) std::memcpy(q.h, pin_ + q.off, q.bytes);
  pending_.clear();
  pin_used_ = 0;
}
Ctx::~Ctx() {
  if (pin_) (void)hipHostFree(pin_);
}
void Ctx::h2d(void *d, const void *h, size_t bytes) {
  // pageable source: the runtime stages it before returning
  PHS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  PHS_HIP(hipStreamSynchronize(s));
}

template <typename T>
static Tall<T> rmv(T *p, int64_t rows, int cols, int bw) {
  Tall<T> t;
  t.p = p;
  t.rows = rows;
  t.cols = cols;
  t.rs = bw;
  t.cs = 1;
  return t;
}
template <typename T>
static Tall<T> none(int64_t rows) {
  Tall<T> t;
  t.p = nullptr;
  t.rows = rows;
  t.cols = 0;
  t.rs = 1;
  t.cs = 1;
  return t;
}

// ------------------------------------------------------------------------
// Block orthonormalisation: T (n x nb, row-major stride bw) against the
// bases [B1 | B2] by two Gram-Schmidt passes (a third when the second still
// removes more than half), then CholQR2 within the block.  Columns whose
// norm drops by more than 1/dep_drop are replaced by random vectors; a
// Cholesky breakdown falls back to shifted CholQR3.
template <typename T>
void orth_block(Ctx &c, T *&Tb, T *&T2b, int64_t n, int nb, int bw, const Tall<T> &B1,
                const Tall<T> &B2, double dep_drop, SmallPool &sp) {
  const Tall<T> none1 = none<T>(n);
  const double u = std::is_same<T, float>::value ? kEps32 / 2 : kEps64 / 2;
  double *n0 = sp.vec(0), *n1 = sp.vec(1);
  double *G = sp.mat(0), *Gram = sp.mat(1), *R1 = sp.mat(2), *Ri1 = sp.mat(3);
  const int ld = kSP;
  bool shifted = false;
  for (int attempt = 0; attempt < 6; ++attempt) {
    Tall<T> Tv = rmv(Tb, n, nb, bw);
    colnorm2(Tv, 0, n, n0, c.sc, c.s);
    int passes = 2;
    for (int pass = 0; pass < passes; ++pass) {
      if (B1.cols + B2.cols > 0) {
        tn(B1, B2, Tv, G, ld, c.sc, c.s);
        nn(B1, B2, G, ld, -1.0, Tv, 1.0, c.s);
      }
      if (pass == 0) colnorm2(Tv, 0, n, n1, c.sc, c.s);
    }
    tn(Tv, none1, Tv, Gram, ld, c.sc, c.s);
    double h0[64], h1[64], hg[64 * 64];
    c.d2h(h0, n0, nb * sizeof(double));
    c.d2h(h1, n1, nb * sizeof(double));
    c.d2h(hg, Gram, (size_t)ld * nb * sizeof(double));
    c.sync();
    bool third = false;
    std::vector<int> dep;
    for (int j = 0; j < nb; ++j) {
      double a0 = std::sqrt(std::max(h0[j], 0.0)), a1 = std::sqrt(std::max(h1[j], 0.0));
      double a2 = std::sqrt(std::max(hg[j + j * ld], 0.0));
      if (!(a0 > 0.0) || !(a2 > dep_drop * a0) || !std::isfinite(a2)) {
        dep.push_back(j);
      } else if (a2 < 0.5 * a1 && B1.cols + B2.cols > 0) {
        third = true;
      }
    }
    if (!dep.empty()) {
      for (int j : dep) {
        Tall<T> col = rmv(Tb + j, n, 1, bw);
        fill_random(col, c.seed, 1000000 + (c.nrand++) * 64, c.s);
        ++c.st->dep_cols;
      }
      continue;
    }
    if (third) {
      tn(B1, B2, Tv, G, ld, c.sc, c.s);
      nn(B1, B2, G, ld, -1.0, Tv, 1.0, c.s);
      tn(Tv, none1, Tv, Gram, ld, c.sc, c.s);
    }
    // CholQR: two passes, or shifted CholQR3 after a breakdown
    int npass = 2;
    double shift = 0.0;
    if (shifted) {
      double tr = 0.0;
      for (int j = 0; j < nb; ++j) tr += hg[j + j * ld];
      shift = 11.0 * ((double)n * nb + (double)nb * (nb + 1)) * u * tr;
      npass = 3;
    }
    bool broke = false;
    for (int q = 0; q < npass; ++q) {
      if (q > 0) tn(rmv(Tb, n, nb, bw), none1, rmv(Tb, n, nb, bw), Gram, ld, c.sc, c.s);
      chol_inv(Gram, ld, nb, q == 0 ? shift : 0.0, R1, Ri1, ld, c.sc.flag, c.s);
      nn(rmv(Tb, n, nb, bw), none1, Ri1, ld, 1.0, rmv(T2b, n, nb, bw), 0.0, c.s);
      std::swap(Tb, T2b);
      int fl = 0;
      c.d2h(&fl, c.sc.flag, sizeof(int));
      c.sync();
      if (fl) {
        broke = true;
        break;
      }
    }
    if (!broke) return;
    shifted = true;
  }
  throw Error(kEbreak, "orthogonalisation failed to produce an independent block");
}
template void orth_block<float>(Ctx &, float *&, float *&, int64_t, int, int, const Tall<float> &,
                                const Tall<float> &, double, SmallPool &);
template void orth_block<double>(Ctx &, double *&, double *&, int64_t, int, int,
                                 const Tall<double> &, const Tall<double> &, double, SmallPool &);

// Left-looking Gram-Schmidt (two passes) on columns [j0, j1) of a
// column-major X against all previous columns; R(:, j) accumulates the
// coefficients when R != nullptr.  Zero (or, if `random_dep`, random)
// replacements for dependent columns.
void cgs_cols(Ctx &c, double *X, int64_t rows, int64_t ld, int j0, int j1, double *R, int ldr,
              bool random_dep, SmallPool &sp) {
  double *g = sp.vec(2), *n2 = sp.vec(3), *n0 = sp.vec(4);
  for (int j = j0; j < j1; ++j) {
    Tall<double> xj = cm(X + (int64_t)j * ld, rows, 1, rows);
    for (int attempt = 0; attempt < 4; ++attempt) {
      if (random_dep) colnorm2(xj, 0, rows, n0, c.sc, c.s);
      if (j > 0) {
        Tall<double> Q = cm(X, rows, j, ld);
        for (int pass = 0; pass < 2; ++pass) {
          tn(Q, none<double>(rows), xj, g, kSP, c.sc, c.s);
          nn(Q, none<double>(rows), g, kSP, -1.0, xj, 1.0, c.s);
          if (R) small_add(j, 1, 1.0, g, kSP, R + (int64_t)j * ldr, ldr, c.s);
        }
      }
      colnorm2(xj, 0, rows, n2, c.sc, c.s);
      if (random_dep) {
        double h[2];
        c.d2h(h, n0, sizeof(double));
        c.d2h(h + 1, n2, sizeof(double));
        c.sync();
        if (!(h[0] > 0.0) || !(std::sqrt(h[1]) > kDepDropF64 * std::sqrt(h[0]))) {
          fill_random(xj, c.seed, 2000000 + (c.nrand++) * 64, c.s);
          ++c.st->dep_cols;
          continue;
        }
      }
      break;
    }
    norm_col(X + (int64_t)j * ld, rows, n2, 1e-300, R ? R + j + (int64_t)j * ldr : nullptr, c.s);
  }
}

// ------------------------------------------------------------------------
// Stage 1: block GD+k on C = A^T A in working precision T.
//
// The steady-state iteration reads the device once: a packed status block
// with the Ritz values, the residual norms and the orthogonality
// diagnostics of the previous basis expansion.  That expansion is done
// without host checks; if its diagnostics show a dependent column or a
// Cholesky breakdown, it is rolled back (the basis, W and H below column p
// are untouched by it) and redone by the checked path.
template <typename T>
Stage1Result run_stage1(Ctx &c, const SpMat<T> &A, const SpMat<T> &At, const Stage1Params &P,
                        Stage1Bufs<T> &bf, SmallPool &sp) {
  const int64_t n = A.n;
  const int k = P.k, b = P.b, bw = P.bw, pmax = P.pmax, pmin = P.pmin;
  const bool largest = P.largest;
  const bool fp32 = std::is_same<T, float>::value;
  const double eps = fp32 ? kEps32 : kEps64;
  const double dep_drop = fp32 ? 1e-4 : kDepDropF64;
  const int ld = kSP;
  const int64_t ldv = basis_ld(n);  // leading dimension of V and W
  T *V[2] = {bf.V[0], bf.V[1]}, *W[2] = {bf.W[0], bf.W[1]};
  int cur = 0, p = 0, nl = 0, nprev = 0;
  T *Tb = bf.Tb, *T2b = bf.T2b, *Rb = bf.Rb;
  double *H = sp.mat(4), *Sa = sp.mat(5), *Y = sp.mat(6), *Hs = sp.mat(7), *prev = sp.mat(8),
         *prev2 = sp.mat(9), *Gb = sp.mat(10), *Sb = sp.mat(34), *G = sp.mat(0),
         *Gram = sp.mat(1), *R1 = sp.mat(2), *Ri1 = sp.mat(3), *G2 = sp.mat(38);
  // packed status block: theta | rn2 | n0 | n1 | n2 | rho2 | flags
  double *stat = sp.vec(22);
  double *theta = stat, *rn2 = stat + 64, *sn0 = stat + 128, *sn1 = stat + 160,
         *sn2v = stat + 192, *rho2 = stat + 224;
  int *sflag = reinterpret_cast<int *>(stat + 256);
  const int kStat = 260;
  int *cnt = c.sc.flag + 8;
  Stage1Result res;
  res.sn2 = P.anorm > 0 ? P.anorm * P.anorm : P.sn2_init;
  std::vector<double> rho_h(bw, 0.0);
  int rho_age = 1 << 30;
  bool warm = false;
  bool gnn_off = false;
  std::vector<double> pc_hist;
  int pw = 0;                 // size of the warm-start eigenvector block
  int pend_nb = 0, pend_p = 0;  // unchecked expansion: width, basis size before
  int64_t last_rebuild = -1000000;  // iteration of the last W = C V rebuild
  int hist_nl = -1;

  // the two products of C X are timed as one group when profiling
  const int pkind = fp32 ? kProfSpmm32 : kProfSpmm64;
  const double cbytes = spmm_bytes(A, bw) + spmm_bytes(At, bw);
  auto applyC = [&](T *X, int nb) {
    if (P.opC) {
      P.opC(X, bf.WTb, bw);
    } else {
      prof_group_begin(pkind, c.s, 2);
      spmm(A, bw, X, bf.Yb, false, c.s);
      spmm(At, bw, bf.Yb, bf.WTb, false, c.s);
      prof_group_end(pkind, c.s, cbytes);
    }
    c.st->mv_stage1 += nb;
  };
  // W_T = C T goes straight into the new columns of W; V's new columns are
  // copied from T unless the caller has written them already
  auto append = [&](int nb, bool v_written) {
    if (P.opC) {
      P.opC(Tb, bf.WTb, bw);
      copy(rmv(bf.WTb, n, nb, bw), cm(W[cur] + (int64_t)p * ldv, n, nb, ldv), c.s);
    } else {
      prof_group_begin(pkind, c.s, 2);
      spmm(A, bw, Tb, bf.Yb, false, c.s);
      if (At.op) {  // an operator writes row-major blocks only
        spmm(At, bw, bf.Yb, bf.WTb, false, c.s);
        copy(rmv(bf.WTb, n, nb, bw), cm(W[cur] + (int64_t)p * ldv, n, nb, ldv), c.s);
      } else {
        spmm(At, bw, bf.Yb, W[cur] + (int64_t)p * ldv, false, c.s, ldv, nb);
      }
      prof_group_end(pkind, c.s, cbytes);
    }
    c.st->mv_stage1 += nb;
    if (!v_written) copy(rmv(Tb, n, nb, bw), cm(V[cur] + (int64_t)p * ldv, n, nb, ldv), c.s);
    // border of H; the previous block's coefficients have no component on
    // the new columns
    TnParts gp;
    tn(cm(V[cur], n, p + nb, ldv), none<T>(n), cm(W[cur] + (int64_t)p * ldv, n, nb, ldv), Gb, ld,
       c.sc, c.s, &gp);
    reduce_border(gp, H, ld, nprev ? prev : nullptr, ld, nprev, c.s);
    p += nb;
  };
  // checked expansion (host decisions on dependence and breakdown)
  auto expand = [&](int nb) {
    orth_block(c, Tb, T2b, n, nb, bw, cm(bf.Xl, n, nl, n), cm(V[cur], n, p, ldv), dep_drop, sp);
    append(nb, false);
  };
  // unchecked expansion: CGS2 + CholQR2, diagnostics left in the status
  // block.  The correction itself is left untouched (a rollback redoes the
  // expansion from it); the passes work in the two other block buffers and
  // the last one also writes the new columns of V.
  auto expand_fast = [&](int nb) {
    T *orig = Tb, *w1 = T2b, *w2 = bf.Fb;
    const Tall<T> B1 = cm(bf.Xl, n, nl, n), B2 = cm(V[cur], n, p, ldv);
    const Tall<T> T0 = rmv(orig, n, nb, bw), T1 = rmv(w1, n, nb, bw), T2 = rmv(w2, n, nb, bw);
    // classical Gram-Schmidt, always twice: a single pass that cancels
    // little (unpreconditioned corrections are nearly orthogonal to V
    // already) still left enough of V in T to stall the largest-mode
    // iteration at the 1e-12 level
    // widths 1, 2 and 4: the second update and the first CholQR product
    // also leave the Gram partials of their output (no separate X^T X pass;
    // at width 8 the 64 float64 accumulators would not fit the registers)
    const bool fused = nb == 1 || nb == 2 || nb == 4;
    TnParts gp;
    tn(B1, B2, T0, G, ld, c.sc, c.s);
    nn(B1, B2, G, ld, -1.0, T1, 1.0, c.s, &T0);
    tn(B1, B2, T1, G2, ld, c.sc, c.s);
    nn<T>(B1, B2, G2, ld, -1.0, T1, 1.0, c.s, nullptr, nullptr, &c.sc, fused ? &gp : nullptr);
    // CholQR2; the first Cholesky also leaves the squared norms of the
    // block before, between and after the two passes in the status block
    CgsDiag dg;
    dg.H1 = G;
    dg.H2 = G2;
    dg.ldh = ld;
    dg.nh = nl + p;
    dg.n0 = sn0;
    dg.n1 = sn1;
    dg.n2 = sn2v;
    // an X^T X Gram (width 8 and up) is reduced across blocks before the
    // Cholesky: its partials (one per block of the product, up to 1024) are
    // too many for the single workgroup of the Cholesky kernel to sum fast
    if (!fused) tn(T1, none<T>(n), T1, Gram, ld, c.sc, c.s);
    chol_inv(Gram, ld, nb, 0.0, R1, Ri1, ld, sflag, c.s, &dg, fused ? &gp : nullptr);
    nn<T>(T1, none<T>(n), Ri1, ld, 1.0, T2, 0.0, c.s, nullptr, nullptr, &c.sc,
          fused ? &gp : nullptr);
    if (!fused) tn(T2, none<T>(n), T2, Gram, ld, c.sc, c.s);
    chol_inv(Gram, ld, nb, 0.0, R1, Ri1, ld, sflag + 1, c.s, nullptr, fused ? &gp : nullptr);
    const Tall<T> Vn = cm(V[cur] + (int64_t)p * ldv, n, nb, ldv);
    nn<T>(T2, none<T>(n), Ri1, ld, 1.0, T1, 0.0, c.s, nullptr, &Vn);
    Tb = w1;
    T2b = w2;
    bf.Fb = orig;
    pend_nb = nb;
    pend_p = p;
    append(nb, true);
  };

  // initial block (Section 5: ones(n,1)/sqrt(n) plus seeded random columns),
  // or a caller-given basis, expanded in chunks of the block width
  {
    int w0 = P.init_cols > 0 ? P.init_cols : b;
    for (int c0 = 0; c0 < w0; c0 += bw) {
      int w = std::min(bw, w0 - c0);
      if (P.init64) {
        copy(cm(const_cast<double *>(P.init64) + (int64_t)c0 * n, n, w, n), rmv(Tb, n, w, bw), c.s);
      } else if (P.init32) {
        copy(cm(const_cast<float *>(P.init32) + (int64_t)c0 * n, n, w, n), rmv(Tb, n, w, bw), c.s);
      } else {
        fill_random(rmv(Tb, n, w, bw), c.seed, 17 + c0, c.s);
        if (c0 == 0) fill_const_col(Tb, n, (int64_t)bw, 1.0 / std::sqrt((double)n), c.s);
      }
      expand(w);
    }
  }
  std::vector<double> hs(kStat), hist;
  const int L = std::max(100, 20 * ((pmax + b - 1) / b));
  int64_t it = 0;
  while (true) {
    ++it;
    double *S = Sa;
    const int nb = std::min(b, p);
    // eigenpairs this iteration uses: the block, or the p_min kept at a
    // restart; a lock recomputes all p
    const int nv = (p + nb > pmax) ? std::min(std::max(pmin, nb), p) : nb;
    // the largest Ritz value (the ||A|| estimate) in smallest mode: at
    // restarts and locks, and every eighth iteration; the running maximum
    // changes slowly and is only used for the stopping thresholds
    const bool want_top = !largest && (nv > nb || it % 8 == 1);
    syev_rr(H, ld, p, nv, largest, theta, S, ld, c.s, want_top);
    // a restart due this iteration goes first: the restarted basis starts
    // with this iteration's Ritz vectors (Y = [S(:, 0:p_min) | prev]), so
    // the Ritz block is its first nb columns and the Ritz kernel reads nb
    // columns of V and W instead of p.  The products go to the other
    // buffers; a lock, rebuild or rollback below discards them.
    const bool restart_due = p + nb > pmax;
    int hc = 0;
    if (restart_due) {
      restart_basis(S, ld, p, pmin, prev, ld, nprev, Y, ld, cnt, c.s);
      hc = std::min(pmin + nprev, p);  // restart_basis fills every column
      nn(cm(V[cur], n, p, ldv), none<T>(n), Y, ld, 1.0, cm(V[1 - cur], n, hc, ldv), 0.0, c.s);
      nn(cm(W[cur], n, p, ldv), none<T>(n), Y, ld, 1.0, cm(W[1 - cur], n, hc, ldv), 0.0, c.s);
      ritz(cm(V[1 - cur], n, nb, ldv), cm(W[1 - cur], n, nb, ldv), sp.eye(), ld, theta, bf.Xb, Rb,
           nb, bw, rn2, nullptr, 0, c.sc, c.s);
    } else {
      ritz(cm(V[cur], n, p, ldv), cm(W[cur], n, p, ldv), S, ld, theta, bf.Xb, Rb, nb, bw, rn2,
           nullptr, 0, c.sc, c.s);
    }
    const bool want_rho = fp32 && rho_age >= 10;
    if (want_rho) {
      // componentwise accuracy floor of float32 C x: || |A|^T |A| |x| ||
      spmm(A, bw, bf.Xb, bf.Yb, true, c.s);
      spmm(At, bw, bf.Yb, bf.WTb, true, c.s);
      colnorm2(rmv(bf.WTb, n, nb, bw), 0, n, rho2, c.sc, c.s);
      c.st->mv_floor += nb;
    }
    c.d2h(hs.data(), stat, kStat * sizeof(double));
    c.sync();
    const double *th_h = hs.data(), *rn_h = hs.data() + 64;
    if (want_rho) {
      for (int j = 0; j < nb; ++j) rho_h[j] = std::sqrt(std::max(hs[224 + j], 0.0));
      rho_age = 0;
    }
    ++rho_age;
    if (pend_nb) {
      // deferred check of the last expansion
      const int *fl = reinterpret_cast<const int *>(hs.data() + 256);
      bool bad = fl[0] || fl[1];
      for (int j = 0; j < pend_nb && !bad; ++j) {
        double a0 = std::sqrt(std::max(hs[128 + j], 0.0)), a1 = std::sqrt(std::max(hs[160 + j], 0.0));
        double a2 = std::sqrt(std::max(hs[192 + j], 0.0));
        if (!(a0 > 0.0) || !(a2 > dep_drop * a0) || !std::isfinite(a2) || a2 < 0.5 * a1) bad = true;
      }
      const int redo = pend_nb;
      pend_nb = 0;
      if (bad) {
        p = pend_p;
        std::swap(Tb, bf.Fb);  // the saved correction block
        expand(redo);
        warm = false;
        ++res.rollbacks;
        continue;
      }
    }
    // largest Ritz value so far: ||A||^2 estimate
    for (int j = 0; j < nv; ++j) res.sn2 = std::max(res.sn2, th_h[j]);
    if (want_top || nv >= p) res.sn2 = std::max(res.sn2, th_h[p - 1]);
    const double sn = std::sqrt(res.sn2);
    const int need = k - nl;
    if (c.verbose && it % 1000 == 0)
      std::fprintf(stderr,
                   "[phsvds] stage 1%s iteration %lld: locked %d/%d, products %lld, "
                   "theta_0 %.9e, ||r_0|| %.3e\n",
                   fp32 ? " (float32)" : "", (long long)it, nl, k,
                   (long long)c.st->mv_stage1, th_h[0], std::sqrt(std::max(rn_h[0], 0.0)));
    if (P.snap) P.snap(it, bf.Xb, Rb, th_h, nb, bf.Xl, nl);
    if (P.hist) {
      if (hist_nl >= 0 && nl != hist_nl) P.hist->push_back(NAN);
      hist_nl = nl;
      const double s0 = std::sqrt(std::max(th_h[0], 1e-300));
      P.hist->push_back(std::log(std::max(std::sqrt(std::max(rn_h[0], 0.0)) / s0, 1e-300)));
    }
    if (P.gnn && !gnn_off && P.gnn_window > 0) {
      // safeguard of the learned preconditioner: fall back to Jacobi when the
      // leading residual has not halved within a window of iterations
      pc_hist.push_back(std::sqrt(std::max(rn_h[0], 0.0)));
      const int Lf = P.gnn_window;
      if ((int)pc_hist.size() >= 2 * Lf) {
        double a = *std::min_element(pc_hist.end() - Lf, pc_hist.end());
        double bprev = *std::min_element(pc_hist.end() - 2 * Lf, pc_hist.end() - Lf);
        if (a > 0.5 * bprev) {
          gnn_off = true;
          ++res.fallbacks;
        }
      }
    }
    std::vector<int> conv;
    auto floor_of = [&](int i) {
      return fp32 ? P.floor * eps * std::max(rho_h[i], 0.0) : P.floor * eps * res.sn2;
    };
    // the user-tolerance part of the test (Section 3.1); in shift-invert
    // its image on C^-1: C r' = -mu r_C for r' = C^-1 x - mu x
    auto rel_of = [&](int i) {
      const double si = std::sqrt(std::max(th_h[i], 0.0));
      return P.si_anorm > 0 ? P.tol * si / P.si_anorm : P.tol * si * sn;
    };
    for (int i = 0; i < std::min(nb, need); ++i) {
      double thr = std::max(rel_of(i), floor_of(i));
      if (std::sqrt(std::max(rn_h[i], 0.0)) < thr) conv.push_back(i);
    }
    bool stag = false;
    if (conv.empty() && need > 0) {
      double fl0 = floor_of(0);
      if (rel_of(0) < fl0) {
        double r0 = std::sqrt(std::max(rn_h[0], 0.0));
        hist.push_back(r0);
        if ((int)hist.size() > 2 * L && r0 < 10.0 * fl0) {
          double a = *std::min_element(hist.end() - L, hist.end());
          double bmin = *std::min_element(hist.begin(), hist.end() - L);
          if (a > 0.9 * bmin) {
            conv.push_back(0);
            stag = true;
          }
        }
      }
    }
    if (!conv.empty() && !stag) {
      // lock on the explicit residual C x - theta x only: the recurrence
      // W s - theta x drifts from it over restarts; on a mismatch rebuild
      // W = C V and H = V^T W
      applyC(bf.Xb, nb);
      std::vector<double> dneg((size_t)kSP * nb, 0.0);
      for (int j = 0; j < nb; ++j) dneg[j + (size_t)j * kSP] = -th_h[j];
      c.h2d(sp.mat(33), dneg.data(), dneg.size() * sizeof(double));
      nn(rmv(bf.Xb, n, nb, bw), none<T>(n), sp.mat(33), ld, 1.0, rmv(bf.WTb, n, nb, bw), 1.0,
         c.s);
      colnorm2(rmv(bf.WTb, n, nb, bw), 0, n, stat + 300, c.sc, c.s);
      double rt[64];
      c.d2h(rt, stat + 300, nb * sizeof(double));
      c.sync();
      bool all_ok = true;
      for (int i : conv) {
        double thr = std::max(rel_of(i), floor_of(i));
        if (!(std::sqrt(std::max(rt[i], 0.0)) < thr)) all_ok = false;
      }
      if (!all_ok && it - last_rebuild <= 10) {
        // rebuilt within the last 10 iterations: the two residuals differ
        // by rounding only, so iterate on without locking
        conv.clear();
      } else if (!all_ok) {
        last_rebuild = it;
        for (int c0 = 0; c0 < p; c0 += bw) {
          int w = std::min(bw, p - c0);
          copy(cm(V[cur] + (int64_t)c0 * ldv, n, w, ldv), rmv(Tb, n, w, bw), c.s);
          applyC(Tb, w);
          copy(rmv(bf.WTb, n, w, bw), cm(W[cur] + (int64_t)c0 * ldv, n, w, ldv), c.s);
        }
        for (int c0 = 0; c0 < p; c0 += 32) {
          int w = std::min(32, p - c0);
          tn(cm(V[cur], n, p, ldv), none<T>(n), cm(W[cur] + (int64_t)c0 * ldv, n, w, ldv),
             H + (int64_t)c0 * ld, ld, c.sc, c.s);
        }
        nprev = 0;
        warm = false;
        ++res.refreshes;
        continue;
      }
    }
    if (!conv.empty()) {
      hist.clear();
      pc_hist.clear();
      for (int i : conv) {
        copy(rmv(bf.Xb + i, n, 1, bw), cm(bf.Xl + (int64_t)nl * n, n, 1, n), c.s);
        res.theta.push_back(th_h[i]);
        res.res.push_back(std::sqrt(std::max(rn_h[i], 0.0)));
        res.tight.push_back(std::sqrt(std::max(rn_h[i], 0.0)) <
                            P.tol * std::sqrt(std::max(th_h[i], 0.0)) * sn);
        ++nl;
        if (c.verbose)
          std::fprintf(stderr, "[phsvds] stage 1 iteration %lld: locked %d/%d, theta %.12e\n",
                       (long long)it, nl, k, th_h[i]);
      }
      // kept basis: an orthonormal basis of the complement of the locked
      // coefficient vectors, starting with the other computed Ritz vectors
      // and completed by coordinate vectors; H is projected onto it
      const int nk = p - (int)conv.size();
      if (nk > 0) {
        std::vector<int> order(conv.begin(), conv.end());
        for (int j = 0; j < nv; ++j)
          if (std::find(conv.begin(), conv.end(), j) == conv.end()) order.push_back(j);
        c.h2d(c.didx, order.data(), nv * sizeof(int));
        gather_cols(S, ld, p, c.didx, nv, Hs, ld, c.s);
        restart_basis(Hs, ld, p, nv, sp.eye(), ld, p - nv, Y, ld, cnt, c.s);
        const double *Yk = Y + (int64_t)conv.size() * ld;
        nn(cm(V[cur], n, p, ldv), none<T>(n), Yk, ld, 1.0, cm(V[1 - cur], n, nk, ldv), 0.0, c.s);
        nn(cm(W[cur], n, p, ldv), none<T>(n), Yk, ld, 1.0, cm(W[1 - cur], n, nk, ldv), 0.0, c.s);
        restart_project(H, ld, p, Yk, ld, nk, nullptr, ld, 0, nullptr, ld, c.s);
        cur = 1 - cur;
      }
      p = nk;
      nprev = 0;
      warm = false;
      if (nl >= k) {
        res.converged = true;
        break;
      }
      if (p == 0) {
        fill_random(rmv(Tb, n, b, bw), c.seed, 3000000 + (c.nrand++) * 64, c.s);
        expand(b);
      }
      continue;
    }
    const bool out_of_budget = res.restarts > P.max_restarts ||
                               c.over_budget() ||
                               (P.max_iters > 0 && it > P.max_iters) || (P.stop && P.stop());
    if (out_of_budget) {
      // the pairs still missing are returned as the leading unlocked Ritz
      // vectors of the current basis (best approximations)
      const int nbest = std::min(need, p);
      if (nbest > 0) {
        syev_rr(H, ld, p, nbest, largest, theta, S, ld, c.s);
        nn(cm(V[cur], n, p, ldv), none<T>(n), S, ld, 1.0, cm(bf.Xl + (int64_t)nl * n, n, nbest, n),
           0.0, c.s);
        res.best_theta.resize(nbest);
        c.d2h(res.best_theta.data(), theta, nbest * sizeof(double));
        c.sync();
      }
      res.nbest = std::max(nbest, 0);
      break;
    }
    // correction T = Prec(R)
    if (P.gnn && !gnn_off) {
      for (int j = 0; j < nb; ++j) {
        copy(rmv(Rb + j, n, 1, bw), cm(bf.Gs, n, 1, n), c.s);
        copy(rmv(bf.Xb + j, n, 1, bw), cm(bf.Gs + n, n, 1, n), c.s);
        P.gnn(bf.Gs, bf.Gs + n, th_h[j], bf.Gs + 2 * n);
        copy(cm(bf.Gs + 2 * n, n, 1, n), rmv(Tb + j, n, 1, bw), c.s);
      }
      c.st->mv_prec += 6 * nb;
    } else if (P.user) {
      // the caller's preconditioner on column-major copies of the block
      copy(rmv(Rb, n, nb, bw), cm(bf.Ub, n, nb, n), c.s);
      P.user(bf.Ub, bf.Ub + (int64_t)n * nb, nb, th_h);
      copy(cm(bf.Ub + (int64_t)n * nb, n, nb, n), rmv(Tb, n, nb, bw), c.s);
    } else if (P.jacobi_d) {
      jacobi_apply<T>(Rb, bf.Xb, P.jacobi_d, theta, n, nb, bw, true, Tb, c.sc, c.s);
    } else {
      std::swap(Tb, Rb);
    }
    if (restart_due) {
      // thick restart + the previous block (GD+k), its products formed
      // before the Ritz block; the count is min(p_min + nprev, p) by
      // construction of restart_basis
      restart_project(H, ld, p, Y, ld, hc, S, ld, nb, prev2, ld, c.s);
      std::swap(prev, prev2);
      nprev = nb;
      cur = 1 - cur;
      p = hc;
      ++res.restarts;
      warm = false;
    } else {
      copy(cm(S, p, nb, ld), cm(prev, p, nb, ld), c.s);  // this iteration's targets
      nprev = nb;
      warm = true;
      pw = p;
      std::swap(Sa, Sb);  // Sb now holds this iteration's eigenvectors
    }
    expand_fast(nb);
  }
  res.iters = it;
  res.nl = nl;
  res.p = p;
  // the basis leaves with leading dimension n (compacted into the other
  // buffer, which is free now, when the padded one differs)
  if (ldv != n && p > 0) copy(cm(V[cur], n, p, ldv), cm(V[1 - cur], n, p, n), c.s);
  res.Vrest = ldv != n ? V[1 - cur] : V[cur];
  bf.Tb = Tb;
  bf.T2b = T2b;
  bf.Rb = Rb;
  return res;
}
template Stage1Result run_stage1<float>(Ctx &, const SpMat<float> &, const SpMat<float> &,
                                        const Stage1Params &, Stage1Bufs<float> &, SmallPool &);
template Stage1Result run_stage1<double>(Ctx &, const SpMat<double> &, const SpMat<double> &,
                                         const Stage1Params &, Stage1Bufs<double> &,
                                         SmallPool &);

// ------------------------------------------------------------------------
// ||C x|| after `iters` steps of power iteration on C = A^T A from a
// counter-based random start, float64: a lower bound on ||A||^2.  x and z
// are n-vectors, y an m-vector (work space).
double power_norm2(Ctx &c, const SpMat<double> &A, const SpMat<double> &At, double *x, double *y,
                   double *z, int iters, SmallPool &sp) {
  const int64_t n = A.n;
  double *nrm = sp.vec(23), *f = sp.vec(23) + 8;
  fill_random(cm(x, n, 1, n), c.seed, 5000000 + (c.nrand++) * 64, c.s);
  double lam = 0.0, h[1];
  for (int it = 0; it <= iters; ++it) {
    colnorm2(cm(x, n, 1, n), 0, n, nrm, c.sc, c.s);
    c.d2h(h, nrm, sizeof(double));
    c.sync();
    const double nx = std::sqrt(std::max(h[0], 0.0));
    if (!(nx > 0.0)) break;
    if (it > 0) lam = nx;  // ||C x_prev||, x_prev of unit norm
    if (it == iters) break;
    const double inv = 1.0 / nx;
    c.h2d(f, &inv, sizeof(double));
    scale_cols(cm(x, n, 1, n), f, c.s);
    spmm(A, 1, x, y, false, c.s);
    spmm(At, 1, y, z, false, c.s);
    std::swap(x, z);
  }
  return lam;
}

// ------------------------------------------------------------------------
// Transition Rayleigh-Ritz on C over Z = orth([X_lock, leading restart
// vectors]), evaluated as the SVD of A Z (same Ritz pairs, no squaring).
void run_transition(Ctx &c, const SpMat<double> &A, const double *Xl, int k, const double *Vr,
                    int nvr, int pmin, double anorm, int bw, TransBufs &tb, SmallPool &sp,
                    std::vector<double> &shifts) {
  const int64_t n = A.n, m = A.m;
  const int extra = std::min(nvr, std::max(0, pmin - k));
  const int pz = k + extra;
  copy(cm(const_cast<double *>(Xl), n, k, n), cm(tb.Z, n, k, n), c.s);
  if (extra) copy(cm(const_cast<double *>(Vr), n, extra, n), cm(tb.Z + (int64_t)k * n, n, extra, n), c.s);
  cgs_cols(c, tb.Z, n, n, 0, pz, nullptr, 0, true, sp);
  for (int c0 = 0; c0 < pz; c0 += bw) {
    int w = std::min(bw, pz - c0);
    copy(cm(tb.Z + (int64_t)c0 * n, n, w, n), rmv(tb.Xn, n, w, bw), c.s);
    spmm(A, bw, tb.Xn, tb.Ym, false, c.s);
    copy(rmv(tb.Ym, m, w, bw), cm(tb.AZ + (int64_t)c0 * m, m, w, m), c.s);
  }
  c.st->mv_rr += pz;
  copy(cm(tb.AZ, m, pz, m), cm(tb.QZ, m, pz, m), c.s);
  cgs_cols(c, tb.QZ, m, m, 0, pz, nullptr, 0, false, sp);
  double *M = sp.mat(11), *Yv = sp.mat(12), *sv = sp.vec(8), *nrm = sp.vec(9);
  for (int c0 = 0; c0 < pz; c0 += 32) {
    int w = std::min(32, pz - c0);
    tn(cm(tb.QZ, m, pz, m), none<double>(m), cm(tb.AZ + (int64_t)c0 * m, m, w, m),
       M + (int64_t)c0 * kSP, kSP, c.sc, c.s);
  }
  svdj(M, kSP, pz, pz, sv, Yv, kSP, c.s);
  nn(cm(tb.Z, n, pz, n), none<double>(n), Yv, kSP, 1.0, cm(tb.Vt, n, k, n), 0.0, c.s);
  nn(cm(tb.AZ, m, pz, m), none<double>(m), Yv, kSP, 1.0, cm(tb.Ut, m, k, m), 0.0, c.s);
  shifts.resize(k);
  c.d2h(shifts.data(), sv, k * sizeof(double));
  finish_left(c, m, k, shifts, anorm, tb, sp);
}

// Left vectors u_i = A v_i / ||A v_i|| of the stage-2 seeds (tb.Ut holds
// A v_i on entry), random and orthogonalised against the others where
// sigma_i <= 10 eps ||A|| (Section 3.3: stage 1 gives them no accuracy).
void finish_left(Ctx &c, int64_t m, int k, const std::vector<double> &shifts, double anorm,
                 TransBufs &tb, SmallPool &sp) {
  double *nrm = sp.vec(9);
  colnorm2(cm(tb.Ut, m, k, m), 0, m, nrm, c.sc, c.s);
  std::vector<double> nh(k);
  c.d2h(nh.data(), nrm, k * sizeof(double));
  c.sync();
  std::vector<double> f(k);
  std::vector<int> tiny;
  for (int i = 0; i < k; ++i) {
    double nv = std::sqrt(std::max(nh[i], 0.0));
    f[i] = nv > 0 ? 1.0 / nv : 0.0;
    if (shifts[i] <= 10.0 * kEps64 * anorm) tiny.push_back(i);
  }
  c.h2d(sp.vec(10), f.data(), k * sizeof(double));
  scale_cols(cm(tb.Ut, m, k, m), sp.vec(10), c.s);
  // left vectors of (numerically) zero singular values carry no accuracy
  // from stage 1: random, orthogonalised against the others (Section 3.3)
  for (int i : tiny) {
    fill_random(cm(tb.Ut + (int64_t)i * m, m, 1, m), c.seed, 4000000 + (c.nrand++) * 64, c.s);
    std::vector<int> others;
    for (int j = 0; j < k; ++j)
      if (std::find(tiny.begin(), tiny.end(), j) == tiny.end()) others.push_back(j);
    // move the random column next to the others and orthogonalise it
    double *tmp = tb.QZ;  // scratch, m x (others + 1)
    for (size_t q = 0; q < others.size(); ++q)
      copy(cm(tb.Ut + (int64_t)others[q] * m, m, 1, m), cm(tmp + (int64_t)q * m, m, 1, m), c.s);
    copy(cm(tb.Ut + (int64_t)i * m, m, 1, m), cm(tmp + (int64_t)others.size() * m, m, 1, m), c.s);
    cgs_cols(c, tmp, m, m, (int)others.size(), (int)others.size() + 1, nullptr, 0, true, sp);
    copy(cm(tmp + (int64_t)others.size() * m, m, 1, m), cm(tb.Ut + (int64_t)i * m, m, 1, m), c.s);
  }
}

// Stage-2 seeds from saved first-stage output: v_i = the given vectors,
// normalised; u_i as finish_left (one product with A each).
void resume_seeds(Ctx &c, const SpMat<double> &A, const double *V, int k,
                  const std::vector<double> &shifts, double anorm, int bw, TransBufs &tb,
                  SmallPool &sp) {
  const int64_t n = A.n, m = A.m;
  copy(cm(const_cast<double *>(V), n, k, n), cm(tb.Vt, n, k, n), c.s);
  double *nrm = sp.vec(9), *f = sp.vec(10);
  colnorm2(cm(tb.Vt, n, k, n), 0, n, nrm, c.sc, c.s);
  std::vector<double> h(k);
  c.d2h(h.data(), nrm, k * sizeof(double));
  c.sync();
  for (int i = 0; i < k; ++i) {
    PHS_REQUIRE(h[i] > 0.0 && std::isfinite(h[i]), kEinval, "init_V has a zero column");
    h[i] = 1.0 / std::sqrt(h[i]);
  }
  c.h2d(f, h.data(), k * sizeof(double));
  scale_cols(cm(tb.Vt, n, k, n), f, c.s);
  for (int c0 = 0; c0 < k; c0 += bw) {
    const int w = std::min(bw, k - c0);
    copy(cm(tb.Vt + (int64_t)c0 * n, n, w, n), rmv(tb.Xn, n, w, bw), c.s);
    spmm(A, bw, tb.Xn, tb.Ym, false, c.s);
    copy(rmv(tb.Ym, m, w, bw), cm(tb.Ut + (int64_t)c0 * m, m, w, m), c.s);
  }
  c.st->mv_rr += k;
  finish_left(c, m, k, shifts, anorm, tb, sp);
}

// ------------------------------------------------------------------------
// Stage 2: GD+k with the refined projection on B (Algorithm 2).
Stage2Result run_stage2(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                        const Stage2Params &P, Stage2Bufs &bf, SmallPool &sp) {
  const int64_t n = A.n, m = A.m, N = n + m;
  const int k2 = P.k2, b = P.b, bw = P.bw, pmax = P.pmax, pmin = P.pmin;
  const int ld = kSP;
  double *V[2] = {bf.V[0], bf.V[1]}, *W[2] = {bf.W[0], bf.W[1]}, *Q[2] = {bf.Q[0], bf.Q[1]};
  int cur = 0, p = 0, nl = 0, nprev = 0;
  double *Tb = bf.Tb, *T2b = bf.T2b, *Rb = bf.Rb;
  double *H = sp.mat(13), *Rq = sp.mat(14), *Ys = sp.mat(15), *Ysl = sp.mat(16),
         *Yr = sp.mat(17), *prev = sp.mat(19), *prev2 = sp.mat(20),
         *Gb = sp.mat(21),
         *G1 = sp.mat(25), *Rc1 = sp.mat(26), *Rci1 = sp.mat(27), *Rc2 = sp.mat(28),
         *Rci2 = sp.mat(29), *Gram = sp.mat(30);
  double *sv = sp.vec(11), *thc = sp.vec(12), *ths = sp.vec(13), *rn2 = sp.vec(14),
         *xt2 = sp.vec(15);
  int *cnt = c.sc.flag + 8;
  Stage2Result res;
  // harmonic mode: the QR is of W itself (target 0), the shifts only order
  // the seeds
  const bool harm = P.extract == 1;
  double shift = harm ? 0.0 : P.shifts[0];
  bool qr_full = true;
  int hist_nl = -1;
  int64_t last_rebuild = -1000000;  // iteration of the last W = B V rebuild
  const double thr = P.tol * P.anorm / std::sqrt(2.0);

  auto applyB = [&](double *X, int nb) {
    spmm(At, bw, X + n * bw, bf.WTb, false, c.s);
    spmm(A, bw, X, bf.WTb + n * bw, false, c.s);
    c.st->mv_stage2 += nb;
  };
  // QR update of W - shift V by the new block (columns p..p+nb): block
  // Gram-Schmidt against Q, then CholQR2 of the remainder when it is well
  // conditioned, column-wise Gram-Schmidt otherwise.
  auto qr_update = [&](int nb) {
    axpby(rmv(bf.WTb, N, nb, bw), rmv(Tb, N, nb, bw), shift, rmv(bf.Cb, N, nb, bw), c.s);
    zero_rows(Rq, ld, p, p + nb, p + nb, c.s);
    Tall<double> Cv = rmv(bf.Cb, N, nb, bw);
    if (p > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        tn(cm(Q[cur], N, p, N), none<double>(N), Cv, G1, ld, c.sc, c.s);
        nn(cm(Q[cur], N, p, N), none<double>(N), G1, ld, -1.0, Cv, 1.0, c.s);
        if (pass == 0)
          small_gemm(false, false, p, nb, nb, 1.0, G1, ld, sp.eye(), ld, 0.0,
                     Rq + (int64_t)p * ld, ld, c.s);
        else
          small_add(p, nb, 1.0, G1, ld, Rq + (int64_t)p * ld, ld, c.s);
      }
    }
    tn(Cv, none<double>(N), Cv, Gram, ld, c.sc, c.s);
    chol_inv(Gram, ld, nb, 0.0, Rc1, Rci1, ld, c.sc.flag, c.s);
    double rd[64 * 64];
    int fl = 0;
    c.d2h(rd, Rc1, (size_t)ld * nb * sizeof(double));
    c.d2h(&fl, c.sc.flag, sizeof(int));
    c.sync();
    double dmax = 0, dmin = 1e300;
    for (int j = 0; j < nb; ++j) {
      dmax = std::max(dmax, std::fabs(rd[j + j * ld]));
      dmin = std::min(dmin, std::fabs(rd[j + j * ld]));
    }
    if (!fl && dmin > 1e-6 * dmax) {
      nn(Cv, none<double>(N), Rci1, ld, 1.0, rmv(bf.C2b, N, nb, bw), 0.0, c.s);
      Tall<double> C2v = rmv(bf.C2b, N, nb, bw);
      tn(C2v, none<double>(N), C2v, Gram, ld, c.sc, c.s);
      chol_inv(Gram, ld, nb, 0.0, Rc2, Rci2, ld, c.sc.flag + 1, c.s);
      nn(C2v, none<double>(N), Rci2, ld, 1.0, cm(Q[cur] + (int64_t)p * N, N, nb, N), 0.0, c.s);
      // R_bb = R2 R1
      small_gemm(false, false, nb, nb, nb, 1.0, Rc2, ld, Rc1, ld, 0.0, Rq + p + (int64_t)p * ld,
                 ld, c.s);
    } else {
      copy(Cv, cm(Q[cur] + (int64_t)p * N, N, nb, N), c.s);
      // coefficients against the new columns only: R(p:p+j, p+j)
      cgs_cols(c, Q[cur], N, N, p, p + nb, Rq, ld, false, sp);
    }
  };
  auto expand2 = [&](int nb) {
    orth_block(c, Tb, T2b, N, nb, bw, cm(bf.Xl, N, nl, N), cm(V[cur], N, p, N), kDepDropF64, sp);
    applyB(Tb, nb);
    copy(rmv(Tb, N, nb, bw), cm(V[cur] + (int64_t)p * N, N, nb, N), c.s);
    copy(rmv(bf.WTb, N, nb, bw), cm(W[cur] + (int64_t)p * N, N, nb, N), c.s);
    TnParts gp;
    tn(cm(V[cur], N, p + nb, N), none<double>(N), rmv(bf.WTb, N, nb, bw), Gb, ld, c.sc, c.s, &gp);
    reduce_border(gp, H, ld, nprev ? prev : nullptr, ld, nprev, c.s);
    if (!qr_full) qr_update(nb);
    p += nb;
  };

  // seeds y_i = [v_i; u_i] / sqrt(2) (Algorithm 2 step 1)
  copy(cm(const_cast<double *>(P.v0), n, k2, n), cm(bf.Y0, n, k2, N), c.s);
  copy(cm(const_cast<double *>(P.u0), m, k2, m), cm(bf.Y0 + n, m, k2, N), c.s);
  {
    std::vector<double> f(k2, 1.0 / std::sqrt(2.0));
    c.h2d(sp.vec(16), f.data(), k2 * sizeof(double));
    scale_cols(cm(bf.Y0, N, k2, N), sp.vec(16), c.s);
  }
  // Krylov fill K_{p_min - k}(B, y_1) by Lanczos with full
  // reorthogonalisation; its last residual is the first correction (step 2)
  const int nk = std::max(0, pmin - k2);
  double *K = Q[1];  // scratch until the first QR
  int npend = 0;
  if (nk > 0) {
    copy(cm(bf.Y0, N, 1, N), cm(K, N, 1, N), c.s);
    cgs_cols(c, K, N, N, 0, 1, nullptr, 0, true, sp);
    for (int i = 0; i < nk; ++i) {
      double *src = K + (int64_t)i * N, *dst = K + (int64_t)(i + 1) * N;
      spmm(At, 1, src + n, dst, false, c.s);
      spmm(A, 1, src, dst + n, false, c.s);
      c.st->mv_stage2 += 1;
      if (i < nk - 1) cgs_cols(c, K, N, N, i + 1, i + 2, nullptr, 0, true, sp);
    }
  }
  {
    // initial basis: seeds (at most p_min of them; the others enter as
    // their targets come up) and the Krylov vectors 2..nk, in chunks
    std::vector<std::pair<double *, int>> cols;
    for (int i = 0; i < std::min(k2, pmin); ++i) cols.push_back({bf.Y0 + (int64_t)i * N, 1});
    for (int i = 1; i < nk; ++i) cols.push_back({K + (int64_t)i * N, 1});
    for (size_t c0 = 0; c0 < cols.size(); c0 += bw) {
      int w = (int)std::min<size_t>(bw, cols.size() - c0);
      for (int q = 0; q < w; ++q)
        copy(cm(cols[c0 + q].first, N, 1, N), rmv(Tb + q, N, 1, bw), c.s);
      expand2(w);
    }
    if (nk > 0) {
      copy(cm(K + (int64_t)nk * N, N, 1, N), rmv(Tb, N, 1, bw), c.s);
      npend = 1;
    }
  }
  std::vector<double> sv_h(pmax), th_h(2 * b + 2), rn_h(bw), xt_h(bw);
  int64_t it = 0;
  while (true) {
    if (npend) {
      expand2(npend);
      npend = 0;
    }
    ++it;
    if (qr_full) {
      axpby(cm(W[cur], N, p, N), cm(V[cur], N, p, N), shift, cm(Q[cur], N, p, N), c.s);
      zero_rows(Rq, ld, 0, p, p, c.s);
      cgs_cols(c, Q[cur], N, N, 0, p, Rq, ld, false, sp);
      qr_full = false;
    }
    int nbal = 0;
    if (harm) {
      // harmonic Ritz vectors for the target 0: with W = Q R, the pencil
      // H y = mu R^T R y, i.e. the eigenpairs (mu, z) of R^-T H R^-1 and
      // y = R^-1 z (mu = 1 / theta_harm), descending in mu; candidates with
      // mu > 0 and balanced halves, |2 ||x_top||^2 - 1| < 0.1 (B's null
      // vectors [0; w] fail it), come first
      double *Ri = sp.mat(18), *Mh = sp.mat(22), *Z = sp.mat(23), *Yh = sp.mat(24),
             *Gt = sp.mat(25);
      double *mu = sp.vec(5), *bal = sp.vec(6);
      tri_inv(Rq, ld, p, Ri, ld, c.s);
      small_gemm(true, false, p, p, p, 1.0, Ri, ld, H, ld, 0.0, Z, ld, c.s);
      small_gemm(false, false, p, p, p, 1.0, Z, ld, Ri, ld, 0.0, Mh, ld, c.s);
      syev_rr(Mh, ld, p, p, true, mu, Z, ld, c.s, false);
      small_gemm(false, false, p, p, p, 1.0, Ri, ld, Z, ld, 0.0, Yh, ld, c.s);
      normalize_small(Yh, ld, p, p, c.s);
      for (int c0 = 0; c0 < p; c0 += 32) {  // Gram of the top halves, 32 columns a launch
        const int w = std::min(32, p - c0);
        tn(cm(V[cur], n, p, N), none<double>(n), cm(V[cur] + (int64_t)c0 * N, n, w, N),
           Gt + (int64_t)c0 * ld, ld, c.sc, c.s);
      }
      rayleigh_small(Gt, ld, p, Yh, ld, p, bal, c.s);
      std::vector<double> mu_h(p), bal_h(p);
      c.d2h(mu_h.data(), mu, p * sizeof(double));
      c.d2h(bal_h.data(), bal, p * sizeof(double));
      c.sync();
      std::vector<int> order(p);
      std::iota(order.begin(), order.end(), 0);
      auto good = [&](int i) { return mu_h[i] > 0.0 && std::fabs(2.0 * bal_h[i] - 1.0) < 0.1; };
      std::stable_sort(order.begin(), order.end(), [&](int a, int q) {
        if (good(a) != good(q)) return good(a);
        return mu_h[a] > mu_h[q];
      });
      for (int i = 0; i < p; ++i) nbal += good(i) ? 1 : 0;
      c.h2d(c.didx, order.data(), p * sizeof(int));
      gather_cols(Yh, ld, p, c.didx, p, Ys, ld, c.s);
      const double lead = mu_h[order[0]];
      std::vector<double> sv0 = {lead != 0.0 ? 1.0 / lead : INFINITY};
      c.h2d(sv, sv0.data(), sizeof(double));
    } else {
      svdj(Rq, ld, p, p, sv, Ys, ld, c.s);
    }
    const int ncand = std::min(p, 2 * b + 1);
    rayleigh_small(H, ld, p, Ys, ld, ncand, thc, c.s);
    c.d2h(th_h.data(), thc, ncand * sizeof(double));
    c.sync();
    // JDQMR expands by the correction of the target alone
    const int bsel = P.method == 1 ? 1 : b;
    std::vector<int> slots = {0};
    for (int q = 1; q < ncand && (int)slots.size() < bsel; ++q)
      if (harm ? q < nbal : th_h[q] > 0.5 * shift) slots.push_back(q);
    int ns = (int)slots.size();
    std::vector<double> ths_h(ns);
    for (int q = 0; q < ns; ++q) ths_h[q] = th_h[slots[q]];
    c.h2d(c.didx, slots.data(), ns * sizeof(int));
    c.h2d(ths, ths_h.data(), ns * sizeof(double));
    gather_cols(Ys, ld, p, c.didx, ns, Ysl, ld, c.s);
    ritz(cm(V[cur], N, p, N), cm(W[cur], N, p, N), Ysl, ld, ths, bf.Xb, Rb, ns, bw, rn2, xt2, n,
         c.sc, c.s);
    c.d2h(rn_h.data(), rn2, ns * sizeof(double));
    c.d2h(xt_h.data(), xt2, ns * sizeof(double));
    c.sync();
    const double r0 = std::sqrt(std::max(rn_h[0], 0.0));
    if (P.hist) {
      if (hist_nl >= 0 && nl != hist_nl) P.hist->push_back(NAN);
      hist_nl = nl;
      P.hist->push_back(std::log(std::max(r0, 1e-300)));
    }
    if (c.verbose && it % 1000 == 0)
      std::fprintf(stderr,
                   "[phsvds] stage 2 iteration %lld: locked %d/%d, products %lld, theta %.12e, "
                   "||r|| %.3e\n",
                   (long long)it, nl, k2, (long long)c.st->mv_stage2, ths_h[0], r0);
    // lock on the B residual test of Section 3.1 and on the triplet
    // residual of the normalised halves (Section 5): for sigma below
    // tol ||A|| an unbalanced x = [v; u] can pass the first alone
    bool lock =
        r0 < thr && triplet_residual(c, bf.Xb, Rb, bw, n, N, ths_h[0], sp) <= P.tol * P.anorm;
    if (lock) {
      // confirm on the explicit product B x: the recurrence W y drifts from
      // it over restarts; on a mismatch rebuild W = B V and H = V^T W, at
      // most once in 10 iterations (as in stage 1)
      applyB(bf.Xb, 1);
      axpby(rmv(bf.WTb, N, 1, bw), rmv(bf.Xb, N, 1, bw), ths_h[0], rmv(bf.Cb, N, 1, bw), c.s);
      double *rx2 = sp.vec(17);
      colnorm2(rmv(bf.Cb, N, 1, bw), 0, N, rx2, c.sc, c.s);
      double hx = 0.0;
      c.d2h(&hx, rx2, sizeof(double));
      c.sync();
      lock = std::sqrt(std::max(hx, 0.0)) < thr &&
             triplet_residual(c, bf.Xb, bf.Cb, bw, n, N, ths_h[0], sp) <= P.tol * P.anorm;
      if (!lock && it - last_rebuild > 10) {
        last_rebuild = it;
        for (int c0 = 0; c0 < p; c0 += bw) {
          const int w = std::min(bw, p - c0);
          copy(cm(V[cur] + (int64_t)c0 * N, N, w, N), rmv(Tb, N, w, bw), c.s);
          applyB(Tb, w);
          copy(rmv(bf.WTb, N, w, bw), cm(W[cur] + (int64_t)c0 * N, N, w, N), c.s);
        }
        for (int c0 = 0; c0 < p; c0 += 32) {
          const int w = std::min(32, p - c0);
          tn(cm(V[cur], N, p, N), none<double>(N), cm(W[cur] + (int64_t)c0 * N, N, w, N),
             H + (int64_t)c0 * ld, ld, c.sc, c.s);
        }
        nprev = 0;
        qr_full = true;
        ++res.refreshes;
        continue;
      }
    }
    if (lock) {
      copy(rmv(bf.Xb, N, 1, bw), cm(bf.Xl + (int64_t)nl * N, N, 1, N), c.s);
      res.theta.push_back(ths_h[0]);
      ++nl;
      if (c.verbose)
        std::fprintf(stderr, "[phsvds] stage 2 iteration %lld: locked %d/%d, sigma %.15e\n",
                     (long long)it, nl, k2, ths_h[0]);
      if (nl >= k2) {
        res.converged = true;
        break;
      }
      // drop the locked direction: V <- V Ys(:, 1:p); the harmonic vectors
      // are not orthonormal, so their orthonormal basis is taken, in order
      double *Yo = Ys;
      if (harm) {
        Yo = sp.mat(26);
        small_qr(Ys, ld, p, p, Yo, ld, sp.mat(27), ld, c.s);
      }
      nn(cm(V[cur], N, p, N), none<double>(N), Yo + ld, ld, 1.0, cm(V[1 - cur], N, p - 1, N), 0.0,
         c.s);
      nn(cm(W[cur], N, p, N), none<double>(N), Yo + ld, ld, 1.0, cm(W[1 - cur], N, p - 1, N), 0.0,
         c.s);
      restart_project(H, ld, p, Yo + ld, ld, p - 1, nullptr, ld, 0, nullptr, ld, c.s);
      cur = 1 - cur;
      p -= 1;
      if (!harm) shift = P.shifts[nl];
      // re-introduce the next initial guess (Algorithm 2 step 11)
      copy(cm(bf.Y0 + (int64_t)nl * N, N, 1, N), rmv(Tb, N, 1, bw), c.s);
      npend = 1;
      nprev = 0;
      qr_full = true;
      continue;
    }
    const bool out_of_budget = res.restarts > P.max_restarts ||
                               c.over_budget() ||
                               (P.max_iters > 0 && it > P.max_iters);
    if (out_of_budget) {
      // best approximations: the target's current vector, then the seeds of
      // the targets not reached
      copy(rmv(bf.Xb, N, 1, bw), cm(bf.Xl + (int64_t)nl * N, N, 1, N), c.s);
      res.best_theta.push_back(ths_h[0]);
      if (k2 - nl - 1 > 0)
        copy(cm(bf.Y0 + (int64_t)(nl + 1) * N, N, k2 - nl - 1, N),
             cm(bf.Xl + (int64_t)(nl + 1) * N, N, k2 - nl - 1, N), c.s);
      for (int j = nl + 1; j < k2; ++j) res.best_theta.push_back(P.shifts[j]);
      res.nbest = k2 - nl;
      break;
    }
    // balance guard for the non-target block members (B's zero and
    // negative eigenvalues must not be taken for singular values)
    std::vector<int> acc = {0};
    for (int q = 1; q < ns; ++q)
      if (std::fabs(2.0 * xt_h[q] - 1.0) < 0.1) acc.push_back(q);
    if ((int)acc.size() < ns) {
      for (size_t q = 0; q < acc.size(); ++q) {
        if ((int)q != acc[q]) {
          copy(rmv(bf.Xb + acc[q], N, 1, bw), rmv(bf.Xb + q, N, 1, bw), c.s);
          copy(rmv(Rb + acc[q], N, 1, bw), rmv(Rb + q, N, 1, bw), c.s);
        }
      }
      std::vector<int> idx2(acc.size());
      for (size_t q = 0; q < acc.size(); ++q) idx2[q] = slots[acc[q]];
      for (size_t q = 0; q < acc.size(); ++q) ths_h[q] = ths_h[acc[q]];
      c.h2d(c.didx, idx2.data(), idx2.size() * sizeof(int));
      gather_cols(Ys, ld, p, c.didx, (int)idx2.size(), Ysl, ld, c.s);
      ns = (int)acc.size();
    }
    // correction t = Prec(r) (step 13)
    if (P.method == 1) {
      // JDQMR: the projected correction equation of the target, by sQMR
      JdInput in;
      in.Q1 = cm(bf.Xl, N, nl, N);
      in.Q2 = rmv(bf.Xb, N, 1, bw);
      in.r = rmv(Rb, N, 1, bw);
      in.theta = ths_h[0];
      in.eta = shift;
      in.thr = thr;
      in.max_inner = P.max_inner;
      in.jacobi_d = P.jacobi_d;
      in.precB = P.precB;
      jd_correction(c, A, At, in, P.jd_work, rmv(Tb, N, 1, bw), sp);
    } else if (P.precB) {
      P.precB(Rb, Tb, ns, bw, ths_h.data());
    } else if (P.jacobi_d) {
      // B-form of the Jacobi preconditioner of C: [f; g] -> [M A^T g; A M f]
      row_scale(Rb, P.jacobi_d, n, bw, true, bf.Cb, c.s);  // M f (top rows)
      spmm(At, bw, Rb + n * bw, Tb, false, c.s);           // A^T g -> top
      row_scale(Tb, P.jacobi_d, n, bw, true, Tb, c.s);     // M A^T g
      spmm(A, bw, bf.Cb, Tb + n * bw, false, c.s);         // A M f -> bottom
      c.st->mv_prec += ns;
    } else {
      std::swap(Tb, Rb);
    }
    if (p + ns > pmax) {
      const double *Yk = Ys;
      if (harm) {
        small_qr(Ys, ld, p, pmin, sp.mat(26), ld, sp.mat(27), ld, c.s);
        Yk = sp.mat(26);
      }
      restart_basis(Yk, ld, p, pmin, prev, ld, nprev, Yr, ld, cnt, c.s);
      int hc = 0;
      c.d2h(&hc, cnt, sizeof(int));
      c.sync();
      nn(cm(V[cur], N, p, N), none<double>(N), Yr, ld, 1.0, cm(V[1 - cur], N, hc, N), 0.0, c.s);
      nn(cm(W[cur], N, p, N), none<double>(N), Yr, ld, 1.0, cm(W[1 - cur], N, hc, N), 0.0, c.s);
      restart_project(H, ld, p, Yr, ld, hc, Ysl, ld, ns, prev2, ld, c.s);
      std::swap(prev, prev2);
      nprev = ns;
      cur = 1 - cur;
      p = hc;
      ++res.restarts;
      // a full QR of W - s V at every restart (Algorithm 2 step 12): updating
      // the factors through a small QR of R Yr carries the rounding of every
      // earlier restart into R, about eps ||W|| each time, which swamps
      // sigma_min(R) when the shift is within 1e-14 ||A|| of the target
      qr_full = true;
    } else {
      small_gemm(false, false, p, ns, ns, 1.0, Ysl, ld, sp.eye(), ld, 0.0, prev, ld, c.s);
      nprev = ns;
    }
    npend = ns;
  }
  res.iters = it;
  res.nl = nl;
  res.Xl = bf.Xl;
  bf.Tb = Tb;
  bf.T2b = T2b;
  bf.Rb = Rb;
  return res;
}

}  // namespace phs
