// Internal interfaces of the PHSVDS host orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <type_traits>
#include <vector>

#include "../../include/phsvds.h"
#include "common.hpp"
#include "kernels.hpp"

namespace phs {

constexpr int kSP = 128;               // leading dimension of small matrices
constexpr double kEps64 = 2.220446049250313e-16;   // float64 spacing at 1
constexpr double kEps32 = 1.1920928955078125e-07;  // float32 spacing at 1
constexpr double kDepDropF64 = 1e-10;  // norm drop that marks a dependent column

// Device pool of small float64 matrices (kSP x kSP) and vectors.
struct SmallPool {
  double *base = nullptr;
  static constexpr int kMats = 40, kVecs = 24, kVecLen = 1024;
  double *mat(int i) const { return base + (int64_t)i * kSP * kSP; }
  double *vec(int i) const { return base + (int64_t)kMats * kSP * kSP + (int64_t)i * kVecLen; }
  double *eye() const { return mat(kMats - 1); }
  static size_t bytes() { return ((size_t)kMats * kSP * kSP + (size_t)kVecs * kVecLen) * 8; }
};

struct Ctx {
  hipStream_t s = nullptr;
  Scratch sc;
  int *didx = nullptr;  // device int scratch (index lists)
  uint64_t seed = 0;
  uint64_t nrand = 0;
  phsvds_stats *st = nullptr;
  int64_t max_mv = 0;  // budget of products with A over the whole solve (0: none)
  bool over_budget() const {
    return max_mv > 0 && st->mv_stage1 + st->mv_rr + st->mv_stage2 > max_mv;
  }
  int verbose = 0;  // progress lines on stderr
  // device-to-host reads go through one pinned staging buffer: d2h queues
  // the copy, sync() waits for the stream and moves the bytes to their
  // destinations (a destination is valid only after the next sync())
  void d2h(void *h, const void *d, size_t bytes);
  void h2d(void *d, const void *h, size_t bytes);
  void sync();
  Ctx() = default;
  Ctx(const Ctx &) = delete;
  Ctx &operator=(const Ctx &) = delete;
  ~Ctx();

 private:
  struct Pending {
    void *h;
    size_t off, bytes;
  };
  char *pin_ = nullptr;
  size_t pin_used_ = 0;
  std::vector<Pending> pending_;
};

struct Stage1Params {
  int k, b, bw, pmax, pmin;
  bool largest;
  double tol, floor, anorm, sn2_init;
  int max_restarts;
  int64_t max_iters;
  const double *jacobi_d;  // diag(C) for the Jacobi preconditioner, or null
  const double *init64;    // initial basis (n x init_cols, column-major) or null
  const float *init32;
  int init_cols;
  // optional per-iteration view of the Ritz block (it, X, R, theta, nb, X_lock, nl),
  // blocks row-major with stride bw, X_lock column-major
  std::function<void(int64_t, const void *, const void *, const double *, int, const void *,
                     int)>
      snap;
  // learned preconditioner: called per column (r, x, theta, t), all length n
  // in working precision; null when not used
  std::function<void(const void *, const void *, double, void *)> gnn;
  int gnn_window = 25;  // safeguard window (iterations); <= 0: never fall back
  // caller's preconditioner: T = M R, n x nb column-major blocks in working
  // precision, theta the nb Ritz values (host); null when not used
  std::function<void(const void *, void *, int, const double *)> user;
  // optional per-iteration history of log(||r_1|| / sqrt(theta_1)) of the
  // leading unlocked pair, NaN where it changed (a lock)
  std::vector<double> *hist = nullptr;
  // the caller's operator in place of C = A^T A (C itself, or C^-1 for
  // shift-invert): Y = op X on row-major n x b blocks; null: A^T (A X)
  std::function<void(const void *, void *, int)> opC;
  // shift-invert: ||A||; the test becomes ||C^-1 x - mu x|| < tol sqrt(mu) / ||A||
  double si_anorm = 0.0;
  // optional early stop, asked before each iteration's budget test (the
  // run then ends as on a spent budget)
  std::function<bool()> stop;
};

template <typename T>
struct Stage1Bufs {
  T *V[2], *W[2], *Xl, *Xb, *Rb, *Tb, *T2b, *WTb, *Yb, *Fb;
  T *Gs;  // 3 n scratch for the learned preconditioner
  T *Ub;  // 2 n bw column-major in/out blocks of the caller's preconditioner
};

double power_norm2(Ctx &c, const SpMat<double> &A, const SpMat<double> &At, double *x, double *y,
                   double *z, int iters, SmallPool &sp);

struct Stage1Result {
  bool converged = false;
  int nl = 0, p = 0;
  int64_t iters = 0, restarts = 0, refreshes = 0, rollbacks = 0, fallbacks = 0;
  double sn2 = 0.0;
  std::vector<double> theta, res;
  std::vector<bool> tight;  // locked by the user tolerance (not by the floor)
  void *Vrest = nullptr;
  // out of budget: the leading unlocked Ritz vectors, stored in Xl after the
  // nl locked ones (best approximations, not converged)
  int nbest = 0;
  std::vector<double> best_theta;
};

struct TransBufs {
  double *Z, *AZ, *QZ, *Vt, *Ut, *Xn, *Ym;
};

struct Stage2Params {
  int k2, b, bw, pmax, pmin;
  double tol, anorm;
  const double *shifts;
  const double *v0, *u0;  // n x k2, m x k2 column-major seeds
  int max_restarts;
  int64_t max_iters;
  const double *jacobi_d;
  int method = 0;             // 0: GD+k, 1: JDQMR (correction equation by sQMR)
  int max_inner = 50;         // JDQMR inner step cap
  double *jd_work = nullptr;  // JDQMR: kJdVectors N-vectors
  // a preconditioner of B other than Jacobi (the B-form of the caller's M
  // of C, the form [M^-1 g; M^-T f] of M ~ A, or the caller's own M of B):
  // T = M_B R for row-major N x ns blocks with row stride ld, theta the ns
  // estimates of B (host); null when not used.  Also used inside JDQMR.
  std::function<void(const double *, double *, int, int, const double *)> precB;
  int extract = 0;  // 0: refined projection at the shifts; 1: harmonic Ritz for target 0
  // optional per-iteration history of log ||r|| of the target, NaN where
  // the target changed (a lock)
  std::vector<double> *hist = nullptr;
};

struct Stage2Bufs {
  double *V[2], *W[2], *Q[2], *Xl, *Y0, *Tb, *T2b, *WTb, *Xb, *Rb, *Cb, *C2b;
};

struct Stage2Result {
  bool converged = false;
  int nl = 0;
  int64_t iters = 0, restarts = 0, refreshes = 0;
  std::vector<double> theta;
  double *Xl = nullptr;
  // out of budget: the target's current vector, then the seeds of the
  // targets not reached, stored in Xl after the nl locked ones
  int nbest = 0;
  std::vector<double> best_theta;
};

template <typename T>
void orth_block(Ctx &c, T *&Tb, T *&T2b, int64_t n, int nb, int bw, const Tall<T> &B1,
                const Tall<T> &B2, double dep_drop, SmallPool &sp);
void cgs_cols(Ctx &c, double *X, int64_t rows, int64_t ld, int j0, int j1, double *R, int ldr,
              bool random_dep, SmallPool &sp);
template <typename T>
Stage1Result run_stage1(Ctx &c, const SpMat<T> &A, const SpMat<T> &At, const Stage1Params &P,
                        Stage1Bufs<T> &bf, SmallPool &sp);
void run_transition(Ctx &c, const SpMat<double> &A, const double *Xl, int k, const double *Vr,
                    int nvr, int pmin, double anorm, int bw, TransBufs &tb, SmallPool &sp,
                    std::vector<double> &shifts);
void finish_left(Ctx &c, int64_t m, int k, const std::vector<double> &shifts, double anorm,
                 TransBufs &tb, SmallPool &sp);
void resume_seeds(Ctx &c, const SpMat<double> &A, const double *V, int k,
                  const std::vector<double> &shifts, double anorm, int bw, TransBufs &tb,
                  SmallPool &sp);
void spmm_op(const phsvds_csr *A, const float *val32, bool trans, bool fp32, int b,
             const void *X, void *Y, void *ws, size_t ws_bytes, hipStream_t s, bool timed);
Stage2Result run_stage2(Ctx &c, const SpMat<double> &A, const SpMat<double> &At,
                        const Stage2Params &P, Stage2Bufs &bf, SmallPool &sp);

}  // namespace phs
