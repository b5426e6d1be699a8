// C ABI of libphsvds: argument checks, workspace planning, setup (CSR of
// A^T, float32 copies, row bins, diag(C)), the two-stage driver and the
// final float64 residual check.  No exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>

#include "gnn.hpp"
#include "harvest.hpp"
#include "jdqmr.hpp"
#include "solver.hpp"

namespace phs {

// Device scratch of the allocation-free transposed product
// (phsvds_spmm_noalloc): the CSR of A^T and the transpose scratch.  Each
// GPU holds its own copy for the life of the process.  In host code
// `scratch` names a host-side stand-in, never the device memory: the device
// address of each GPU's copy comes from hipGetSymbolAddress and is the only
// thing passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err;

// Device address of this GPU's `scratch`, looked up once per device with
// that device current (the calling thread's current device).
void *noalloc_scratch() {
  static std::mutex mu;
  static void *addr[64] = {};
  int dev = -1;
  PHS_HIP(hipGetDevice(&dev));
  PHS_REQUIRE(dev >= 0 && dev < 64, kEinval, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(-3, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = p;
  }
  return addr[dev];
}

double wall() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

template <typename F>
int guarded(F &&f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error &e) {
    g_err = e.what();
    return e.code;
  } catch (const std::exception &e) {
    g_err = e.what();
    return PHSVDS_EBREAKDOWN;
  }
}

struct Dims {
  int64_t m, n, nnz;
  int k, b, bw, pmax, pmin;
  bool fp32, cont, jac;
  int gw = 0;        // width of the learned preconditioner (0: not used)
  bool cg = false;   // harvest buffers
  bool jd = false;   // JDQMR work vectors
  bool dyn = false;  // dynamic switching: the current approximations
  // blocks for the caller's preconditioner: always planned, since the
  // workspace size is fixed before the preconditioner is known
  bool user = true;
};

// row-major view with row stride ld
template <typename T>
Tall<T> rmv_(T *p, int64_t rows, int cols, int ld) {
  Tall<T> t;
  t.p = p;
  t.rows = rows;
  t.cols = cols;
  t.rs = ld;
  t.cs = 1;
  return t;
}

int width_for(int b) {
  int w = 1;
  while (w < b) w *= 2;
  return w;
}

bool make_dims(int64_t m, int64_t n, int64_t nnz, int k, const phsvds_opts &o, Dims &d) {
  d.m = m;
  d.n = n;
  d.nnz = nnz;
  d.k = k;
  d.b = o.block > 0 ? o.block : 1;
  if (d.b > 16) return false;
  d.bw = width_for(d.b);
  // locked vectors leave the basis, so k is not bounded by p_max (<= 64,
  // the size of the small dense problems)
  d.pmax = o.max_basis > 0 ? o.max_basis : std::min(64, std::max(35, 2 * k + 2 * d.b));
  d.pmax = (int)std::min<int64_t>(d.pmax, n);  // a basis cannot outgrow the space
  d.pmin = o.min_restart > 0 ? o.min_restart : std::max(21, (int)std::ceil(0.6 * d.pmax));
  d.pmin = std::min(d.pmin, d.pmax - 2 * d.b);
  d.fp32 = o.stage1_fp32 != 0;
  d.cont = d.fp32 && o.fp64_continue != 0;
  d.jac = false;
  d.gw = o.gnn_width;
  d.jd = o.stage2_method == 1;
  d.dyn = o.dynamic != 0;
  if (o.stage2_method != 0 && o.stage2_method != 1) return false;
  if (o.max_inner < 0) return false;
  if (d.gw != 0 && d.gw != 8 && d.gw != 16 && d.gw != 32) return false;
  return d.pmax <= 64 && d.pmin >= d.b && d.pmin >= 1 && k >= 1 && k <= 64;
}

template <typename T>
void take_stage1(Arena &ar, const Dims &d, Stage1Bufs<T> &b) {
  for (int i = 0; i < 2; ++i) {
    b.V[i] = ar.take<T>(basis_ld(d.n) * d.pmax);
    b.W[i] = ar.take<T>(basis_ld(d.n) * d.pmax);
  }
  b.Xl = ar.take<T>(d.n * d.k);
  b.Xb = ar.take<T>(d.n * d.bw);
  b.Rb = ar.take<T>(d.n * d.bw);
  b.Tb = ar.take<T>(d.n * d.bw);
  b.T2b = ar.take<T>(d.n * d.bw);
  b.WTb = ar.take<T>(d.n * d.bw);
  b.Fb = ar.take<T>(d.n * d.bw);
  b.Yb = ar.take<T>(d.m * d.bw);
  b.Gs = ar.take<T>(3 * d.n);
  b.Ub = d.user ? ar.take<T>(2 * d.n * d.bw) : nullptr;
}

struct Plan {
  int64_t *trp;
  int32_t *tci;
  double *tva;
  char *tws;
  size_t tws_bytes;
  int32_t *binA, *binAt, *pinv;
  char *binWs;
  size_t binWs_bytes;
  float *va32, *tva32;
  double *diagC;
  Scratch sc;
  int *didx;
  double *pool;
  Stage1Bufs<float> s32;
  Stage1Bufs<double> s64;
  double *Xs, *Vr64;
  TransBufs tb;
  Stage2Bufs s2;
  double *Vf, *Uf, *AV, *RU, *RV, *Fx, *Fy;
  double *jd;  // JDQMR work vectors
  double *ub;  // stage-2 blocks of the caller's preconditioner
  double *dynV;  // dynamic switching: the latest approximations (n x k)
  GnnGraph gg;
  GnnBufs gb;
  CgBufs cg;
};

void carve(Arena &ar, const Dims &d, Plan &p) {
  const int64_t m = d.m, n = d.n, N = m + n, nnz = d.nnz;
  const int pz = std::max(d.k, d.pmin);
  p.trp = ar.take<int64_t>(n + 1);
  p.tci = ar.take<int32_t>(std::max<int64_t>(nnz, 1));
  p.tva = ar.take<double>(std::max<int64_t>(nnz, 1));
  p.tws_bytes = transpose_ws_bytes(m, n, nnz);
  p.tws = ar.take<char>(p.tws_bytes);
  p.binA = ar.take<int32_t>(m);
  p.binAt = ar.take<int32_t>(n);
  p.pinv = ar.take<int32_t>(std::max<int64_t>(m, 1));
  p.binWs_bytes = bin_ws_bytes(std::max(m, n));
  p.binWs = ar.take<char>(p.binWs_bytes);
  p.va32 = d.fp32 ? ar.take<float>(nnz) : nullptr;
  p.tva32 = d.fp32 ? ar.take<float>(nnz) : nullptr;
  p.diagC = ar.take<double>(n);
  p.sc.part = ar.take<double>(kPartCap);
  p.sc.aux = ar.take<double>(kAuxCap);
  p.sc.flag = ar.take<int>(64);
  p.didx = ar.take<int>(256);
  p.pool = ar.take<double>(SmallPool::bytes() / 8);
  if (d.fp32) take_stage1<float>(ar, d, p.s32);
  if (!d.fp32 || d.cont) take_stage1<double>(ar, d, p.s64);
  p.Xs = ar.take<double>(n * d.k);
  p.Vr64 = ar.take<double>(n * d.pmax);
  p.tb.Z = ar.take<double>(n * pz);
  p.tb.AZ = ar.take<double>(m * pz);
  p.tb.QZ = ar.take<double>(m * pz);
  p.tb.Vt = ar.take<double>(n * d.k);
  p.tb.Ut = ar.take<double>(m * d.k);
  p.tb.Xn = ar.take<double>(n * d.bw);
  p.tb.Ym = ar.take<double>(m * d.bw);
  for (int i = 0; i < 2; ++i) {
    p.s2.V[i] = ar.take<double>(N * d.pmax);
    p.s2.W[i] = ar.take<double>(N * d.pmax);
    p.s2.Q[i] = ar.take<double>(N * d.pmax);
  }
  p.s2.Xl = ar.take<double>(N * d.k);
  p.s2.Y0 = ar.take<double>(N * d.k);
  double **blk[] = {&p.s2.Tb, &p.s2.T2b, &p.s2.WTb, &p.s2.Xb, &p.s2.Rb, &p.s2.Cb, &p.s2.C2b};
  for (double **q : blk) *q = ar.take<double>(N * d.bw);
  p.Vf = ar.take<double>(n * d.k);
  p.Uf = ar.take<double>(m * d.k);
  p.AV = ar.take<double>(m * d.k);
  p.RU = ar.take<double>(n * d.k);
  p.RV = ar.take<double>(m * d.k);
  p.Fx = ar.take<double>(std::max(n, m) * 8);
  p.Fy = ar.take<double>(std::max(n, m) * 8);
  p.jd = d.jd ? ar.take<double>(N * kJdVectors) : nullptr;
  p.ub = d.user ? ar.take<double>(2 * n * d.bw) : nullptr;
  p.dynV = d.dyn ? ar.take<double>(n * d.k) : nullptr;
  if (d.gw > 0) gnn_carve(ar, m, n, nnz, d.gw, p.gg, p.gb);
  if (d.cg) carve_cg(ar, m, n, d.bw, p.cg);
}

// Y (rows_out x w, column-major) = op(A) X (column-major), in chunks of 8.
void apply_cols(Ctx &c, const SpMat<double> &A, const double *X, int w, double *Y, double *Fx,
                double *Fy) {
  for (int c0 = 0; c0 < w; c0 += 8) {
    int cw = std::min(8, w - c0);
    Tall<double> src = cm(const_cast<double *>(X) + c0 * A.n, A.n, cw, A.n);
    Tall<double> fx = {Fx, A.n, cw, 8, 1};
    copy(src, fx, c.s);
    spmm(A, 8, Fx, Fy, false, c.s);
    Tall<double> fy = {Fy, A.m, cw, 8, 1};
    copy(fy, cm(Y + c0 * A.m, A.m, cw, A.m), c.s);
  }
}

__global__ void k_sign_fix(double *V, int64_t n, double *U, int64_t m) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  double *v = V + (int64_t)j * n;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    double a = fabs(v[i]);
    if (a > best) {
      best = a;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double a = bv[threadIdx.x + o];
      int64_t ai = bi[threadIdx.x + o];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ai < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  const double sg = v[bi[0]] < 0 ? -1.0 : 1.0;
  __syncthreads();
  if (sg < 0) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v[i] = -v[i];
    double *u = U + (int64_t)j * m;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) u[i] = -u[i];
  }
}

}  // namespace

// Workspace of a transposed product: the CSR of A^T (row pointers, columns,
// float64 values, and float32 values for a float32 product), then the
// transpose scratch.
size_t spmm_t_ws_bytes(int64_t m, int64_t n, int64_t nnz, bool fp32) {
  Arena ar;
  ar.dry = true;
  ar.take<int64_t>(n + 1);
  ar.take<int32_t>(std::max<int64_t>(nnz, 1));
  ar.take<double>(std::max<int64_t>(nnz, 1));
  if (fp32) ar.take<float>(std::max<int64_t>(nnz, 1));
  ar.take<char>(transpose_ws_bytes(m, n, nnz));
  return ar.used;
}

void spmm_op(const phsvds_csr *A, const float *val32, bool trans, bool fp32, int b,
             const void *X, void *Y, void *ws, size_t ws_bytes, hipStream_t s, bool timed) {
  PHS_REQUIRE(A && X && Y, kEinval, "null argument");
  PHS_REQUIRE(A->m >= 0 && A->n >= 0 && A->nnz >= 0 && A->nnz < (int64_t(1) << 31), kEinval,
              "bad CSR sizes");
  PHS_REQUIRE(b == 1 || b == 2 || b == 4 || b == 8 || b == 16 || b == 32, kEinval,
              "block width must be 1, 2, 4, 8, 16 or 32");
  if (!trans) {
    PHS_REQUIRE(!fp32 || val32, kEinval, "float32 product needs val32");
    if (fp32) {
      SpMat<float> S;
      S.m = A->m; S.n = A->n; S.nnz = A->nnz;
      S.rowptr = A->rowptr; S.colind = A->colind; S.val = val32;
      if (timed) spmm(S, b, (const float *)X, (float *)Y, false, s);
      else spmm_untimed(S, b, (const float *)X, (float *)Y, s);
    } else {
      SpMat<double> S;
      S.m = A->m; S.n = A->n; S.nnz = A->nnz;
      S.rowptr = A->rowptr; S.colind = A->colind; S.val = A->val;
      if (timed) spmm(S, b, (const double *)X, (double *)Y, false, s);
      else spmm_untimed(S, b, (const double *)X, (double *)Y, s);
    }
    return;
  }
  PHS_REQUIRE(A->val, kEinval, "a transposed product needs the float64 values of A");
  PHS_REQUIRE(ws && ws_bytes >= spmm_t_ws_bytes(A->m, A->n, A->nnz, fp32), kEnomem,
              "spmm: workspace too small for the transpose");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  const int64_t nz = std::max<int64_t>(A->nnz, 1);
  int64_t *trp = ar.take<int64_t>(A->n + 1);
  int32_t *tci = ar.take<int32_t>(nz);
  double *tva = ar.take<double>(nz);
  float *tva32 = fp32 ? ar.take<float>(nz) : nullptr;
  const size_t tws = transpose_ws_bytes(A->m, A->n, A->nnz);
  char *tw = ar.take<char>(tws);
  csr_transpose(A->m, A->n, A->nnz, A->rowptr, A->colind, A->val, trp, tci, tva, tw, tws, s);
  if (fp32) {
    copy(cm(tva, A->nnz, 1, A->nnz), cm(tva32, A->nnz, 1, A->nnz), s);
    SpMat<float> S;
    S.m = A->n; S.n = A->m; S.nnz = A->nnz;
    S.rowptr = trp; S.colind = tci; S.val = tva32;
    if (timed) spmm(S, b, (const float *)X, (float *)Y, false, s);
    else spmm_untimed(S, b, (const float *)X, (float *)Y, s);
  } else {
    SpMat<double> S;
    S.m = A->n; S.n = A->m; S.nnz = A->nnz;
    S.rowptr = trp; S.colind = tci; S.val = tva;
    if (timed) spmm(S, b, (const double *)X, (double *)Y, false, s);
    else spmm_untimed(S, b, (const double *)X, (double *)Y, s);
  }
}

__global__ void k_scale_by_cols(int64_t nnz, const int32_t *ci, const double *va,
                                const double *d, double *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const double dj = d[ci[p]];
  out[p] = dj > 0.0 ? va[p] / sqrt(dj) : va[p];
}

void jacobi_scaled_values(const phsvds_csr *A, double *val_out, void *ws, size_t ws_bytes,
                          hipStream_t s) {
  PHS_REQUIRE(ws && ws_bytes >= spmm_t_ws_bytes(A->m, A->n, A->nnz, false) +
                                    (size_t)A->n * sizeof(double) + 256,
              kEnomem, "jacobi_scaled_values: workspace too small");
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  const int64_t nz = std::max<int64_t>(A->nnz, 1);
  int64_t *trp = ar.take<int64_t>(A->n + 1);
  int32_t *tci = ar.take<int32_t>(nz);
  double *tva = ar.take<double>(nz);
  const size_t tws = transpose_ws_bytes(A->m, A->n, A->nnz);
  char *tw = ar.take<char>(tws);
  double *d = ar.take<double>(A->n);
  csr_transpose(A->m, A->n, A->nnz, A->rowptr, A->colind, A->val, trp, tci, tva, tw, tws, s);
  SpMat<double> At;
  At.m = A->n;
  At.n = A->m;
  At.nnz = A->nnz;
  At.rowptr = trp;
  At.colind = tci;
  At.val = tva;
  col_sq_norms(At, d, s);
  if (A->nnz) {
    k_scale_by_cols<<<cdiv(A->nnz, 256), 256, 0, s>>>(A->nnz, A->colind, A->val, d, val_out);
    PHS_CHECK_LAUNCH();
  }
}

namespace {

int svds_impl(const phsvds_csr *Ain, const phsvds_operator *Aop, int k, double tol,
              const phsvds_precond *Pc, const phsvds_opts *oin, void *ws, size_t ws_bytes,
              void *stream, double *sigma, double *Uout, double *Vout, double *resnorm,
              phsvds_stats *stats) {
  const double t0 = wall();
  PHS_REQUIRE((Ain || (Aop && Aop->apply)) && sigma && Uout && Vout && resnorm, kEinval,
              "null argument");
  phsvds_opts o;
  phsvds_default_opts(&o);
  if (oin) o = *oin;
  phsvds_stats stl;
  std::memset(&stl, 0, sizeof(stl));
  const int64_t m = Ain ? Ain->m : Aop->m, n = Ain ? Ain->n : Aop->n, nnz = Ain ? Ain->nnz : 0;
  if (!Ain) {
    const int pk = Pc ? Pc->kind : PHSVDS_PREC_NONE;
    PHS_REQUIRE(pk == PHSVDS_PREC_NONE || pk == PHSVDS_PREC_USER || pk == PHSVDS_PREC_USER_A,
                kEinval, "an operator for A takes no JACOBI or GNN preconditioner");
    PHS_REQUIRE(!o.stage1_fp32, kEinval, "an operator for A runs in float64 only");
  }
  PHS_REQUIRE(m >= n && n >= 1 && nnz >= 0 && nnz < (int64_t(1) << 31), kEinval,
              "need m >= n >= 1 and nnz < 2^31");
  PHS_REQUIRE(tol > 0, kEinval, "tol must be positive");
  PHS_REQUIRE(k <= n, kEinval, "k must not exceed n");
  int pkind = Pc ? Pc->kind : PHSVDS_PREC_NONE;
  PHS_REQUIRE(pkind == PHSVDS_PREC_NONE || pkind == PHSVDS_PREC_JACOBI ||
                  pkind == PHSVDS_PREC_GNN || pkind == PHSVDS_PREC_USER ||
                  pkind == PHSVDS_PREC_USER_A,
              kEinval, "unsupported preconditioner kind");
  PHS_REQUIRE(pkind != PHSVDS_PREC_USER || Pc->user_apply || Pc->user_apply_B, kEinval,
              "a USER preconditioner needs user_apply or user_apply_B");
  PHS_REQUIRE(pkind != PHSVDS_PREC_USER_A || Pc->user_solve, kEinval,
              "a USER_A preconditioner needs user_solve");
  bool resume = o.init_V && o.shifts;
  PHS_REQUIRE(!o.shifts || o.init_V, kEinval, "shifts need init_V");
  PHS_REQUIRE(!o.c_apply || (!o.stage1_fp32 && !o.dynamic), kEinval,
              "an operator for C needs stage1_fp32 = 0 and dynamic = 0");
  PHS_REQUIRE(!o.c_inverse || (o.c_apply && o.which == 0 && pkind == PHSVDS_PREC_NONE &&
                               !resume),
              kEinval, "shift-invert needs c_apply, the smallest end and no preconditioner");
  PHS_REQUIRE(!o.dynamic || (o.which == 0 && !o.stage1_fp32 && o.stage2_method == 0 &&
                             !o.init_V && pkind != PHSVDS_PREC_GNN),
              kEinval,
              "dynamic switching needs the smallest end, float64, stage2_method 0, no init_V "
              "and no GNN preconditioner");
  PHS_REQUIRE(!resume || (o.k0 >= k && o.which == 0 && o.stage2 != -1), kEinval,
              "resuming the second stage needs k0 >= k, the smallest end and stage2 >= 0");
  Dims d;
  PHS_REQUIRE(make_dims(m, n, nnz, k, o, d), kEinval,
              "unsupported sizes: need 1 <= k <= 64, block <= 16, max_basis <= 64 and "
              "n >= 3 block (the basis is capped at n and must hold a restart plus a block)");
  d.jac = pkind == PHSVDS_PREC_JACOBI || pkind == PHSVDS_PREC_GNN;
  PHS_REQUIRE(!o.init_V || resume || (o.k0 >= 1 && o.k0 <= d.pmin), kEinval,
              "init_V without shifts needs 1 <= k0 <= p_min");
  PHS_REQUIRE(!o.dynamic || k <= d.pmin, kEinval, "dynamic switching needs k <= p_min");
  if (pkind != PHSVDS_PREC_GNN) d.gw = 0;
  if (pkind == PHSVDS_PREC_GNN) {
    PHS_REQUIRE(Pc->gnn_weights && (Pc->gnn_width == 8 || Pc->gnn_width == 16 ||
                                    Pc->gnn_width == 32),
                kEinval, "GNN preconditioner needs weights and width 8, 16 or 32");
    PHS_REQUIRE(o.gnn_width == Pc->gnn_width, kEinval,
                "opts.gnn_width must equal the preconditioner's width (workspace sizing)");
  }
  const int gwin = (Pc && Pc->fallback_window != 0) ? Pc->fallback_window : 25;
  const bool largest = o.which == 1;
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  Plan pl{};
  carve(ar, d, pl);
  Ctx c;
  c.s = (hipStream_t)stream;
  c.sc = pl.sc;
  c.didx = pl.didx;
  c.seed = o.seed;
  c.st = &stl;
  c.max_mv = o.max_matvecs;
  c.verbose = o.verbose;
  SmallPool sp;
  sp.base = pl.pool;
  {
    // identity used to copy small matrices through small_gemm
    std::vector<double> eye((size_t)kSP * kSP, 0.0);
    for (int i = 0; i < kSP; ++i) eye[i + (size_t)i * kSP] = 1.0;
    c.h2d(sp.eye(), eye.data(), eye.size() * sizeof(double));
  }
  // ---------------------------------------------------------------- setup
  SpMat<double> A64, At64;
  A64.m = m;
  A64.n = n;
  A64.nnz = nnz;
  At64.m = n;
  At64.n = m;
  At64.nnz = nnz;
  OpHook hook;
  bool row_perm = false;  // row space in bin order (set below)
  if (Aop) {
    // the caller's operator (Section 3.3): every product of the path goes
    // through it, on the solver's stream
    hook.f = [&](const void *X, void *Y, int b, bool trans, bool fp64) {
      const int rc = Aop->apply(Aop->ctx, X, Y, b, trans ? 1 : 0, fp64 ? 1 : 0, c.s);
      if (rc != 0) throw Error(PHSVDS_EUSER, "operator returned " + std::to_string(rc));
    };
    A64.op = &hook;
    At64.op = &hook;
    At64.op_trans = true;
  } else {
    A64.rowptr = Ain->rowptr;
    A64.colind = Ain->colind;
    A64.val = Ain->val;
    csr_transpose(m, n, nnz, Ain->rowptr, Ain->colind, Ain->val, pl.trp, pl.tci, pl.tva,
                  pl.tws, pl.tws_bytes, c.s);
    At64.rowptr = pl.trp;
    At64.colind = pl.tci;
    At64.val = pl.tva;
    build_bins(m, A64.rowptr, pl.binA, pl.binWs, pl.binWs_bytes, A64.bins, &A64.nbins, c.s);
    A64.binrows = pl.binA;
    if (A64.nbins == 1) A64.nbins = 0;
    build_bins(n, At64.rowptr, pl.binAt, pl.binWs, pl.binWs_bytes, At64.bins, &At64.nbins, c.s);
    At64.binrows = pl.binAt;
    if (At64.nbins == 1) At64.nbins = 0;
    // rows of A of several length classes: the row space (A X, the left
    // vectors, the top of B's vectors) is kept in bin order, so that the
    // long rows, which A^T gathers most often, share cache lines.  Products
    // and sums over the columns are unchanged (A^T takes each row in its
    // original order); U is returned in the caller's order.  Not with the
    // preconditioner forms that take row-space vectors from the caller.
    row_perm = A64.nbins >= 2 && pkind != PHSVDS_PREC_USER_A && !(Pc && Pc->user_apply_B);
    if (row_perm) {
      permute_row_space(m, nnz, pl.binA, pl.pinv, pl.tci, c.s);
      A64.slot_out = true;
    }
  }
  SpMat<float> A32, At32;
  if (d.fp32) {
    copy(cm(const_cast<double *>(Ain->val), nnz, 1, nnz), cm(pl.va32, nnz, 1, nnz), c.s);
    copy(cm(pl.tva, nnz, 1, nnz), cm(pl.tva32, nnz, 1, nnz), c.s);
    A32.m = m; A32.n = n; A32.nnz = nnz; A32.rowptr = A64.rowptr; A32.colind = A64.colind;
    A32.val = pl.va32; A32.nbins = A64.nbins; A32.binrows = A64.binrows;
    A32.slot_out = A64.slot_out;
    std::memcpy(A32.bins, A64.bins, sizeof(A64.bins));
    At32.m = n; At32.n = m; At32.nnz = nnz; At32.rowptr = At64.rowptr; At32.colind = At64.colind;
    At32.val = pl.tva32; At32.nbins = At64.nbins; At32.binrows = At64.binrows;
    std::memcpy(At32.bins, At64.bins, sizeof(At64.bins));
  }
  if (d.jac) col_sq_norms(At64, pl.diagC, c.s);
  if (d.gw && pkind == PHSVDS_PREC_GNN) gnn_prepare(*Ain, pl.gg, c.s);
  c.sync();
  const double t1 = wall();
  stl.t_setup = t1 - t0;
  // -------------------------------------------------------------- stage 1
  Stage1Params P1{};
  P1.k = k;
  P1.b = d.b;
  P1.bw = d.bw;
  P1.pmax = d.pmax;
  P1.pmin = d.pmin;
  P1.largest = largest || o.c_inverse;
  P1.tol = tol;
  P1.floor = o.floor_factor > 0 ? o.floor_factor : 10.0;
  P1.anorm = o.anorm;
  P1.sn2_init = 0.0;
  P1.max_restarts = o.max_restarts > 0 ? o.max_restarts : 10000;
  P1.max_iters = 0;
  P1.jacobi_d = d.jac ? pl.diagC : nullptr;
  P1.init64 = o.init_V ? o.init_V : o.init_block;
  P1.init32 = nullptr;
  P1.init_cols = o.init_V ? o.k0 : d.b;
  // the caller's preconditioner (float32 blocks in a float32 first stage)
  auto user_call = [&](const void *R, void *T, int nb, const double *th, int fp64) {
    const int rc = Pc->user_apply(Pc->user_ctx, R, T, n, nb, th, fp64, c.s);
    if (rc != 0)
      throw Error(PHSVDS_EUSER, "user preconditioner returned " + std::to_string(rc));
  };
  auto solve_call = [&](const void *X, void *Y, int nb, int trans, int fp64) {
    const int rc = Pc->user_solve(Pc->user_ctx, X, Y, nb, trans, fp64, c.s);
    if (rc != 0) throw Error(PHSVDS_EUSER, "user solve returned " + std::to_string(rc));
  };
  // stage-1 hook in the working precision fp64: M R, or M^-1 (M^-T R) for
  // M ~ A through the m-row intermediate Ym (free while the correction is
  // formed)
  auto stage1_hook = [&](bool fp64, void *Ym) -> std::function<void(const void *, void *, int,
                                                                    const double *)> {
    if (pkind == PHSVDS_PREC_USER && Pc->user_apply)
      return [&, fp64](const void *R, void *T, int nb, const double *th) {
        user_call(R, T, nb, th, fp64 ? 1 : 0);
      };
    if (pkind == PHSVDS_PREC_USER_A)
      return [&, fp64, Ym](const void *R, void *T, int nb, const double *) {
        solve_call(R, Ym, nb, 1, fp64 ? 1 : 0);
        solve_call(Ym, T, nb, 0, fp64 ? 1 : 0);
      };
    return nullptr;
  };
  P1.user = d.fp32 ? stage1_hook(false, pl.s32.Yb) : stage1_hook(true, pl.s64.Yb);
  double si_anorm = 0.0;
  if (o.c_apply) {
    P1.opC = [&](const void *X, void *Y, int b) {
      const int rc = o.c_apply(o.c_ctx, X, Y, b, 1, c.s);
      if (rc != 0) throw Error(PHSVDS_EUSER, "C operator returned " + std::to_string(rc));
    };
    if (o.c_inverse) {
      // shift-invert: the running maximum is of C^-1's spectrum, ||A||
      // comes from the caller or from power iteration on A^T A
      si_anorm = o.anorm > 0 ? o.anorm
                             : std::sqrt(power_norm2(c, A64, At64, pl.tb.Xn, pl.tb.Ym, pl.tb.Z,
                                                     12, sp));
      if (!(o.anorm > 0)) stl.mv_prec += 12;
      P1.si_anorm = si_anorm;
      P1.anorm = 0.0;
    }
  }
  // stage-2 preconditioner of B on row-major N x ns blocks (row stride ldr),
  // through the column-major scratch blocks Cb and C2b (free while the
  // correction is formed, also inside JDQMR)
  const int64_t Nt = m + n;
  double *cb1 = pl.s2.Cb, *cb2 = pl.s2.C2b, *ub = pl.ub;
  auto stage2_hook =
      [&]() -> std::function<void(const double *, double *, int, int, const double *)> {
    if (pkind == PHSVDS_PREC_USER && Pc->user_apply_B)
      // the caller's own preconditioner of B
      return [&](const double *R, double *T, int ns, int ldr, const double *th) {
        copy(rmv_(const_cast<double *>(R), Nt, ns, ldr), cm(cb1, Nt, ns, Nt), c.s);
        const int rc = Pc->user_apply_B(Pc->user_ctx, cb1, cb2, Nt, ns, th, 1, c.s);
        if (rc != 0)
          throw Error(PHSVDS_EUSER, "user B-preconditioner returned " + std::to_string(rc));
        copy(cm(cb2, Nt, ns, Nt), rmv_(T, Nt, ns, ldr), c.s);
      };
    if (pkind == PHSVDS_PREC_USER)
      // B-form of the caller's M of C: [f; g] -> [M A^T g; A M f], theta of
      // C the squared estimates
      return [&](const double *R, double *T, int ns, int ldr, const double *th) {
        std::vector<double> th2(ns);
        for (int q = 0; q < ns; ++q) th2[q] = th[q] * th[q];
        const int64_t off = n * ns;
        copy(rmv_(const_cast<double *>(R), n, ns, ldr), cm(ub, n, ns, n), c.s);  // f
        user_call(ub, ub + off, ns, th2.data(), 1);                               // M f
        copy(cm(ub + off, n, ns, n), rmv_(cb1, n, ns, ldr), c.s);
        spmm(A64, ldr, cb1, T + n * ldr, false, c.s);                  // A M f -> bottom
        spmm(At64, ldr, R + n * ldr, cb2, false, c.s);                 // A^T g
        copy(rmv_(cb2, n, ns, ldr), cm(ub, n, ns, n), c.s);
        user_call(ub, ub + off, ns, th2.data(), 1);
        copy(cm(ub + off, n, ns, n), rmv_(T, n, ns, ldr), c.s);        // M A^T g -> top
        stl.mv_prec += ns;
      };
    if (pkind == PHSVDS_PREC_USER_A)
      // M ~ A: [f; g] -> [M^-1 g; M^-T f] (Section 4)
      return [&](const double *R, double *T, int ns, int ldr, const double *) {
        copy(rmv_(const_cast<double *>(R) + n * ldr, m, ns, ldr), cm(cb1, m, ns, m), c.s);
        solve_call(cb1, cb2, ns, 0, 1);                                // M^-1 g
        copy(cm(cb2, n, ns, n), rmv_(T, n, ns, ldr), c.s);
        copy(rmv_(const_cast<double *>(R), n, ns, ldr), cm(cb1, n, ns, n), c.s);
        solve_call(cb1, cb2, ns, 1, 1);                                // M^-T f
        copy(cm(cb2, m, ns, m), rmv_(T + n * ldr, m, ns, ldr), c.s);
      };
    return nullptr;
  };
  // saved first-stage output for a second stage alone: the caller's, or
  // the dynamic phase's when it chose B
  const double *resume_V = o.init_V;
  std::vector<double> resume_shifts;
  if (resume) resume_shifts.assign(o.shifts, o.shifts + k);
  int s2_extract = 0;
  if (o.dynamic) {
    // ------------------------------------ dynamic switching (Section 4.1)
    const double an0 = o.anorm > 0 ? o.anorm
                                   : std::sqrt(power_norm2(c, A64, At64, pl.tb.Xn, pl.tb.Ym,
                                                           pl.tb.Z, 12, sp));
    if (!(o.anorm > 0)) stl.mv_prec += 12;
    P1.anorm = an0;
    const int init_iter = o.init_iter > 0 ? o.init_iter : 50;
    const int max_switch = o.max_switch > 0 ? o.max_switch : 8;
    std::vector<double> sig;  // estimates of the columns of dynV, ascending
    int ncols = 0;
    bool first = true;
    auto seg_rate = [](const std::vector<double> &h) {
      double sum = 0.0;
      int cnt = 0;
      for (size_t i = 1; i < h.size(); ++i)
        if (!std::isnan(h[i]) && !std::isnan(h[i - 1])) sum += h[i] - h[i - 1], ++cnt;
      return cnt ? std::exp(sum / cnt) : 1.0;
    };
    // dynV <- the given columns of X (ld ldx) in ascending order of |est|
    auto take = [&](const double *X, int64_t ldx, std::vector<double> est, bool normalise) {
      const int nc = (int)est.size();
      std::vector<int> ord(nc);
      std::iota(ord.begin(), ord.end(), 0);
      for (double &e : est) e = std::fabs(e);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int q) { return est[a] < est[q]; });
      for (int i = 0; i < nc; ++i)
        copy(cm(const_cast<double *>(X) + (int64_t)ord[i] * ldx, n, 1, n),
             cm(pl.dynV + (int64_t)i * n, n, 1, n), c.s);
      if (normalise && nc) {
        double *nrm = sp.vec(7);
        colnorm2(cm(pl.dynV, n, nc, n), 0, n, nrm, c.sc, c.s);
        std::vector<double> nh(nc);
        c.d2h(nh.data(), nrm, nc * sizeof(double));
        c.sync();
        for (double &x : nh) x = x > 0 ? 1.0 / std::sqrt(x) : 0.0;
        c.h2d(sp.vec(7), nh.data(), nc * sizeof(double));
        scale_cols(cm(pl.dynV, n, nc, n), sp.vec(7), c.s);
      }
      sig.assign(nc, 0.0);
      for (int i = 0; i < nc; ++i) sig[i] = est[ord[i]];
      ncols = nc;
    };
    auto run = [&](bool onB, int iters) -> std::pair<double, int> {
      std::vector<double> h;
      if (!onB) {
        Stage1Params Q = P1;
        Q.max_iters = iters;
        Q.hist = &h;
        Q.init64 = first ? o.init_block : pl.dynV;
        Q.init_cols = first ? d.b : ncols;
        Stage1Result r = run_stage1<double>(c, A64, At64, Q, pl.s64, sp);
        stl.iters1 += r.iters;
        stl.restarts1 += r.restarts;
        stl.refreshes += r.refreshes;
        stl.rollbacks += r.rollbacks;
        std::vector<double> th(r.theta);
        th.insert(th.end(), r.best_theta.begin(), r.best_theta.end());
        for (double &t : th) t = std::sqrt(std::max(t, 0.0));
        take(pl.s64.Xl, n, th, false);
        first = false;
        return {seg_rate(h), r.nl};
      }
      resume_seeds(c, A64, pl.dynV, ncols, sig, an0, d.bw, pl.tb, sp);
      Stage2Params Q{};
      Q.k2 = ncols;
      Q.b = d.b;
      Q.bw = d.bw;
      Q.pmax = d.pmax;
      Q.pmin = d.pmin;
      Q.tol = tol;
      Q.anorm = an0;
      Q.shifts = sig.data();
      Q.v0 = pl.tb.Vt;
      Q.u0 = pl.tb.Ut;
      Q.max_restarts = P1.max_restarts;
      Q.max_iters = iters;
      Q.jacobi_d = pkind == PHSVDS_PREC_JACOBI ? pl.diagC : nullptr;
      Q.method = 0;
      Q.extract = 1;
      Q.precB = stage2_hook();
      Q.hist = &h;
      Stage2Result r = run_stage2(c, A64, At64, Q, pl.s2, sp);
      stl.iters2 += r.iters;
      stl.restarts2 += r.restarts;
      stl.refreshes += r.refreshes;
      std::vector<double> th(r.theta);
      th.insert(th.end(), r.best_theta.begin(), r.best_theta.end());
      take(r.Xl, m + n, th, true);
      return {seg_rate(h), r.nl};
    };
    // Algorithm 3: first tests on C and on B, then runs of the faster one
    double rate[2] = {1.0, 1.0};
    int num_conv = 0, last = 0, found = -1;
    auto record = [&](int on, int iters, std::pair<double, int> out) {
      rate[on] = out.first;
      num_conv += out.second;
      if (stl.dyn_runs < 16) {
        stl.dyn_on[stl.dyn_runs] = on + 1;
        stl.dyn_iters[stl.dyn_runs] = iters;
        stl.dyn_locked[stl.dyn_runs] = out.second;
        stl.dyn_rate[stl.dyn_runs] = out.first;
      }
      ++stl.dyn_runs;
      last = on;
      if (out.second >= k) found = on;
    };
    record(0, init_iter, run(false, init_iter));
    if (found < 0) record(1, init_iter, run(true, init_iter));
    int nsw = 0, j = 0;
    while (found < 0 && nsw < max_switch) {
      const int choice = rate[0] <= rate[1] ? 0 : 1;
      if ((nsw == 0 && num_conv > 0) || num_conv > 1) break;
      j = choice == last ? j + 1 : j / 2;
      const int iters = init_iter << std::min(j, 20);
      ++nsw;
      record(choice, iters, run(choice == 1, iters));
    }
    const int choice = found >= 0 ? found : (rate[0] <= rate[1] ? 0 : 1);
    stl.dyn_choice = choice + 1;
    stl.dyn_found = found >= 0 ? 1 : 0;
    if (choice == 0) {
      // the two-stage method from the latest approximations
      P1.init64 = pl.dynV;
      P1.init_cols = ncols;
    } else {
      // GD+k on B (harmonic) from them, as a second stage alone
      resume = true;
      resume_V = pl.dynV;
      resume_shifts = sig;
      s2_extract = 1;
    }
  }
  if (pkind == PHSVDS_PREC_GNN && !(o.anorm > 0)) {
    // a smoothing preconditioner keeps the top of the spectrum out of the
    // basis, so the largest Ritz value no longer estimates ||A||^2: start
    // the running maximum from power iteration on C (a lower bound)
    P1.sn2_init = power_norm2(c, A64, At64, pl.tb.Xn, pl.tb.Ym, pl.tb.Z, 12, sp);
    stl.mv_prec += 12;
  }
  Stage1Result r1;
  const double *Xl64 = nullptr, *Vr64 = nullptr;
  int nvr = 0;
  if (resume) {
    // saved first-stage output: the given vectors and shifts stand for the
    // locked pairs of stage 1; every pair goes through the second stage
    r1.converged = true;
    r1.nl = k;
    for (int i = 0; i < k; ++i) {
      r1.theta.push_back(resume_shifts[i] * resume_shifts[i]);
      r1.res.push_back(0.0);
      r1.tight.push_back(false);
    }
    if (o.dynamic) {
      r1.sn2 = P1.anorm * P1.anorm;
    } else {
      r1.sn2 = o.anorm > 0 ? o.anorm * o.anorm
                           : power_norm2(c, A64, At64, pl.tb.Xn, pl.tb.Ym, pl.tb.Z, 12, sp);
      if (!(o.anorm > 0)) stl.mv_prec += 12;
    }
    Xl64 = resume_V;
  } else {
  auto gnn32 = [&](const void *r, const void *x, double th, void *t) {
    gnn_forward(*Ain, pl.gg, pl.gb, Pc->gnn_weights, d.gw, (const float *)r, (const float *)x,
                th, (float *)t, c.s);
  };
  auto gnn64 = [&](const void *r, const void *x, double th, void *t) {
    copy(cm((double *)r, n, 1, n), cm(pl.gb.rf, n, 1, n), c.s);
    copy(cm((double *)x, n, 1, n), cm(pl.gb.xf, n, 1, n), c.s);
    gnn_forward(*Ain, pl.gg, pl.gb, Pc->gnn_weights, d.gw, pl.gb.rf, pl.gb.xf, th, pl.gb.tout,
                c.s);
    copy(cm(pl.gb.tout, n, 1, n), cm((double *)t, n, 1, n), c.s);
  };
  if (d.fp32) {
    if (d.gw && pkind == PHSVDS_PREC_GNN) P1.gnn = gnn32;
    P1.gnn_window = gwin;
    r1 = run_stage1<float>(c, A32, At32, P1, pl.s32, sp);
    stl.fp32_locked = r1.nl;
    stl.iters1 += r1.iters;
    stl.restarts1 += r1.restarts;
    if (d.cont) {
      // continue stage 1 in float64 from the float32 basis
      const int extra = std::min(r1.p, std::max(0, d.pmin - r1.nl));
      double *init = pl.s64.V[1];
      copy(cm(pl.s32.Xl, n, r1.nl, n), cm(init, n, r1.nl, n), c.s);
      if (extra)
        copy(cm((float *)r1.Vrest, n, extra, n), cm(init + (int64_t)r1.nl * n, n, extra, n), c.s);
      Stage1Params P2 = P1;
      if (d.gw && pkind == PHSVDS_PREC_GNN) P2.gnn = gnn64;
      P2.user = stage1_hook(true, pl.s64.Yb);
      P2.init64 = init;
      P2.init_cols = r1.nl + extra;
      P2.sn2_init = r1.sn2;
      if (P2.init_cols < d.b) P2.init_cols = d.b;
      r1 = run_stage1<double>(c, A64, At64, P2, pl.s64, sp);
      Xl64 = pl.s64.Xl;
      Vr64 = (const double *)r1.Vrest;
      nvr = r1.p;
    } else {
      // float32 results move to float64 buffers (re-sorted below)
      copy(cm(pl.s32.Xl, n, r1.nl + r1.nbest, n), cm(pl.Xs, n, r1.nl + r1.nbest, n), c.s);
      copy(cm((float *)r1.Vrest, n, r1.p, n), cm(pl.Vr64, n, r1.p, n), c.s);
      Xl64 = pl.Xs;
      Vr64 = pl.Vr64;
      nvr = r1.p;
    }
  } else {
    if (d.gw && pkind == PHSVDS_PREC_GNN) P1.gnn = gnn64;
    P1.gnn_window = gwin;
    r1 = run_stage1<double>(c, A64, At64, P1, pl.s64, sp);
    Xl64 = pl.s64.Xl;
    Vr64 = (const double *)r1.Vrest;
    nvr = r1.p;
  }
  }  // first stage
  if (o.c_inverse) {
    // eigenvalues mu of C^-1 -> theta = 1 / mu of C (sorted below)
    for (double &t : r1.theta) t = 1.0 / std::max(t, 1e-300);
    for (double &t : r1.best_theta) t = 1.0 / std::max(t, 1e-300);
    r1.sn2 = si_anorm * si_anorm;
  }
  stl.iters1 += d.fp32 && !d.cont ? 0 : r1.iters;
  stl.restarts1 += d.fp32 && !d.cont ? 0 : r1.restarts;
  stl.fallbacks += r1.fallbacks;
  stl.refreshes += r1.refreshes;
  stl.rollbacks += r1.rollbacks;
  c.sync();
  const double t2 = wall();
  stl.t_stage1 = t2 - t1;
  const double sn = std::sqrt(r1.sn2);
  stl.anorm_est = sn;
  const double an = o.anorm > 0 ? o.anorm : (o.dynamic ? P1.anorm : sn);
  const int nl = r1.nl;
  // best approximations of the pairs not converged follow the locked ones
  const int nbest = r1.nbest, ntot = nl + nbest;
  // sort the locked pairs (ascending, or descending for largest)
  std::vector<int> ord(nl);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    return largest ? r1.theta[a] > r1.theta[b] : r1.theta[a] < r1.theta[b];
  });
  double *Xs = (Xl64 == pl.Xs) ? pl.tb.Vt : pl.Xs;  // sorted copy
  std::vector<double> s1(nl);
  std::vector<bool> tight(nl);
  for (int i = 0; i < nl; ++i) {
    copy(cm(const_cast<double *>(Xl64) + (int64_t)ord[i] * n, n, 1, n),
         cm(Xs + (int64_t)i * n, n, 1, n), c.s);
    s1[i] = std::sqrt(std::max(r1.theta[ord[i]], 0.0));
    tight[i] = r1.tight[ord[i]];
    if (i < 64) stl.res_stage1[i] = r1.res[ord[i]];
  }
  if (nbest)
    copy(cm(const_cast<double *>(Xl64) + (int64_t)nl * n, n, nbest, n),
         cm(Xs + (int64_t)nl * n, n, nbest, n), c.s);
  if (Xs == pl.tb.Vt) {  // keep Xs away from the transition outputs
    copy(cm(pl.tb.Vt, n, ntot, n), cm(pl.Vf, n, ntot, n), c.s);
    Xs = pl.Vf;
  }
  // stage-2 entry (Section 3.1): pairs whose stage-1 test was floor-limited
  int need2 = 0;
  if (!largest && o.stage2 != -1 && nl > 0) {
    if (o.stage2 == 1 || resume) {
      need2 = nl;
    } else {
      for (int i = 0; i < nl; ++i) {
        bool floor_limited =
            d.fp32 && !d.cont ? !tight[i] : (tol * s1[i] < P1.floor * kEps64 * sn);
        if (floor_limited) need2 = i + 1;
      }
    }
  }
  stl.stage2_pairs = need2;
  bool conv = r1.converged && nl == k;
  double *Vsrc = Xs, *Usrc = nullptr;
  if (need2 > 0) {
    std::vector<double> shifts;
    if (resume)
      resume_seeds(c, A64, Xs, nl, s1, an, d.bw, pl.tb, sp), shifts = s1;
    else
      run_transition(c, A64, Xs, nl, Vr64, nvr, d.pmin, an, d.bw, pl.tb, sp, shifts);
    Stage2Params P2{};
    P2.k2 = need2;
    P2.b = d.b;
    P2.bw = d.bw;
    P2.pmax = d.pmax;
    P2.pmin = d.pmin;
    P2.tol = tol;
    P2.anorm = an;
    P2.shifts = shifts.data();
    P2.v0 = pl.tb.Vt;
    P2.u0 = pl.tb.Ut;
    P2.max_restarts = P1.max_restarts;
    P2.max_iters = 0;
    P2.jacobi_d = pkind == PHSVDS_PREC_JACOBI ? pl.diagC : nullptr;
    P2.method = o.stage2_method;
    P2.extract = s2_extract;
    P2.precB = stage2_hook();
    P2.max_inner = o.max_inner > 0 ? o.max_inner : 50;
    P2.jd_work = pl.jd;
    Stage2Result r2 = run_stage2(c, A64, At64, P2, pl.s2, sp);
    stl.iters2 = r2.iters;
    stl.restarts2 = r2.restarts;
    stl.refreshes += r2.refreshes;
    conv = conv && r2.converged;
    // assemble: stage-2 pairs from [v; u], the rest from the transition
    const int64_t N = m + n;
    copy(cm(pl.tb.Vt, n, nl, n), cm(pl.Vf, n, nl, n), c.s);
    copy(cm(pl.tb.Ut, m, nl, m), cm(pl.Uf, m, nl, m), c.s);
    if (r2.nl) {
      copy(cm(r2.Xl, n, r2.nl, N), cm(pl.Vf, n, r2.nl, n), c.s);
      copy(cm(r2.Xl + n, m, r2.nl, N), cm(pl.Uf, m, r2.nl, m), c.s);
    }
    if (nbest && Xs != pl.Vf)
      copy(cm(Xs + (int64_t)nl * n, n, nbest, n), cm(pl.Vf + (int64_t)nl * n, n, nbest, n), c.s);
    Vsrc = pl.Vf;
    Usrc = pl.Uf;
  } else {
    if (Xs != pl.Vf) copy(cm(Xs, n, ntot, n), cm(pl.Vf, n, ntot, n), c.s);
    Vsrc = pl.Vf;
  }
  c.sync();
  const double t3 = wall();
  stl.t_stage2 = t3 - t2;
  // ------------------------------------------- final float64 check (Sec. 5)
  double *nrm = sp.vec(20);
  std::vector<double> f(ntot), nh(ntot);
  if (ntot > 0) {
    colnorm2(cm(Vsrc, n, ntot, n), 0, n, nrm, c.sc, c.s);
    c.d2h(nh.data(), nrm, ntot * sizeof(double));
    c.sync();
    for (int i = 0; i < ntot; ++i) f[i] = nh[i] > 0 ? 1.0 / std::sqrt(nh[i]) : 0.0;
    c.h2d(sp.vec(21), f.data(), ntot * sizeof(double));
    scale_cols(cm(Vsrc, n, ntot, n), sp.vec(21), c.s);
    apply_cols(c, A64, Vsrc, ntot, pl.AV, pl.Fx, pl.Fy);
    stl.mv_final += ntot;
    if (!Usrc) {
      copy(cm(pl.AV, m, ntot, m), cm(pl.Uf, m, ntot, m), c.s);
      Usrc = pl.Uf;
    }
    if (nbest)  // left vectors of the best approximations: A v / ||A v||
      copy(cm(pl.AV + (int64_t)nl * m, m, nbest, m), cm(pl.Uf + (int64_t)nl * m, m, nbest, m),
           c.s);
    colnorm2(cm(Usrc, m, ntot, m), 0, m, nrm, c.sc, c.s);
    c.d2h(nh.data(), nrm, ntot * sizeof(double));
    c.sync();
    for (int i = 0; i < ntot; ++i) f[i] = nh[i] > 0 ? 1.0 / std::sqrt(nh[i]) : 0.0;
    c.h2d(sp.vec(21), f.data(), ntot * sizeof(double));
    scale_cols(cm(Usrc, m, ntot, m), sp.vec(21), c.s);
  }
  std::vector<double> sig(ntot, 0.0), res(ntot, 0.0);
  if (ntot > 0) {
    double *G = sp.mat(31);
    for (int c0 = 0; c0 < ntot; c0 += 32) {
      int w = std::min(32, ntot - c0);
      tn(cm(Usrc, m, ntot, m), cm<double>(nullptr, m, 0, m), cm(pl.AV + (int64_t)c0 * m, m, w, m),
         G + (int64_t)c0 * kSP, kSP, c.sc, c.s);
    }
    std::vector<double> gh((size_t)kSP * ntot);
    c.d2h(gh.data(), G, gh.size() * sizeof(double));
    c.sync();
    std::vector<double> flip(ntot, 1.0), dneg((size_t)kSP * kSP, 0.0);
    for (int i = 0; i < ntot; ++i) {
      sig[i] = gh[i + (size_t)i * kSP];
      if (sig[i] < 0) {
        flip[i] = -1.0;
        sig[i] = -sig[i];
      }
      dneg[i + (size_t)i * kSP] = -sig[i];
    }
    c.h2d(sp.vec(21), flip.data(), ntot * sizeof(double));
    scale_cols(cm(Usrc, m, ntot, m), sp.vec(21), c.s);
    c.h2d(sp.mat(32), dneg.data(), dneg.size() * sizeof(double));
    // r_v = A v - sigma u ; r_u = A^T u - sigma v
    copy(cm(pl.AV, m, ntot, m), cm(pl.RV, m, ntot, m), c.s);
    nn(cm(Usrc, m, ntot, m), cm<double>(nullptr, m, 0, m), sp.mat(32), kSP, 1.0, cm(pl.RV, m, ntot, m),
       1.0, c.s);
    apply_cols(c, At64, Usrc, ntot, pl.RU, pl.Fx, pl.Fy);
    nn(cm(Vsrc, n, ntot, n), cm<double>(nullptr, n, 0, n), sp.mat(32), kSP, 1.0, cm(pl.RU, n, ntot, n),
       1.0, c.s);
    std::vector<double> a(ntot), bq(ntot);
    colnorm2(cm(pl.RV, m, ntot, m), 0, m, nrm, c.sc, c.s);
    c.d2h(a.data(), nrm, ntot * sizeof(double));
    c.sync();
    colnorm2(cm(pl.RU, n, ntot, n), 0, n, nrm, c.sc, c.s);
    c.d2h(bq.data(), nrm, ntot * sizeof(double));
    c.sync();
    for (int i = 0; i < ntot; ++i) res[i] = std::sqrt(a[i] + bq[i]);
  }
  // order, sign convention, outputs
  std::vector<int> fo(ntot);
  std::iota(fo.begin(), fo.end(), 0);
  std::stable_sort(fo.begin(), fo.end(),
                   [&](int a, int b) { return largest ? sig[a] > sig[b] : sig[a] < sig[b]; });
  for (int i = 0; i < k; ++i) {
    if (i < ntot) {
      int j = fo[i];
      copy(cm(Vsrc + (int64_t)j * n, n, 1, n), cm(Vout + (int64_t)i * n, n, 1, n), c.s);
      if (row_perm)
        unpermute_rows(m, 1, pl.binA, Usrc + (int64_t)j * m, Uout + (int64_t)i * m, c.s);
      else
        copy(cm(Usrc + (int64_t)j * m, m, 1, m), cm(Uout + (int64_t)i * m, m, 1, m), c.s);
      sigma[i] = sig[j];
      resnorm[i] = res[j];
    } else {
      PHS_HIP(hipMemsetAsync(Vout + (int64_t)i * n, 0, n * sizeof(double), c.s));
      PHS_HIP(hipMemsetAsync(Uout + (int64_t)i * m, 0, m * sizeof(double), c.s));
      sigma[i] = NAN;
      resnorm[i] = INFINITY;
    }
  }
  if (ntot > 0) {
    k_sign_fix<<<std::min(ntot, k), 256, 0, c.s>>>(Vout, n, Uout, m);
    PHS_CHECK_LAUNCH();
  }
  c.sync();
  stl.t_total = wall() - t0;
  if (stats) *stats = stl;
  bool ok = conv && nl == k;
  for (int i = 0; i < nl && ok; ++i) ok = res[i] <= tol * an * (1.0 + 1e-8);
  return ok ? PHSVDS_OK : PHSVDS_NOT_CONVERGED;
}


int harvest_impl(const phsvds_csr *Ain, int k, int every, int max_pairs, double tol,
                 double cg_tol, int cg_maxit, double shift_scale, const phsvds_opts *oin,
                 void *ws, size_t ws_bytes,
                 void *stream, double *Rout, double *Xout, double *Tout, double *theta_out,
                 int *count_out, phsvds_stats *stats) {
  PHS_REQUIRE(Ain && Rout && Xout && Tout && theta_out && count_out, kEinval, "null argument");
  phsvds_opts o;
  phsvds_default_opts(&o);
  if (oin) o = *oin;
  o.stage1_fp32 = 0;
  const int64_t m = Ain->m, n = Ain->n, nnz = Ain->nnz;
  PHS_REQUIRE(m >= n && n >= 1 && every >= 1 && max_pairs >= 0, kEinval, "bad harvest sizes");
  PHS_REQUIRE(shift_scale >= 0.0 && shift_scale <= 1.0, kEinval, "shift_scale must be in [0, 1]");
  Dims d;
  PHS_REQUIRE(make_dims(m, n, nnz, k, o, d), kEinval, "unsupported sizes");
  d.cg = true;
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  Plan pl{};
  carve(ar, d, pl);
  phsvds_stats stl;
  std::memset(&stl, 0, sizeof(stl));
  Ctx c;
  c.s = (hipStream_t)stream;
  c.sc = pl.sc;
  c.didx = pl.didx;
  c.seed = o.seed;
  c.st = &stl;
  SmallPool sp;
  sp.base = pl.pool;
  {
    std::vector<double> eye((size_t)kSP * kSP, 0.0);
    for (int i = 0; i < kSP; ++i) eye[i + (size_t)i * kSP] = 1.0;
    c.h2d(sp.eye(), eye.data(), eye.size() * sizeof(double));
  }
  SpMat<double> A64, At64;
  A64.m = m; A64.n = n; A64.nnz = nnz;
  A64.rowptr = Ain->rowptr; A64.colind = Ain->colind; A64.val = Ain->val;
  csr_transpose(m, n, nnz, Ain->rowptr, Ain->colind, Ain->val, pl.trp, pl.tci, pl.tva, pl.tws,
                pl.tws_bytes, c.s);
  At64.m = n; At64.n = m; At64.nnz = nnz;
  At64.rowptr = pl.trp; At64.colind = pl.tci; At64.val = pl.tva;
  Stage1Params P1{};
  P1.k = k; P1.b = d.b; P1.bw = d.bw; P1.pmax = d.pmax; P1.pmin = d.pmin;
  P1.largest = false; P1.tol = tol; P1.floor = 10.0; P1.anorm = o.anorm;
  P1.max_restarts = o.max_restarts > 0 ? o.max_restarts : 10000;
  P1.init64 = o.init_block; P1.init_cols = d.b;
  int count = 0;
  // stop once max_pairs are written (the solve itself need not converge),
  // or after 50 times the iterations that could fill them
  P1.stop = [&]() { return count >= max_pairs; };
  P1.max_iters = (int64_t)every * 50 * ((max_pairs + d.b - 1) / d.b + 1);
  P1.snap = [&](int64_t it, const void *Xb, const void *Rb, const double *th, int nb,
                const void *Xl, int nl) {
    if (it % every || count >= max_pairs) return;
    std::vector<int> ok = projected_cg_block(c, A64, At64, (const double *)Xl, nl,
                                             (const double *)Xb, nb, d.bw, th, shift_scale,
                                             (const double *)Rb, cg_tol, cg_maxit, pl.cg, sp);
    for (int j = 0; j < nb && count < max_pairs; ++j) {
      if (!ok[j]) continue;
      Tall<double> src;
      src.rows = n; src.cols = 1; src.rs = d.bw; src.cs = 1;
      src.p = const_cast<double *>((const double *)Rb) + j;
      copy(src, cm(Rout + (int64_t)count * n, n, 1, n), c.s);
      src.p = const_cast<double *>((const double *)Xb) + j;
      copy(src, cm(Xout + (int64_t)count * n, n, 1, n), c.s);
      src.p = pl.cg.T + j;
      copy(src, cm(Tout + (int64_t)count * n, n, 1, n), c.s);
      theta_out[count] = th[j];
      ++count;
    }
  };
  run_stage1<double>(c, A64, At64, P1, pl.s64, sp);
  c.sync();
  *count_out = count;
  if (stats) *stats = stl;
  return PHSVDS_OK;
}

}  // namespace
}  // namespace phs

using namespace phs;

extern "C" {

void phsvds_default_opts(phsvds_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->which = 0;
  o->block = 1;
  o->stage1_fp32 = 0;
  o->fp64_continue = 1;
  o->stage2 = 0;
  o->max_restarts = 10000;
  o->seed = 1;
  o->floor_factor = 10.0;
  o->stage2_method = 1;
  o->max_inner = 50;
}

const char *phsvds_version(void) { return "phsvds-mi355x 0.1 (gfx950)"; }

const char *phsvds_last_error(void) { return g_err.c_str(); }

int phsvds_spmm_f64(const phsvds_csr *A, int b, const double *X, double *Y, int absval,
                    void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(A && X && Y, kEinval, "null argument");
    SpMat<double> S;
    S.m = A->m;
    S.n = A->n;
    S.nnz = A->nnz;
    S.rowptr = A->rowptr;
    S.colind = A->colind;
    S.val = A->val;
    spmm(S, b, X, Y, absval != 0, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_rr_eig(const double *H, int ldh, int p, int nvec, int largest, double *theta,
                  double *S, int lds, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(H && theta && S, kEinval, "null argument");
    PHS_REQUIRE(ldh >= p && lds >= p, kEinval, "leading dimension below p");
    syev_rr(H, ldh, p, nvec, largest != 0, theta, S, lds, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_small_svd(const double *M, int ldm, int rows, int cols, double *sv, double *Y, int ldy,
                     void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(M && sv && Y, kEinval, "null argument");
    PHS_REQUIRE(ldm >= rows && ldy >= cols, kEinval, "leading dimension too small");
    svdj(M, ldm, rows, cols, sv, Y, ldy, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_spmm_f32(const phsvds_csr *A, const float *val32, int b, const float *X, float *Y,
                    int absval, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(A && val32 && X && Y, kEinval, "null argument");
    SpMat<float> S;
    S.m = A->m;
    S.n = A->n;
    S.nnz = A->nnz;
    S.rowptr = A->rowptr;
    S.colind = A->colind;
    S.val = val32;
    spmm(S, b, X, Y, absval != 0, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

size_t phsvds_spmm_ws_bytes(const phsvds_csr *A, int trans, int fp32) {
  if (!A || !trans) return 0;
  return spmm_t_ws_bytes(A->m, A->n, A->nnz, fp32 != 0);
}

int phsvds_spmm(const phsvds_csr *A, const float *val32, int trans, int fp32, int b,
                const void *X, void *Y, void *ws, size_t ws_bytes, void *stream) {
  return guarded([&]() {
    spmm_op(A, val32, trans != 0, fp32 != 0, b, X, Y, ws, ws_bytes, (hipStream_t)stream, true);
    return PHSVDS_OK;
  });
}

size_t phsvds_jacobi_ws_bytes(const phsvds_csr *A) {
  if (!A) return 0;
  return spmm_t_ws_bytes(A->m, A->n, A->nnz, false) + (size_t)A->n * sizeof(double) + 256;
}

int phsvds_jacobi_scaled_values(const phsvds_csr *A, double *val_out, void *ws,
                                size_t ws_bytes, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(A && val_out && A->val, kEinval, "null argument");
    jacobi_scaled_values(A, val_out, ws, ws_bytes, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_spmm_noalloc(const phsvds_csr *A, const float *val32, int trans, int fp32, int b,
                        const void *X, void *Y, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(A, kEinval, "null argument");
    void *ws = nullptr;
    size_t need = 0;
    if (trans) {
      need = spmm_t_ws_bytes(A->m, A->n, A->nnz, fp32 != 0);
      PHS_REQUIRE(need <= kNoAllocScratchBytes, kEnomem,
                  "phsvds_spmm_noalloc: this transposed product needs " + std::to_string(need) +
                      " bytes of scratch, above the " + std::to_string(kNoAllocScratchBytes) +
                      " the library holds per GPU");
      ws = noalloc_scratch();
    }
    spmm_op(A, val32, trans != 0, fp32 != 0, b, X, Y, ws, need, (hipStream_t)stream, false);
    return PHSVDS_OK;
  });
}

size_t phsvds_tsgemm_ws_bytes(void) { return (size_t)kPartCap * sizeof(double); }

int phsvds_tsgemm_tn(int fp32, int64_t rows, int nx, int ny, const void *X, int64_t ldx,
                     const void *Y, int64_t ldy, int layout, double *G, int ldg, void *ws,
                     size_t ws_bytes, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(X && Y && G && ws, kEinval, "null argument");
    PHS_REQUIRE((layout & ~3) == 0, kEinval, "tsgemm_tn: unknown layout bits");
    const bool ycol = (layout & 1) != 0, xrow = (layout & 2) != 0;
    PHS_REQUIRE(rows >= 1 && nx >= 1 && nx <= 128 && ny >= 1 && ny <= 32, kEinval,
                "tsgemm_tn: need rows >= 1, 1 <= nx <= 128, 1 <= ny <= 32");
    PHS_REQUIRE((xrow ? ldx >= nx : ldx >= rows) && ldg >= nx && (ycol ? ldy >= rows : ldy >= ny),
                kEinval, "tsgemm_tn: leading dimension too small");
    PHS_REQUIRE(ws_bytes >= (size_t)kPartCap * sizeof(double), kEnomem,
                "tsgemm_tn: workspace too small");
    Scratch sc;
    sc.part = (double *)ws;
    const hipStream_t s = (hipStream_t)stream;
    if (fp32) {
      float *xp = (float *)const_cast<void *>(X), *yp = (float *)const_cast<void *>(Y);
      Tall<float> x = xrow ? Tall<float>{xp, rows, nx, ldx, 1} : cm(xp, rows, nx, ldx);
      Tall<float> y = ycol ? cm(yp, rows, ny, ldy) : Tall<float>{yp, rows, ny, ldy, 1};
      tn(x, cm<float>(nullptr, rows, 0, rows), y, G, ldg, sc, s);
    } else {
      double *xp = (double *)const_cast<void *>(X), *yp = (double *)const_cast<void *>(Y);
      Tall<double> x = xrow ? Tall<double>{xp, rows, nx, ldx, 1} : cm(xp, rows, nx, ldx);
      Tall<double> y = ycol ? cm(yp, rows, ny, ldy) : Tall<double>{yp, rows, ny, ldy, 1};
      tn(x, cm<double>(nullptr, rows, 0, rows), y, G, ldg, sc, s);
    }
    return PHSVDS_OK;
  });
}

int phsvds_tsgemm_nn(int fp32, int64_t rows, int nx, int ny, double alpha, const void *X,
                     int64_t ldx, const double *S, int lds, double beta, void *Y, int64_t ldy,
                     void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(X && S && Y, kEinval, "null argument");
    PHS_REQUIRE(rows >= 1 && nx >= 1 && nx <= 160 && ny >= 1 && ny <= 64, kEinval,
                "tsgemm_nn: need rows >= 1, 1 <= nx <= 160, 1 <= ny <= 64");
    PHS_REQUIRE(ldx >= rows && ldy >= rows && lds >= nx, kEinval,
                "tsgemm_nn: leading dimension too small");
    const hipStream_t s = (hipStream_t)stream;
    if (fp32) {
      nn(cm((float *)const_cast<void *>(X), rows, nx, ldx), cm<float>(nullptr, rows, 0, rows), S,
         lds, alpha, cm((float *)Y, rows, ny, ldy), beta, s);
    } else {
      nn(cm((double *)const_cast<void *>(X), rows, nx, ldx), cm<double>(nullptr, rows, 0, rows),
         S, lds, alpha, cm((double *)Y, rows, ny, ldy), beta, s);
    }
    return PHSVDS_OK;
  });
}

size_t phsvds_transpose_ws_bytes(const phsvds_csr *A) {
  if (!A) return 0;
  return transpose_ws_bytes(A->m, A->n, A->nnz);
}

int phsvds_csr_transpose(const phsvds_csr *A, int64_t *t_rowptr, int32_t *t_colind,
                         double *t_val, void *ws, size_t ws_bytes, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(A && t_rowptr && t_colind && t_val, kEinval, "null argument");
    PHS_REQUIRE(ws_bytes >= transpose_ws_bytes(A->m, A->n, A->nnz), kEnomem,
                "transpose workspace too small");
    csr_transpose(A->m, A->n, A->nnz, A->rowptr, A->colind, A->val, t_rowptr, t_colind, t_val,
                  ws, ws_bytes, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int k, const phsvds_opts *oin,
                           size_t *bytes) {
  return guarded([&]() {
    PHS_REQUIRE(bytes, kEinval, "null argument");
    phsvds_opts o;
    phsvds_default_opts(&o);
    if (oin) o = *oin;
    Dims d;
    PHS_REQUIRE(m >= n && n >= 1 && make_dims(m, n, nnz, k, o, d), kEinval,
                "unsupported sizes: need m >= n, 1 <= k <= 64, block <= 16, max_basis <= 64");
    Arena ar;
    ar.dry = true;
    Plan pl{};
    carve(ar, d, pl);
    *bytes = ar.used;
    return PHSVDS_OK;
  });
}

int phsvds_harvest_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int k,
                                   const phsvds_opts *oin, size_t *bytes) {
  return guarded([&]() {
    PHS_REQUIRE(bytes, kEinval, "null argument");
    phsvds_opts o;
    phsvds_default_opts(&o);
    if (oin) o = *oin;
    o.stage1_fp32 = 0;
    Dims d;
    PHS_REQUIRE(m >= n && n >= 1 && make_dims(m, n, nnz, k, o, d), kEinval, "unsupported sizes");
    d.cg = true;
    Arena ar;
    ar.dry = true;
    Plan pl{};
    carve(ar, d, pl);
    *bytes = ar.used;
    return PHSVDS_OK;
  });
}

int phsvds_harvest(const phsvds_csr *A, int k, int every, int max_pairs, double tol,
                   double cg_tol, int cg_maxit, double shift_scale, const phsvds_opts *opts,
                   void *workspace, size_t ws_bytes, void *stream, double *R, double *X,
                   double *T, double *theta, int *count, phsvds_stats *stats) {
  return guarded([&]() {
    return harvest_impl(A, k, every, max_pairs, tol, cg_tol, cg_maxit, shift_scale, opts,
                        workspace, ws_bytes, stream, R, X, T, theta, count, stats);
  });
}

int64_t phsvds_gnn_nweights(int width) { return gnn_nweights(width); }

size_t phsvds_gnn_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int width) {
  Arena ar;
  ar.dry = true;
  GnnGraph g;
  GnnBufs b;
  gnn_carve(ar, m, n, nnz, width, g, b);
  return ar.used;
}

static void gnn_views(const phsvds_csr *A, int width, void *gws, size_t bytes, GnnGraph &g,
                      GnnBufs &b) {
  PHS_REQUIRE(A && gws, kEinval, "null argument");
  PHS_REQUIRE(width == 8 || width == 16 || width == 32, kEinval, "width must be 8, 16 or 32");
  Arena ar;
  ar.base = (char *)gws;
  ar.size = bytes;
  gnn_carve(ar, A->m, A->n, A->nnz, width, g, b);
}

int phsvds_gnn_prepare(const phsvds_csr *A, int width, void *gws, size_t bytes, void *stream) {
  return guarded([&]() {
    GnnGraph g;
    GnnBufs b;
    gnn_views(A, width, gws, bytes, g, b);
    gnn_prepare(*A, g, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_gnn_forward(const phsvds_csr *A, int width, void *gws, size_t bytes, const float *w,
                       const float *r, const float *x, double theta, float *t, void *stream) {
  return guarded([&]() {
    GnnGraph g;
    GnnBufs b;
    gnn_views(A, width, gws, bytes, g, b);
    PHS_REQUIRE(w && r && x && t, kEinval, "null argument");
    gnn_forward(*A, g, b, w, width, r, x, theta, t, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_gnn_loss_grad(const phsvds_csr *A, int width, void *gws, size_t bytes, const float *w,
                         const float *r, const float *x, double theta, const float *tstar,
                         double *grad, double *loss, void *stream) {
  return guarded([&]() {
    GnnGraph g;
    GnnBufs b;
    gnn_views(A, width, gws, bytes, g, b);
    PHS_REQUIRE(w && r && x && tstar && grad && loss, kEinval, "null argument");
    gnn_loss_grad(*A, g, b, w, width, r, x, theta, tstar, b.tout, grad, loss,
                  (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_gnn_residual_loss_grad(const phsvds_csr *A, int width, void *gws, size_t bytes,
                                  const float *w, const float *r, const float *x, double theta,
                                  double *grad, double *loss, void *stream) {
  return guarded([&]() {
    GnnGraph g;
    GnnBufs b;
    gnn_views(A, width, gws, bytes, g, b);
    PHS_REQUIRE(w && r && x && grad && loss, kEinval, "null argument");
    gnn_loss_grad(*A, g, b, w, width, r, x, theta, nullptr, b.tout, grad, loss,
                  (hipStream_t)stream, 1);
    return PHSVDS_OK;
  });
}

int phsvds_gnn_adam(float *w, float *m, float *v, const double *grad, int64_t nw, int step,
                    double lr, double grad_scale, void *stream) {
  return guarded([&]() {
    PHS_REQUIRE(w && m && v && grad && nw > 0 && step >= 1, kEinval, "bad Adam arguments");
    gnn_adam(w, m, v, grad, nw, step, lr, grad_scale, (hipStream_t)stream);
    return PHSVDS_OK;
  });
}

int phsvds_svds(const phsvds_csr *A, int k, double tol, const phsvds_precond *P,
                const phsvds_opts *opts, void *workspace, size_t ws_bytes, void *stream,
                double *sigma, double *U, double *V, double *resnorm, phsvds_stats *stats) {
  return guarded([&]() {
    return svds_impl(A, nullptr, k, tol, P, opts, workspace, ws_bytes, stream, sigma, U, V,
                     resnorm, stats);
  });
}

int phsvds_svds_op(const phsvds_operator *A, int k, double tol, const phsvds_precond *P,
                   const phsvds_opts *opts, void *workspace, size_t ws_bytes, void *stream,
                   double *sigma, double *U, double *V, double *resnorm, phsvds_stats *stats) {
  return guarded([&]() {
    PHS_REQUIRE(A, kEinval, "null operator");
    return svds_impl(nullptr, A, k, tol, P, opts, workspace, ws_bytes, stream, sigma, U, V,
                     resnorm, stats);
  });
}

}  // extern "C"
