// Learned preconditioner: a message-passing network over the graph of
// C = A^T A, float32 on the device (forward, back-propagation, Adam).
//
// Per node j (width w, three layers):
//   h0_j = [u_j, u_j d_j / max(d_j - tau, d_j/10), d_j, tau],  u = rh / sqrt(d),
//          rh = r sqrt(n)/||r||, d = diag(C)/mean(diag C), tau = theta/mean(diag C)
//   pre^l = h^{l-1} Ws_l + b_l + Ch (h^{l-1} Wm_l),  h^l = relu(pre^l)
//   Ch    = D^-1/2 A^T A D^-1/2 (two float32 SpMMs of width w)
//   t_j   = ((I - x x^T) t~)_j,  t~_j = (h^3 wo + h0_1)_j ||r|| / (sqrt(n) mean(diag C) sqrt(d_j))
// Input and output both carry D^-1/2, so the network's linear part, a
// polynomial q in Ch, acts as the symmetric D^-1/2 q(Ch) D^-1/2; h0_1 through
// the readout is exactly the Jacobi step r / max(diag C - theta, diag C / 10),
// so the network learns a correction to the Jacobi preconditioner.
// The node-wise dense layers run one thread per node with the weights in
// LDS; aggregation reuses the row-major SpMM kernels at width w.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "gnn.hpp"
#include "prof.hpp"

namespace phs {

int64_t gnn_nweights(int w, int nin) { return 2LL * nin * w + w + 2LL * (2LL * w * w + w) + w; }

GnnOffsets gnn_offsets(int w, int nin) {
  GnnOffsets o;
  int64_t at = 0;
  o.Ws[0] = at; at += (int64_t)nin * w;
  o.Wm[0] = at; at += (int64_t)nin * w;
  o.b[0] = at; at += w;
  for (int l = 1; l < 3; ++l) {
    o.Ws[l] = at; at += (int64_t)w * w;
    o.Wm[l] = at; at += (int64_t)w * w;
    o.b[l] = at; at += w;
  }
  o.wo = at; at += w;
  o.total = at;
  return o;
}

void gnn_carve(Arena &ar, int64_t m, int64_t n, int64_t nnz, int w, GnnGraph &g, GnnBufs &b) {
  g.trp = ar.take<int64_t>(n + 1);
  g.tci = ar.take<int32_t>(std::max<int64_t>(nnz, 1));
  g.tva = ar.take<double>(std::max<int64_t>(nnz, 1));
  g.tws_bytes = transpose_ws_bytes(m, n, nnz);
  g.tws = ar.take<char>(g.tws_bytes);
  g.va32 = ar.take<float>(std::max<int64_t>(nnz, 1));
  g.tva32 = ar.take<float>(std::max<int64_t>(nnz, 1));
  g.d64 = ar.take<double>(n);
  g.dn = ar.take<float>(n);
  g.isd = ar.take<float>(n);
  g.meta = ar.take<double>(8);
  b.h0 = ar.take<float>(n * kGnnIn);
  for (int l = 0; l < 3; ++l) {
    b.pre[l] = ar.take<float>(n * w);
    b.h[l] = ar.take<float>(n * w);
  }
  b.S = ar.take<float>(n * w);
  b.M = ar.take<float>(n * w);
  b.Z = ar.take<float>(n * w);
  b.Ym = ar.take<float>(m * w);
  b.delta = ar.take<float>(n * w);
  b.dh = ar.take<float>(n * w);
  b.traw = ar.take<float>(n);
  b.g = ar.take<float>(n);
  b.tout = ar.take<float>(n);
  b.rf = ar.take<float>(n);
  b.xf = ar.take<float>(n);
  b.vec = ar.take<double>(64);
  b.G = ar.take<double>(64 * 64);
  b.sc.part = ar.take<double>(kPartCap);
  b.sc.aux = ar.take<double>(kAuxCap);
  b.sc.flag = ar.take<int>(64);
}

__global__ void k_to_float(const double *a, float *b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

__global__ __launch_bounds__(256) void k_gnn_diag(const double *d64, int64_t n, float *dn,
                                                  float *isd, double *meta) {
  // single block: mean of diag(C), then normalised diagonal and D^-1/2
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += d64[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    dn[i] = (float)(d64[i] / mean);
    isd[i] = (float)(1.0 / sqrt(d64[i] > 0 ? d64[i] : 1.0));
  }
  if (threadIdx.x == 0) meta[0] = mean;
}

void gnn_prepare(const phsvds_csr &A, GnnGraph &g, hipStream_t s) {
  const int64_t m = A.m, n = A.n, nnz = A.nnz;
  csr_transpose(m, n, nnz, A.rowptr, A.colind, A.val, g.trp, g.tci, g.tva, g.tws, g.tws_bytes, s);
  int64_t blocks = std::min<int64_t>(cdiv(std::max<int64_t>(nnz, 1), 256), 8192);
  k_to_float<<<(unsigned)blocks, 256, 0, s>>>(A.val, g.va32, nnz);
  k_to_float<<<(unsigned)blocks, 256, 0, s>>>(g.tva, g.tva32, nnz);
  SpMat<double> At;
  At.m = n;
  At.n = m;
  At.nnz = nnz;
  At.rowptr = g.trp;
  At.colind = g.tci;
  At.val = g.tva;
  col_sq_norms(At, g.d64, s);
  k_gnn_diag<<<1, 256, 0, s>>>(g.d64, n, g.dn, g.isd, g.meta);
  PHS_CHECK_LAUNCH();
}

static void views(const phsvds_csr &A, const GnnGraph &g, SpMat<float> &A32, SpMat<float> &At32) {
  A32.m = A.m;
  A32.n = A.n;
  A32.nnz = A.nnz;
  A32.rowptr = A.rowptr;
  A32.colind = A.colind;
  A32.val = g.va32;
  At32.m = A.n;
  At32.n = A.m;
  At32.nnz = A.nnz;
  At32.rowptr = g.trp;
  At32.colind = g.tci;
  At32.val = g.tva32;
}

// ------------------------------------------------------------- kernels
// h0 from r (norm ||r||^2 in nr2[0]), theta and the normalised diagonal.
__global__ void k_gnn_feat(const float *r, int64_t n, const float *dn, const double *meta,
                           double theta, const double *nr2, float *h0) {
  const double nr = sqrt(fmax(nr2[0], 1e-300));
  const double sc = sqrt((double)n) / nr;
  const double tau = theta / meta[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = dn[i];
    const double u = r[i] * sc / sqrt(d);
    const double den = fmax(d - tau, 0.1 * d);
    h0[i * kGnnIn + 0] = (float)u;
    h0[i * kGnnIn + 1] = (float)(u * d / den);
    h0[i * kGnnIn + 2] = (float)d;
    h0[i * kGnnIn + 3] = (float)tau;
  }
}

// Rows of K floats (K a multiple of 4, 16-byte aligned) moved as float4.
template <int K>
__device__ inline void load_row(const float *__restrict__ p, float (&o)[K]) {
  static_assert(K % 4 == 0, "row width must be a multiple of 4");
#pragma unroll
  for (int q = 0; q < K / 4; ++q) {
    const float4 u = reinterpret_cast<const float4 *>(p)[q];
    o[4 * q] = u.x;
    o[4 * q + 1] = u.y;
    o[4 * q + 2] = u.z;
    o[4 * q + 3] = u.w;
  }
}
template <int K>
__device__ inline void store_row(float *__restrict__ p, const float (&o)[K]) {
#pragma unroll
  for (int q = 0; q < K / 4; ++q)
    reinterpret_cast<float4 *>(p)[q] =
        make_float4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
}

// S = h Ws + b ; M = D^-1/2 (h Wm)   (h: n x FIN, outputs n x W).  One
// thread per node: its input row is loaded whole before the products; the
// weights are wavefront-uniform reads (scalar loads, no LDS traffic).  One
// node per thread and no loop over nodes, so the weight loads stay next to
// their products instead of being hoisted (2 W FIN values would not fit in
// scalar registers).
template <int W, int FIN>
__global__ __launch_bounds__(256) void k_gnn_dense(const float *__restrict__ h, int64_t n,
                                                   const float *__restrict__ Ws,
                                                   const float *__restrict__ Wm,
                                                   const float *__restrict__ bias,
                                                   const float *__restrict__ isd,
                                                   float *__restrict__ S, float *__restrict__ M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float hv[FIN];
    load_row<FIN>(h + i * FIN, hv);
    const float sc = isd[i];
    float as[W], am[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      as[c] = bias[c];
      am[c] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < FIN; ++k)
#pragma unroll
      for (int c = 0; c < W; ++c) {
        as[c] = fmaf(hv[k], Ws[k * W + c], as[c]);
        am[c] = fmaf(hv[k], Wm[k * W + c], am[c]);
      }
#pragma unroll
    for (int c = 0; c < W; ++c) am[c] *= sc;
    store_row<W>(S + i * W, as);
    store_row<W>(M + i * W, am);
  }
}

// pre = S + D^-1/2 Z ; h = relu(pre)
__global__ void k_gnn_combine(const float *S, const float *Z, const float *isd, int64_t n, int w,
                              float *pre, float *h) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * w;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float p = S[e] + isd[e / w] * Z[e];
    pre[e] = p;
    h[e] = p > 0.f ? p : 0.f;
  }
}

// traw_i = (h3_i . wo + h0_i1) * scale, scale = ||r|| / (sqrt(n) mean(diag C))
template <int W>
__global__ __launch_bounds__(256) void k_gnn_readout(const float *__restrict__ h,
                                                     const float *__restrict__ h0,
                                                     const float *__restrict__ dn, int64_t n,
                                                     const float *__restrict__ wo,
                                                     const double *nr2, const double *meta,
                                                     float *__restrict__ traw) {
  const double scale = sqrt(fmax(nr2[0], 0.0)) / (sqrt((double)n) * meta[0]);
  float wv[W];
#pragma unroll
  for (int c = 0; c < W; ++c) wv[c] = wo[c];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float hr[W];
    load_row<W>(h + i * W, hr);
    float s = h0[i * kGnnIn + 1];
#pragma unroll
    for (int c = 0; c < W; ++c) s = fmaf(hr[c], wv[c], s);
    traw[i] = (float)(s * scale / sqrt((double)dn[i]));
  }
}

// g_j /= sqrt(d_j)
__global__ void k_scale_isd(float *g, const float *dn, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    g[i] = (float)((double)g[i] / sqrt((double)dn[i]));
}

// y = a - coef[0] * x   (coef on the device, scaled by mul)
__global__ void k_axpy_dev(const float *a, const float *x, const double *coef, double mul,
                           int64_t n, float *y) {
  const float cf = (float)(coef[0] * mul);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - cf * x[i];
}

// gradient of the loss w.r.t. the projected output: g = 2 (t - t*) / ||t*||^2
__global__ void k_gnn_lossgrad(const float *t, const float *ts, const double *tsn2, int64_t n,
                               float *g) {
  const double f = 2.0 / fmax(tsn2[0], 1e-300);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    g[i] = (float)(f * ((double)t[i] - (double)ts[i]));
}

// delta = dh (o) [pre > 0]; for the last layer dh = scale * g (x) wo
__global__ void k_gnn_delta_top(const float *graw, const float *wo, const double *nr2,
                                const double *meta, const float *pre, int64_t n, int w,
                                float *delta) {
  const double scale = sqrt(fmax(nr2[0], 0.0)) / (sqrt((double)n) * meta[0]);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * w;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / w;
    const int c = (int)(e % w);
    delta[e] = pre[e] > 0.f ? (float)(scale * graw[i] * wo[c]) : 0.f;
  }
}

// dh_prev = delta Ws^T + dM Wm^T (n x W: the previous layer has width W),
// then masked by the previous layer's pre-activation into delta_prev.  Rows
// are loaded whole before the products; weights are wavefront-uniform reads.
template <int W>
__global__ __launch_bounds__(256) void k_gnn_back_dense(const float *__restrict__ delta,
                                                        const float *__restrict__ dM, int64_t n,
                                                        const float *__restrict__ Ws,
                                                        const float *__restrict__ Wm,
                                                        const float *__restrict__ pre_prev,
                                                        float *__restrict__ delta_prev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float dl[W], dm[W], pp[W], out[W];
    load_row<W>(delta + i * W, dl);
    load_row<W>(dM + i * W, dm);
    load_row<W>(pre_prev + i * W, pp);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      float sacc = 0.f;
#pragma unroll
      for (int c = 0; c < W; ++c)
        sacc = fmaf(dl[c], Ws[k * W + c], fmaf(dm[c], Wm[k * W + c], sacc));
      out[k] = pp[k] > 0.f ? sacc : 0.f;
    }
    store_row<W>(delta_prev + i * W, out);
  }
}

__global__ void k_row_scale_f(float *x, const float *s, int64_t n, int w) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * w;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= s[e / w];
}

// grad[off + i*w + c] += G[i + c*ldg]  (column-major double -> row-major)
__global__ void k_grad_acc(const double *G, int ldg, int fin, int w, double *grad) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < fin * w; e += gridDim.x * blockDim.x) {
    int i = e / w, c = e % w;
    grad[e] += G[i + (int64_t)c * ldg];
  }
}

__global__ void k_adam(float *w, float *m, float *v, const double *g, int64_t nw, double gscale,
                       double lr, double b1, double b2, double eps, double bc1, double bc2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double gg = g[e] * gscale;
    const double mk = b1 * (double)m[e] + (1 - b1) * gg;
    const double vk = b2 * (double)v[e] + (1 - b2) * gg * gg;
    m[e] = (float)mk;
    v[e] = (float)vk;
    w[e] = (float)((double)w[e] - lr * (mk / bc1) / (sqrt(vk / bc2) + eps));
  }
}

static unsigned grid_for(int64_t work) {
  int64_t b = cdiv(std::max<int64_t>(work, 1), 256);
  return (unsigned)std::min<int64_t>(b, 8192);
}

// one thread per node (kernels without a loop over nodes)
static unsigned node_grid(int64_t n) {
  PHS_REQUIRE(n <= (int64_t)256 * 0x7fffffff, kEinval, "gnn: too many nodes");
  return (unsigned)cdiv(std::max<int64_t>(n, 1), 256);
}

template <typename F>
static void dispatch_w(int w, F &&f) {
  switch (w) {
    case 8: f(std::integral_constant<int, 8>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    default: throw Error(kEinval, "gnn: width must be 8, 16 or 32");
  }
}

// Ch Z for Z n x w (row-major, float32): D^-1/2 A^T A D^-1/2 Z, in place on
// out (n x w), using b.Ym as the m x w intermediate.
static void apply_Ch(const SpMat<float> &A32, const SpMat<float> &At32, const GnnGraph &g,
                     GnnBufs &b, int w, float *Z_in_scaled, float *out, hipStream_t s) {
  spmm(A32, w, Z_in_scaled, b.Ym, false, s);
  spmm(At32, w, b.Ym, out, false, s);
}

void gnn_forward(const phsvds_csr &A, const GnnGraph &g, GnnBufs &b, const float *wts, int w,
                 const float *r, const float *x, double theta, float *t, hipStream_t s) {
  const int64_t n = A.n;
  SpMat<float> A32, At32;
  views(A, g, A32, At32);
  const GnnOffsets o = gnn_offsets(w, kGnnIn);
  colnorm2(cm(const_cast<float *>(r), n, 1, n), 0, n, b.vec, b.sc, s);
  k_gnn_feat<<<grid_for(n), 256, 0, s>>>(r, n, g.dn, g.meta, theta, b.vec, b.h0);
  const float *hin = b.h0;
  int fin = kGnnIn;
  for (int l = 0; l < 3; ++l) {
    dispatch_w(w, [&](auto WW) {
      constexpr int W = decltype(WW)::value;
      if (l == 0)
        k_gnn_dense<W, kGnnIn><<<node_grid(n), 256, 0, s>>>(hin, n, wts + o.Ws[l],
                                                           wts + o.Wm[l], wts + o.b[l], g.isd,
                                                           b.S, b.M);
      else
        k_gnn_dense<W, W><<<node_grid(n), 256, 0, s>>>(hin, n, wts + o.Ws[l], wts + o.Wm[l],
                                                      wts + o.b[l], g.isd, b.S, b.M);
    });
    apply_Ch(A32, At32, g, b, w, b.M, b.Z, s);
    k_gnn_combine<<<grid_for(n * w), 256, 0, s>>>(b.S, b.Z, g.isd, n, w, b.pre[l], b.h[l]);
    hin = b.h[l];
    fin = w;
  }
  dispatch_w(w, [&](auto WW) {
    constexpr int W = decltype(WW)::value;
    k_gnn_readout<W><<<grid_for(n), 256, 0, s>>>(b.h[2], b.h0, g.dn, n, wts + o.wo, b.vec,
                                                 g.meta, b.traw);
  });
  // t = traw - x (x^T traw)
  tn(cm(const_cast<float *>(x), n, 1, n), cm<float>(nullptr, n, 0, n), cm(b.traw, n, 1, n),
     b.vec + 1, 1, b.sc, s);
  k_axpy_dev<<<grid_for(n), 256, 0, s>>>(b.traw, x, b.vec + 1, 1.0, n, t);
  PHS_CHECK_LAUNCH();
}

// e = a - c (float32)
__global__ void k_sub_f(const float *a, const float *c, int64_t n, float *e) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    e[i] = a[i] - c[i];
}

// g *= f / den[0]
__global__ void k_scale_by(float *g, int64_t n, const double *den, double f) {
  const double c = f / fmax(den[0], 1e-300);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    g[i] = (float)(c * (double)g[i]);
}

// loss[0] += num[0] / den[0]
__global__ void k_ratio_acc(const double *num, const double *den, double *loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) loss[0] += num[0] / fmax(den[0], 1e-300);
}

void gnn_loss_grad(const phsvds_csr &A, const GnnGraph &g, GnnBufs &b, const float *wts, int w,
                   const float *r, const float *x, double theta, const float *tstar, float *t,
                   double *grad, double *loss_dev, hipStream_t s, int kind) {
  const int64_t n = A.n;
  SpMat<float> A32, At32;
  views(A, g, A32, At32);
  const GnnOffsets o = gnn_offsets(w, kGnnIn);
  gnn_forward(A, g, b, wts, w, r, x, theta, t, s);
  if (kind == 1) {
    // loss = ||C t - r||^2 / ||r||^2 ; g = 2 C (C t - r) / ||r||^2, with
    // C t from two float32 products (b.M holds e until the backward pass)
    spmm(A32, 1, t, b.Ym, false, s);
    spmm(At32, 1, b.Ym, b.M, false, s);
    k_sub_f<<<grid_for(n), 256, 0, s>>>(b.M, r, n, b.M);
    colnorm2(cm(b.M, n, 1, n), 0, n, b.vec + 3, b.sc, s);
    colnorm2(cm(const_cast<float *>(r), n, 1, n), 0, n, b.vec + 2, b.sc, s);
    k_ratio_acc<<<1, 64, 0, s>>>(b.vec + 3, b.vec + 2, loss_dev);
    spmm(A32, 1, b.M, b.Ym, false, s);
    spmm(At32, 1, b.Ym, b.g, false, s);
    k_scale_by<<<grid_for(n), 256, 0, s>>>(b.g, n, b.vec + 2, 2.0);
    PHS_CHECK_LAUNCH();
  } else {
    // loss = ||t - t*||^2 / ||t*||^2 ; g = 2 (t - t*)/||t*||^2
    colnorm2(cm(const_cast<float *>(tstar), n, 1, n), 0, n, b.vec + 2, b.sc, s);
    k_gnn_lossgrad<<<grid_for(n), 256, 0, s>>>(t, tstar, b.vec + 2, n, b.g);
    // loss_dev[0] += ||g||^2 ||t*||^2 / 4  (= ||t - t*||^2 / ||t*||^2)
    colnorm2(cm(b.g, n, 1, n), 0, n, b.vec + 3, b.sc, s);
    gnn_loss_acc(b.vec + 3, b.vec + 2, loss_dev, s);
  }
  // graw = (I - x x^T) g
  tn(cm(const_cast<float *>(x), n, 1, n), cm<float>(nullptr, n, 0, n), cm(b.g, n, 1, n),
     b.vec + 4, 1, b.sc, s);
  k_axpy_dev<<<grid_for(n), 256, 0, s>>>(b.g, x, b.vec + 4, 1.0, n, b.g);
  // through the per-node output scale 1 / sqrt(d_j)
  k_scale_isd<<<grid_for(n), 256, 0, s>>>(b.g, g.dn, n);
  // dwo = scale * h3^T graw
  {
    tn(rm(b.h[2], n, w), cm<float>(nullptr, n, 0, n), cm(b.g, n, 1, n), b.G, 64, b.sc, s);
    // scale folded in by a 1 x w accumulation with factor: use the delta kernel path
  }
  k_gnn_delta_top<<<grid_for(n * w), 256, 0, s>>>(b.g, wts + o.wo, b.vec, g.meta, b.pre[2], n, w,
                                                  b.delta);
  PHS_CHECK_LAUNCH();
  gnn_scale_acc(b.G, 64, w, b.vec, g.meta, n, grad + o.wo, s);
  for (int l = 2; l >= 0; --l) {
    const int fin = l == 0 ? kGnnIn : w;
    const float *hin = l == 0 ? b.h0 : b.h[l - 1];
    // dWs = hin^T delta ; db = sum delta ; dM = Ch delta ; dWm = hin^T dM
    tn(rm(const_cast<float *>(hin), n, fin), cm<float>(nullptr, n, 0, n), rm(b.delta, n, w), b.G,
       64, b.sc, s);
    k_grad_acc<<<grid_for(fin * w), 256, 0, s>>>(b.G, 64, fin, w, grad + o.Ws[l]);
    colsum_acc(rm(b.delta, n, w), grad + o.b[l], b.sc, s);
    copy(rm(b.delta, n, w), rm(b.M, n, w), s);
    k_row_scale_f<<<grid_for(n * w), 256, 0, s>>>(b.M, g.isd, n, w);
    apply_Ch(A32, At32, g, b, w, b.M, b.Z, s);
    k_row_scale_f<<<grid_for(n * w), 256, 0, s>>>(b.Z, g.isd, n, w);  // dM
    tn(rm(const_cast<float *>(hin), n, fin), cm<float>(nullptr, n, 0, n), rm(b.Z, n, w), b.G, 64,
       b.sc, s);
    k_grad_acc<<<grid_for(fin * w), 256, 0, s>>>(b.G, 64, fin, w, grad + o.Wm[l]);
    if (l > 0) {
      dispatch_w(w, [&](auto WW) {
        constexpr int W = decltype(WW)::value;
        k_gnn_back_dense<W><<<node_grid(n), 256, 0, s>>>(b.delta, b.Z, n, wts + o.Ws[l],
                                                        wts + o.Wm[l], b.pre[l - 1], b.dh);
      });
      std::swap(b.delta, b.dh);
    }
    PHS_CHECK_LAUNCH();
  }
}

void gnn_adam(float *w, float *m, float *v, const double *g, int64_t nw, int step, double lr,
              double gscale, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  k_adam<<<grid_for(nw), 256, 0, s>>>(w, m, v, g, nw, gscale, lr, b1, b2, 1e-8,
                                      1.0 - std::pow(b1, step), 1.0 - std::pow(b2, step));
  PHS_CHECK_LAUNCH();
}

// grad_wo[c] += scale * G[c]  (G: w x 1 column, scale from ||r||)
__global__ void k_scale_acc(const double *G, int w, const double *nr2, const double *meta,
                            int64_t n, double *gout) {
  const double scale = sqrt(fmax(nr2[0], 0.0)) / (sqrt((double)n) * meta[0]);
  for (int c = threadIdx.x; c < w; c += blockDim.x) gout[c] += scale * G[c];
}

void gnn_scale_acc(const double *G, int ldg, int w, const double *nr2, const double *meta,
                   int64_t n, double *gout, hipStream_t s) {
  (void)ldg;
  k_scale_acc<<<1, 64, 0, s>>>(G, w, nr2, meta, n, gout);
  PHS_CHECK_LAUNCH();
}

// loss += ||g||^2 ||t*||^2 / 4
__global__ void k_loss_acc(const double *g2, const double *ts2, double *loss) {
  if (threadIdx.x == 0) loss[0] += 0.25 * g2[0] * ts2[0];
}

void gnn_loss_acc(const double *g2, const double *ts2, double *loss, hipStream_t s) {
  k_loss_acc<<<1, 64, 0, s>>>(g2, ts2, loss);
  PHS_CHECK_LAUNCH();
}

// out[c] += sum_i X(i, c) (row-major float block)
__global__ __launch_bounds__(256) void k_colsum(const float *X, int64_t n, int w, double *part) {
  __shared__ double red[256];
  for (int c = 0; c < w; ++c) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      s += X[i * w + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * w + c] = red[0];
    __syncthreads();
  }
}

__global__ void k_colsum_fin(const double *part, int nblk, int w, double *out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= w) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * w + c];
  out[c] += s;
}

void colsum_acc(const Tall<float> &X, double *out, const Scratch &sc, hipStream_t s) {
  int64_t blocks = std::min<int64_t>(cdiv(std::max<int64_t>(X.rows, 1), 1024), 256);
  k_colsum<<<(unsigned)blocks, 256, 0, s>>>(X.p, X.rows, X.cols, sc.part);
  k_colsum_fin<<<1, 64, 0, s>>>(sc.part, (int)blocks, X.cols, out);
  PHS_CHECK_LAUNCH();
}

}  // namespace phs
