// Small dense float64 kernels, one workgroup each (p <= 64).
//
// The projected problems of the method -- the eigendecomposition of the
// Rayleigh-Ritz matrix H (Algorithm 2 step 8), the SVD of the refined
// projection factor R (step 9), Cholesky factors for CholQR, restart
// rotations -- are at most 64 x 64.  They run in LDS inside one workgroup:
// cyclic Jacobi for the symmetric eigenproblem and one-sided (Hestenes)
// Jacobi for the SVD, both with round-robin pair ordering so that the p/2
// rotations of a round are applied in parallel.  Jacobi methods compute
// small eigenvalues and singular values to high relative accuracy, which
// the refined projection needs near convergence.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace phs {

constexpr int kSmallMax = 64;
constexpr int kLd = kSmallMax + 1;  // LDS row padding

__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Round-robin (circle method) pairing of P (even) indices: in round r,
// pair k is (a, b) with a < b.
__device__ inline void rr_pair(int P, int r, int k, int &a, int &b) {
  const int M = P - 1;
  if (k == 0) {
    a = r % M;
    b = M;
  } else {
    a = (r + k) % M;
    b = (r - k + M) % M;
  }
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
}

// ---------------------------------------------------------- syevj
__global__ __launch_bounds__(256) void k_syevj(const double *H, int ldh, int p, int P,
                                               bool desc, double *theta, double *Sout,
                                               int lds) {
  __shared__ double a[kSmallMax * kLd];
  __shared__ double v[kSmallMax * kLd];
  __shared__ double cs[kSmallMax / 2][2];
  __shared__ int pr[kSmallMax / 2][2];
  __shared__ int nrot;
  const int t = threadIdx.x;
  for (int idx = t; idx < P * P; idx += blockDim.x) {
    int i = idx % P, j = idx / P;
    a[i * kLd + j] = (i < p && j < p) ? 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh])
                                      : 0.0;
    v[i * kLd + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int half = P / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < P - 1; ++r) {
      if (t < half) {
        int i, j;
        rr_pair(P, r, t, i, j);
        pr[t][0] = i;
        pr[t][1] = j;
        double aij = a[i * kLd + j], aii = a[i * kLd + i], ajj = a[j * kLd + j];
        double c = 1.0, s = 0.0;
        if (aij != 0.0 && fabs(aij) > 1e-300 &&
            fabs(aij) > 2.220446049250313e-16 * sqrt(fabs(aii) * fabs(ajj))) {
          double tau = (ajj - aii) / (2.0 * aij);
          double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          atomicAdd(&nrot, 1);
        }
        cs[t][0] = c;
        cs[t][1] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = t; idx < half * P; idx += blockDim.x) {
        int k = idx / P, col = idx % P;
        double c = cs[k][0], s = cs[k][1];
        if (s == 0.0) continue;
        int i = pr[k][0], j = pr[k][1];
        double ai = a[i * kLd + col], aj = a[j * kLd + col];
        a[i * kLd + col] = c * ai - s * aj;
        a[j * kLd + col] = s * ai + c * aj;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int idx = t; idx < half * P; idx += blockDim.x) {
        int k = idx / P, row = idx % P;
        double c = cs[k][0], s = cs[k][1];
        if (s == 0.0) continue;
        int i = pr[k][0], j = pr[k][1];
        double ai = a[row * kLd + i], aj = a[row * kLd + j];
        a[row * kLd + i] = c * ai - s * aj;
        a[row * kLd + j] = s * ai + c * aj;
        double vi = v[row * kLd + i], vj = v[row * kLd + j];
        v[row * kLd + i] = c * vi - s * vj;
        v[row * kLd + j] = s * vi + c * vj;
      }
      __syncthreads();
      if (t < half && cs[t][1] != 0.0) {
        int i = pr[t][0], j = pr[t][1];
        a[i * kLd + j] = 0.0;
        a[j * kLd + i] = 0.0;
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  // sort: rank of each diagonal entry (ties by index)
  for (int i = t; i < p; i += blockDim.x) {
    double di = a[i * kLd + i];
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      double dj = a[j * kLd + j];
      bool before = desc ? (dj > di || (dj == di && j < i)) : (dj < di || (dj == di && j < i));
      rank += before;
    }
    theta[rank] = di;
    for (int row = 0; row < p; ++row) Sout[row + (int64_t)rank * lds] = v[row * kLd + i];
  }
}

void syevj(const double *H, int ldh, int p, bool descending, double *theta, double *S, int lds,
           hipStream_t s) {
  PHS_REQUIRE(p >= 1 && p <= kSmallMax, kEinval, "syevj: size out of range");
  int P = p + (p & 1);
  if (P < 2) P = 2;
  k_syevj<<<1, 256, 0, s>>>(H, ldh, p, P, descending, theta, S, lds);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------------ svdj
// One-sided Jacobi on the columns of M (rows x cols), rows <= 2 * 64.
constexpr int kSvdRows = 2 * kSmallMax;
__global__ __launch_bounds__(256) void k_svdj(const double *M, int ldm, int rows, int cols,
                                              int P, double *sv, double *Yout, int ldy) {
  __shared__ double g[kSmallMax * kSvdRows];  // column-major, ld = kSvdRows
  __shared__ double y[kSmallMax * kSmallMax];  // column-major, ld = kSmallMax
  __shared__ double cs[kSmallMax / 2][2];
  __shared__ int nrot;
  const int t = threadIdx.x;
  for (int idx = t; idx < P * kSvdRows; idx += blockDim.x) {
    int i = idx % kSvdRows, j = idx / kSvdRows;
    g[j * kSvdRows + i] = (i < rows && j < cols) ? M[i + (int64_t)j * ldm] : 0.0;
  }
  for (int idx = t; idx < P * kSmallMax; idx += blockDim.x) {
    int i = idx % kSmallMax, j = idx / kSmallMax;
    y[j * kSmallMax + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int half = P / 2;
  // 256 threads: groups of G = 256 / half threads per pair (power of two)
  int G = 1;
  while (G * 2 * half <= 256 && G < 64) G *= 2;
  const int pair = t / G, lane = t % G;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < P - 1; ++r) {
      int i = 0, j = 0;
      double al = 0, be = 0, ga = 0;
      if (pair < half) {
        rr_pair(P, r, pair, i, j);
        for (int k = lane; k < rows; k += G) {
          double gi = g[i * kSvdRows + k], gj = g[j * kSvdRows + k];
          al += gi * gi;
          be += gj * gj;
          ga += gi * gj;
        }
      }
      for (int off = G / 2; off > 0; off >>= 1) {
        al += __shfl_xor(al, off, G);
        be += __shfl_xor(be, off, G);
        ga += __shfl_xor(ga, off, G);
      }
      if (pair < half && lane == 0) {
        double c = 1.0, s = 0.0;
        if (ga != 0.0 && fabs(ga) > 2.220446049250313e-16 * sqrt(al * be)) {
          double zeta = (be - al) / (2.0 * ga);
          double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          atomicAdd(&nrot, 1);
        }
        cs[pair][0] = c;
        cs[pair][1] = s;
      }
      __syncthreads();
      if (pair < half) {
        double c = cs[pair][0], s = cs[pair][1];
        if (s != 0.0) {
          for (int k = lane; k < rows; k += G) {
            double gi = g[i * kSvdRows + k], gj = g[j * kSvdRows + k];
            g[i * kSvdRows + k] = c * gi - s * gj;
            g[j * kSvdRows + k] = s * gi + c * gj;
          }
          for (int k = lane; k < cols; k += G) {
            double yi = y[i * kSmallMax + k], yj = y[j * kSmallMax + k];
            y[i * kSmallMax + k] = c * yi - s * yj;
            y[j * kSmallMax + k] = s * yi + c * yj;
          }
        }
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  __shared__ double nrm[kSmallMax];
  for (int j = t; j < cols; j += blockDim.x) {
    double s2 = 0.0;
    for (int k = 0; k < rows; ++k) s2 += g[j * kSvdRows + k] * g[j * kSvdRows + k];
    nrm[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = t; j < cols; j += blockDim.x) {
    int rank = 0;
    for (int q = 0; q < cols; ++q) rank += (nrm[q] < nrm[j]) || (nrm[q] == nrm[j] && q < j);
    sv[rank] = nrm[j];
    for (int k = 0; k < cols; ++k) Yout[k + (int64_t)rank * ldy] = y[j * kSmallMax + k];
  }
}

void svdj(const double *M, int ldm, int rows, int cols, double *sv, double *Y, int ldy,
          hipStream_t s) {
  PHS_REQUIRE(cols >= 1 && cols <= kSmallMax && rows >= cols && rows <= kSvdRows, kEinval,
              "svdj: size out of range");
  int P = cols + (cols & 1);
  if (P < 2) P = 2;
  k_svdj<<<1, 256, 0, s>>>(M, ldm, rows, cols, P, sv, Y, ldy);
  PHS_CHECK_LAUNCH();
}

// -------------------------------------------------------- chol_inv
__global__ __launch_bounds__(256) void k_chol_inv(const double *G, int ldg, int w, double shift,
                                                  double *Rg, double *Ri, int ldr, int *flag) {
  __shared__ double r[kSmallMax * kLd];  // r[i * kLd + j], upper triangle used
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int idx = t; idx < w * w; idx += blockDim.x) {
    int i = idx % w, j = idx / w;
    r[i * kLd + j] = 0.5 * (G[i + (int64_t)j * ldg] + G[j + (int64_t)i * ldg]) +
                     (i == j ? shift : 0.0);
  }
  __syncthreads();
  // right-looking: after step k, row k holds R(k, k:w)
  for (int k = 0; k < w; ++k) {
    if (t == 0) {
      double d = r[k * kLd + k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        d = 1.0;
      }
      r[k * kLd + k] = sqrt(d);
    }
    __syncthreads();
    double piv = r[k * kLd + k];
    for (int j = k + 1 + t; j < w; j += blockDim.x) r[k * kLd + j] /= piv;
    __syncthreads();
    for (int idx = t; idx < (w - k - 1) * (w - k - 1); idx += blockDim.x) {
      int i = k + 1 + idx / (w - k - 1), j = k + 1 + idx % (w - k - 1);
      if (j >= i) r[i * kLd + j] -= r[k * kLd + i] * r[k * kLd + j];
    }
    __syncthreads();
  }
  // write R, then Rinv column by column (thread per column, back substitution)
  for (int idx = t; idx < w * w; idx += blockDim.x) {
    int i = idx % w, j = idx / w;
    Rg[i + (int64_t)j * ldr] = (j >= i) ? r[i * kLd + j] : 0.0;
  }
  for (int j = t; j < w; j += blockDim.x) {
    // solve R x = e_j; x_i = 0 for i > j
    for (int i = w - 1; i >= 0; --i) {
      double x = 0.0;
      if (i <= j) {
        double sacc = (i == j) ? 1.0 : 0.0;
        for (int q = i + 1; q <= j; ++q) sacc -= r[i * kLd + q] * Ri[q + (int64_t)j * ldr];
        x = sacc / r[i * kLd + i];
      }
      Ri[i + (int64_t)j * ldr] = x;
    }
  }
  __syncthreads();
  if (t == 0) flag[0] = bad;
}

void chol_inv(const double *G, int ldg, int w, double shift, double *R, double *Rinv, int ldr,
              int *flag, hipStream_t s) {
  PHS_REQUIRE(w >= 1 && w <= kSmallMax, kEinval, "chol_inv: size out of range");
  k_chol_inv<<<1, 256, 0, s>>>(G, ldg, w, shift, R, Rinv, ldr, flag);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------ small gemm
__global__ __launch_bounds__(256) void k_small_gemm(bool ta, bool tb, int M, int N, int K,
                                                    double alpha, const double *A, int lda,
                                                    const double *B, int ldb, double beta,
                                                    double *C, int ldc) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < M * N;
       idx += gridDim.x * blockDim.x) {
    int i = idx % M, j = idx / M;
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
      double av = ta ? A[k + (int64_t)i * lda] : A[i + (int64_t)k * lda];
      double bv = tb ? B[j + (int64_t)k * ldb] : B[k + (int64_t)j * ldb];
      s = fma(av, bv, s);
    }
    double c = alpha * s;
    if (beta != 0.0) c += beta * C[i + (int64_t)j * ldc];
    C[i + (int64_t)j * ldc] = c;
  }
}

void small_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
                const double *B, int ldb, double beta, double *C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  k_small_gemm<<<cdiv((int64_t)M * N, 256), 256, 0, s>>>(ta, tb, M, N, K, alpha, A, lda, B, ldb,
                                                         beta, C, ldc);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------ MGS2 helpers (restart, QR)
// Orthogonalise column `c` of q (rows x *, ld kSvdRows in LDS) against
// columns [0, upto) twice; returns the norms before and after.
__device__ inline void mgs2_col(double *q, int rows, int c, int upto, double *red, double *rcoef,
                                double &n0, double &n2) {
  const int t = threadIdx.x;
  double s = 0.0;
  for (int k = t; k < rows; k += blockDim.x) s += q[c * kSvdRows + k] * q[c * kSvdRows + k];
  n0 = sqrt(block_sum(s, red));
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < upto; ++j) {
      double d = 0.0;
      for (int k = t; k < rows; k += blockDim.x) d += q[j * kSvdRows + k] * q[c * kSvdRows + k];
      d = block_sum(d, red);
      for (int k = t; k < rows; k += blockDim.x) q[c * kSvdRows + k] -= d * q[j * kSvdRows + k];
      if (rcoef && t == 0) rcoef[j] += d;
      __syncthreads();
    }
  }
  s = 0.0;
  for (int k = t; k < rows; k += blockDim.x) s += q[c * kSvdRows + k] * q[c * kSvdRows + k];
  n2 = sqrt(block_sum(s, red));
}

__global__ __launch_bounds__(256) void k_restart_basis(const double *K, int ldk, int rows,
                                                       int kc, const double *P, int ldp, int pc,
                                                       double *Y, int ldy, int *count) {
  __shared__ double q[kSmallMax * kSvdRows];
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int idx = t; idx < rows * kc; idx += blockDim.x) {
    int i = idx % rows, j = idx / rows;
    q[j * kSvdRows + i] = K[i + (int64_t)j * ldk];
  }
  __syncthreads();
  int cur = kc;
  for (int c = 0; c < pc && cur < kSmallMax; ++c) {
    for (int k = t; k < rows; k += blockDim.x) q[cur * kSvdRows + k] = P[k + (int64_t)c * ldp];
    __syncthreads();
    double n0, n2;
    mgs2_col(q, rows, cur, cur, red, nullptr, n0, n2);
    if (n0 > 0.0 && n2 > 1e-8 * n0) {
      for (int k = t; k < rows; k += blockDim.x) q[cur * kSvdRows + k] /= n2;
      ++cur;
    }
    __syncthreads();
  }
  for (int idx = t; idx < rows * cur; idx += blockDim.x) {
    int i = idx % rows, j = idx / rows;
    Y[i + (int64_t)j * ldy] = q[j * kSvdRows + i];
  }
  if (t == 0) count[0] = cur;
}

void restart_basis(const double *K, int ldk, int rows, int kc, const double *P, int ldp, int pc,
                   double *Y, int ldy, int *count, hipStream_t s) {
  PHS_REQUIRE(rows <= kSvdRows && kc + pc <= kSmallMax + 32 && kc <= kSmallMax, kEinval,
              "restart_basis: size out of range");
  k_restart_basis<<<1, 256, 0, s>>>(K, ldk, rows, kc, P, ldp, pc, Y, ldy, count);
  PHS_CHECK_LAUNCH();
}

__global__ __launch_bounds__(256) void k_small_qr(const double *M, int ldm, int rows, int cols,
                                                  double *Q, int ldq, double *R, int ldr) {
  __shared__ double q[kSmallMax * kSvdRows];
  __shared__ double red[256];
  __shared__ double rc[kSmallMax];
  const int t = threadIdx.x;
  for (int idx = t; idx < rows * cols; idx += blockDim.x) {
    int i = idx % rows, j = idx / rows;
    q[j * kSvdRows + i] = M[i + (int64_t)j * ldm];
  }
  for (int idx = t; idx < cols * cols; idx += blockDim.x) R[idx % cols + (int64_t)(idx / cols) * ldr] = 0.0;
  __syncthreads();
  for (int c = 0; c < cols; ++c) {
    if (t < kSmallMax) rc[t] = 0.0;
    __syncthreads();
    double n0, n2;
    mgs2_col(q, rows, c, c, red, rc, n0, n2);
    double inv = n2 > 0.0 ? 1.0 / n2 : 0.0;
    for (int k = t; k < rows; k += blockDim.x) q[c * kSvdRows + k] *= inv;
    if (t == 0) {
      for (int j = 0; j < c; ++j) R[j + (int64_t)c * ldr] = rc[j];
      R[c + (int64_t)c * ldr] = n2;
    }
    __syncthreads();
  }
  for (int idx = t; idx < rows * cols; idx += blockDim.x) {
    int i = idx % rows, j = idx / rows;
    Q[i + (int64_t)j * ldq] = q[j * kSvdRows + i];
  }
}

void small_qr(const double *M, int ldm, int rows, int cols, double *Q, int ldq, double *R,
              int ldr, hipStream_t s) {
  PHS_REQUIRE(rows <= kSvdRows && cols <= kSmallMax && cols <= rows, kEinval,
              "small_qr: size out of range");
  k_small_qr<<<1, 256, 0, s>>>(M, ldm, rows, cols, Q, ldq, R, ldr);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------------ misc
__global__ void k_h_border(double *H, int ldh, int p, int nb, const double *G, int ldg) {
  const int tot = (p + nb) * nb;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += gridDim.x * blockDim.x) {
    int i = idx % (p + nb), c = idx / (p + nb);
    double gv = G[i + (int64_t)c * ldg];
    if (i < p) {
      H[i + (int64_t)(p + c) * ldh] = gv;
      H[(p + c) + (int64_t)i * ldh] = gv;
    } else {
      int r = i - p;
      double sym = 0.5 * (gv + G[(p + c) + (int64_t)r * ldg]);
      H[i + (int64_t)(p + c) * ldh] = sym;
    }
  }
}

void h_border(double *H, int ldh, int p, int nb, const double *G, int ldg, hipStream_t s) {
  k_h_border<<<cdiv((int64_t)(p + nb) * nb, 256), 256, 0, s>>>(H, ldh, p, nb, G, ldg);
  PHS_CHECK_LAUNCH();
}

__global__ void k_gather_cols(const double *A, int lda, int rows, const int *idx, int nc,
                              double *B, int ldb) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * nc;
       e += gridDim.x * blockDim.x) {
    int i = e % rows, c = e / rows;
    B[i + (int64_t)c * ldb] = A[i + (int64_t)idx[c] * lda];
  }
}

void gather_cols(const double *A, int lda, int rows, const int *idx, int nc, double *B, int ldb,
                 hipStream_t s) {
  if (rows * nc == 0) return;
  k_gather_cols<<<cdiv((int64_t)rows * nc, 256), 256, 0, s>>>(A, lda, rows, idx, nc, B, ldb);
  PHS_CHECK_LAUNCH();
}

__global__ void k_set_diag(double *H, int ldh, int nc, const double *d, const int *idx) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nc * nc; e += gridDim.x * blockDim.x) {
    int i = e % nc, j = e / nc;
    H[i + (int64_t)j * ldh] = (i == j) ? d[idx[i]] : 0.0;
  }
}

void set_diag(double *H, int ldh, int nc, const double *d, const int *idx, hipStream_t s) {
  if (nc == 0) return;
  k_set_diag<<<cdiv((int64_t)nc * nc, 256), 256, 0, s>>>(H, ldh, nc, d, idx);
  PHS_CHECK_LAUNCH();
}

__global__ void k_zero_rows(double *A, int lda, int r0, int r1, int nc) {
  const int nr = r1 - r0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nr * nc; e += gridDim.x * blockDim.x)
    A[r0 + e % nr + (int64_t)(e / nr) * lda] = 0.0;
}

void zero_rows(double *A, int lda, int r0, int r1, int nc, hipStream_t s) {
  if (r1 <= r0 || nc <= 0) return;
  k_zero_rows<<<cdiv((int64_t)(r1 - r0) * nc, 256), 256, 0, s>>>(A, lda, r0, r1, nc);
  PHS_CHECK_LAUNCH();
}

__global__ void k_rayleigh_small(const double *H, int ldh, int p, const double *Y, int ldy,
                                 int nc, double *theta) {
  __shared__ double red[256];
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      int i = e % p, j = e / p;
      s += Y[i + (int64_t)c * ldy] * H[i + (int64_t)j * ldh] * Y[j + (int64_t)c * ldy];
    }
    double tot = block_sum(s, red);
    if (threadIdx.x == 0) theta[c] = tot;
  }
}

void rayleigh_small(const double *H, int ldh, int p, const double *Y, int ldy, int nc,
                    double *theta, hipStream_t s) {
  if (nc <= 0) return;
  k_rayleigh_small<<<1, 256, 0, s>>>(H, ldh, p, Y, ldy, nc, theta);
  PHS_CHECK_LAUNCH();
}

}  // namespace phs

namespace phs {

__global__ void k_small_add(int M, int N, double alpha, const double *A, int lda, double *B,
                            int ldb) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * N; e += gridDim.x * blockDim.x) {
    int i = e % M, j = e / M;
    B[i + (int64_t)j * ldb] += alpha * A[i + (int64_t)j * lda];
  }
}

void small_add(int M, int N, double alpha, const double *A, int lda, double *B, int ldb,
               hipStream_t s) {
  if (M * N <= 0) return;
  k_small_add<<<cdiv((int64_t)M * N, 256), 256, 0, s>>>(M, N, alpha, A, lda, B, ldb);
  PHS_CHECK_LAUNCH();
}

}  // namespace phs
