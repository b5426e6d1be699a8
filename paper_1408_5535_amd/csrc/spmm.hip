// Sparse matrix times block of vectors, CSR, row-major blocks (gfx950).
//
// Y = A X with A m x n in CSR and X (n x B), Y (m x B) stored row-major, so
// that every nonzero a_ic gathers one contiguous B-vector x_c (B * sizeof(T)
// bytes: 32-64 B for B = 8), loaded by the 16-byte lanes of one slot.  G
// slots of a wavefront share a row: each walks the row's nonzeros with
// stride G and keeps partial sums in registers; the G partials are combined
// with cross-lane shuffles.  G is
// chosen from the row-length distribution: 1 lane per row for the grid
// operators (2-4 nonzeros per row), wider groups for random rows, and the
// rows of a power-law matrix are split into length bins, each launched with
// its own G (long rows get a whole wavefront).
//
// The CSR transpose is built on the device: column counts by atomics, an
// exclusive scan, an atomic scatter, then a per-row sort that restores
// column order (so A^T products are deterministic).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace phs {

// rows: optional list of row indices (a length bin); nullptr = all rows.
// A row is handled by G nonzero slots x VL vector lanes: the b-vector row of
// X that a nonzero gathers (b * sizeof(T) bytes) is split into VL chunks of
// 16 B, one per lane, so the VL lanes of a slot load one contiguous row
// together (one cache line request per nonzero instead of one per 16 B).
// Each slot takes every G-th nonzero of the row, kSpU at a time (their
// indices and values first, then kSpU independent gathers); the G slots'
// partial sums are combined by shuffles and the VL lanes of slot 0 store
// their chunks of the Y row (or, with ycm > 0, the first ycols values of
// the row into a column-major Y with leading dimension ycm).
constexpr int kSpU = 4;

template <typename T, int B>
struct SpVec {  // lanes per X row and values per lane
  static constexpr int VL = (B * (int)sizeof(T)) >= 16 ? (B * (int)sizeof(T)) / 16 : 1;
  static constexpr int CW = B / VL;
};

template <typename T, int CW>
__device__ inline void load_chunk(const T *__restrict__ p, T (&o)[CW]) {
  if constexpr (CW * sizeof(T) == 16) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    __builtin_memcpy(o, &u, 16);
  } else {
#pragma unroll
    for (int i = 0; i < CW; ++i) o[i] = p[i];
  }
}

template <typename T, int CW>
__device__ inline void store_chunk(T *__restrict__ p, const T (&o)[CW]) {
  if constexpr (CW * sizeof(T) == 16) {
    uint4 u;
    __builtin_memcpy(&u, o, 16);
    *reinterpret_cast<uint4 *>(p) = u;
  } else {
#pragma unroll
    for (int i = 0; i < CW; ++i) p[i] = o[i];
  }
}

// Workgroups are dispatched to the eight XCDs round robin, and each XCD has
// its own L2.  The logical block index hands XCD x runs of xc consecutive
// blocks (x-th run of every eight), so that rows whose X neighbourhoods
// overlap (the grid operators reach back N rows) share one L2, while the
// blocks in flight still cover one compact window of rows.  The tail that
// does not fill eight runs is split into eight contiguous pieces.  Runs of
// 32-256 blocks measured alike (7% faster than plain round robin on the
// N = 512 grid, unchanged at N = 1024); one contiguous eighth per XCD was 5%
// slower at N = 1024.
__device__ inline int64_t xcd_block() {
  constexpr int kXcd = 8, xc = 64;
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t base = nb / (kXcd * xc) * (kXcd * xc);
  if (b < base) {
    const int64_t x = b % kXcd, k = b / kXcd;
    return ((k / xc) * kXcd + x) * xc + k % xc;
  }
  const int64_t bb = b - base, nt = nb - base;
  const int64_t x = bb % kXcd, k = bb / kXcd, q = nt / kXcd, r = nt % kXcd;
  return base + (x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k);
}

template <typename T, int B, int G, bool ABS>
__global__ __launch_bounds__(256) void k_spmm(int64_t nrows, const int32_t *__restrict__ rows,
                                              int64_t yslot, const int64_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const T *__restrict__ va,
                                              const T *__restrict__ X, T *__restrict__ Y,
                                              int64_t ycm, int ycols) {
  constexpr int VL = SpVec<T, B>::VL, CW = SpVec<T, B>::CW, GL = G * VL;
  const int64_t gid = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t slot = gid / GL;
  const int lig = (int)(threadIdx.x % GL);
  const int g = lig / VL, part = lig % VL;
  if (slot >= nrows) return;  // a whole group leaves together
  const int64_t row = rows ? (int64_t)rows[slot] : slot;
  T acc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) acc[j] = T(0);
  const int64_t end = rp[row + 1];
  const T *Xp = X + part * CW;
  for (int64_t p0 = rp[row] + g; p0 < end; p0 += (int64_t)G * kSpU) {
    int64_t c[kSpU];
    T a[kSpU];
#pragma unroll
    for (int u = 0; u < kSpU; ++u) {
      const int64_t p = p0 + (int64_t)u * G;
      const bool in = p < end;
      c[u] = in ? ci[p] : 0;
      a[u] = in ? va[p] : T(0);  // zero weight for the padding slots
    }
    // padding slots gather nothing (rows of the grid operators are shorter
    // than kSpU, and whole wavefronts then skip those loads)
    T x[kSpU][CW];
#pragma unroll
    for (int u = 0; u < kSpU; ++u) {
      if (p0 + (int64_t)u * G < end) {
        load_chunk<T, CW>(Xp + c[u] * B, x[u]);
      } else {
#pragma unroll
        for (int j = 0; j < CW; ++j) x[u][j] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < kSpU; ++u) {
      T au = a[u];
      if constexpr (ABS) {
        au = fabs(au);
#pragma unroll
        for (int j = 0; j < CW; ++j) x[u][j] = fabs(x[u][j]);
      }
#pragma unroll
      for (int j = 0; j < CW; ++j) acc[j] = fma(au, x[u][j], acc[j]);
    }
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int j = 0; j < CW; ++j) acc[j] += __shfl_xor(acc[j], off * VL, GL);
    }
  }
  if (g == 0) {
    // the result row goes to the row's own index, or (yslot >= 0) to its
    // position yslot + slot in the order of the bins
    const int64_t yr = yslot >= 0 ? yslot + slot : row;
    if (ycm == 0) {
      store_chunk<T, CW>(Y + yr * B + part * CW, acc);
    } else {
#pragma unroll
      for (int j = 0; j < CW; ++j)
        if (part * CW + j < ycols) Y[yr + (int64_t)(part * CW + j) * ycm] = acc[j];
    }
  }
}

template <typename T, int B, bool ABS>
static void launch_g(int G, int64_t nrows, const int32_t *rows, int64_t yslot, const int64_t *rp,
                     const int32_t *ci, const T *va, const T *X, T *Y, int64_t ycm, int ycols,
                     hipStream_t s) {
  if (nrows <= 0) return;
  constexpr int VL = SpVec<T, B>::VL;
  constexpr int Gmax = 64 / VL;  // a row group stays inside one wavefront
  if (G > Gmax) G = Gmax;
  const int64_t threads = nrows * G * VL;
  dim3 grid(cdiv(threads, 256));
  switch (G) {
    case 1: k_spmm<T, B, 1, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols); break;
    case 2: k_spmm<T, B, 2, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols); break;
    case 4: k_spmm<T, B, 4, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols); break;
    case 8: k_spmm<T, B, 8, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols); break;
    case 16:
      if constexpr (Gmax >= 16)
        k_spmm<T, B, 16, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols);
      break;
    case 32:
      if constexpr (Gmax >= 32)
        k_spmm<T, B, 32, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols);
      break;
    default:
      if constexpr (Gmax >= 64)
        k_spmm<T, B, 64, ABS><<<grid, 256, 0, s>>>(nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols);
      break;
  }
  PHS_CHECK_LAUNCH();
}

template <typename T, bool ABS>
static void launch_b(int b, int G, int64_t nrows, const int32_t *rows, int64_t yslot,
                     const int64_t *rp,
                     const int32_t *ci, const T *va, const T *X, T *Y, int64_t ycm, int ycols,
                     hipStream_t s) {
  switch (b) {
    case 1: launch_g<T, 1, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    case 2: launch_g<T, 2, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    case 4: launch_g<T, 4, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    case 8: launch_g<T, 8, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    case 16: launch_g<T, 16, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    case 32: launch_g<T, 32, ABS>(G, nrows, rows, yslot, rp, ci, va, X, Y, ycm, ycols, s); break;
    default: throw Error(kEinval, "spmm: block width must be 1, 2, 4, 8, 16 or 32");
  }
}

template <typename T>
void spmm_launch(const SpMat<T> &A, int b, const T *X, T *Y, bool absval, int64_t ycm,
                 int ycols, hipStream_t s);

int lanes_for_length(double avg) {
  if (avg <= 4) return 1;
  if (avg <= 8) return 2;
  if (avg <= 20) return 4;
  if (avg <= 40) return 8;
  if (avg <= 80) return 16;
  if (avg <= 160) return 32;
  return 64;
}

template <typename T>
void spmm(const SpMat<T> &A, int b, const T *X, T *Y, bool absval, hipStream_t s, int64_t ycm,
          int ycols) {
  const int kind = sizeof(T) == 8 ? kProfSpmm64 : kProfSpmm32;
  PHS_REQUIRE(ycm == 0 || (ycm >= A.m && ycols >= 1 && ycols <= b), kEinval,
              "spmm: bad column-major output");
  if (A.op) {
    // the caller's operator: row-major blocks only, no |A|
    PHS_REQUIRE(ycm == 0 && !absval, kEinval, "spmm: operator products are plain row-major");
    A.op->f(X, Y, b, A.op_trans, sizeof(T) == 8);
    return;
  }
  prof_begin(kind, s);
  spmm_launch(A, b, X, Y, absval, ycm, ycols, s);
  // algorithmic bytes: values + column indices + row pointers + X + Y
  prof_end(kind, s,
           (double)A.nnz * (sizeof(T) + 4) + (double)(A.m + 1) * 8 +
               (double)A.n * b * sizeof(T) + (double)A.m * b * sizeof(T));
}

template <typename T>
void spmm_launch(const SpMat<T> &A, int b, const T *X, T *Y, bool absval, int64_t ycm,
                 int ycols, hipStream_t s) {
  if (A.nbins == 0) {
    const int G = lanes_for_length(A.m ? (double)A.nnz / (double)A.m : 0.0);
    if (absval)
      launch_b<T, true>(b, G, A.m, nullptr, -1, A.rowptr, A.colind, A.val, X, Y, ycm, ycols, s);
    else
      launch_b<T, false>(b, G, A.m, nullptr, -1, A.rowptr, A.colind, A.val, X, Y, ycm, ycols, s);
    return;
  }
  for (int k = 0; k < A.nbins; ++k) {
    const Bin &bn = A.bins[k];
    const int64_t ys = A.slot_out ? bn.offset : -1;
    if (absval)
      launch_b<T, true>(b, bn.lanes, bn.count, A.binrows + bn.offset, ys, A.rowptr, A.colind,
                        A.val, X, Y, ycm, ycols, s);
    else
      launch_b<T, false>(b, bn.lanes, bn.count, A.binrows + bn.offset, ys, A.rowptr, A.colind,
                         A.val, X, Y, ycm, ycols, s);
  }
}
template <typename T>
void spmm_untimed(const SpMat<T> &A, int b, const T *X, T *Y, hipStream_t s) {
  if (A.op) {
    A.op->f(X, Y, b, A.op_trans, sizeof(T) == 8);
    return;
  }
  spmm_launch(A, b, X, Y, false, 0, 0, s);
}
template void spmm_untimed<float>(const SpMat<float> &, int, const float *, float *,
                                  hipStream_t);
template void spmm_untimed<double>(const SpMat<double> &, int, const double *, double *,
                                   hipStream_t);
template void spmm<float>(const SpMat<float> &, int, const float *, float *, bool, hipStream_t,
                          int64_t, int);
template void spmm<double>(const SpMat<double> &, int, const double *, double *, bool,
                           hipStream_t, int64_t, int);

// ---------------------------------------------------------------- transpose
__global__ void k_count_cols(int64_t nnz, const int32_t *__restrict__ ci, int32_t *cnt) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[ci[p]], 1);
}

// Exclusive scan of n int32 counts into n+1 int64 offsets: tile sums,
// a single-block scan of the tile sums, then per-tile scans.
constexpr int kScanTile = 1024;
__global__ __launch_bounds__(256) void k_tile_sums(int64_t n, const int32_t *cnt, int64_t *tsum) {
  __shared__ int64_t red[256];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int i = threadIdx.x; i < kScanTile; i += 256)
    if (base + i < n) s += cnt[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_scan_tiles(int64_t ntiles, int64_t *tsum) {
  // sequential over chunks of 256, parallel within a chunk
  __shared__ int64_t buf[256];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c = 0; c < ntiles; c += 256) {
    int64_t i = c + threadIdx.x;
    int64_t v = i < ntiles ? tsum[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int64_t t = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < ntiles) tsum[i] = carry + buf[threadIdx.x] - v;  // exclusive
    __syncthreads();
    if (threadIdx.x == 255) carry += buf[255];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_tile_scan(int64_t n, const int32_t *cnt,
                                                   const int64_t *tsum, int64_t *out) {
  __shared__ int64_t buf[kScanTile];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int i = threadIdx.x; i < kScanTile; i += 256) buf[i] = (base + i < n) ? cnt[base + i] : 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = tsum[blockIdx.x];
    for (int i = 0; i < kScanTile; ++i) {
      int64_t v = buf[i];
      buf[i] = run;
      run += v;
    }
    if (base + kScanTile >= n) out[n] = run;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kScanTile; i += 256)
    if (base + i < n) out[base + i] = buf[i];
}

__global__ void k_scatter_t(int64_t m, const int64_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, const double *__restrict__ va,
                            const int64_t *__restrict__ trp, int32_t *fill, int32_t *tci,
                            double *tva) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
    int c = ci[p];
    int64_t pos = trp[c] + atomicAdd(&fill[c], 1);
    tci[pos] = (int32_t)r;
    tva[pos] = va[p];
  }
}

__global__ void k_sort_short(int64_t n, const int64_t *__restrict__ trp, int32_t *tci,
                             double *tva, int32_t *longlist, int32_t *nlong) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t a = trp[r], e = trp[r + 1];
  if (e - a > 32) {
    longlist[atomicAdd(nlong, 1)] = (int32_t)r;
    return;
  }
  for (int64_t i = a + 1; i < e; ++i) {
    int32_t key = tci[i];
    double v = tva[i];
    int64_t j = i - 1;
    while (j >= a && tci[j] > key) {
      tci[j + 1] = tci[j];
      tva[j + 1] = tva[j];
      --j;
    }
    tci[j + 1] = key;
    tva[j + 1] = v;
  }
}

// One block per long row: the rank of each (distinct) key is its position.
__global__ __launch_bounds__(256) void k_sort_long(const int32_t *longlist,
                                                   const int64_t *__restrict__ trp,
                                                   int32_t *tci, double *tva, int32_t *tmpc,
                                                   double *tmpv) {
  const int64_t r = longlist[blockIdx.x];
  const int64_t a = trp[r], len = trp[r + 1] - a;
  for (int64_t i = threadIdx.x; i < len; i += 256) {
    int32_t key = tci[a + i];
    int64_t rank = 0;
    for (int64_t j = 0; j < len; ++j) rank += tci[a + j] < key;
    tmpc[a + rank] = key;
    tmpv[a + rank] = tva[a + i];
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < len; i += 256) {
    tci[a + i] = tmpc[a + i];
    tva[a + i] = tmpv[a + i];
  }
}

// Zero fill by a kernel (no memset node in the stream's work).
template <typename T>
__global__ void k_zero(T *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = T(0);
}
template <typename T>
void zero_fill(T *p, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  k_zero<T><<<cdiv(count, 256), 256, 0, s>>>(p, count);
  PHS_CHECK_LAUNCH();
}

// Validity of a CSR input: bit 1 row pointers (rp[0] = 0, non-decreasing,
// rp[m] = nnz), bit 2 a column index outside [0, n), bit 4 a row not
// strictly increasing (unsorted or duplicate columns).
__global__ __launch_bounds__(256) void k_csr_check(int64_t m, int64_t n, int64_t nnz,
                                                   const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, int32_t *flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > m) return;
  int bad = 0;
  if (r == 0 && rp[0] != 0) bad |= 1;
  if (r == m) {
    if (rp[m] != nnz) bad |= 1;
  } else {
    const int64_t a = rp[r], b = rp[r + 1];
    if (b < a || a < 0 || b > nnz) {
      bad |= 1;
    } else {
      int32_t prev = -1;
      for (int64_t q = a; q < b; ++q) {
        const int32_t c = ci[q];
        if (c < 0 || c >= n) bad |= 2;
        if (c <= prev) bad |= 4;
        prev = c;
      }
    }
  }
  if (bad) atomicOr(flag, bad);
}

size_t transpose_ws_bytes(int64_t m, int64_t n, int64_t nnz) {
  Arena ar;
  ar.dry = true;
  ar.take<int32_t>(16);                 // validity flag, long-row counter
  ar.take<int32_t>(n);                  // counts / fill
  ar.take<int64_t>(cdiv(n, kScanTile));  // tile sums
  ar.take<int32_t>(n + 1);              // long rows (+ counter)
  ar.take<int32_t>(nnz);
  ar.take<double>(nnz);
  (void)m;
  return ar.used;
}

void csr_transpose(int64_t m, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci,
                   const double *va, int64_t *trp, int32_t *tci, double *tva, void *ws,
                   size_t ws_bytes, hipStream_t s) {
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  int32_t *flags = ar.take<int32_t>(16);  // [0] validity, [1] long-row count
  int32_t *cnt = ar.take<int32_t>(n);
  int64_t ntiles = cdiv(n, kScanTile);
  int64_t *tsum = ar.take<int64_t>(ntiles);
  int32_t *longl = ar.take<int32_t>(n + 1);
  int32_t *tmpc = ar.take<int32_t>(nnz);
  double *tmpv = ar.take<double>(nnz);
  int32_t *nlong = flags + 1;
  zero_fill(flags, 16, s);
  k_csr_check<<<cdiv(m + 1, 256), 256, 0, s>>>(m, n, nnz, rp, ci, flags);
  PHS_CHECK_LAUNCH();
  int32_t hf = 0;
  PHS_HIP(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PHS_HIP(hipStreamSynchronize(s));
  PHS_REQUIRE(!(hf & 1), kEinval, "CSR: row pointers must start at 0, not decrease, end at nnz");
  PHS_REQUIRE(!(hf & 2), kEinval, "CSR: column index outside [0, n)");
  PHS_REQUIRE(!(hf & 4), kEinval, "CSR: columns of a row must be sorted and distinct");
  zero_fill(cnt, n, s);
  if (nnz) k_count_cols<<<cdiv(nnz, 256), 256, 0, s>>>(nnz, ci, cnt);
  PHS_CHECK_LAUNCH();
  if (n) {
    k_tile_sums<<<ntiles, 256, 0, s>>>(n, cnt, tsum);
    k_scan_tiles<<<1, 256, 0, s>>>(ntiles, tsum);
    k_tile_scan<<<ntiles, 256, 0, s>>>(n, cnt, tsum, trp);
    PHS_CHECK_LAUNCH();
  } else {
    zero_fill(trp, 1, s);
  }
  zero_fill(cnt, n, s);
  if (m) k_scatter_t<<<cdiv(m, 256), 256, 0, s>>>(m, rp, ci, va, trp, cnt, tci, tva);
  if (n) k_sort_short<<<cdiv(n, 256), 256, 0, s>>>(n, trp, tci, tva, longl, nlong);
  PHS_CHECK_LAUNCH();
  int32_t nl = 0;
  PHS_HIP(hipMemcpyAsync(&nl, nlong, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PHS_HIP(hipStreamSynchronize(s));
  if (nl > 0) {
    k_sort_long<<<nl, 256, 0, s>>>(longl, trp, tci, tva, tmpc, tmpv);
    PHS_CHECK_LAUNCH();
  }
}

// Row-length bins for skewed matrices: rows are grouped by the lane count
// their length calls for, so that each launch has uniform work per group.
__device__ inline int bin_of(int64_t len) {
  int g = 0;
  for (int lim = 4; g < 6 && len > lim; lim *= 2) ++g;  // 0..6 -> 1..64 lanes
  return g;
}

// Per-block counts in LDS, one global atomic per bin and block (the totals).
__global__ __launch_bounds__(256) void k_bin_count(int64_t m, const int64_t *__restrict__ rp,
                                                   int32_t *cnt) {
  __shared__ int32_t h[8];
  if (threadIdx.x < 8) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) atomicAdd(&h[bin_of(rp[r + 1] - rp[r])], 1);
  __syncthreads();
  if (threadIdx.x < 7 && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// Each block's count per bin, bin-major: bc[g * nblk + block].
__global__ __launch_bounds__(256) void k_bin_blkcount(int64_t m, const int64_t *__restrict__ rp,
                                                      int64_t nblk, int32_t *bc) {
  __shared__ int32_t h[8];
  if (threadIdx.x < 8) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) atomicAdd(&h[bin_of(rp[r + 1] - rp[r])], 1);
  __syncthreads();
  if (threadIdx.x < 7) bc[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Places each row at the exclusive scan of the block counts (bin-major)
// plus its rank among the block's rows of its bin (wavefront ballots), so
// that the rows of every bin come in ascending order.
__global__ __launch_bounds__(256) void k_bin_place(int64_t m, const int64_t *__restrict__ rp,
                                                   int64_t nblk, const int64_t *off,
                                                   int32_t *rows) {
  __shared__ int32_t wc[4][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = r < m ? bin_of(rp[r + 1] - rp[r]) : -1;
  int rank = 0;
  for (int b = 0; b < 7; ++b) {
    const unsigned long long bal = __ballot(g == b);
    if (g == b) rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wc[w][b] = __popcll(bal);
  }
  __syncthreads();
  if (g >= 0) {
    int pre = 0;
    for (int v = 0; v < w; ++v) pre += wc[v][g];
    rows[off[g * nblk + blockIdx.x] + pre + rank] = (int32_t)r;
  }
}

size_t bin_ws_bytes(int64_t m) {
  const int64_t nblk = cdiv(std::max<int64_t>(m, 1), 256), E = 7 * nblk;
  Arena ar;
  ar.dry = true;
  ar.take<int32_t>(16);               // totals per bin
  ar.take<int32_t>(E);                // block counts
  ar.take<int64_t>(cdiv(E, kScanTile));  // tile sums
  ar.take<int64_t>(E + 1);            // their exclusive scan
  return ar.used;
}

// Row-length bins, with rows[] listing the rows of bin 0, then bin 1, ...
// each in ascending order (a permutation of 0..m-1 that depends only on the
// row lengths).
void build_bins(int64_t m, const int64_t *rp, int32_t *rows, void *ws, size_t ws_bytes, Bin *bins,
                int *nbins, hipStream_t s) {
  const int64_t nblk = cdiv(std::max<int64_t>(m, 1), 256), E = 7 * nblk;
  Arena ar;
  ar.base = (char *)ws;
  ar.size = ws_bytes;
  int32_t *tot = ar.take<int32_t>(16);
  int32_t *bc = ar.take<int32_t>(E);
  int64_t *tsum = ar.take<int64_t>(cdiv(E, kScanTile));
  int64_t *off = ar.take<int64_t>(E + 1);
  zero_fill(tot, 16, s);
  if (m > 0) {
    k_bin_count<<<cdiv(m, 256), 256, 0, s>>>(m, rp, tot);
    k_bin_blkcount<<<nblk, 256, 0, s>>>(m, rp, nblk, bc);
    PHS_CHECK_LAUNCH();
    const int64_t ntiles = cdiv(E, kScanTile);
    k_tile_sums<<<ntiles, 256, 0, s>>>(E, bc, tsum);
    k_scan_tiles<<<1, 256, 0, s>>>(ntiles, tsum);
    k_tile_scan<<<ntiles, 256, 0, s>>>(E, bc, tsum, off);
    k_bin_place<<<nblk, 256, 0, s>>>(m, rp, nblk, off, rows);
    PHS_CHECK_LAUNCH();
  }
  int32_t cnt[7] = {0, 0, 0, 0, 0, 0, 0};
  PHS_HIP(hipMemcpyAsync(cnt, tot, 7 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PHS_HIP(hipStreamSynchronize(s));
  int nb = 0, o = 0;
  for (int g = 0; g < 7; ++g) {
    if (cnt[g] > 0) {
      bins[nb].offset = o;
      bins[nb].count = cnt[g];
      bins[nb].lanes = 1 << g;
      ++nb;
    }
    o += cnt[g];
  }
  *nbins = nb;
}

// inv[rows[q]] = q
__global__ void k_invert_perm(int64_t m, const int32_t *__restrict__ rows, int32_t *inv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) inv[rows[q]] = (int32_t)q;
}
// ci[p] <- inv[ci[p]]
__global__ void k_remap_idx(int64_t nnz, const int32_t *__restrict__ inv, int32_t *ci) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) ci[p] = inv[ci[p]];
}
// dst[rows[q]] = src[q] for each of w columns (ld m)
__global__ void k_unpermute_cols(int64_t m, int w, const int32_t *__restrict__ rows,
                                 const double *__restrict__ src, double *dst) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const int64_t r = rows[q];
  for (int j = 0; j < w; ++j) dst[r + (int64_t)j * m] = src[q + (int64_t)j * m];
}

void permute_row_space(int64_t m, int64_t nnz, const int32_t *rows, int32_t *inv, int32_t *tci,
                       hipStream_t s) {
  if (m <= 0) return;
  k_invert_perm<<<cdiv(m, 256), 256, 0, s>>>(m, rows, inv);
  if (nnz > 0) k_remap_idx<<<cdiv(nnz, 256), 256, 0, s>>>(nnz, inv, tci);
  PHS_CHECK_LAUNCH();
}

void unpermute_rows(int64_t m, int w, const int32_t *rows, const double *src, double *dst,
                    hipStream_t s) {
  if (m <= 0 || w <= 0) return;
  k_unpermute_cols<<<cdiv(m, 256), 256, 0, s>>>(m, w, rows, src, dst);
  PHS_CHECK_LAUNCH();
}

}  // namespace phs
