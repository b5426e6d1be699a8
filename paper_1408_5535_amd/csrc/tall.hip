// Tall-skinny block kernels (N x p with N up to ~10^7, p <= 128).
//
// These carry the dense work of the GD+k iteration: projections X^T Y
// (Rayleigh-Ritz borders, Gram-Schmidt coefficients, Gram matrices), basis
// updates X S (Ritz vectors, restarts, Gram-Schmidt updates), residuals and
// norms.  All of them stream the tall operands once from HBM; the small
// operand lives in LDS.  Reductions go through per-block partials and a
// second pass in float64, in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"
#include "wave.hpp"

namespace phs {

template <typename T>
struct TV {  // trivially copyable kernel argument
  const T *p;
  int64_t rows;
  int cols;
  int64_t rs, cs;
};
template <typename T>
static TV<T> tv(const Tall<T> &t) {
  return TV<T>{t.p, t.rows, t.cols, t.rs, t.cs};
}

// ---------------------------------------------------------------- X^T Y
// One wavefront per output tile of kTnCX x kTnCY entries; the waves of a
// workgroup cover all tiles for one slab of rows, so the slab of Y is read
// from HBM once and served from cache to the other tiles.  With fewer tiles
// than waves, reps = waves / tiles waves share a tile and split its rows;
// their sums are added in LDS in a fixed order.  Lanes walk the rows
// (consecutive lanes, consecutive rows: coalesced for column-major X), kTnU
// rows per lane in flight, products accumulated in T registers.  Each wave
// reduces its tile over its lanes; one partial per block and entry goes to
// `part`, which a second kernel (or the consumer) adds in a fixed order.
constexpr int kTnCX = 4, kTnCY = 4, kTnMaxWaves = 4;
template <typename T>
struct TnRows {  // rows per lane in flight: float 4, double 2 (register budget)
  static constexpr int U = sizeof(T) == 4 ? 4 : 2;
};

// acc += X(rows, tile columns)^T Y(rows, tile columns) over the rows
// r = rs + lane + 64 U q (q = 0, 1, ...) below r1, taken U at a time with
// stride `step` between groups.
template <typename T>
__device__ inline void tn_tile(const TV<T> &x1, const TV<T> &x2, const TV<T> &y, int i0, int j0,
                               int64_t rs, int64_t r1, int64_t step, int lane,
                               T (&acc)[kTnCX][kTnCY]) {
  constexpr int U = TnRows<T>::U;
  const int nx = x1.cols + x2.cols, ny = y.cols;
  // column bases (uniform); columns past the operand read as zero
  const T *xp[kTnCX];
  bool in1[kTnCX];  // column from x1 (else x2): selects the row stride
#pragma unroll
  for (int a = 0; a < kTnCX; ++a) {
    const int i = i0 + a;
    in1[a] = i < x1.cols;
    xp[a] = in1[a] ? x1.p + (int64_t)i * x1.cs
                   : x2.p + (int64_t)(i < nx ? i - x1.cols : 0) * x2.cs;
  }
  const T *yp[kTnCY];
#pragma unroll
  for (int c = 0; c < kTnCY; ++c) yp[c] = y.p + (int64_t)(j0 + c < ny ? j0 + c : 0) * y.cs;
#pragma unroll
  for (int a = 0; a < kTnCX; ++a)
#pragma unroll
    for (int c = 0; c < kTnCY; ++c) acc[a][c] = T(0);
  for (int64_t rb = rs + lane; rb < r1; rb += step) {
    T xr[U][kTnCX], yr[U][kTnCY];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = rb + (int64_t)u * 64;
      const bool in = r < r1;
      const int64_t o1 = r * x1.rs, o2 = r * x2.rs, oy = r * y.rs;
#pragma unroll
      for (int a = 0; a < kTnCX; ++a)
        xr[u][a] = (in && i0 + a < nx) ? xp[a][in1[a] ? o1 : o2] : T(0);
#pragma unroll
      for (int c = 0; c < kTnCY; ++c) yr[u][c] = (in && j0 + c < ny) ? yp[c][oy] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int a = 0; a < kTnCX; ++a)
#pragma unroll
        for (int c = 0; c < kTnCY; ++c) acc[a][c] = fma(xr[u][a], yr[u][c], acc[a][c]);
  }
}

template <typename T>
__global__ __launch_bounds__(64 * kTnMaxWaves) void k_tn(TV<T> x1, TV<T> x2, TV<T> y,
                                                         int64_t rpb, double *part) {
  constexpr int U = TnRows<T>::U;
  const int nx = x1.cols + x2.cols, ny = y.cols;
  const int tx = (nx + kTnCX - 1) / kTnCX, ty = (ny + kTnCY - 1) / kTnCY, ntile = tx * ty;
  const int E = nx * ny;
  const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t N = y.rows;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
  T acc[kTnCX][kTnCY];
  if (ntile < nw) {
    // reps waves per tile (the launch makes nw a multiple of ntile)
    __shared__ double red[kTnMaxWaves][kTnCX * kTnCY];
    const int reps = nw / ntile, tile = w % ntile, sub = w / ntile;
    const int i0 = (tile / ty) * kTnCX, j0 = (tile % ty) * kTnCY;
    tn_tile(x1, x2, y, i0, j0, r0 + (int64_t)sub * 64 * U, r1, (int64_t)64 * U * reps, lane, acc);
#pragma unroll
    for (int a = 0; a < kTnCX; ++a)
#pragma unroll
      for (int c = 0; c < kTnCY; ++c) {
        const double v = wave_total((double)acc[a][c]);
        if (lane == 0) red[w][a * kTnCY + c] = v;
      }
    __syncthreads();
    if (sub == 0 && lane < kTnCX * kTnCY) {
      const int a = lane / kTnCY, c = lane % kTnCY, i = i0 + a, j = j0 + c;
      double v = red[tile][lane];
      for (int q = 1; q < reps; ++q) v += red[tile + q * ntile][lane];
      if (i < nx && j < ny) part[(int64_t)blockIdx.x * E + i * ny + j] = v;
    }
    return;
  }
  for (int tile = w; tile < ntile; tile += nw) {
    const int i0 = (tile / ty) * kTnCX, j0 = (tile % ty) * kTnCY;
    tn_tile(x1, x2, y, i0, j0, r0, r1, (int64_t)64 * U, lane, acc);
    // wave sums (DPP rows, then the four row sums in a fixed order); lane 0
    // writes the block's partial of every entry of the tile (float64)
#pragma unroll
    for (int a = 0; a < kTnCX; ++a)
#pragma unroll
      for (int c = 0; c < kTnCY; ++c) {
        const double v = wave_total((double)acc[a][c]);
        const int i = i0 + a, j = j0 + c;
        if (lane == 0 && i < nx && j < ny) part[(int64_t)blockIdx.x * E + i * ny + j] = v;
      }
  }
}

// Entry e of G from the block partials, one wavefront: lane l sums partials
// l, l+64, ... and the lane sums are combined in the fixed order of
// wave_total.
__device__ inline double sum_parts(const double *part, int np, int E, int e) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = threadIdx.x;
  // two rounds of four at a time (eight loads in flight), same order
  for (; b + 448 < np; b += 512) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + 64 * u) * E + e];
    s0 += v[0];
    s1 += v[1];
    s2 += v[2];
    s3 += v[3];
    s0 += v[4];
    s1 += v[5];
    s2 += v[6];
    s3 += v[7];
  }
  for (; b + 192 < np; b += 256) {
    s0 += part[(int64_t)b * E + e];
    s1 += part[(int64_t)(b + 64) * E + e];
    s2 += part[(int64_t)(b + 128) * E + e];
    s3 += part[(int64_t)(b + 192) * E + e];
  }
  for (; b < np; b += 64) s0 += part[(int64_t)b * E + e];
  return wave_total((s0 + s1) + (s2 + s3));
}

__global__ __launch_bounds__(64) void k_reduce_parts(const double *part, int np, int nx, int ny,
                                                     double *G, int ldg) {
  const int E = nx * ny, e = blockIdx.x;
  const double s = sum_parts(part, np, E, e);
  if (threadIdx.x == 0) G[e / ny + (int64_t)(e % ny) * ldg] = s;
}

// G = V^T W_new ((p + nb) x nb, from the partials) written as the border of
// H: H(i, p+c) = H(p+c, i) = G(i, c) for i < p, and the new diagonal block
// symmetrised, H(p+r, p+c) = (G(p+r, c) + G(p+c, r)) / 2.  The extra last
// block zeroes rows p..p+nb-1 of Z (nz columns), if given.
__global__ __launch_bounds__(64) void k_reduce_border(const double *part, int np, int nx, int nb,
                                                      double *H, int ldh, double *Z, int ldz,
                                                      int nz) {
  const int E = nx * nb, e = blockIdx.x, p = nx - nb;
  if (e == E) {
    for (int q = threadIdx.x; q < nb * nz; q += 64) Z[(p + q % nb) + (int64_t)(q / nb) * ldz] = 0.0;
    return;
  }
  const int i = e / nb, c = e % nb;
  const double g = sum_parts(part, np, E, e);
  if (i < p) {
    if (threadIdx.x == 0) {
      H[i + (int64_t)(p + c) * ldh] = g;
      H[(p + c) + (int64_t)i * ldh] = g;
    }
  } else {
    const int r = i - p;
    const double gm = sum_parts(part, np, E, (p + c) * nb + r);
    if (threadIdx.x == 0) H[i + (int64_t)(p + c) * ldh] = 0.5 * (g + gm);
  }
}

void reduce_border(const TnParts &pt, double *H, int ldh, double *Z, int ldz, int nz,
                   hipStream_t s) {
  PHS_REQUIRE(pt.nx >= pt.ny && pt.ny >= 1, kEinval, "reduce_border: partials do not match");
  const int E = pt.nx * pt.ny;
  k_reduce_border<<<E + (Z && nz > 0 ? 1 : 0), 64, 0, s>>>(pt.part, pt.np, pt.nx, pt.ny, H, ldh,
                                                         Z, ldz, nz);
  PHS_CHECK_LAUNCH();
}

// ----------------------------------------------------- X^T Y on MFMA
// For long operands (the basis spills out of the caches) the contraction
// runs on the matrix cores: 16 x 16 x 4 MFMA tiles (float32 or float64),
// wave w of a block owning columns 16w..16w+15 of X and all (<= 16) columns
// of Y.  Rows are staged through LDS in chunks of 64: each lane loads its
// row of the wave's 16 X columns (every load instruction a coalesced run of
// 64 consecutive rows of one column), the block loads the Y chunk, and the
// 16 K-steps of the chunk read their operands from LDS (row pitch 17, no
// bank conflicts); the next chunk's global loads are issued before the
// MFMAs of the current one.  Operand layout of the 16x16x4 instructions:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[r][l % 16] in accumulator v = 0..3 with r = 4 (l / 16) + v (float32) or
// r = l / 16 + 4 v (float64).  One partial per block and entry, as k_tn
// leaves them.
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D held in accumulator v of lane l (column l % 16)
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the float64 instruction interleaves the lane groups over D's rows
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};

constexpr int kTmRows = 64, kTmPitch = 17, kTmMaxWaves = 8;

// A row of a row-major block, NB values at p (16-byte aligned), written by
// 16-byte stores: one instruction then covers whole rows of the wavefront's
// lanes instead of one value of each (element-wise stores of the row-major
// outputs halved the rate of the Ritz block and slowed the X S kernel by a
// fifth).
template <typename T, int NB>
__device__ inline void store_row16(T *p, const T (&v)[NB]) {
  constexpr int VW = 16 / (int)sizeof(T);
  static_assert(NB % VW == 0, "row not a multiple of 16 bytes");
  typedef T vec __attribute__((ext_vector_type(VW)));
#pragma unroll
  for (int c = 0; c < NB; c += VW) {
    vec a;
#pragma unroll
    for (int u = 0; u < VW; ++u) a[u] = v[c + u];
    *reinterpret_cast<vec *>(p + c) = a;
  }
}
template <typename T, int NB>
constexpr bool row16_ok() {
  return NB % (16 / (int)sizeof(T)) == 0;
}
// The NB values of a row at p (16-byte aligned) by 16-byte loads.
template <typename T, int NB>
__device__ inline void load_row16(const T *p, T (&v)[NB]) {
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VW)));
#pragma unroll
  for (int c = 0; c < NB; c += VW) {
    const vec a = *reinterpret_cast<const vec *>(p + c);
#pragma unroll
    for (int u = 0; u < VW; ++u) v[c + u] = a[u];
  }
}

template <typename T>
__device__ inline T tall_at(const TV<T> &x1, const TV<T> &x2, int64_t r, int i) {
  return i < x1.cols ? x1.p[r * x1.rs + (int64_t)i * x1.cs]
                     : x2.p[r * x2.rs + (int64_t)(i - x1.cols) * x2.cs];
}

template <typename T>
__global__ __launch_bounds__(64 * kTmMaxWaves) void k_tn_mfma(TV<T> x1, TV<T> x2, TV<T> y,
                                                               int64_t rpb, double *part) {
  extern __shared__ char tm_lds[];
  const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T *ys = reinterpret_cast<T *>(tm_lds);
  T *xs = ys + kTmRows * kTmPitch + w * kTmRows * kTmPitch;
  const int nx = x1.cols + x2.cols, ny = y.cols;
  const int i0 = 16 * w;
  const bool active = i0 < nx;
  const int64_t N = y.rows;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
  // Y chunk loads: 64 x 16 values over the block, consecutive threads on
  // consecutive rows (column-major Y) or on consecutive columns (row-major)
  const bool ycm = y.rs == 1;
  const int per = (kTmRows * 16 + blockDim.x - 1) / blockDim.x;  // <= 4 (>= 256 threads)
  T xr[16], yr[4];
  auto load = [&](int64_t rc) {
    const int64_t r = rc + lane;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int i = i0 + c;
      xr[c] = (active && r < r1 && i < nx) ? tall_at(x1, x2, r, i) : T(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * (int)blockDim.x;
      if (q < per && e < kTmRows * 16) {
        const int rr = ycm ? e % kTmRows : e / 16, cc = ycm ? e / kTmRows : e % 16;
        const int64_t ry = rc + rr;
        yr[q] = (ry < r1 && cc < ny) ? y.p[ry * y.rs + (int64_t)cc * y.cs] : T(0);
      }
    }
  };
  typename Mfma16<T>::v4 acc = {T(0), T(0), T(0), T(0)};
  if (r0 < r1) load(r0);
  for (int64_t rc = r0; rc < r1; rc += kTmRows) {
    __syncthreads();  // the previous chunk's operands are consumed
#pragma unroll
    for (int c = 0; c < 16; ++c) xs[lane * kTmPitch + c] = xr[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * (int)blockDim.x;
      if (q < per && e < kTmRows * 16) {
        const int rr = ycm ? e % kTmRows : e / 16, cc = ycm ? e / kTmRows : e % 16;
        ys[rr * kTmPitch + cc] = yr[q];
      }
    }
    __syncthreads();
    if (rc + kTmRows < r1) load(rc + kTmRows);
    if (active) {
#pragma unroll
      for (int k = 0; k < kTmRows / 4; ++k) {
        const int row = 4 * k + (lane >> 4), col = lane & 15;
        acc = Mfma16<T>::op(xs[row * kTmPitch + col], ys[row * kTmPitch + col], acc);
      }
    }
  }
  (void)nw;
  if (active) {
    const int E = nx * ny, j = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + Mfma16<T>::row(lane, v);
      if (i < nx && j < ny) part[(int64_t)blockIdx.x * E + i * ny + j] = (double)acc[v];
    }
  }
}

// G = X^T X for a row-major block of NB columns (row stride NB, rows
// 16-byte aligned) on long operands.  Each thread takes whole rows with
// 16-byte loads, two rows ahead of their products, so a wave reads 64
// consecutive rows as one contiguous run (the column-at-a-time loads of the
// MFMA kernel touch every line of the block once per column); the upper
// triangle of the products is accumulated in float64 (exact products of
// float32 values).  The block's sums (wave reductions, then the waves in a
// fixed order) go out as a full NB x NB partial, entry (i, j) at i NB + j.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_gram_rows(const T *__restrict__ X, int64_t N, int64_t rpb,
                                                   double *part) {
  constexpr int NE = NB * (NB + 1) / 2;
  constexpr int RU = 2;
  double acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) acc[e] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
  const int64_t step = blockDim.x;
  for (int64_t rb = r0 + threadIdx.x; rb < r1; rb += RU * step) {
    T x[RU][NB];
#pragma unroll
    for (int q = 0; q < RU; ++q) {
      const int64_t r = rb + q * step;
      if (r < r1) {
        load_row16<T, NB>(X + r * NB, x[q]);
      } else {
#pragma unroll
        for (int i = 0; i < NB; ++i) x[q][i] = T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < RU; ++q) {
      int e = 0;
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = i; j < NB; ++j, ++e)
          acc[e] = fma((double)x[q][i], (double)x[q][j], acc[e]);
    }
  }
  __shared__ double red[4][NE];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const double v = wave_total(acc[e]);
    if (lane == 0) red[w][e] = v;
  }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  for (int e = threadIdx.x; e < NE; e += blockDim.x) {
    double v = red[0][e];
    for (int q = 1; q < nw; ++q) v += red[q][e];
    int i = 0, rem = e;
    while (rem >= NB - i) rem -= NB - i, ++i;
    const int j = i + rem;
    part[(int64_t)blockIdx.x * NB * NB + i * NB + j] = v;
    part[(int64_t)blockIdx.x * NB * NB + j * NB + i] = v;
  }
}

// LDS bytes a workgroup may use on the current device (read once).
int device_lds_max() {
  static int lds_max = -1;
  if (lds_max < 0) {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      lds_max = v;
    else
      lds_max = 65536;
  }
  return lds_max;
}

// Row count from which X^T Y takes the MFMA kernel.
constexpr int64_t kTnMfmaRows = 65536;

template <typename T>
void tn(const Tall<T> &X1, const Tall<T> &X2, const Tall<T> &Y, double *G, int ldg,
        const Scratch &sc, hipStream_t s, TnParts *keep) {
  const int nx = X1.cols + X2.cols, ny = Y.cols;
  if (nx == 0 || ny == 0) return;
  PHS_REQUIRE(nx <= 128 && ny <= 32, kEinval, "tn: operand too wide");
  PHS_REQUIRE(X1.rows == Y.rows && (X2.cols == 0 || X2.rows == Y.rows), kEinval,
              "tn: row counts differ");
  const int lds_max = device_lds_max();
  const int waves_m = std::max(4, (nx + 15) / 16);
  const size_t shm_m = (size_t)(1 + waves_m) * kTmRows * kTmPitch * sizeof(T);
  // the Gram matrix of a whole row-major block of 8 columns
  if (X2.cols == 0 && X1.p == Y.p && nx == 8 && ny == 8 && X1.cs == 1 && Y.cs == 1 &&
      X1.rs == 8 && Y.rs == 8 && X1.rows == Y.rows && Y.rows >= kTnMfmaRows &&
      ((uintptr_t)X1.p & 15) == 0) {
    const int64_t N = Y.rows, E = 64;
    const int64_t nblk = std::min<int64_t>(1024, kPartCap / E);
    const int64_t rpb = (N + nblk - 1) / nblk;
    const int nb_used = (int)((N + rpb - 1) / rpb);
    prof_begin(kProfTn, s);
    k_gram_rows<T, 8><<<nb_used, 256, 0, s>>>(X1.p, N, rpb, sc.part);
    if (keep) {
      *keep = TnParts{sc.part, nb_used, nx, ny};
    } else {
      k_reduce_parts<<<(int)E, 64, 0, s>>>(sc.part, nb_used, nx, ny, G, ldg);
    }
    PHS_CHECK_LAUNCH();
    prof_end(kProfTn, s, (double)Y.rows * nx * sizeof(T));
    return;
  }
  if (ny <= 16 && Y.rows >= kTnMfmaRows && shm_m <= (size_t)lds_max) {
    const int64_t N = Y.rows, E = (int64_t)nx * ny;
    const int waves = waves_m;
    // about four blocks per compute unit, slabs a multiple of the chunk,
    // and the partials within their buffer
    int64_t nblk = std::min<int64_t>(1024, kPartCap / E);
    int64_t rpb = ((N + nblk - 1) / nblk + kTmRows - 1) / kTmRows * kTmRows;
    nblk = (N + rpb - 1) / rpb;
    const size_t shm = shm_m;
    prof_begin(kProfTn, s);
    k_tn_mfma<T><<<(int)nblk, 64 * waves, shm, s>>>(tv(X1), tv(X2), tv(Y), rpb, sc.part);
    if (keep) {
      *keep = TnParts{sc.part, (int)nblk, nx, ny};
    } else {
      k_reduce_parts<<<(int)E, 64, 0, s>>>(sc.part, (int)nblk, nx, ny, G, ldg);
    }
    PHS_CHECK_LAUNCH();
    prof_end(kProfTn, s, (double)Y.rows * (nx + ny) * sizeof(T));
    return;
  }
  const int tiles = ((nx + kTnCX - 1) / kTnCX) * ((ny + kTnCY - 1) / kTnCY);
  // fewer tiles than waves: several waves per tile (a multiple of the tiles)
  const int waves = tiles < kTnMaxWaves ? tiles * (kTnMaxWaves / tiles) : kTnMaxWaves;
  const int64_t N = Y.rows, E = (int64_t)nx * ny;
  // about 2048 waves in flight, slabs a multiple of 64 * kTnU rows, and the
  // partials within their buffer
  int64_t nblk = (2048 + waves - 1) / waves;
  const int64_t unit = 64 * TnRows<T>::U * (tiles < kTnMaxWaves ? waves / tiles : 1);
  int64_t rpb = ((N + nblk - 1) / nblk + unit - 1) / unit * unit;
  if (rpb < unit) rpb = unit;
  nblk = (N + rpb - 1) / rpb;
  const int64_t cap = kPartCap / E;
  if (nblk > cap) {
    nblk = cap;
    rpb = ((N + nblk - 1) / nblk + unit - 1) / unit * unit;
    nblk = (N + rpb - 1) / rpb;
  }
  if (nblk < 1) nblk = 1;
  prof_begin(kProfTn, s);
  k_tn<T><<<(int)nblk, 64 * waves, 0, s>>>(tv(X1), tv(X2), tv(Y), rpb, sc.part);
  if (keep) {
    *keep = TnParts{sc.part, (int)nblk, nx, ny};
  } else {
    k_reduce_parts<<<(int)E, 64, 0, s>>>(sc.part, (int)nblk, nx, ny, G, ldg);
  }
  PHS_CHECK_LAUNCH();
  prof_end(kProfTn, s, (double)Y.rows * (nx + ny) * sizeof(T));
}

// One wavefront per entry: lane l sums partials l, l+64, ... and the 64
// lane sums are combined by the fixed DPP / lane order of wave_total.
__device__ inline double wave_sum(double v) { return wave_total(v); }

// ------------------------------------------------------------------ X S

// Y = alpha X S + beta Z (Z defaults to Y itself), optionally also written
// to a second output Y2 in another layout.
template <typename T>
struct NnOut {
  T *y;
  int64_t yrs, ycs;
  const T *z;
  int64_t zrs, zcs;
  T *y2;
  int64_t y2rs, y2cs;
};

// NT output columns per thread (4, 8 or 16: the narrowest tile that holds
// ny, or 16 with several column tiles; a 32-column tile for the restart
// products measured no faster than two 16-column tiles).  With NG > 0 (then
// ny == NG and one column tile) the kernel also forms the Gram matrix Y^T Y
// of its output: each thread accumulates its rows in float64, and every
// block writes its partial (entry (i, j) at i * NG + j) to gpart for the
// consumer to reduce.
template <typename T, int NG, int NT>
__global__ __launch_bounds__(NG > 0 ? 1024 : 256) void k_nn(TV<T> x1, TV<T> x2, const double *S,
                                                             int lds, int ny, double alpha,
                                                             double beta, NnOut<T> o,
                                                             double *gpart, int ntl) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ss = reinterpret_cast<T *>(smem);
  const int nx = x1.cols + x2.cols;
  // row block and column tile: with several tiles the 1-D grid gives the
  // tiles of one row block to consecutive blocks of one XCD (blocks go to
  // the eight XCDs round robin), so that the rows of X they all read are
  // fetched into that XCD's L2 once; the row-block count is a multiple of 8
  int64_t rb = blockIdx.x, nrb = gridDim.x;
  int tb = 0;
  if (ntl > 1) {
    const int64_t x = blockIdx.x % 8, k = blockIdx.x / 8;
    tb = (int)(k % ntl);
    rb = (k / ntl) * 8 + x;
    nrb = gridDim.x / ntl;
  }
  const int c0 = tb * NT;
  const int nc = min(NT, ny - c0);
  // S tile into LDS, four loads in flight per thread before their stores
  for (int idx0 = threadIdx.x; idx0 < nx * NT; idx0 += 4 * blockDim.x) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * blockDim.x, j = idx / NT, c = idx % NT;
      v[u] = (idx < nx * NT && c < nc) ? (T)S[j + (int64_t)(c0 + c) * lds] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (idx0 + u * blockDim.x < nx * NT) ss[idx0 + u * blockDim.x] = v[u];
  }
  __syncthreads();
  const int64_t N = x1.cols ? x1.rows : x2.rows;
  double g[NG > 0 ? NG : 1][NG > 0 ? NG : 1];
  if constexpr (NG > 0) {
#pragma unroll
    for (int a = 0; a < NG; ++a)
#pragma unroll
      for (int c = 0; c < NG; ++c) g[a][c] = 0.0;
  }
  // the output is a whole row-major block of NT columns: 16-byte row stores
  const bool yrow16 = row16_ok<T, NT>() && o.ycs == 1 && o.yrs == NT && c0 == 0 && nc == NT &&
                      ((uintptr_t)o.y & 15) == 0;
  // Z by 16-byte row loads too, for float32 rows (float64 rows measured
  // slower that way in the Gram variant)
  const bool zrow16 = row16_ok<T, NT>() && sizeof(T) == 4 && beta != 0.0 && o.zcs == 1 &&
                      o.zrs == NT && c0 == 0 && nc == NT && ((uintptr_t)o.z & 15) == 0;
  for (int64_t r = rb * blockDim.x + threadIdx.x; r < N; r += nrb * blockDim.x) {
    T acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = T(0);
    for (int j = 0; j < x1.cols; ++j) {
      T xv = x1.p[r * x1.rs + (int64_t)j * x1.cs];
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[c] = fma(xv, ss[j * NT + c], acc[c]);
    }
    for (int j = 0; j < x2.cols; ++j) {
      T xv = x2.p[r * x2.rs + (int64_t)j * x2.cs];
#pragma unroll
      for (int c = 0; c < NT; ++c)
        acc[c] = fma(xv, ss[(x1.cols + j) * NT + c], acc[c]);
    }
    T zr[NT];
    if constexpr (row16_ok<T, NT>()) {
      if (zrow16) load_row16<T, NT>(o.z + r * o.zrs, zr);
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      if (c < nc) {
        const int64_t col = c0 + c;
        T v = (T)alpha * acc[c];
        if (beta != 0.0) v += (T)beta * (zrow16 ? zr[c] : o.z[r * o.zrs + col * o.zcs]);
        if (!yrow16) o.y[r * o.yrs + col * o.ycs] = v;
        if (o.y2) o.y2[r * o.y2rs + col * o.y2cs] = v;
        acc[c] = v;
      }
    }
    if constexpr (row16_ok<T, NT>()) {
      if (yrow16) store_row16<T, NT>(o.y + r * o.yrs, acc);
    }
    if constexpr (NG > 0) {
#pragma unroll
      for (int a = 0; a < NG; ++a)
#pragma unroll
        for (int c = 0; c < NG; ++c) g[a][c] = fma((double)acc[a], (double)acc[c], g[a][c]);
    }
  }
  if constexpr (NG > 0) {
    // block partial: wave sums, then the waves in a fixed order
    __shared__ double red[16][NG * NG];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int a = 0; a < NG; ++a)
#pragma unroll
      for (int c = 0; c < NG; ++c) {
        const double v = wave_total(g[a][c]);
        if (lane == 0) red[w][a * NG + c] = v;
      }
    __syncthreads();
    if (threadIdx.x < NG * NG) {
      const int e = threadIdx.x;
      double v = red[0][e];
      for (int q = 1; q < nw; ++q) v += red[q][e];
      gpart[(int64_t)blockIdx.x * NG * NG + e] = v;
    }
  }
}

// One element through a raw buffer view (loads past the view's byte extent
// return zero).
template <typename T>
__device__ inline T raw_load(__amdgpu_buffer_rsrc_t rs, int off) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}
// One element stored through a raw buffer view at byte offset voff + soff
// (soff uniform over the wave).
template <typename T>
__device__ inline void raw_store(T v, __amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(unsigned __attribute__((ext_vector_type(2))), v), rs, voff, soff, 0);
}

// X S on the matrix cores for long operands, computed as (X S)^T = S^T X^T
// with 16 x 16 x 4 MFMA tiles: lane l supplies S(k0 + l/16, 16t + l%16)
// (from LDS) and X(r0 + l%16, k0 + l/16), so each X load instruction reads
// four runs of 16 consecutive rows, and receives (X S)(r0 + l%16, 16t + r)
// with r the accumulator's row of D: every store instruction writes runs of
// 16 consecutive rows of one output column.  A wave owns 16 rows at a time
// and all NT column tiles of the output (one X operand feeds NT MFMAs).
// The K dimension is taken KS steps of 4 columns per pass (S zero padded to
// whole passes): the KS loads of a pass are issued before its MFMAs, and
// neither carries a branch, so each MFMA waits for its own load only.
// Row r of X reaches output row r only, so rows past N may hold anything.
// BUF: X is one column-major operand (ld >= N) read through a buffer view
// of its extent, so columns past nx load as zero and each load is one
// 32-bit offset, and a plain product's column-major output is stored through
// a buffer view, its per-column offset uniform over the wave; otherwise every
// load reads an in-bounds element (row and column clamped) and columns past
// nx are zeroed where they are used.  The row offsets are rebuilt each tile
// (the empty asm hides them from the loop), so that the KS load offsets and
// the stores' column offsets are not held in registers across the loop.
// (The float64 buffer path asks for at least five waves per SIMD: left to
// itself the scheduler holds S operands of later steps in registers and the
// kernel runs four waves, 6% slower.)
template <typename T, int NT, int KS, bool PLAIN, bool BUF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && BUF ? 5 : 1)))
void k_nn_mfma(TV<T> x1, TV<T> x2, const double *S, int lds, int ny, double alpha, double beta,
               NnOut<T> o) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ss = reinterpret_cast<T *>(smem);  // S(k, c) at k * 16 NT + c, zero padded
  const int nx = x1.cols + x2.cols, W = 16 * NT;
  const int nk = (nx + 4 * KS - 1) / (4 * KS) * (4 * KS);
  for (int idx = threadIdx.x; idx < nk * W; idx += blockDim.x) {
    const int k = idx / W, c = idx % W;
    ss[idx] = (k < nx && c < ny) ? (T)S[k + (int64_t)c * lds] : T(0);
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t N = x1.cols ? x1.rows : x2.rows;
  const int64_t ntile = (N + 15) / 16;
  const int lr = lane & 15, lk = lane >> 4;
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)x1.p, (short)0, BUF ? (int)((N + (int64_t)(nx - 1) * x1.cs) * sizeof(T)) : 0,
      0x00020000);
  const int ldb = BUF ? (int)(x1.cs * sizeof(T)) : 0;
  const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)o.y, (short)0, BUF ? (int)((N + (int64_t)(ny - 1) * o.ycs) * sizeof(T)) : 0,
      0x00020000);
  const int ldy = BUF ? (int)(o.ycs * sizeof(T)) : 0;
  // the lane's part of the output column (the rest is uniform over the wave)
  const int lcol = Mfma16<T>::row(lane, 0);
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    const int64_t r = tile * 16 + lr;
    const bool rin = r < N;
    typename Mfma16<T>::v4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = typename Mfma16<T>::v4{T(0), T(0), T(0), T(0)};
    for (int k0 = 0; k0 < nk; k0 += 4 * KS) {
      T xb[KS];
      if constexpr (BUF) {
        int off = (int)r * (int)sizeof(T) + (k0 + lk) * ldb;
        asm("" : "+v"(off));
#pragma unroll
        for (int u = 0; u < KS; ++u) xb[u] = raw_load<T>(xr, off + 4 * u * ldb);
      } else {
        const int64_t rr = rin ? r : N - 1;
#pragma unroll
        for (int u = 0; u < KS; ++u) xb[u] = tall_at(x1, x2, rr, min(k0 + 4 * u + lk, nx - 1));
      }
#pragma unroll
      for (int u = 0; u < KS; ++u) {
        const int k = k0 + 4 * u + lk;
        const T xv = (BUF || k < nx) ? xb[u] : T(0);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = Mfma16<T>::op(ss[k * W + 16 * t + lr], xv, acc[t]);
      }
    }
    if constexpr (BUF && PLAIN) {
      int yoff = (int)r * (int)sizeof(T) + lcol * ldy;
      asm("" : "+v"(yoff));
      if (rin) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int cu = 16 * t + Mfma16<T>::row(0, v);  // uniform part of the column
            if (cu + lcol < ny) raw_store<T>((T)alpha * acc[t][v], yr, yoff, cu * ldy);
          }
        }
      }
    } else if (rin) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t col = 16 * t + Mfma16<T>::row(lane, v);
          if (col < ny) {
            T y = (T)alpha * acc[t][v];
            if constexpr (!PLAIN) {
              if (beta != 0.0) y += (T)beta * o.z[r * o.zrs + col * o.zcs];
              if (o.y2) o.y2[r * o.y2rs + col * o.y2cs] = y;
            }
            o.y[r * o.yrs + col * o.ycs] = y;
          }
        }
      }
    }
  }
}

// The float32 plain product of k_nn_mfma with each lane on a pair of
// consecutive rows: an 8-byte load gives the X operands of two MFMA tiles
// (rows r0 + 2j and r0 + 2j + 1 for the operand column j) that share every
// S operand, and an 8-byte store writes both outputs, so one load or store
// instruction covers four whole 128-byte runs of a column where the 16-row
// tile covers four halves.  Needs even leading dimensions and 8-byte aligned
// X and Y: the byte extents are then rounded up to 8 without reaching the
// next column, so a pair is wholly inside or wholly past the view.
template <int NT, int KS>
__global__ __launch_bounds__(256) void k_nn_mfma_pair(TV<float> x1, const double *S, int lds,
                                                       int ny, double alpha, NnOut<float> o) {
  extern __shared__ __align__(16) unsigned char smem[];
  float *ss = reinterpret_cast<float *>(smem);  // S(k, c) at k * 16 NT + c, zero padded
  const int nx = x1.cols, W = 16 * NT;
  const int nk = (nx + 4 * KS - 1) / (4 * KS) * (4 * KS);
  for (int idx = threadIdx.x; idx < nk * W; idx += blockDim.x) {
    const int k = idx / W, c = idx % W;
    ss[idx] = (k < nx && c < ny) ? (float)S[k + (int64_t)c * lds] : 0.0f;
  }
  __syncthreads();
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t N = x1.rows;
  const int64_t ntile = (N + 31) / 32;
  const int lr = lane & 15, lk = lane >> 4;
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)x1.p, (short)0, (int)(((N + (int64_t)(nx - 1) * x1.cs) * 4 + 7) & ~(int64_t)7),
      0x00020000);
  const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)o.y, (short)0, (int)(((N + (int64_t)(ny - 1) * o.ycs) * 4 + 7) & ~(int64_t)7),
      0x00020000);
  const unsigned ldb = (unsigned)(x1.cs * 4);
  const int ldy = (int)(o.ycs * 4);
  const int lcol = Mfma16<float>::row(lane, 0);
  const float al = (float)alpha;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    const int64_t r = tile * 32 + 2 * lr;  // rows r and r + 1
    Mfma16<float>::v4 a0[NT], a1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      a0[t] = Mfma16<float>::v4{0.0f, 0.0f, 0.0f, 0.0f};
      a1[t] = a0[t];
    }
    for (int k0 = 0; k0 < nk; k0 += 4 * KS) {
      f2 xb[KS];
      unsigned off = (unsigned)r * 4u + (unsigned)(k0 + lk) * ldb;
      asm("" : "+v"(off));
#pragma unroll
      for (int u = 0; u < KS; ++u)
        xb[u] = __builtin_bit_cast(
            f2, __builtin_amdgcn_raw_buffer_load_b64(xr, (int)(off + 4u * (unsigned)u * ldb), 0, 0));
#pragma unroll
      for (int u = 0; u < KS; ++u) {
        const int k = k0 + 4 * u + lk;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float sv = ss[k * W + 16 * t + lr];
          a0[t] = Mfma16<float>::op(sv, xb[u].x, a0[t]);
          a1[t] = Mfma16<float>::op(sv, xb[u].y, a1[t]);
        }
      }
    }
    if (r < N) {
      const bool two = r + 1 < N;
      int yoff = (int)r * 4 + lcol * ldy;
      asm("" : "+v"(yoff));
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cu = 16 * t + Mfma16<float>::row(0, v);  // uniform part of the column
          if (cu + lcol < ny) {
            const f2 y2 = {al * a0[t][v], al * a1[t][v]};
            if (two)
              __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, y2), yr, yoff, cu * ldy, 0);
            else
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, y2.x), yr, yoff,
                                                    cu * ldy, 0);
          }
        }
      }
    }
  }
}

// K-steps of 4 columns per pass of k_nn_mfma for nx columns of X: the
// fewest wasted steps among passes of 8, 9, 12, 13 or 16 (restarts from 33
// and from 50 columns take 9 and 13 steps exactly; a zero-padded step costs
// its MFMAs, 3-9% of the kernel's time at those widths).
inline int nnm_ksteps(int nx) {
  const int steps = (nx + 3) / 4;
  int best = 16, waste = 1 << 30;
  for (int ks : {16, 13, 12, 9, 8}) {
    const int w = (steps + ks - 1) / ks * ks - steps;
    if (w < waste) best = ks, waste = w;
  }
  return best;
}

// Row count from which X S (without the Gram output) takes the MFMA kernel.
constexpr int64_t kNnMfmaRows = 65536;

template <typename T>
void nn(const Tall<T> &X1, const Tall<T> &X2, const double *S, int lds, double alpha,
        const Tall<T> &Y, double beta, hipStream_t s, const Tall<T> *Z, const Tall<T> *Y2,
        const Scratch *gsc, TnParts *gram) {
  const int nx = X1.cols + X2.cols, ny = Y.cols;
  if (ny == 0 || Y.rows == 0) return;
  PHS_REQUIRE(nx <= 160, kEinval, "nn: operand too wide");
  PHS_REQUIRE(!Z || (Z->rows == Y.rows && Z->cols == Y.cols), kEinval, "nn: Z shape");
  PHS_REQUIRE(!Y2 || (Y2->rows == Y.rows && Y2->cols == Y.cols), kEinval, "nn: Y2 shape");
  PHS_REQUIRE(!gram || (gsc && (ny == 1 || ny == 2 || ny == 4)), kEinval,
              "nn: the Gram output needs 1, 2 or 4 columns");
  if (nx == 0 && beta == 1.0 && !Z && !Y2 && !gram) return;
  const int nt_m = (ny + 15) / 16;
  // one column-major operand whose padded extent fits a 31-bit byte offset
  // goes through a buffer view, with the fewest wasted K-steps
  const int ks_b = nnm_ksteps(nx), nk_b = (nx + 4 * ks_b - 1) / (4 * ks_b) * (4 * ks_b);
  const bool buf = X2.cols == 0 && X1.rs == 1 && X1.cs >= X1.rows &&
                   (double)(nk_b + 1) * (double)X1.cs * sizeof(T) < 2147483648.0 &&
                   Y.rs == 1 && Y.cs >= Y.rows &&
                   (double)(16 * nt_m + 1) * (double)Y.cs * sizeof(T) < 2147483648.0;
  const int ks_m = buf ? ks_b : 16;
  const size_t shm_m =
      (size_t)((nx + 4 * ks_m - 1) / (4 * ks_m) * (4 * ks_m)) * 16 * nt_m * sizeof(T);
  // (up to 16 output columns the vector kernel streams X faster: its loads
  // are runs of 64 rows, the MFMA operand's runs of 16)
  if (!gram && nx > 0 && ny > 16 && ny <= 64 && Y.rows >= kNnMfmaRows &&
      shm_m <= (size_t)device_lds_max()) {
    const int nt = nt_m;
    const size_t shm = shm_m;
    NnOut<T> o{Y.p, Y.rs, Y.cs, Z ? Z->p : Y.p, Z ? Z->rs : Y.rs, Z ? Z->cs : Y.cs,
               Y2 ? Y2->p : nullptr, Y2 ? Y2->rs : 0, Y2 ? Y2->cs : 0};
    const int64_t tiles = (Y.rows + 15) / 16;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + 3) / 4, 2048);
    prof_begin(kProfNn, s);
    // plain products (Y = alpha X S, the restarts) store one output only,
    // which keeps the hoisted store offsets out of the registers
    const bool plain = beta == 0.0 && !Z && !Y2;
    // float32 plain products in row pairs: even leading dimensions, 8-byte
    // aligned operands
    const bool pair = sizeof(T) == 4 && plain && buf && X1.cs % 2 == 0 && Y.cs % 2 == 0 &&
                      ((uintptr_t)X1.p & 7) == 0 && ((uintptr_t)Y.p & 7) == 0;
    const unsigned grid2 = (unsigned)std::min<int64_t>(((Y.rows + 31) / 32 + 3) / 4, 2048);
#define PHS_NNK(NT_, KS_, BUF_)                                                                  \
  do {                                                                                           \
    if constexpr (sizeof(T) == 4 && BUF_) {                                                      \
      if (pair) {                                                                                \
        k_nn_mfma_pair<NT_, KS_><<<grid2, 256, shm, s>>>(tv(X1), S, lds, ny, alpha, o);          \
        break;                                                                                   \
      }                                                                                          \
    }                                                                                            \
    if (plain)                                                                                   \
      k_nn_mfma<T, NT_, KS_, true, BUF_>                                                         \
          <<<grid, 256, shm, s>>>(tv(X1), tv(X2), S, lds, ny, alpha, beta, o);                   \
    else                                                                                         \
      k_nn_mfma<T, NT_, KS_, false, BUF_>                                                        \
          <<<grid, 256, shm, s>>>(tv(X1), tv(X2), S, lds, ny, alpha, beta, o);                   \
  } while (0)
#define PHS_NNM(NT_)                                     \
  do {                                                   \
    if (!buf) PHS_NNK(NT_, 16, false);                   \
    else if (ks_m == 16) PHS_NNK(NT_, 16, true);         \
    else if (ks_m == 13) PHS_NNK(NT_, 13, true);         \
    else if (ks_m == 12) PHS_NNK(NT_, 12, true);         \
    else if (ks_m == 9) PHS_NNK(NT_, 9, true);           \
    else PHS_NNK(NT_, 8, true);                          \
  } while (0)
    switch (nt) {
      case 1: PHS_NNM(1); break;
      case 2: PHS_NNM(2); break;
      case 3: PHS_NNM(3); break;
      default: PHS_NNM(4); break;
    }
#undef PHS_NNM
#undef PHS_NNK
    PHS_CHECK_LAUNCH();
    prof_end(kProfNn, s, (double)Y.rows * (nx + ny * (beta != 0.0 ? 2 : 1)) * sizeof(T));
    return;
  }
  // with the Gram partials: blocks of 1024 threads, at most 256 of them (each
  // thread then takes several rows), so that the consumer adds few partials
  // while as many waves are in flight as with 1024 blocks of 256
  const int threads = gram ? 1024 : 256;
  int64_t blocks = cdiv(Y.rows, threads);
  if (blocks > 4096) blocks = 4096;
  if (gram && blocks > 256) blocks = 256;
  const int nt = ny <= 4 ? 4 : ny <= 8 ? 8 : 16;
  const int ntl = (int)cdiv(ny, nt);
  if (ntl > 1) blocks = cdiv(blocks, 8) * 8;
  const unsigned grid = (unsigned)(blocks * ntl);
  size_t shm = (size_t)(nx > 0 ? nx : 1) * nt * sizeof(T);
  Tall<T> a = X1, b = X2;
  if (a.cols == 0 && b.cols == 0) a.rows = Y.rows;
  NnOut<T> o{Y.p, Y.rs, Y.cs, Z ? Z->p : Y.p, Z ? Z->rs : Y.rs, Z ? Z->cs : Y.cs,
             Y2 ? Y2->p : nullptr, Y2 ? Y2->rs : 0, Y2 ? Y2->cs : 0};
  prof_begin(kProfNn, s);
  double *gp = gram ? gsc->part : nullptr;
#define PHS_NN(NG, NT) \
  k_nn<T, NG, NT><<<grid, threads, shm, s>>>(tv(a), tv(b), S, lds, ny, alpha, beta, o, gp, ntl)
  if (!gram) {
    if (nt == 4) PHS_NN(0, 4);
    else if (nt == 8) PHS_NN(0, 8);
    else PHS_NN(0, 16);
  } else {
    switch (ny) {
      case 1: PHS_NN(1, 4); break;
      case 2: PHS_NN(2, 4); break;
      default: PHS_NN(4, 4); break;
    }
  }
#undef PHS_NN
  if (gram) *gram = TnParts{gp, (int)blocks, ny, ny};
  PHS_CHECK_LAUNCH();
  prof_end(kProfNn, s, (double)Y.rows * (nx + ny * (beta != 0.0 ? 2 : 1)) * sizeof(T));
}

// ---------------------------------------------------------- Ritz block
constexpr int kRitzMax = 32;

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ritz(TV<T> V, TV<T> W, const double *S, int lds,
                                              const double *theta, T *X, T *R, int ldx,
                                              int64_t ntop, double *part) {
  constexpr int nb = NB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int p = V.cols;
  T *ss = reinterpret_cast<T *>(smem);
  double *red = reinterpret_cast<double *>(smem + ((p * kRitzMax * sizeof(T) + 15) & ~15));
  // S block into LDS, eight loads in flight per thread before their stores
  for (int idx0 = threadIdx.x; idx0 < p * kRitzMax; idx0 += 8 * blockDim.x) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = idx0 + u * blockDim.x, j = idx / kRitzMax, c = idx % kRitzMax;
      v[u] = (idx < p * kRitzMax && c < nb) ? (T)S[j + (int64_t)c * lds] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (idx0 + u * blockDim.x < p * kRitzMax) ss[idx0 + u * blockDim.x] = v[u];
  }
  __shared__ T th[kRitzMax];
  if (threadIdx.x < kRitzMax) th[threadIdx.x] = threadIdx.x < nb ? (T)theta[threadIdx.x] : T(0);
  __syncthreads();
  double rs[NB], xs[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) rs[c] = xs[c] = 0.0;
  const int64_t N = V.rows;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * blockDim.x) {
    T ax[NB], aw[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) ax[c] = aw[c] = T(0);
    // eight columns of V and W (sixteen loads) in flight before their
    // products; columns past p are not read
    for (int j0 = 0; j0 < p; j0 += 8) {
      T v[8], w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u;
        v[u] = j < p ? V.p[r + (int64_t)j * V.cs] : T(0);
        w[u] = j < p ? W.p[r + (int64_t)j * W.cs] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (j0 + u < p) {
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            const T sv = ss[(j0 + u) * kRitzMax + c];
            ax[c] = fma(v[u], sv, ax[c]);
            aw[c] = fma(w[u], sv, aw[c]);
          }
        }
      }
    }
    T rrv[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      T rr = aw[c] - th[c] * ax[c];
      rrv[c] = rr;
      rs[c] += (double)rr * (double)rr;
      if (r < ntop) xs[c] += (double)ax[c] * (double)ax[c];
    }
    if constexpr (row16_ok<T, NB>()) {
      if (ldx == NB && (((uintptr_t)X | (uintptr_t)R) & 15) == 0) {
        store_row16<T, NB>(X + r * ldx, ax);
        store_row16<T, NB>(R + r * ldx, rrv);
        continue;
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      X[r * ldx + c] = ax[c];
      R[r * ldx + c] = rrv[c];
    }
  }
  // block reduction of the 2 nb sums
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    red[threadIdx.x] = rs[c];
    red[256 + threadIdx.x] = xs[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        red[threadIdx.x] += red[threadIdx.x + o];
        red[256 + threadIdx.x] += red[256 + threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[(int64_t)blockIdx.x * 2 * nb + c] = red[0];
      part[(int64_t)blockIdx.x * 2 * nb + nb + c] = red[256];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_reduce_vec(const double *part, int nblk, int E,
                                                   double *out0, double *out1, int split) {
  const int e = blockIdx.x;
  // lane l adds partials l, l + 64, ... in order; eight loads in flight
  double s = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * 64;
      v[u] = part[(int64_t)(b < nblk ? b : b0) * E + e];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u * 64 < nblk) s += v[u];
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    if (e < split) {
      if (out0) out0[e] = s;
    } else if (out1) {
      out1[e - split] = s;
    }
  }
}

template <typename T>
void ritz(const Tall<T> &V, const Tall<T> &W, const double *S, int lds, const double *theta,
          T *X, T *R, int nb, int ldx, double *rn2, double *xt2, int64_t ntop, const Scratch &sc,
          hipStream_t s) {
  PHS_REQUIRE(nb <= kRitzMax && V.rs == 1 && W.rs == 1, kEinval, "ritz: bad operands");
  int64_t blocks = cdiv(V.rows, 256);
  if (blocks > 1024) blocks = 1024;
  size_t shm = ((V.cols * kRitzMax * sizeof(T) + 15) & ~(size_t)15) + 512 * sizeof(double);
  prof_begin(kProfRitz, s);
#define PHS_RITZ(NB)                                                                       \
  k_ritz<T, NB><<<(unsigned)blocks, 256, shm, s>>>(tv(V), tv(W), S, lds, theta, X, R, ldx, ntop, \
                                                    sc.part)
  switch (nb) {
    case 1: PHS_RITZ(1); break;
    case 2: PHS_RITZ(2); break;
    case 3: PHS_RITZ(3); break;
    case 4: PHS_RITZ(4); break;
    case 5: PHS_RITZ(5); break;
    case 6: PHS_RITZ(6); break;
    case 7: PHS_RITZ(7); break;
    case 8: PHS_RITZ(8); break;
    case 16: PHS_RITZ(16); break;
    case 32: PHS_RITZ(32); break;
    default: throw Error(kEinval, "ritz: unsupported block width");
  }
#undef PHS_RITZ
  k_reduce_vec<<<2 * nb, 64, 0, s>>>(sc.part, (int)blocks, 2 * nb, rn2, xt2, nb);
  PHS_CHECK_LAUNCH();
  prof_end(kProfRitz, s, (double)V.rows * (2.0 * V.cols + 2.0 * nb) * sizeof(T));
}

// ------------------------------------------------------------ col norms
template <typename T>
__global__ __launch_bounds__(256) void k_colnorm2(TV<T> x, int64_t r0, int64_t r1,
                                                  double *part) {
  __shared__ double red[256];
  for (int j = 0; j < x.cols; ++j) {
    double acc = 0.0;
    for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1;
         r += (int64_t)gridDim.x * blockDim.x) {
      double v = (double)x.p[r * x.rs + (int64_t)j * x.cs];
      acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * x.cols + j] = red[0];
    __syncthreads();
  }
}

// Row-major block (row stride W a power of two <= 256, unit column
// stride): the rows [r0, r1) are one contiguous run of (r1 - r0) W values,
// read in order; with a thread count that is a multiple of W, thread t
// always meets column t mod W.
template <typename T>
__global__ __launch_bounds__(256) void k_colnorm2_rm(TV<T> x, int64_t r0, int64_t r1,
                                                     double *part) {
  __shared__ double red[256];
  const int W = (int)x.rs;
  const int c = threadIdx.x & (W - 1);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (c < x.cols) {
    const int64_t hi = r1 * W, S = (int64_t)gridDim.x * blockDim.x;
    int64_t e = r0 * W + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e + 3 * S < hi; e += 4 * S) {
      const double v0 = (double)x.p[e], v1 = (double)x.p[e + S];
      const double v2 = (double)x.p[e + 2 * S], v3 = (double)x.p[e + 3 * S];
      a0 = fma(v0, v0, a0);
      a1 = fma(v1, v1, a1);
      a2 = fma(v2, v2, a2);
      a3 = fma(v3, v3, a3);
    }
    for (; e < hi; e += S) {
      const double v = (double)x.p[e];
      a0 = fma(v, v, a0);
    }
  }
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int o = 128; o >= W; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < x.cols) part[(int64_t)blockIdx.x * x.cols + threadIdx.x] = red[threadIdx.x];
}

template <typename T>
void colnorm2(const Tall<T> &X, int64_t r0, int64_t r1, double *out, const Scratch &sc,
              hipStream_t s) {
  if (X.cols == 0) return;
  const bool rm = X.rs > 1 && X.cs == 1 && X.rs <= 256 && (X.rs & (X.rs - 1)) == 0 &&
                  X.cols <= X.rs;
  int64_t blocks;
  if (rm) {
    blocks = cdiv((r1 - r0 > 0 ? r1 - r0 : 1) * X.rs, 256 * 8);
    if (blocks > 2048) blocks = 2048;
    k_colnorm2_rm<T><<<(unsigned)blocks, 256, 0, s>>>(tv(X), r0, r1, sc.part);
    k_reduce_vec<<<X.cols, 64, 0, s>>>(sc.part, (int)blocks, X.cols, out, nullptr, X.cols);
    PHS_CHECK_LAUNCH();
    return;
  }
  blocks = cdiv(r1 - r0 > 0 ? r1 - r0 : 1, 256 * 4);
  if (blocks > 512) blocks = 512;
  k_colnorm2<T><<<(unsigned)blocks, 256, 0, s>>>(tv(X), r0, r1, sc.part);
  k_reduce_vec<<<X.cols, 64, 0, s>>>(sc.part, (int)blocks, X.cols, out, nullptr, X.cols);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------- element-wise
// One row per thread, columns in chunks of eight whose loads all precede
// their stores: consecutive lanes take consecutive rows, so column-major
// sides are coalesced and a row-major side is read or written one whole row
// per lane.
template <typename Ti, typename To>
__global__ void k_copy(TV<Ti> a, To *bp, int64_t brs, int64_t bcs) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Ti *src = a.p + i * a.rs;
    To *dst = bp + i * brs;
    for (int j0 = 0; j0 < a.cols; j0 += 8) {
      Ti v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < a.cols) v[u] = src[(int64_t)(j0 + u) * a.cs];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < a.cols) dst[(int64_t)(j0 + u) * bcs] = (To)v[u];
    }
  }
}

template <typename Ti, typename To>
void copy(const Tall<Ti> &src, const Tall<To> &dst, hipStream_t s) {
  const int64_t n = src.rows * src.cols;
  if (n == 0) return;
  PHS_REQUIRE(src.rows == dst.rows && src.cols == dst.cols, kEinval, "copy: shape mismatch");
  int64_t blocks = cdiv(src.rows, 256);
  if (blocks > 8192) blocks = 8192;
  k_copy<Ti, To><<<(unsigned)blocks, 256, 0, s>>>(tv(src), dst.p, dst.rs, dst.cs);
  PHS_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_scale_cols(T *p, int64_t rows, int cols, int64_t rs, int64_t cs,
                             const double *f) {
  const int64_t n = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = rs == 1 ? idx % rows : idx / cols;
    int64_t j = rs == 1 ? idx / rows : idx % cols;
    p[i * rs + j * cs] *= (T)f[j];
  }
}

template <typename T>
void scale_cols(const Tall<T> &X, const double *f, hipStream_t s) {
  const int64_t n = X.rows * X.cols;
  if (n == 0) return;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 8192) blocks = 8192;
  k_scale_cols<T><<<(unsigned)blocks, 256, 0, s>>>(X.p, X.rows, X.cols, X.rs, X.cs, f);
  PHS_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_axpby(TV<T> x, TV<T> z, double shift, T *yp, int64_t yrs, int64_t ycs) {
  const int64_t n = x.rows * x.cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = yrs == 1 ? idx % x.rows : idx / x.cols;
    int64_t j = yrs == 1 ? idx / x.rows : idx % x.cols;
    yp[i * yrs + j * ycs] = x.p[i * x.rs + j * x.cs] - (T)shift * z.p[i * z.rs + j * z.cs];
  }
}

template <typename T>
void axpby(const Tall<T> &X, const Tall<T> &Z, double shift, const Tall<T> &Y, hipStream_t s) {
  const int64_t n = X.rows * X.cols;
  if (n == 0) return;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 8192) blocks = 8192;
  k_axpby<T><<<(unsigned)blocks, 256, 0, s>>>(tv(X), tv(Z), shift, Y.p, Y.rs, Y.cs);
  PHS_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_fill_random(T *p, int64_t rows, int cols, int64_t rs, int64_t cs,
                              uint64_t seed, uint64_t sid) {
  const int64_t n = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = idx % rows, j = idx / rows;
    p[i * rs + j * cs] = (T)stream_uniform(seed, sid + (uint64_t)j, (uint64_t)i);
  }
}

template <typename T>
void fill_random(const Tall<T> &X, uint64_t seed, uint64_t sid, hipStream_t s) {
  const int64_t n = X.rows * X.cols;
  if (n == 0) return;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 8192) blocks = 8192;
  k_fill_random<T><<<(unsigned)blocks, 256, 0, s>>>(X.p, X.rows, X.cols, X.rs, X.cs, seed, sid);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------------ Jacobi
// den = d - theta, clamped away from 0 by 1e-3 d (sign kept).
__device__ inline double jac_den(double d, double th) {
  double den = d - th, lim = 1e-3 * d;
  if (fabs(den) < lim) den = den >= 0 ? lim : -lim;
  return den;
}

// Pass 1: T = M r with M = (diag(C) - theta)^-1, or, for the Olsen form,
// only the block partials of x^T M r and x^T M x.  All loads of a row
// precede its stores.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_jacobi1(const T *__restrict__ R, const T *__restrict__ X,
                                                 const double *__restrict__ d,
                                                 const double *__restrict__ theta, int64_t n,
                                                 int ldx, bool olsen, T *__restrict__ Tout,
                                                 double *__restrict__ part) {
  __shared__ double red[2][256];
  double th[NB], a[NB], b[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    th[c] = theta[c];
    a[c] = b[c] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double di = d[i];
    T rv[NB], xv[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) rv[c] = R[i * ldx + c];
    if (olsen) {
#pragma unroll
      for (int c = 0; c < NB; ++c) xv[c] = X[i * ldx + c];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double rd = 1.0 / jac_den(di, th[c]);
        const double x = (double)xv[c];
        a[c] = fma(x, (double)rv[c] * rd, a[c]);
        b[c] = fma(x * x, rd, b[c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) Tout[i * ldx + c] = (T)((double)rv[c] / jac_den(di, th[c]));
    }
  }
  if (!olsen) return;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    red[0][threadIdx.x] = a[c];
    red[1][threadIdx.x] = b[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        red[0][threadIdx.x] += red[0][threadIdx.x + o];
        red[1][threadIdx.x] += red[1][threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[(int64_t)blockIdx.x * 2 * NB + c] = red[0][0];
      part[(int64_t)blockIdx.x * 2 * NB + NB + c] = red[1][0];
    }
    __syncthreads();
  }
}

// Pass 2 of the Olsen form: T = M (r - e x), e = x^T M r / x^T M x.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_jacobi2(const T *__restrict__ R, const T *__restrict__ X,
                                                 const double *__restrict__ d,
                                                 const double *__restrict__ theta, int64_t n,
                                                 int ldx, const double *__restrict__ dots,
                                                 T *__restrict__ Tout) {
  // R and X by 16-byte row loads
  const bool v16 = ldx == NB && (((uintptr_t)R | (uintptr_t)X) & 15) == 0;
  double th[NB], e[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    th[c] = theta[c];
    e[c] = dots[NB + c] != 0.0 ? dots[c] / dots[NB + c] : 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double di = d[i];
    T rv[NB], xv[NB];
    bool done = false;
    if constexpr (row16_ok<T, NB>()) {
      if (v16) {
        load_row16<T, NB>(R + i * ldx, rv);
        load_row16<T, NB>(X + i * ldx, xv);
        done = true;
      }
    }
    if (!done) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        rv[c] = R[i * ldx + c];
        xv[c] = X[i * ldx + c];
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      Tout[i * ldx + c] = (T)(((double)rv[c] - e[c] * (double)xv[c]) / jac_den(di, th[c]));
  }
}

template <typename T>
void jacobi_apply(const T *R, const T *X, const double *d, const double *theta, int64_t n,
                  int nb, int ldx, bool olsen, T *Tout, const Scratch &sc, hipStream_t s) {
  PHS_REQUIRE(nb <= kRitzMax, kEinval, "jacobi: block too wide");
  PHS_REQUIRE(R != Tout && X != Tout, kEinval, "jacobi: output aliases an input");
  int64_t blocks = cdiv(n, 256);
  if (blocks > 1024) blocks = 1024;
#define PHS_JAC(NB)                                                                         \
  case NB:                                                                                  \
    k_jacobi1<T, NB><<<(unsigned)blocks, 256, 0, s>>>(R, X, d, theta, n, ldx, olsen, Tout,  \
                                                      sc.part);                             \
    if (olsen) {                                                                            \
      k_reduce_vec<<<2 * NB, 64, 0, s>>>(sc.part, (int)blocks, 2 * NB, sc.aux, nullptr,     \
                                         2 * NB);                                           \
      k_jacobi2<T, NB><<<(unsigned)blocks, 256, 0, s>>>(R, X, d, theta, n, ldx, sc.aux, Tout); \
    }                                                                                       \
    break;
  switch (nb) {
    PHS_JAC(1)
    PHS_JAC(2)
    PHS_JAC(3)
    PHS_JAC(4)
    PHS_JAC(5)
    PHS_JAC(6)
    PHS_JAC(7)
    PHS_JAC(8)
    PHS_JAC(16)
    PHS_JAC(32)
    default: throw Error(kEinval, "jacobi: unsupported block width");
  }
#undef PHS_JAC
  PHS_CHECK_LAUNCH();
}

__global__ void k_col_sq_norms(int64_t n, const int64_t *rp, const double *va, double *d) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int64_t p = rp[j]; p < rp[j + 1]; ++p) s += va[p] * va[p];
  d[j] = s;
}

void col_sq_norms(const SpMat<double> &At, double *d, hipStream_t s) {
  if (At.m == 0) return;
  k_col_sq_norms<<<cdiv(At.m, 256), 256, 0, s>>>(At.m, At.rowptr, At.val, d);
  PHS_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_row_scale(const T *X, const double *w, int64_t n, int b, bool inv, T *Y) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * b;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = idx / b;
    Y[idx] = inv ? (T)((double)X[idx] / w[i]) : (T)((double)X[idx] * w[i]);
  }
}

template <typename T>
void row_scale(const T *X, const double *w, int64_t n, int b, bool inv, T *Y, hipStream_t s) {
  if (n * b == 0) return;
  int64_t blocks = cdiv(n * b, 256);
  if (blocks > 8192) blocks = 8192;
  k_row_scale<T><<<(unsigned)blocks, 256, 0, s>>>(X, w, n, b, inv, Y);
  PHS_CHECK_LAUNCH();
}

#define PHS_INST(T)                                                                           \
  template void tn<T>(const Tall<T> &, const Tall<T> &, const Tall<T> &, double *, int,      \
                      const Scratch &, hipStream_t, TnParts *);                              \
  template void nn<T>(const Tall<T> &, const Tall<T> &, const double *, int, double,         \
                      const Tall<T> &, double, hipStream_t, const Tall<T> *,                 \
                      const Tall<T> *, const Scratch *, TnParts *);                          \
  template void ritz<T>(const Tall<T> &, const Tall<T> &, const double *, int, const double *, \
                        T *, T *, int, int, double *, double *, int64_t, const Scratch &,     \
                        hipStream_t);                                                         \
  template void colnorm2<T>(const Tall<T> &, int64_t, int64_t, double *, const Scratch &,     \
                            hipStream_t);                                                     \
  template void scale_cols<T>(const Tall<T> &, const double *, hipStream_t);                  \
  template void axpby<T>(const Tall<T> &, const Tall<T> &, double, const Tall<T> &,           \
                         hipStream_t);                                                        \
  template void fill_random<T>(const Tall<T> &, uint64_t, uint64_t, hipStream_t);             \
  template void jacobi_apply<T>(const T *, const T *, const double *, const double *, int64_t, \
                                int, int, bool, T *, const Scratch &, hipStream_t);           \
  template void row_scale<T>(const T *, const double *, int64_t, int, bool, T *, hipStream_t);
PHS_INST(float)
PHS_INST(double)
template void copy<float, float>(const Tall<float> &, const Tall<float> &, hipStream_t);
template void copy<double, double>(const Tall<double> &, const Tall<double> &, hipStream_t);
template void copy<float, double>(const Tall<float> &, const Tall<double> &, hipStream_t);
template void copy<double, float>(const Tall<double> &, const Tall<float> &, hipStream_t);

}  // namespace phs

namespace phs {

// Normalise column j of a column-major X from its squared norm n2 (device):
// X(:, j) /= sqrt(n2), or zeroed when n2 is below tiny; Rjj = sqrt(n2).
template <typename T>
__global__ void k_norm_col(T *x, int64_t rows, const double *n2, double tiny, double *Rjj) {
  const double nv = sqrt(fmax(n2[0], 0.0));
  const double f = nv > tiny ? 1.0 / nv : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] * f);
  if (blockIdx.x == 0 && threadIdx.x == 0 && Rjj) Rjj[0] = nv > tiny ? nv : 0.0;
}

template <typename T>
void norm_col(T *x, int64_t rows, const double *n2, double tiny, double *Rjj, hipStream_t s) {
  int64_t blocks = cdiv(rows, 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_norm_col<T><<<(unsigned)blocks, 256, 0, s>>>(x, rows, n2, tiny, Rjj);
  PHS_CHECK_LAUNCH();
}
template void norm_col<float>(float *, int64_t, const double *, double, double *, hipStream_t);
template void norm_col<double>(double *, int64_t, const double *, double, double *, hipStream_t);

template <typename T>
__global__ void k_fill_const(T *p, int64_t rows, int64_t rs, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i * rs] = v;
}

template <typename T>
void fill_const_col(T *p, int64_t rows, int64_t rs, double v, hipStream_t s) {
  int64_t blocks = cdiv(rows, 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_fill_const<T><<<(unsigned)blocks, 256, 0, s>>>(p, rows, rs, (T)v);
  PHS_CHECK_LAUNCH();
}
template void fill_const_col<float>(float *, int64_t, int64_t, double, hipStream_t);
template void fill_const_col<double>(double *, int64_t, int64_t, double, hipStream_t);

}  // namespace phs
