// Small dense float64 kernels, one workgroup each (p <= 64).
//
// The projected problems of the method -- the eigenpairs of the
// Rayleigh-Ritz matrix H (Algorithm 1; Algorithm 2 step 8), the SVD of the
// refined projection factor R (step 9), Cholesky factors for CholQR, QR and
// triangular inverses, restart rotations -- are at most 64 x 64 and run in
// LDS inside one workgroup.  The symmetric eigenproblem computes only the
// eigenpairs an iteration uses: Householder tridiagonalisation, Sturm
// multisection for the wanted eigenvalues (one point per lane), inverse
// iteration with Gram-Schmidt inside clusters, and the reflectors applied
// back.  The SVD is one-sided (Hestenes) Jacobi with round-robin pair
// ordering, so the p/2 rotations of a round run in parallel; it computes
// small singular values to high relative accuracy, which the refined
// projection needs near convergence.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "wave.hpp"

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

// ---------------------------------------------------------- syev
// Rayleigh-Ritz eigenproblem H s = theta s of the search space (p <= 64),
// float64, one workgroup of four wavefronts; lane t of each wave works on
// row t of H in LDS.  Steps 1, 2 and 4 use all four waves, the inverse
// iteration (step 3) runs on wave 0.
//  1. Householder reduction H = Q T Q^T to tridiagonal T, last row first;
//     the reflectors stay in the rows of H they annihilate.
//  2. Selected eigenvalues of T by multisection of Sturm sequences: the
//     eigenvalue of rank r is bracketed by the lanes of one group, each
//     evaluating the count at one interior point per step; the group keeps
//     the subinterval below the first point whose count exceeds the rank.
//  3. Eigenvectors of T by inverse iteration, one lane per vector;
//     vectors of nearly equal eigenvalues are orthogonalised between
//     sweeps, those of a cluster (eigenvalues within 1e-3 ||T||) after the
//     last sweep.
//  4. s = Q y by applying the reflectors, each vector held in the
//     registers of a lane group.
// Outputs: theta[0..nvec) and S(:, 0..nvec) for the nvec eigenpairs at the
// wanted end (ascending, or descending if `desc`), and (if other_end)
// theta[p-1], the eigenvalue at the other end.  Other entries are not
// written.
constexpr int kPadRows = kSmallMax + 8;

// Step 2 with Q points per lane and L lanes per eigenvalue (Q * L <= 64).
template <int Q>
__device__ void multisect(const double *ds, const double *e2s, int n, int ne, int nvec, int L,
                          bool desc, double lo, double hi, double *lamv) {
  const double eps = 2.220446049250313e-16;
  const int t = threadIdx.x;
  const int slot = t / L, sub = t % L;
  const bool act = slot < ne;
  const int rank = act ? (slot < nvec ? slot : n - 1) : 0;
  const int jidx = desc ? n - 1 - rank : rank;
  const int P = Q * L;
  const int base = (t & 63) - sub;  // first lane of the group in its wave
  const unsigned long long gmask = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
  double a0 = lo - eps, b0 = hi + eps;
  // width 2 + 2 eps down to below 1e-2 eps: a factor 2^59.7
  const int nst = (int)ceil(59.8 / log2((double)(P + 1))) + 1;
  for (int it = 0; it < nst; ++it) {
    const double w = (b0 - a0) / (double)(P + 1);
    double x[Q], pm[Q], pc[Q];
    int cnt[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      x[k] = a0 + (double)(k * L + sub + 1) * w;
      pm[k] = 1.0;
      pc[k] = ds[0] - x[k];
      if (pc[k] == 0.0) pc[k] = -1e-290;
      cnt[k] = pc[k] < 0.0;
    }
    // p_i = (d_i - x) p_{i-1} - e_i^2 p_{i-2}; rows past n are padded with
    // d = 4, e = 0 (no sign change); the pair is rescaled every 8 rows
    for (int i0 = 1; i0 < n; i0 += 8) {
      double dv[8], ev[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        dv[u] = ds[i0 + u];
        ev[u] = e2s[i0 + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          double pn = fma(dv[u] - x[k], pc[k], -ev[u] * pm[k]);
          // an exact zero takes the sign opposite to its predecessor
          if (pn == 0.0) pn = -copysign(1e-290, pc[k]);
          // sign change: the sign bits of the high words differ
          cnt[k] += (int)(((unsigned)__double2hiint(pn) ^ (unsigned)__double2hiint(pc[k])) >> 31);
          pm[k] = pc[k];
          pc[k] = pn;
        }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        int ex;
        frexp(fmax(fabs(pm[k]), fabs(pc[k])), &ex);
        pm[k] = ldexp(pm[k], -ex);
        pc[k] = ldexp(pc[k], -ex);
      }
    }
    // bit k*L + sub of the group mask: point k*L + sub lies above the
    // eigenvalue
    unsigned long long above = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k)
      above |= ((__ballot(act && cnt[k] > jidx) >> base) & gmask) << (k * L);
    const int j = above ? __ffsll((long long)above) - 1 : P;
    const double na = j > 0 ? a0 + (double)j * w : a0;
    const double nb = j < P ? a0 + (double)(j + 1) * w : b0;
    a0 = na;
    b0 = fmax(nb, na);
  }
  if (act && sub == 0) lamv[slot] = 0.5 * (a0 + b0);
}

// Step 4 with G lanes per vector, R = 64 / G rows per lane in registers.
template <int G>
__device__ void apply_reflectors(const double *a, const double *rh, const double *y, int n,
                                 int nvec, const double *lamv, double tnorm, double *theta,
                                 double *Sout, int lds) {
  constexpr int R = kSmallMax / G;
  const int t = threadIdx.x;
  const int c = t / G, sub = t % G;
  const bool act = c < nvec;
  double yr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = sub + r * G;
    yr[r] = (act && k < n) ? y[k * kLd + c] : 0.0;
  }
  for (int i = 2; i < n; ++i) {
    const double ih = rh[i];
    if (ih == 0.0) continue;
    // reflector entries k < i, masked without branches
    double av[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = sub + r * G;
      const double x = a[i * kLd + k];
      av[r] = k < i ? x : 0.0;
    }
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int r = 0; r < R; r += 2) {
      d0 = fma(av[r], yr[r], d0);
      if (r + 1 < R) d1 = fma(av[r + 1], yr[r + 1], d1);
    }
    const double sc = group_sum<G>(d0 + d1) * ih;
#pragma unroll
    for (int r = 0; r < R; ++r) yr[r] = fma(-sc, av[r], yr[r]);
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = sub + r * G;
      if (k < n) Sout[k + (int64_t)c * lds] = yr[r];
    }
    if (sub == 0) theta[c] = lamv[c] * tnorm;
  }
}

__global__ __launch_bounds__(256) void k_syev(const double *H, int ldh, int p, int nvec, bool desc,
                                             bool other_end, double *theta, double *Sout,
                                             int lds) {
  __shared__ double a[kSmallMax * kLd];   // H, then the reflectors
  __shared__ double y[kPadRows * kLd];    // eigenvectors of T, column per vector
  __shared__ double uu[kSmallMax * kLd];  // 1 / pivots of (T - lambda I) / ||T||
  __shared__ double ll[kPadRows * kLd];   // multipliers
  __shared__ double vv[kPadRows], pq[kPadRows], hh[kSmallMax], rh[kSmallMax];
  __shared__ double pp[4 * kSmallMax];  // partial products of the four waves
  __shared__ double d[kSmallMax], e[kSmallMax + 1], ds[kPadRows], e2s[kPadRows], es1[kSmallMax];
  __shared__ double lamv[kSmallMax + 1];
  __shared__ int cstart[kSmallMax], tstart[kSmallMax];
  // wave 0 runs step 3; all four waves run steps 1, 2 and 4
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool w0 = w == 0;
  const int n = p;
  const double eps = 2.220446049250313e-16;
  // symmetric part of H: lane t writes row t, wave w the columns k = w mod 4;
  // columns n..63 are zero (the chunks of step 1 read up to column 63 with
  // weight 0, and LDS left by an earlier kernel may hold NaN patterns)
  if (t < n) {
#pragma unroll 4
    for (int k = w; k < n; k += 4)
      a[t * kLd + k] = 0.5 * (H[t + (int64_t)k * ldh] + H[k + (int64_t)t * ldh]);
    for (int k = n + w; k < kSmallMax; k += 4) a[t * kLd + k] = 0.0;
  }
  if (w0) {
    hh[t] = 0.0;
    rh[t] = 0.0;
    vv[t] = 0.0;
    pq[t] = 0.0;
    if (t < kPadRows - kSmallMax) {
      vv[kSmallMax + t] = 0.0;
      pq[kSmallMax + t] = 0.0;
    }
  }
  __syncthreads();
  // 1. reduction of row i onto position i - 1 (l = i - 1).  Every wave
  //    forms the reflector from row i itself and, after the cross-wave sum
  //    of A v, the vector q itself (identical values in every wave, so
  //    every wave takes the same branches); the product A v and the
  //    rank-two update are split into column blocks of 16, one per wave.
  //    Each wave keeps its own copies of v and q (in uu and ll, unused
  //    until step 3), so a step has two block barriers: after the partial
  //    products, and after the update.
  const int kb = 16 * w;  // this wave's column block
  double *vw = uu + w * kSmallMax, *qw = ll + w * kSmallMax;
  for (int i = n - 1; i >= 2; --i) {
    const int l = i - 1;
    const double xi = (t <= l) ? a[i * kLd + t] : 0.0;
    double scale = 1.0, xs = xi, f = a[i * kLd + l];
    double sigma = wave_total(xi * xi);
    if (!(sigma > 1e-280 && sigma < 1e280)) {  // rare: scale by the 1-norm first
      scale = wave_total(fabs(xi));
      if (scale == 0.0) {
        if (threadIdx.x == 0) e[i] = 0.0;
        continue;  // hh[i] stays 0: no reflector
      }
      const double isc = 1.0 / scale;
      xs = xi * isc;
      f *= isc;
      sigma = wave_total(xs * xs);
    }
    const double g = f >= 0 ? -sqrt(sigma) : sqrt(sigma);
    const double h = sigma - f * g;
    const double ih = 1.0 / h;
    const double v = (t == l) ? f - g : xs;  // reflector I - v v^T / h; 0 past l
    vw[t] = v;
    if (threadIdx.x == 0) {
      e[i] = scale * g;
      hh[i] = h;
      rh[i] = ih;
    }
    wave_sync();
    // partial (A v)_t over this wave's column block (v is 0 past l)
    {
      double s0 = 0.0, s1 = 0.0;
      if (t <= l) {
#pragma unroll
        for (int c8 = 0; c8 < 16; c8 += 8) {
          if (kb + c8 > l) break;
          double av[8], vk[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            av[u] = a[t * kLd + kb + c8 + u];
            vk[u] = vw[kb + c8 + u];
          }
          s0 = fma(av[0], vk[0], s0); s1 = fma(av[1], vk[1], s1);
          s0 = fma(av[2], vk[2], s0); s1 = fma(av[3], vk[3], s1);
          s0 = fma(av[4], vk[4], s0); s1 = fma(av[5], vk[5], s1);
          s0 = fma(av[6], vk[6], s0); s1 = fma(av[7], vk[7], s1);
        }
      }
      pp[w * kSmallMax + t] = s0 + s1;
    }
    __syncthreads();
    const double pj = (t <= l) ? ((pp[t] + pp[kSmallMax + t]) +
                                  (pp[2 * kSmallMax + t] + pp[3 * kSmallMax + t])) * ih
                               : 0.0;
    const double K = wave_total(v * pj) * (0.5 * ih);
    const double qj = (t <= l) ? pj - K * v : 0.0;
    qw[t] = qj;
    wave_sync();
    // rank-two update of this wave's column block; columns past l see
    // q = v = 0 and stay unchanged
    if (t <= l) {
#pragma unroll
      for (int c8 = 0; c8 < 16; c8 += 8) {
        if (kb + c8 > l) break;
        double qk[8], vk[8], av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          qk[u] = qw[kb + c8 + u];
          vk[u] = vw[kb + c8 + u];
          av[u] = a[t * kLd + kb + c8 + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          a[t * kLd + kb + c8 + u] = av[u] - (v * qk[u] + qj * vk[u]);
      }
      if (w0) a[i * kLd + t] = v;
    }
    __syncthreads();
  }
  if (w0) {
    if (t == 0) {
      e[0] = 0.0;
      e[n] = 0.0;
      if (n >= 2) e[1] = a[1 * kLd + 0];
    }
    if (t < n) d[t] = a[t * kLd + t];
  }
  __syncthreads();
  // T scaled to unit norm (Gershgorin bound)
  double lo = 1e300, hi = -1e300;
  if (t < n) {
    const double r = fabs(e[t]) + fabs(e[t + 1]);
    lo = d[t] - r;
    hi = d[t] + r;
  }
  lo = -wave_max(-lo);
  hi = wave_max(hi);
  double tnorm = fmax(fabs(lo), fabs(hi));
  if (!(tnorm > 0.0)) tnorm = 1.0;
  const double sc = 1.0 / tnorm;
  if (w0) {
    ds[t] = t < n ? d[t] * sc : 4.0;
    e2s[t] = (t > 0 && t < n) ? (e[t] * sc) * (e[t] * sc) : 0.0;
    if (t < kPadRows - kSmallMax) {
      ds[kSmallMax + t] = 4.0;
      e2s[kSmallMax + t] = 0.0;
    }
  }
  __syncthreads();
  // 2. multisection.  Slots 0..nvec-1: ranks 0..nvec-1; slot nvec (if
  //    nvec < n): rank n-1.  Rank r is ascending index r, or n-1-r if desc.
  {
    const int ne = (other_end && nvec < n) ? nvec + 1 : nvec;
    // one point per lane: the recurrences are issue-bound, so a second or
    // fourth interleaved point per lane costs nearly its full time while
    // adding under one bit per step (p = 35: 4 + 1 eigenvalues 24.5 -> 17.6
    // us, 21 + 1 eigenvalues 53.1 -> 26.7 us against 2 and 4 points per lane)
    int L = 64;
    while (L * ne > 256) L >>= 1;
    multisect<1>(ds, e2s, n, ne, nvec, L, desc, lo * sc, hi * sc, lamv);
  }
  __syncthreads();
  if (w0) {
  // 3. inverse iteration on (T - lambda I)/||T|| = L U without pivoting,
  //    tiny pivots replaced; two sweeps from a pseudo-random start (the
  //    shift is accurate to rounding, so each sweep reduces every other
  //    component by gap / rounding).  Rows n..n+7 of the column are
  //    zero padding (multiplier 0), so the chunked loops need no guards.
  if (t < nvec) {
    const int c = t;
    const double lam = lamv[c];
    const double tiny = 1e-3 * eps;
    double u = ds[0] - lam;
    if (fabs(u) < tiny) u = tiny;
    double ru = 1.0 / u;  // one division per row: the multiplier reuses it
    uu[c] = ru;
    ll[c] = 0.0;
    // rows eight at a time (e and ds of the chunk loaded together; rows
    // past n are padding: ds = 4, e = 0, results unused)
    for (int i0 = 1; i0 < n; i0 += 8) {
      double ev[8], dv[8];
#pragma unroll
      for (int u8 = 0; u8 < 8; ++u8) {
        ev[u8] = i0 + u8 < n ? e[i0 + u8] : 0.0;
        dv[u8] = ds[i0 + u8];
      }
#pragma unroll
      for (int u8 = 0; u8 < 8; ++u8) {
        const int i = i0 + u8;
        const double es = ev[u8] * sc;
        const double li = es * ru;
        u = dv[u8] - lam - li * es;
        if (fabs(u) < tiny) u = tiny;
        ru = 1.0 / u;
        if (i < n) {
          ll[i * kLd + c] = li;
          uu[i * kLd + c] = ru;
        }
      }
    }
    for (int i = 0; i < n; ++i) {
      uint32_t hsh = (uint32_t)(i * kSmallMax + c + 1) * 0x9E3779B9u;
      hsh ^= hsh >> 16; hsh *= 0x85EBCA6Bu; hsh ^= hsh >> 13; hsh *= 0xC2B2AE35u; hsh ^= hsh >> 16;
      y[i * kLd + c] = (double)(hsh >> 8) * (2.0 / 16777216.0) - 1.0;
    }
    for (int i = n; i < n + 8; ++i) {
      y[i * kLd + c] = 0.0;
      ll[i * kLd + c] = 0.0;
    }
    int st = c, tt = c;
    while (st > 0 && fabs(lamv[st] - lamv[st - 1]) <= 1e-3) --st;
    while (tt > 0 && fabs(lamv[tt] - lamv[tt - 1]) <= 1e-10) --tt;
    cstart[c] = st;
    tstart[c] = tt;
  }
  // superdiagonal of the scaled T, shared: es1[i] = e_{i+1} / ||T||
  es1[t] = (t + 1 < n) ? e[t + 1] * sc : 0.0;
  wave_sync();
  constexpr int kSweeps = 2;
  for (int sweep = 0; sweep < kSweeps; ++sweep) {
    if (t < nvec) {
      const int c = t;
      // L w = y
      double w = y[c];
      double big = 0.0;
      for (int i0 = 1; i0 < n; i0 += 8) {
        double yv[8], lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          yv[u] = y[(i0 + u) * kLd + c];
          lv[u] = ll[(i0 + u) * kLd + c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          w = yv[u] - lv[u] * w;
          yv[u] = w;
          big = fmax(big, fabs(w));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) y[(i0 + u) * kLd + c] = yv[u];
      }
      // U x = w, bottom up; rows below 0 go to padding row n + 7
      double x = y[(n - 1) * kLd + c] * uu[(n - 1) * kLd + c];
      y[(n - 1) * kLd + c] = x;
      big = fmax(big, fabs(x));
      for (int i0 = n - 2; i0 >= 0; i0 -= 8) {
        double yv[8], uv[8], ev[8];
        int row[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 - u;
          row[u] = i >= 0 ? i : n + 7;
          yv[u] = y[row[u] * kLd + c];
          uv[u] = i >= 0 ? uu[row[u] * kLd + c] : 0.0;
          ev[u] = es1[i >= 0 ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          x = (yv[u] - ev[u] * x) * uv[u];
          yv[u] = x;
          big = fmax(big, fabs(x));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) y[row[u] * kLd + c] = i0 - u >= 0 ? yv[u] : 0.0;
      }
      if (!(big < 1e150)) {
        // growth beyond 1e150 (tiny pivots in a row): the sweep is redone
        // from the start vector scaled by 1e-200
        for (int i = 0; i < n; ++i) {
          uint32_t hsh = (uint32_t)(i * kSmallMax + c + 1) * 0x9E3779B9u;
          hsh ^= hsh >> 16; hsh *= 0x85EBCA6Bu; hsh ^= hsh >> 13; hsh *= 0xC2B2AE35u;
          hsh ^= hsh >> 16;
          y[i * kLd + c] = ((double)(hsh >> 8) * (2.0 / 16777216.0) - 1.0) * 1e-200;
        }
        double w2 = y[c];
        for (int i = 1; i < n; ++i) {
          w2 = y[i * kLd + c] - ll[i * kLd + c] * w2;
          y[i * kLd + c] = w2;
        }
        double x2 = y[(n - 1) * kLd + c] * uu[(n - 1) * kLd + c];
        y[(n - 1) * kLd + c] = x2;
        for (int i = n - 2; i >= 0; --i) {
          x2 = (y[i * kLd + c] - es1[i] * x2) * uu[i * kLd + c];
          y[i * kLd + c] = x2;
        }
      }
      // normalise (entries below 1e150 after a good sweep: no overflow)
      double s0 = 0.0, s1 = 0.0;
      for (int i0 = 0; i0 < n; i0 += 8) {
        double yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = y[(i0 + u) * kLd + c];
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          const double a0 = fabs(yv[u]) < 1e300 ? yv[u] : 0.0;
          const double a1 = fabs(yv[u + 1]) < 1e300 ? yv[u + 1] : 0.0;
          s0 = fma(a0, a0, s0);
          s1 = fma(a1, a1, s1);
        }
      }
      const double s2 = s0 + s1;
      const bool ok = s2 > 0.0 && s2 < 1e300;
      const double in2 = ok ? 1.0 / sqrt(s2) : 0.0;
      for (int i0 = 0; i0 < n; i0 += 8) {
        double yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = y[(i0 + u) * kLd + c];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (i0 + u < n) y[(i0 + u) * kLd + c] = fabs(yv[u]) < 1e300 ? yv[u] * in2 : 0.0;
      }
      if (!ok) y[(c % n) * kLd + c] = 1.0;
    }
    wave_sync();
    // Gram-Schmidt: between sweeps against vectors of eigenvalues within
    // 1e-10 ||T||, after the last sweep within 1e-3 ||T||; lanes split the
    // dot products, then the rows; repeated when the first pass cancels
    // more than half
    const int *start = sweep == kSweeps - 1 ? cstart : tstart;
    for (int c = 1; c < nvec; ++c) {
      const int st = start[c];
      if (st == c) continue;
      for (int pass = 0; pass < 2; ++pass) {
        if (t >= st && t < c) {
          double s0 = 0.0, s1 = 0.0;
          for (int i0 = 0; i0 < n; i0 += 8) {
            double yk[8], yc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              yk[u] = y[(i0 + u) * kLd + t];
              yc[u] = y[(i0 + u) * kLd + c];
            }
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
              if (i0 + u < n) s0 = fma(yk[u], yc[u], s0);
              if (i0 + u + 1 < n) s1 = fma(yk[u + 1], yc[u + 1], s1);
            }
          }
          pq[t] = s0 + s1;
        }
        wave_sync();
        double yi = 0.0;
        if (t < n) {
          yi = y[t * kLd + c];
          for (int k0 = st; k0 < c; k0 += 8) {
            double pv[8], yv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int k = k0 + u < c ? k0 + u : c - 1;
              pv[u] = k0 + u < c ? pq[k] : 0.0;
              yv[u] = y[t * kLd + k];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) yi = fma(-pv[u], yv[u], yi);
          }
        }
        const double nrm = sqrt(wave_total(yi * yi));
        if (t < n) y[t * kLd + c] = nrm > 0 ? yi / nrm : 0.0;
        wave_sync();
        if (nrm > 0.5) break;
      }
    }
  }
  }  // wave 0
  __syncthreads();
  // 4. s = P_{n-1} ... P_2 y
  {
    int G = 16;
    while (G > 4 && G * nvec > 256) G >>= 1;
    switch (G) {
      case 16: apply_reflectors<16>(a, rh, y, n, nvec, lamv, tnorm, theta, Sout, lds); break;
      case 8: apply_reflectors<8>(a, rh, y, n, nvec, lamv, tnorm, theta, Sout, lds); break;
      default: apply_reflectors<4>(a, rh, y, n, nvec, lamv, tnorm, theta, Sout, lds); break;
    }
    if (threadIdx.x == 0 && other_end && nvec < n) theta[n - 1] = lamv[nvec] * tnorm;
  }
}

void syev_rr(const double *H, int ldh, int p, int nvec, bool descending, double *theta,
             double *S, int lds, hipStream_t s, bool other_end) {
  PHS_REQUIRE(p >= 1 && p <= kSmallMax && nvec >= 1 && nvec <= p, kEinval,
              "syev: size out of range");
  k_syev<<<1, 256, 0, s>>>(H, ldh, p, nvec, descending, other_end, theta, S, lds);
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
  // eight loads in flight per thread before their stores
  for (int idx0 = t; idx0 < P * kSvdRows; idx0 += 8 * blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = idx0 + u * blockDim.x, i = idx % kSvdRows, j = idx / kSvdRows;
      v[u] = (idx < P * kSvdRows && i < rows && j < cols) ? M[i + (int64_t)j * ldm] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = idx0 + u * blockDim.x;
      if (idx < P * kSvdRows) g[idx] = v[u];
    }
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
                                                  double *Rg, double *Ri, int ldr, int *flag,
                                                  CgsDiag dg, const double *part, int np) {
  __shared__ double r[kSmallMax * kLd];   // r[i * kLd + j], upper triangle used
  __shared__ double ri[kSmallMax * kLd];  // R^{-1}, same layout
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  if (part) {
    // G from the block partials of X^T X (entry i * w + j of each block):
    // groups of tpe lanes per entry, fixed summation order
    const int E = w * w;
    int tpe = 1;
    while (tpe * 2 * E <= 256 && tpe < 64) tpe *= 2;
    const int grp = t / tpe, sub = t % tpe, ngrp = 256 / tpe;
    for (int e0 = 0; e0 < E; e0 += ngrp) {
      const int e = e0 + grp;
      // sixteen partials per lane in flight at a time (the padding past np
      // rereads the last partial with weight 0)
      double sv = 0.0;
      if (e < E) {
        for (int b0 = sub; b0 < np; b0 += 16 * tpe) {
          double pv[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int b = b0 + u * tpe;
            pv[u] = part[(int64_t)(b < np ? b : np - 1) * E + e];
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) sv += b0 + u * tpe < np ? pv[u] : 0.0;
        }
      }
      for (int o = tpe / 2; o > 0; o >>= 1) sv += __shfl_xor(sv, o, tpe);
      if (sub == 0 && e < E) r[(e / w) * kLd + e % w] = sv;
    }
    __syncthreads();
  }
  // G(i, j): from the partials (in r) or from global memory
  auto gij = [&](int i, int j) { return part ? r[i * kLd + j] : G[i + (int64_t)j * ldg]; };
  if (dg.n2 && t < w) {
    // squared column norms around two Gram-Schmidt passes from the final
    // Gram matrix and the two coefficient blocks
    double h1 = 0.0, h2 = 0.0;
    for (int i0 = 0; i0 < dg.nh; i0 += 16) {
      double c1[16], c2[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t i = i0 + u < dg.nh ? i0 + u : dg.nh - 1;
        c1[u] = dg.H1[i + (int64_t)t * dg.ldh];
        c2[u] = dg.H2[i + (int64_t)t * dg.ldh];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double m = i0 + u < dg.nh ? 1.0 : 0.0;
        h1 = fma(m * c1[u], c1[u], h1);
        h2 = fma(m * c2[u], c2[u], h2);
      }
    }
    const double a2 = gij(t, t);
    dg.n2[t] = a2;
    dg.n1[t] = a2 + h2;
    dg.n0[t] = a2 + h2 + h1;
  }
  if (part) {
    // symmetrise in place: pairs (i < j) by one thread each
    for (int idx = t; idx < w * w; idx += blockDim.x) {
      int i = idx % w, j = idx / w;
      if (i < j) {
        const double v = 0.5 * (r[i * kLd + j] + r[j * kLd + i]);
        r[i * kLd + j] = v;
        r[j * kLd + i] = v;
      } else if (i == j) {
        r[i * kLd + i] += shift;
      }
    }
  } else {
    for (int idx = t; idx < w * w; idx += blockDim.x) {
      int i = idx % w, j = idx / w;
      r[i * kLd + j] = 0.5 * (G[i + (int64_t)j * ldg] + G[j + (int64_t)i * ldg]) +
                       (i == j ? shift : 0.0);
    }
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
  // Rinv column by column in LDS (thread per column, back substitution),
  // then R and Rinv to global memory
  for (int j = t; j < w; j += blockDim.x) {
    // solve R x = e_j; x_i = 0 for i > j
    for (int i = w - 1; i >= 0; --i) {
      double x = 0.0;
      if (i <= j) {
        double sacc = (i == j) ? 1.0 : 0.0;
        for (int q = i + 1; q <= j; ++q) sacc -= r[i * kLd + q] * ri[q * kLd + j];
        x = sacc / r[i * kLd + i];
      }
      ri[i * kLd + j] = x;
    }
  }
  __syncthreads();
  for (int idx = t; idx < w * w; idx += blockDim.x) {
    int i = idx % w, j = idx / w;
    Rg[i + (int64_t)j * ldr] = (j >= i) ? r[i * kLd + j] : 0.0;
    Ri[i + (int64_t)j * ldr] = ri[i * kLd + j];
  }
  if (t == 0) flag[0] = bad;
}

void chol_inv(const double *G, int ldg, int w, double shift, double *R, double *Rinv, int ldr,
              int *flag, hipStream_t s, const CgsDiag *dg, const TnParts *pt) {
  PHS_REQUIRE(!pt || (pt->nx == w && pt->ny == w && pt->np >= 1), kEinval,
              "chol_inv: partials do not match");
  PHS_REQUIRE(w >= 1 && w <= kSmallMax, kEinval, "chol_inv: size out of range");
  PHS_REQUIRE(!dg || (dg->nh >= 0 && dg->ldh >= dg->nh), kEinval,
              "chol_inv: bad diagnostics operands");
  k_chol_inv<<<1, 256, 0, s>>>(G, ldg, w, shift, R, Rinv, ldr, flag, dg ? *dg : CgsDiag{},
                               pt ? pt->part : nullptr, pt ? pt->np : 0);
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
#pragma unroll 8
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

// Projection of the Rayleigh-Ritz matrix onto a restart basis, one launch:
// H <- Y^T (H Y) (H p x p in, hc x hc out, Y p x hc) and, if S is given,
// Q = Y^T S (hc x ns).  Same arithmetic as the two or three small_gemm
// calls it replaces (each entry one fma chain in index order).
__global__ __launch_bounds__(256) void k_restart_project(double *H, int ldh, int p,
                                                         const double *Y, int ldy, int hc,
                                                         const double *S, int lds, int ns,
                                                         double *Q, int ldq) {
  __shared__ double h[kSmallMax * kLd], y[kSmallMax * kLd], hy[kSmallMax * kLd];
  const int t = threadIdx.x;
  for (int e = t; e < p * p; e += 256) h[(e % p) + (e / p) * kLd] = H[e % p + (int64_t)(e / p) * ldh];
  for (int e = t; e < p * hc; e += 256)
    y[(e % p) + (e / p) * kLd] = Y[e % p + (int64_t)(e / p) * ldy];
  __syncthreads();
  // HY = H Y
  for (int e = t; e < p * hc; e += 256) {
    const int i = e % p, j = e / p;
    double acc = 0.0;
    for (int k = 0; k < p; ++k) acc = fma(h[i + k * kLd], y[k + j * kLd], acc);
    hy[i + j * kLd] = acc;
  }
  __syncthreads();
  // H = Y^T (H Y); Q = Y^T S
  for (int e = t; e < hc * hc; e += 256) {
    const int i = e % hc, j = e / hc;
    double acc = 0.0;
    for (int k = 0; k < p; ++k) acc = fma(y[k + i * kLd], hy[k + j * kLd], acc);
    H[i + (int64_t)j * ldh] = acc;
  }
  if (S) {
    for (int e = t; e < hc * ns; e += 256) {
      const int i = e % hc, j = e / hc;
      double acc = 0.0;
      for (int k = 0; k < p; ++k) acc = fma(y[k + i * kLd], S[k + (int64_t)j * lds], acc);
      Q[i + (int64_t)j * ldq] = acc;
    }
  }
}

void restart_project(double *H, int ldh, int p, const double *Y, int ldy, int hc,
                     const double *S, int lds, int ns, double *Q, int ldq, hipStream_t s) {
  PHS_REQUIRE(p >= 1 && p <= kSmallMax && hc >= 0 && hc <= p && (!S || (ns >= 0 && Q)),
              kEinval, "restart_project: size out of range");
  if (hc == 0) return;
  k_restart_project<<<1, 256, 0, s>>>(H, ldh, p, Y, ldy, hc, S, lds, ns, Q, ldq);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------ MGS2 helpers (restart, QR)
// Single-wavefront Gram-Schmidt helpers for small coefficient spaces
// (rows <= 64): lane r owns row r of every column, dot products are wave
// reductions, so no workgroup barriers are needed.

// Orthogonalise column c of q (ld kLd, lane r owns row r for the update)
// against columns [0, c), twice.  The c dot products of a pass are computed
// in parallel (lane j forms q_j^T x from LDS, rows eight at a time), then
// every lane updates its row; coefficients accumulate into rc if given.
// With reject > 0, a column whose norm after the first pass is at most
// reject * n0 is returned after that pass (n2 = that norm): the second pass
// could only shrink it further, and the caller discards such a column.
__device__ inline void wave_cgs2(double *q, int rows, int c, double *xs, double *dots, double *rc,
                                 double &n0, double &n2, double reject = 0.0) {
  const int r = threadIdx.x;
  double x = (r < rows) ? q[c * kLd + r] : 0.0;
  n0 = sqrt(wave_total(x * x));
  for (int pass = 0; pass < 2; ++pass) {
    xs[r] = x;  // zero past rows
    __syncthreads();
    if (r < c) {
      double d0 = 0.0, d1 = 0.0;
      for (int k0 = 0; k0 < rows; k0 += 8) {
        double qv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          qv[u] = q[r * kLd + k0 + u];  // rows past `rows` meet xs = 0
          xv[u] = xs[k0 + u];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          d0 = fma(qv[u], xv[u], d0);
          d1 = fma(qv[u + 1], xv[u + 1], d1);
        }
      }
      dots[r] = d0 + d1;
      if (rc) rc[r] += d0 + d1;
    }
    __syncthreads();
    // eight coefficients at a time, their loads in flight together; the
    // padding past c reads column c - 1 with coefficient 0
    double acc = x;
    for (int j0 = 0; j0 < c; j0 += 8) {
      double dv[8], qv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u < c ? j0 + u : c - 1;
        dv[u] = j0 + u < c ? dots[j] : 0.0;
        qv[u] = q[j * kLd + r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma(-dv[u], qv[u], acc);
    }
    x = (r < rows) ? acc : 0.0;
    if (pass == 0 && reject > 0.0) {
      const double n1 = sqrt(wave_total(x * x));
      if (!(n1 > reject * n0)) {
        q[c * kLd + r] = x;
        n2 = n1;
        __syncthreads();
        return;
      }
    }
  }
  q[c * kLd + r] = x;
  n2 = sqrt(wave_total(x * x));
  __syncthreads();
}

// Columns [0, nc) of a column-major global matrix into LDS (ld kLd), row r
// per lane: eight loads in flight before their stores.
__device__ inline void load_cols_lds(double *q, const double *src, int ld, int rows, int nc,
                                     int r) {
  for (int j0 = 0; j0 < nc; j0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (j0 + u < nc && r < rows) ? src[r + (int64_t)(j0 + u) * ld] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u < nc) q[(j0 + u) * kLd + r] = v[u];
  }
}

// Y = [K | orth(P against K)]; a dependent column of P is replaced by the
// next coordinate vector that is independent, so the count is always
// min(kc + pc, rows).
__global__ __launch_bounds__(64) void k_restart_basis(const double *K, int ldk, int rows, int kc,
                                                      const double *P, int ldp, int pc, double *Y,
                                                      int ldy, int *count) {
  __shared__ double q[kSmallMax * kLd + 8];  // column-major, ld kLd (no bank conflicts)
  __shared__ double xs[kSmallMax + 8], dots[kSmallMax];
  const int r = threadIdx.x;
  if (r < 8) xs[kSmallMax + r] = 0.0;
  // every column the kernel reads has its 64 rows written first; the reads
  // past them (row 64 of a column, and the tail of the array) meet zeros
  q[r * kLd + kSmallMax] = 0.0;
  if (r < 8) q[kSmallMax * kLd + r] = 0.0;
  __syncthreads();
  load_cols_lds(q, K, ldk, rows, kc, r);
  __syncthreads();
  int cur = kc, unit = 0;
  const int want = min(kc + pc, min(rows, kSmallMax));
  for (int c = 0; cur < want; ++c) {
    for (int attempt = 0; attempt < rows + 1; ++attempt) {
      double x;
      if (c < pc && attempt == 0) {
        x = r < rows ? P[r + (int64_t)c * ldp] : 0.0;
      } else {
        x = (r == unit) ? 1.0 : 0.0;
        ++unit;
      }
      q[cur * kLd + r] = x;
      __syncthreads();
      double n0, n2;
      wave_cgs2(q, rows, cur, xs, dots, nullptr, n0, n2, 1e-8);
      if (n0 > 0.0 && n2 > 1e-8 * n0) {
        q[cur * kLd + r] /= n2;
        ++cur;
        __syncthreads();
        break;
      }
    }
  }
  if (r < rows)
    for (int j = 0; j < cur; ++j) Y[r + (int64_t)j * ldy] = q[j * kLd + r];
  if (r == 0) count[0] = cur;
}

void restart_basis(const double *K, int ldk, int rows, int kc, const double *P, int ldp, int pc,
                   double *Y, int ldy, int *count, hipStream_t s) {
  PHS_REQUIRE(rows <= kSmallMax && kc <= kSmallMax, kEinval, "restart_basis: size out of range");
  k_restart_basis<<<1, 64, 0, s>>>(K, ldk, rows, kc, P, ldp, pc, Y, ldy, count);
  PHS_CHECK_LAUNCH();
}

__global__ __launch_bounds__(64) void k_small_qr(const double *M, int ldm, int rows, int cols,
                                                 double *Q, int ldq, double *R, int ldr) {
  __shared__ double q[kSmallMax * kLd + 8];  // column-major, ld kLd
  __shared__ double rc[kSmallMax], xs[kSmallMax + 8], dots[kSmallMax];
  const int r = threadIdx.x;
  if (r < 8) xs[kSmallMax + r] = 0.0;
  // the columns read are written first (64 rows each); row 64 of a column
  // and the tail of the array meet zeros
  q[r * kLd + kSmallMax] = 0.0;
  if (r < 8) q[kSmallMax * kLd + r] = 0.0;
  __syncthreads();
  load_cols_lds(q, M, ldm, rows, cols, r);
  for (int e = r; e < cols * cols; e += 64) R[e % cols + (int64_t)(e / cols) * ldr] = 0.0;
  for (int c = 0; c < cols; ++c) {
    rc[r] = 0.0;
    __syncthreads();
    double n0, n2;
    wave_cgs2(q, rows, c, xs, dots, rc, n0, n2);
    double inv = n2 > 0.0 ? 1.0 / n2 : 0.0;
    q[c * kLd + r] *= inv;
    if (r < c) R[r + (int64_t)c * ldr] = rc[r];
    if (r == 0) R[c + (int64_t)c * ldr] = n2;
  }
  if (r < rows)
    for (int j = 0; j < cols; ++j) Q[r + (int64_t)j * ldq] = q[j * kLd + r];
}

void small_qr(const double *M, int ldm, int rows, int cols, double *Q, int ldq, double *R,
              int ldr, hipStream_t s) {
  PHS_REQUIRE(rows <= kSmallMax && cols <= rows, kEinval, "small_qr: size out of range");
  k_small_qr<<<1, 64, 0, s>>>(M, ldm, rows, cols, Q, ldq, R, ldr);
  PHS_CHECK_LAUNCH();
}

// ------------------------------------------------------------ misc
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

// Inverse of an upper-triangular R (p x p, p <= 64) by back substitution,
// one column per thread; diagonal entries below 1e-14 max|R_jj| in size are
// raised to that size (keeping their sign) so a nearly singular R gives a
// large but finite inverse.
__global__ __launch_bounds__(64) void k_tri_inv(const double *R, int ldr, int p, double *Ri,
                                                 int ldri) {
  __shared__ double dmax;
  const int j = threadIdx.x;
  if (j == 0) {
    double mx = 0.0;
    for (int i = 0; i < p; ++i) mx = fmax(mx, fabs(R[i + (int64_t)i * ldr]));
    dmax = mx;
  }
  __syncthreads();
  if (j >= p) return;
  const double fl = 1e-14 * dmax;
  auto diag = [&](int i) {
    double d = R[i + (int64_t)i * ldr];
    if (fabs(d) < fl) d = d < 0.0 ? -fl : fl;
    return d;
  };
  double *x = Ri + (int64_t)j * ldri;
  for (int i = p - 1; i >= 0; --i) {
    if (i > j) {
      x[i] = 0.0;
      continue;
    }
    double sacc = (i == j) ? 1.0 : 0.0;
    for (int l = i + 1; l <= j; ++l) sacc -= R[i + (int64_t)l * ldr] * x[l];
    x[i] = dmax > 0.0 ? sacc / diag(i) : 0.0;
  }
}

void tri_inv(const double *R, int ldr, int p, double *Ri, int ldri, hipStream_t s) {
  PHS_REQUIRE(p >= 1 && p <= kSmallMax, kEinval, "tri_inv: size out of range");
  k_tri_inv<<<1, 64, 0, s>>>(R, ldr, p, Ri, ldri);
  PHS_CHECK_LAUNCH();
}

// Columns 0..nc-1 of Y (p rows) scaled to unit 2-norm (zero columns stay).
__global__ void k_normalize_small(double *Y, int ldy, int p, int nc) {
  __shared__ double red[256];
  for (int c = 0; c < nc; ++c) {
    double sacc = 0.0;
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      const double v = Y[i + (int64_t)c * ldy];
      sacc += v * v;
    }
    const double tot = block_sum(sacc, red);
    const double f = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
    for (int i = threadIdx.x; i < p; i += blockDim.x) Y[i + (int64_t)c * ldy] *= (tot > 0.0 ? f : 1.0);
    __syncthreads();
  }
}

void normalize_small(double *Y, int ldy, int p, int nc, hipStream_t s) {
  if (nc <= 0 || p <= 0) return;
  k_normalize_small<<<1, 256, 0, s>>>(Y, ldy, p, nc);
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
