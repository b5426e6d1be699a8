// Host-side launchers of the PHSVDS device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

namespace phs {

// ------------------------------------------------------------------ sparse
struct Bin {
  int32_t offset, count, lanes;
};

// The caller's operator in place of a CSR (Section 3.3: products with A
// and A^T given as functions): Y = op(A) X for row-major blocks of width b,
// X n x b and Y m x b for A (trans false), the other way round for A^T.
struct OpHook {
  std::function<void(const void *X, void *Y, int b, bool trans, bool fp64)> f;
};

// CSR matrix on the device in working precision T, or the caller's
// operator (op set: only m, n and op_trans are meaningful).
template <typename T>
struct SpMat {
  int64_t m = 0, n = 0, nnz = 0;
  const int64_t *rowptr = nullptr;
  const int32_t *colind = nullptr;
  const T *val = nullptr;
  int nbins = 0;  // 0: one launch over all rows
  Bin bins[8];
  const int32_t *binrows = nullptr;
  // binned products write the result of row binrows[q] to row q (the row
  // space of the result is in bin order)
  bool slot_out = false;
  const OpHook *op = nullptr;
  bool op_trans = false;  // this SpMat is A^T of the operator
};

int lanes_for_length(double avg);
template <typename T>
void spmm(const SpMat<T> &A, int b, const T *X, T *Y, bool absval, hipStream_t s,
          int64_t ycm = 0, int ycols = 0);
// The same product without the profiling hooks (which record events).
template <typename T>
void spmm_untimed(const SpMat<T> &A, int b, const T *X, T *Y, hipStream_t s);
// Algorithmic HBM bytes of one Y = A X at block width b: values and column
// indices once, row pointers once, X once, Y once (the count spmm records
// for each launch it times).
template <typename T>
inline double spmm_bytes(const SpMat<T> &A, int b) {
  return (double)A.nnz * (sizeof(T) + 4) + (double)(A.m + 1) * 8 +
         (double)A.n * b * sizeof(T) + (double)A.m * b * sizeof(T);
}
size_t transpose_ws_bytes(int64_t m, int64_t n, int64_t nnz);
// Y = op(A) X for a caller CSR (the C ABI's product): op = A, or A^T built
// into ws (spmm_t_ws_bytes bytes) on every call.
size_t spmm_t_ws_bytes(int64_t m, int64_t n, int64_t nnz, bool fp32);
void csr_transpose(int64_t m, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci,
                   const double *va, int64_t *trp, int32_t *tci, double *tva, void *ws,
                   size_t ws_bytes, hipStream_t s);
// Row-length bins: rows lists the rows of each bin in ascending order, the
// bins one after another (bin_ws_bytes(m) bytes of scratch).
size_t bin_ws_bytes(int64_t m);
void build_bins(int64_t m, const int64_t *rp, int32_t *rows, void *ws, size_t ws_bytes, Bin *bins,
                int *nbins, hipStream_t s);
// Row space in bin order: inv = rows^-1, and the column indices of A^T
// (rows of A) renumbered through it, so that products A X written by slot
// (SpMat::slot_out) feed A^T directly.
void permute_row_space(int64_t m, int64_t nnz, const int32_t *rows, int32_t *inv, int32_t *tci,
                       hipStream_t s);
// dst[rows[q], j] = src[q, j] for w columns of length m (ld m).
void unpermute_rows(int64_t m, int w, const int32_t *rows, const double *src, double *dst,
                    hipStream_t s);

// ------------------------------------------------------------- tall blocks
// A tall matrix view: element (i, j) at p[i * rs + j * cs].  Column-major
// storage has rs = 1, cs = ld; a row-major block of width w has rs = w, cs = 1.
template <typename T>
struct Tall {
  T *p = nullptr;
  int64_t rows = 0;
  int cols = 0;
  int64_t rs = 1, cs = 0;
  T *col(int j) const { return p + (int64_t)j * cs; }
};
template <typename T>
inline Tall<T> cm(T *p, int64_t rows, int cols, int64_t ld) {
  Tall<T> t;
  t.p = p;
  t.rows = rows;
  t.cols = cols;
  t.rs = 1;
  t.cs = ld;
  return t;
}
template <typename T>
inline Tall<T> rm(T *p, int64_t rows, int cols) {
  Tall<T> t;
  t.p = p;
  t.rows = rows;
  t.cols = cols;
  t.rs = cols;
  t.cs = 1;
  return t;
}

// Reduction scratch for the tall-skinny products.
struct Scratch {
  double *part = nullptr;  // partial sums, kPartCap doubles
  double *aux = nullptr;   // small results, kAuxCap doubles
  int *flag = nullptr;     // status flags (64 ints)
};
constexpr int64_t kPartCap = 1 << 21;
// Leading dimension of the first stage's bases (V, W): n rounded up to 64
// elements, so that every column starts on a 256-byte boundary and the
// tall-skinny kernels move whole cache lines whatever n is.
inline int64_t basis_ld(int64_t n) { return (n + 63) / 64 * 64; }
constexpr int64_t kAuxCap = 1 << 16;

// Block partials of a product X^T Y left for a consumer kernel to reduce:
// np blocks of nx * ny doubles, entry (i, j) at offset i * ny + j.
struct TnParts {
  const double *part = nullptr;
  int np = 0, nx = 0, ny = 0;
};
// G (nx x ny, ld ldg, float64) = X^T Y, X = [X1 | X2] (X2 may have 0 cols).
// With keep, the final reduction is left to the consumer: G is not written
// and keep describes the partials (valid until the next use of sc.part).
template <typename T>
void tn(const Tall<T> &X1, const Tall<T> &X2, const Tall<T> &Y, double *G, int ldg,
        const Scratch &sc, hipStream_t s, TnParts *keep = nullptr);
// The border of H from the partials of G = V^T W_new ((p + nb) x nb, kept by
// tn): H(0:p+nb, p:p+nb) = G, H(p:p+nb, 0:p) = G(0:p)^T, the new diagonal
// block symmetrised; with Z given, rows p..p+nb-1 of Z (nz columns) are
// zeroed in the same launch (reduction and border copy in one kernel).
void reduce_border(const TnParts &pt, double *H, int ldh, double *Z, int ldz, int nz,
                   hipStream_t s);
// Y = alpha * [X1 | X2] S + beta * Z, S float64 (nx x ny, ld lds); Z is Y
// itself unless given.  If Y2 is given the result is written there too.
// With gram (and gsc), the launch also leaves the block partials of the Gram
// matrix Y^T Y (float64, ny of 1, 2 or 4) in gsc->part and describes them in
// *gram, as tn does with keep.
template <typename T>
void nn(const Tall<T> &X1, const Tall<T> &X2, const double *S, int lds, double alpha,
        const Tall<T> &Y, double beta, hipStream_t s, const Tall<T> *Z = nullptr,
        const Tall<T> *Y2 = nullptr, const Scratch *gsc = nullptr, TnParts *gram = nullptr);
// Ritz block: X = V S, R = W S - X diag(theta) (row-major outputs, row stride ldx),
// rn2[j] = ||R_:,j||^2; if ntop > 0 also xt2[j] = ||X_{0:ntop, j}||^2.
template <typename T>
void ritz(const Tall<T> &V, const Tall<T> &W, const double *S, int lds, const double *theta,
          T *X, T *R, int nb, int ldx, double *rn2, double *xt2, int64_t ntop,
          const Scratch &sc, hipStream_t s);
// out[j] = sum_i X(i, j)^2 over rows [r0, r1) (float64 result, device).
template <typename T>
void colnorm2(const Tall<T> &X, int64_t r0, int64_t r1, double *out, const Scratch &sc,
              hipStream_t s);
// dst = src elementwise (any layouts, same shape), with type conversion.
template <typename Ti, typename To>
void copy(const Tall<Ti> &src, const Tall<To> &dst, hipStream_t s);
// X(:, j) *= f[j] (f on device).
template <typename T>
void scale_cols(const Tall<T> &X, const double *f, hipStream_t s);
// Y = X - shift * Z (same shapes).
template <typename T>
void axpby(const Tall<T> &X, const Tall<T> &Z, double shift, const Tall<T> &Y, hipStream_t s);
// Column j of X := counter-based uniform(-0.5, 0.5) stream (seed, stream_id + j).
template <typename T>
void fill_random(const Tall<T> &X, uint64_t seed, uint64_t stream_id, hipStream_t s);
// Jacobi: T = (d - theta_j)^-1 R, Olsen form if olsen (X = Ritz block).
template <typename T>
void jacobi_apply(const T *R, const T *X, const double *d, const double *theta, int64_t n,
                  int nb, int ldx, bool olsen, T *Tout, const Scratch &sc, hipStream_t s);
// d[j] = ||A_:,j||^2 from the CSR of A^T (row j of A^T is column j of A).
void col_sq_norms(const SpMat<double> &At, double *d, hipStream_t s);
// element-wise multiply rows: Y(i, :) = X(i, :) * w[i] (or / w[i] if inv).
template <typename T>
void row_scale(const T *X, const double *w, int64_t n, int b, bool inv, T *Y, hipStream_t s);

// -------------------------------------------------- small dense (float64)
// Selected eigenpairs of the symmetric H (p x p, ld ldh, p <= 64; one
// workgroup): the nvec at the wanted end (ascending, or descending if
// `descending`) in theta[0..nvec), S(:, 0..nvec) (ld lds), and, if
// other_end, the eigenvalue at the other end in theta[p-1] (without it the
// multisection has one group fewer to run).  H is not modified.
void syev_rr(const double *H, int ldh, int p, int nvec, bool descending, double *theta,
             double *S, int lds, hipStream_t s, bool other_end = true);
// One-sided Jacobi SVD of M (rows x cols, ld ldm, rows >= cols): singular
// values ascending in sv, right vectors in Y (cols x cols, ld ldy).
void svdj(const double *M, int ldm, int rows, int cols, double *sv, double *Y, int ldy,
          hipStream_t s);
// Cholesky G + shift I = R^T R (w x w) and Rinv = R^-1 (upper triangular,
// ld ldr).  flag[0] = 1 on breakdown (non-positive pivot).
// Optional diagnostics of a block after two classical Gram-Schmidt passes
// T1 = T0 - Q H1, T2 = T1 - Q H2 against an orthonormal Q (nh columns) when
// G = T2^T T2: n2 = diag(G), n1 = n2 + colsum(H2^2), n0 = n1 + colsum(H1^2)
// (the squared column norms of T2, T1 and T0).
struct CgsDiag {
  const double *H1 = nullptr, *H2 = nullptr;
  int ldh = 0, nh = 0;
  double *n0 = nullptr, *n1 = nullptr, *n2 = nullptr;
};
// With pt, G is the reduction of the partials pt (X^T X) and the G argument
// is not read.
void chol_inv(const double *G, int ldg, int w, double shift, double *R, double *Rinv, int ldr,
              int *flag, hipStream_t s, const CgsDiag *dg = nullptr,
              const TnParts *pt = nullptr);
// C = alpha op(A) op(B) + beta C, all small float64.
void small_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
                const double *B, int ldb, double beta, double *C, int ldc, hipStream_t s);
// Y = [K | orth(P against K)] (rows x min(kc + pc, rows)); a dependent
// column of P is replaced by an independent coordinate vector, so
// count[0] = min(kc + pc, rows) always.
void restart_basis(const double *K, int ldk, int rows, int kc, const double *P, int ldp, int pc,
                   double *Y, int ldy, int *count, hipStream_t s);
// H <- Y^T H Y (p x p -> hc x hc) and, with S given, Q = Y^T S (hc x ns),
// in one launch (the restart projection of the Rayleigh-Ritz matrix).
void restart_project(double *H, int ldh, int p, const double *Y, int ldy, int hc,
                     const double *S, int lds, int ns, double *Q, int ldq, hipStream_t s);
// Thin QR by two-pass modified Gram-Schmidt: M (rows x cols) = Q R.
void small_qr(const double *M, int ldm, int rows, int cols, double *Q, int ldq, double *R,
              int ldr, hipStream_t s);
// Copy columns idx[0..nc) of A (rows x *) into B; idx on device.
void gather_cols(const double *A, int lda, int rows, const int *idx, int nc, double *B, int ldb,
                 hipStream_t s);
// H = diag(d[idx[0..nc)]).
void set_diag(double *H, int ldh, int nc, const double *d, const int *idx, hipStream_t s);
// Zero rows [r0, r1) of a small matrix with nc columns.
void zero_rows(double *A, int lda, int r0, int r1, int nc, hipStream_t s);
// theta[j] = y_j^T H y_j for columns of Y (p x nc).
void rayleigh_small(const double *H, int ldh, int p, const double *Y, int ldy, int nc,
                    double *theta, hipStream_t s);

// Ri = R^-1 for upper-triangular R (p x p, p <= 64); diagonal entries below
// 1e-14 max|R_jj| are raised to that size (sign kept).
void tri_inv(const double *R, int ldr, int p, double *Ri, int ldri, hipStream_t s);
// Scale columns 0..nc-1 of Y (p rows) to unit 2-norm (zero columns stay).
void normalize_small(double *Y, int ldy, int p, int nc, hipStream_t s);

// B += alpha A (small).
void small_add(int M, int N, double alpha, const double *A, int lda, double *B, int ldb,
               hipStream_t s);
// Normalise a column from its squared norm on the device (zero if tiny).
template <typename T>
void norm_col(T *x, int64_t rows, const double *n2, double tiny, double *Rjj, hipStream_t s);
// p[i * rs] = v for i < rows.
template <typename T>
void fill_const_col(T *p, int64_t rows, int64_t rs, double v, hipStream_t s);

}  // namespace phs
