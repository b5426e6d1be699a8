// Learned preconditioner (message-passing network) on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/phsvds.h"
#include "common.hpp"
#include "kernels.hpp"

namespace phs {

constexpr int kGnnIn = 4;     // node input features
constexpr int kGnnMaxW = 32;  // largest hidden width

struct GnnOffsets {
  int64_t Ws[3], Wm[3], b[3], wo, total;
};

// Per-matrix device data: CSR of A^T, float32 values, diag(C) normalised
// and D^-1/2, mean(diag C) in meta[0].
struct GnnGraph {
  int64_t *trp;
  int32_t *tci;
  double *tva;
  char *tws;
  size_t tws_bytes;
  float *va32, *tva32, *dn, *isd;
  double *d64, *meta;
};

struct GnnBufs {
  float *h0, *pre[3], *h[3], *S, *M, *Z, *Ym, *delta, *dh, *traw, *g, *tout, *rf, *xf;
  double *vec, *G;
  Scratch sc;
};

int64_t gnn_nweights(int w, int nin = kGnnIn);
GnnOffsets gnn_offsets(int w, int nin = kGnnIn);
void gnn_carve(Arena &ar, int64_t m, int64_t n, int64_t nnz, int w, GnnGraph &g, GnnBufs &b);
void gnn_prepare(const phsvds_csr &A, GnnGraph &g, hipStream_t s);
void gnn_forward(const phsvds_csr &A, const GnnGraph &g, GnnBufs &b, const float *wts, int w,
                 const float *r, const float *x, double theta, float *t, hipStream_t s);
void gnn_loss_grad(const phsvds_csr &A, const GnnGraph &g, GnnBufs &b, const float *wts, int w,
                   const float *r, const float *x, double theta, const float *tstar, float *t,
                   double *grad, double *loss_dev, hipStream_t s, int kind = 0);
void gnn_adam(float *w, float *m, float *v, const double *g, int64_t nw, int step, double lr,
              double gscale, hipStream_t s);
void gnn_scale_acc(const double *G, int ldg, int w, const double *nr2, const double *meta,
                   int64_t n, double *gout, hipStream_t s);
void gnn_loss_acc(const double *g2, const double *ts2, double *loss, hipStream_t s);
void colsum_acc(const Tall<float> &X, double *out, const Scratch &sc, hipStream_t s);

}  // namespace phs
