// Network internals shared by net.cpp and the solver (capi.cpp).
#pragma once

#include "net.h"

#define HELM_NET_LAYERS 8

struct NetLayer {
  int cin, cout, relu;
  int cin_pad, cout_pad, kpad;  // forward implicit GEMM
  int cob, kbpad;               // backward-data implicit GEMM (input channels, K)
  float *w, *b, *dw, *db, *mw, *vw, *mb, *vb;
  unsigned char* mask;  // 1 for real (non-padding) weights
  bf16 *wt, *wb;
};

struct helm_net;
struct NetSolveBufs;

int net_dim(const helm_net* n);  // 2 or 3  // activation buffers of one solver context's network applications

// Buffers for network applications on up to B solver-grid images of ngrid^dim points,
// owned by the solver context that reserves them (one network may serve several contexts
// of different sizes); freed by net_bufs_destroy.
NetSolveBufs* net_bufs_create(helm_net* n, int B, int ngrid);
void net_bufs_destroy(NetSolveBufs* b);
// Preconditioner application on B <= the reserved count of images (ngrid^dim): features
// from the basis vectors v (scaled by vscale and in_gain) and the coefficient contrast,
// z = out_gain * network output for the right-hand sides in `mask`.  Returns
// hipErrorInvalidValue (and launches nothing) when B or ngrid do not fit the buffers.
hipError_t net_apply(helm_net* n, NetSolveBufs* bufs, hipStream_t s, int B, int ngrid, const c32* v, long long v_stride,
               const float* vscale, int vs_stride, float in_gain, const c32* coef, c32 cb, float out_gain, c32* z,
               long long z_stride, const int* mask);
