// Pieces shared by the H*v kernels (kernels.hip, stream.hip): per-lane complex
// accumulators, the launch parameters, streaming loads and stores, and the fused
// Lanczos epilogue with its per-block partial sums.
#pragma once

#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "ftlm_internal.hpp"

namespace ftlm {

// ------------------------------------------------------------------ helpers
template <typename R, int KC>
struct Acc {
  R re[KC];
  R im[KC];
};

template <typename R, int KC>
__device__ __forceinline__ void acc_zero(Acc<R, KC> &a) {
#pragma unroll
  for (int q = 0; q < KC; q++) a.re[q] = a.im[q] = R(0);
}

// a += c * x[0..KC)
template <typename R, int KC>
__device__ __forceinline__ void mac(Acc<R, KC> &a, Cx<R> c, const Cx<R> *__restrict__ x) {
  Cx<R> xv[KC];
#pragma unroll
  for (int q = 0; q < KC; q++) xv[q] = x[q];
#pragma unroll
  for (int q = 0; q < KC; q++) {
    a.re[q] = fma(c.re, xv[q].re, a.re[q]);
    a.re[q] = fma(-c.im, xv[q].im, a.re[q]);
    a.im[q] = fma(c.re, xv[q].im, a.im[q]);
    a.im[q] = fma(c.im, xv[q].re, a.im[q]);
  }
}

template <typename R, int KC>
__device__ __forceinline__ void mac_real(Acc<R, KC> &a, R c, const Cx<R> *__restrict__ x) {
#pragma unroll
  for (int q = 0; q < KC; q++) {
    Cx<R> xv = x[q];
    a.re[q] = fma(c, xv.re, a.re[q]);
    a.im[q] = fma(c, xv.im, a.im[q]);
  }
}

// ------------------------------------------------------------------ H*v
struct HvParams {
  int K;             // row stride in columns
  uint32_t ntile;    // number of 256-row tiles
  const void *v;
  void *w;
  const double *scale;  // per-column scale of v (or nullptr)
  // Lanczos epilogue
  int lanczos;
  const void *xprev;
  const void *ov1;
  const double *sx_prev;
  const double *beta_prev;
  double *part;
  unsigned *counter;
  double *alpha_out, *yre_out, *yim_out;
};

// Streaming (non-temporal) loads and stores for vectors touched once per pass
// (partial sums of w, the Lanczos epilogue's operands): keeping them out of L2
// leaves it to the window's v tiles that the outer pairs gather.
template <typename R>
using V2 = R __attribute__((ext_vector_type(2)));

template <typename R>
__device__ __forceinline__ Cx<R> ld_stream(const Cx<R> *p) {
  const V2<R> v = __builtin_nontemporal_load(reinterpret_cast<const V2<R> *>(p));
  return Cx<R>{v.x, v.y};
}

template <typename R>
__device__ __forceinline__ void st_stream(Cx<R> *p, const Cx<R> &x) {
  V2<R> v;
  v.x = x.re;
  v.y = x.im;
  __builtin_nontemporal_store(v, reinterpret_cast<V2<R> *>(p));
}

template <typename R, int KC, bool STREAM = false>
__device__ __forceinline__ void hv_epilogue(const HvParams &P, uint32_t row, int c0,
                                            const Acc<R, KC> &acc, const Cx<R> *own,
                                            double (&red)[3][KC]) {
  Cx<R> *w = reinterpret_cast<Cx<R> *>(P.w) + (size_t)row * P.K + c0;
  if (!P.lanczos) {
#pragma unroll
    for (int q = 0; q < KC; q++) {
      R sc = P.scale ? (R)P.scale[c0 + q] : R(1);
      w[q] = Cx<R>{acc.re[q] * sc, acc.im[q] * sc};
    }
    return;
  }
  const Cx<R> *xp = P.xprev ? reinterpret_cast<const Cx<R> *>(P.xprev) + (size_t)row * P.K + c0 : nullptr;
  const Cx<R> *o1 = P.ov1 ? reinterpret_cast<const Cx<R> *>(P.ov1) + (size_t)row * P.K + c0 : nullptr;
#pragma unroll
  for (int q = 0; q < KC; q++) {
    const double sx = P.scale[c0 + q];
    double wr = (double)acc.re[q] * sx, wi = (double)acc.im[q] * sx;
    if (xp) {
      const double bp = P.beta_prev[c0 + q] * P.sx_prev[c0 + q];
      Cx<R> a = STREAM ? ld_stream(xp + q) : xp[q];
      wr -= bp * (double)a.re;
      wi -= bp * (double)a.im;
    }
    Cx<R> out{(R)wr, (R)wi};
    if (STREAM) st_stream(w + q, out);
    else w[q] = out;
    Cx<R> xo = own[q];
    // alpha partial uses the stored (rounded) w so that the update sees the same numbers
    red[0][q] += (double)xo.re * (double)out.re + (double)xo.im * (double)out.im;
    if (o1) {
      Cx<R> ov = STREAM ? ld_stream(o1 + q) : o1[q];
      red[1][q] += (double)ov.re * (double)xo.re + (double)ov.im * (double)xo.im;
      red[2][q] += (double)ov.re * (double)xo.im - (double)ov.im * (double)xo.re;
    }
  }
}

template <int KC, int NT = kBlock>
__device__ __forceinline__ void hv_finish(const HvParams &P, double (&red)[3][KC]) {
  if (!P.lanczos) return;
  block_partials_store<3, KC, NT>(red, P.part, blockIdx.y * gridDim.x + blockIdx.x);
}

}  // namespace ftlm
