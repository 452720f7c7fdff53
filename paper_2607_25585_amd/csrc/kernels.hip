// HIP kernels (gfx950) of the FTLM hot path.
//
//  * hv_half / hv_gen : matrix-free w = H v on the product basis (Sec. 2.1),
//    gather form, one row per lane and KC column vectors per lane, optional
//    fused Lanczos epilogue (w -= beta_{j-1} v_{j-1}; alpha_j and y_j partials).
//  * gaussian / copy_start : start vectors of Eqs. (E-1-1), (E-1-2) and their norms.
//  * update : u = w - alpha_j v_j, beta_j = |u| (Lanczos recursion of Sec. 2.3).
//  * tridiag : Krylov eigenpairs by implicit QL (Bowdler, Martin, Reinsch and
//    Wilkinson, Numer. Math. 11 (1968)) tracking two rows of the eigenvector
//    matrix.
//  * boltzmann : the sums of Eqs. (E-2-C) and (E-2-D) in log-sum-exp form.
//
// Every reduction is a fixed-order tree (wave shuffles, LDS, then one block that
// sums the per-block partials in block order), so results are bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "device_reduce.hpp"
#include "ftlm_internal.hpp"
#include "hv_common.hpp"

namespace ftlm {

// Table pointers passed separately as __restrict__ kernel arguments (reads at
// wave-uniform addresses then use the scalar data cache).
template <typename R>
struct UniformTabs {
  const Cx<R> *pc, *czp, *czm;
  const int2 *pij;
  const R *pzz;
};

template <typename R>
static inline UniformTabs<R> uniform_tabs(const DevTables<R> &tb, bool half) {
  return UniformTabs<R>{half ? tb.pc_half : tb.pc, tb.czp, tb.czm, tb.pij, tb.pzz};
}

// alpha_j and y_j of every column from the H*v kernel's per-block partials
// (layout [cb][bx][3][KC], gx blocks along x): one block per (column,
// quantity), each summing its partials in block order, so the sums are those
// of one block taking them in turn but the columns do not wait on each other.
template <int KC>
__global__ __launch_bounds__(kBlock) void hv_lanczos_finish(HvParams P, unsigned gx) {
  const int c = blockIdx.x / 3, a = blockIdx.x % 3;
  if (a != 0 && !P.ov1) return;
  const int cb = c / KC, q = c % KC;
  double s = block_sum_strided(P.part + ((size_t)cb * gx * 3 + a) * KC + q, gx, (size_t)3 * KC);
  s *= P.scale[c];
  if (threadIdx.x == 0) {
    if (a == 0) P.alpha_out[c] = s;
    else if (a == 1) P.yre_out[c] = s;
    else P.yim_out[c] = s;
  }
}

static void launch_hv_finish(const HvParams &P, unsigned gx, unsigned gy, int kc, hipStream_t s) {
  const dim3 grid(3 * gy * (unsigned)kc);
  switch (kc) {
    case 8: hipLaunchKernelGGL(hv_lanczos_finish<8>, grid, dim3(kBlock), 0, s, P, gx); break;
    case 4: hipLaunchKernelGGL(hv_lanczos_finish<4>, grid, dim3(kBlock), 0, s, P, gx); break;
    case 2: hipLaunchKernelGGL(hv_lanczos_finish<2>, grid, dim3(kBlock), 0, s, P, gx); break;
    default: hipLaunchKernelGGL(hv_lanczos_finish<1>, grid, dim3(kBlock), 0, s, P, gx); break;
  }
}

// Spin-1/2 systems with N >= 8: tile = 256 rows whose low 8 bits run over the
// lanes; bits >= 8 (the tile index) are uniform over the block.
template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void hv_half(HamGeom g, DevTables<R> tb, const int2 *__restrict__ pij,
                                                  const R *__restrict__ pzz, HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, np = g.npair;
  Cx<R> *s_pc = reinterpret_cast<Cx<R> *>(smem);   // [np][4]
  Cx<R> *s_hf = s_pc + 4 * np;                     // [n][2]
  Cx<R> *s_fh = s_hf + 2 * n;                      // [n][2] high part of F (per tile)
  R *s_hd = reinterpret_cast<R *>(s_fh + 2 * n);   // [n][2]
  R *s_phi = s_hd + 2 * n;                         // [8]
  R *s_dt = s_phi + 8;                             // [n]
  const int t = threadIdx.x;
  const int c0 = blockIdx.y * KC;
  for (int i = t; i < 4 * np; i += kBlock) s_pc[i] = tb.pc_half[i];
  for (int i = t; i < 2 * n; i += kBlock) {
    s_hf[i] = tb.hflip[i];
    s_hd[i] = tb.hdiag[(i >> 1) * 16 + (i & 1)];
  }
  __syncthreads();
  // low-bit part of the diagonal (identical for every tile)
  R dlow = 0;
  for (int k = 0; k < kLowBits; k++) dlow += s_hd[2 * k + ((t >> k) & 1)];
  for (int p = 0; p < np; p++) {
    const int2 ij = pij[p];
    if (ij.y >= kLowBits) continue;
    const R mm = (((t >> ij.x) ^ (t >> ij.y)) & 1) ? R(-0.25) : R(0.25);
    dlow = fma(pzz[p], mm, dlow);
  }
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v) + c0;
  double red[3][KC];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int q = 0; q < KC; q++) red[a][q] = 0.0;

  for (uint32_t tile = blockIdx.x; tile < P.ntile; tile += gridDim.x) {
    const uint32_t hi = tile << kLowBits;  // row bits >= 8
    __syncthreads();
    if (t < 2 * n) {
      const int k = t >> 1, sel = t & 1;
      R fr = 0, fi = 0;
      for (int l = kLowBits; l < n; l++) {
        if (l == k) continue;
        const R ml = ((hi >> l) & 1) ? R(0.5) : R(-0.5);
        const Cx<R> c = tb.cz_half[(k * n + l) * 2 + sel];
        fr = fma(c.re, ml, fr);
        fi = fma(c.im, ml, fi);
      }
      s_fh[t] = Cx<R>{fr, fi};
    } else if (t >= 64 && t < 64 + kLowBits) {
      const int i = t - 64;
      R ph = 0;
      for (int j = kLowBits; j < n; j++) ph = fma(tb.zz[i * n + j], ((hi >> j) & 1) ? R(0.5) : R(-0.5), ph);
      s_phi[i] = ph;
    } else if (t >= 128 && t < 128 + n - kLowBits) {
      const int k = kLowBits + (t - 128);
      const R mk = ((hi >> k) & 1) ? R(0.5) : R(-0.5);
      R acc = s_hd[2 * k + ((hi >> k) & 1)];
      for (int j = k + 1; j < n; j++) acc = fma(tb.zz[k * n + j] * mk, ((hi >> j) & 1) ? R(0.5) : R(-0.5), acc);
      s_dt[k - kLowBits] = acc;
    }
    __syncthreads();
    R diag = dlow;
    for (int k = 0; k < n - kLowBits; k++) diag += s_dt[k];
#pragma unroll
    for (int i = 0; i < kLowBits; i++) diag = fma(((t >> i) & 1) ? R(0.5) : R(-0.5), s_phi[i], diag);

    const uint32_t row = hi | (uint32_t)t;
    Acc<R, KC> acc;
    acc_zero(acc);
    const Cx<R> *own = v + (size_t)row * P.K;
    mac_real(acc, diag, own);
    // single-site flips: h_k[b][1-b] + F_k (s^{+-}_k s^z_l pieces)
    for (int k = 0; k < n; k++) {
      const int b = (row >> k) & 1;
      const Cx<R> a1 = s_hf[2 * k + b], a2 = s_fh[2 * k + b];
      const Cx<R> a3 = tb.lowf[(k * 2 + b) * 256 + t];
      const Cx<R> c{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im};
      mac(acc, c, v + (size_t)(row ^ (1u << k)) * P.K);
    }
    // pair flips: exactly one of the four ladder pairs connects each row
    for (int p = 0; p < np; p++) {
      const int2 ij = pij[p];
      const int type = (((row >> ij.x) & 1) << 1) | ((row >> ij.y) & 1);
      const Cx<R> c = s_pc[4 * p + type];
      mac(acc, c, v + (size_t)(row ^ ((1u << ij.x) | (1u << ij.y))) * P.K);
    }
    hv_epilogue<R, KC>(P, row, c0, acc, own, red);
  }
  hv_finish<KC>(P, red);
}

// Spin-1/2 systems with N >= 11, one column per block: the block owns a tile of
// 2048 rows (sites 0..10 vary, 8 rows per thread: lane bits 0..7, row slot q =
// bits 8..10) staged in LDS.  Terms flipping only tile sites read LDS.  For
// every outer site a the partner tile (tile with bit a flipped) is staged once
// and serves the single flip of a and all mixed pairs (i < 11, a).  Pairs of two
// outer sites read the partner tile straight from global memory (one use each).
template <typename R>
__global__ __launch_bounds__(kBlock, 2) void hv_tile(HamGeom g, DevTables<R> tb, const int2 *__restrict__ pij,
                                                     const Cx<R> *__restrict__ pch, const R *__restrict__ pzz,
                                                     HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int Q = kRowsPerThread;
  const int n = g.n, np = g.npair, n_in = g.n_ll, n_out0 = g.n_ll + g.n_lh;
  Cx<R> *own = reinterpret_cast<Cx<R> *>(smem);   // [2048]
  Cx<R> *part = own + kTileRows;                  // [2048]
  Cx<R> *s_pc = part + kTileRows;                 // [n_in][4]
  Cx<R> *s_fmh = s_pc + 4 * n_in;                 // [n][2][Q]
  Cx<R> *s_hf = s_fmh + 2 * Q * n;                // [n][2]
  R *s_hd = reinterpret_cast<R *>(s_hf + 2 * n);  // [n][2]
  R *s_dmh = s_hd + 2 * n;                        // [Q]
  R *s_phi = s_dmh + Q;                           // [8][Q]
  R *s_term = s_phi + 8 * Q;                      // [32][Q]
  const int t = threadIdx.x;
  const int c0 = blockIdx.y;
  const int K = P.K;
  for (int i = t; i < 4 * n_in; i += kBlock) s_pc[i] = pch[i];
  for (int i = t; i < 2 * n; i += kBlock) {
    s_hf[i] = tb.hflip[i];
    s_hd[i] = tb.hdiag[(i >> 1) * 16 + (i & 1)];
  }
  __syncthreads();
  R dlow = 0;
  for (int k = 0; k < kLowBits; k++) dlow += s_hd[2 * k + ((t >> k) & 1)];
  for (int p = 0; p < n_in; p++) {
    const int2 ij = pij[p];
    if (ij.y >= kLowBits) continue;
    dlow = fma(pzz[p], (((t >> ij.x) ^ (t >> ij.y)) & 1) ? R(-0.25) : R(0.25), dlow);
  }
  R mlane[kLowBits];
#pragma unroll
  for (int i = 0; i < kLowBits; i++) mlane[i] = ((t >> i) & 1) ? R(0.5) : R(-0.5);
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v);
  const uint32_t ntile = g.dim >> kTileBits;
  double red[3][1] = {{0.0}, {0.0}, {0.0}};

  for (uint32_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const uint32_t base = tile << kTileBits;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; q++) own[q * kBlock + t] = v[(size_t)(base + q * kBlock + t) * K + c0];
    // per-tile uniform parts: rows of slot q have bits 8..10 = q and bits >= 11 = base
    for (int e = t; e < 2 * Q * n; e += kBlock) {
      const int k = e / (2 * Q), sel = (e / Q) & 1, q = e % Q;
      const uint32_t rb = base | ((uint32_t)q << kLowBits);
      R fr = 0, fi = 0;
      for (int l = kLowBits; l < n; l++) {
        if (l == k) continue;
        const R ml = ((rb >> l) & 1) ? R(0.5) : R(-0.5);
        const Cx<R> c = tb.cz_half[(k * n + l) * 2 + sel];
        fr = fma(c.re, ml, fr);
        fi = fma(c.im, ml, fi);
      }
      s_fmh[e] = Cx<R>{fr, fi};
    }
    if (t < 24 * Q) {
      const int k = kLowBits + t / Q, q = t % Q;
      if (k < n) {
        const uint32_t rb = base | ((uint32_t)q << kLowBits);
        const R mk = ((rb >> k) & 1) ? R(0.5) : R(-0.5);
        R acc = s_hd[2 * k + ((rb >> k) & 1)];
        for (int j = k + 1; j < n; j++) acc = fma(tb.zz[k * n + j] * mk, ((rb >> j) & 1) ? R(0.5) : R(-0.5), acc);
        s_term[(k - kLowBits) * Q + q] = acc;
      }
    } else if (t < 24 * Q + 8 * Q) {
      const int i = (t - 24 * Q) / Q, q = (t - 24 * Q) % Q;
      const uint32_t rb = base | ((uint32_t)q << kLowBits);
      R ph = 0;
      for (int j = kLowBits; j < n; j++) ph = fma(tb.zz[i * n + j], ((rb >> j) & 1) ? R(0.5) : R(-0.5), ph);
      s_phi[i * Q + q] = ph;
    }
    __syncthreads();
    if (t < Q) {
      R d = 0;
      for (int k = kLowBits; k < n; k++) d += s_term[(k - kLowBits) * Q + t];
      s_dmh[t] = d;
    }
    __syncthreads();

    Cx<R> acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      R dg = dlow + s_dmh[q];
#pragma unroll
      for (int i = 0; i < kLowBits; i++) dg = fma(mlane[i], s_phi[i * Q + q], dg);
      const Cx<R> x = own[q * kBlock + t];
      acc[q] = Cx<R>{dg * x.re, dg * x.im};
    }
    // single flips of tile sites
#pragma unroll 1
    for (int k = 0; k < kTileBits; k++) {
      if (!((g.single_mask >> k) & 1u)) continue;
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const int r = q * kBlock + t;
        const int b = (r >> k) & 1;
        const Cx<R> a1 = s_hf[2 * k + b], a2 = tb.lowf[(k * 2 + b) * 256 + t], a3 = s_fmh[(k * 2 + b) * Q + q];
        const Cx<R> c{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im};
        const Cx<R> x = own[r ^ (1 << k)];
        acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
        acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
      }
    }
    // pairs inside the tile
#pragma unroll 1
    for (int p = 0; p < n_in; p++) {
      const int2 ij = pij[p];
      const int mask = (1 << ij.x) | (1 << ij.y);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const int r = q * kBlock + t;
        const int type = (((r >> ij.x) & 1) << 1) | ((r >> ij.y) & 1);
        const Cx<R> c = s_pc[4 * p + type];
        const Cx<R> x = own[r ^ mask];
        acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
        acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
      }
    }
    // outer sites: stage the partner tile once, then its single flip and mixed pairs
#pragma unroll 1
    for (int a = kTileBits; a < n; a++) {
      const bool single_a = (g.single_mask >> a) & 1u;
      if (!single_a && g.mx_off[a + 1] == g.mx_off[a]) continue;  // uniform: no term needs this tile
      __syncthreads();
      const uint32_t pb = base ^ (1u << a);
#pragma unroll
      for (int q = 0; q < Q; q++) part[q * kBlock + t] = v[(size_t)(pb + q * kBlock + t) * K + c0];
      __syncthreads();
      const int ba = (base >> a) & 1;
#pragma unroll
      for (int q = 0; q < Q; q++) {
        if (!single_a) break;
        const Cx<R> a1 = s_hf[2 * a + ba], a2 = tb.lowf[(a * 2 + ba) * 256 + t], a3 = s_fmh[(a * 2 + ba) * Q + q];
        const Cx<R> c{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im};
        const Cx<R> x = part[q * kBlock + t];
        acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
        acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
      }
      const int p1 = g.mx_off[a + 1];
#pragma unroll 1
      for (int p = g.mx_off[a]; p < p1; p++) {
        const int i = pij[p].x;
        const Cx<R> clo = pch[4 * p + ba], chi = pch[4 * p + 2 + ba];
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const int r = q * kBlock + t;
          const Cx<R> c = ((r >> i) & 1) ? chi : clo;
          const Cx<R> x = part[r ^ (1 << i)];
          acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
          acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
        }
      }
    }
    // pairs of two outer sites: partner tile read once from global memory
#pragma unroll 1
    for (int p = n_out0; p < np; p++) {
      const int2 ij = pij[p];
      const int type = (((base >> ij.x) & 1) << 1) | ((base >> ij.y) & 1);
      const Cx<R> c = pch[4 * p + type];
      const uint32_t pb = base ^ (1u << ij.x) ^ (1u << ij.y);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const Cx<R> x = v[(size_t)(pb + q * kBlock + t) * K + c0];
        acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
        acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
      }
    }
#pragma unroll
    for (int q = 0; q < Q; q++) {
      Acc<R, 1> a1;
      a1.re[0] = acc[q].re;
      a1.im[0] = acc[q].im;
      // the epilogue reads the own value through a pointer with the column stride of v
      hv_epilogue<R, 1>(P, base + q * kBlock + t, c0, a1, v + (size_t)(base + q * kBlock + t) * K + c0, red);
    }
  }
  hv_finish<1>(P, red);
}

// Windowed pass (any spins, one column per block).  The block stages the
// window of rows that share the digits of every inactive site, applies from LDS
// the terms this pass owns, and accumulates into w.  Thread t owns window rows
// t + 256 q (q < RPT); loops run term-outer / row-inner so that each term's
// metadata is read once per window and the row updates issue back to back.
// POW2: every active site is a spin 1/2 (window digits = bits of the row).
// The window-uniform parts of the diagonal and of the s^{+-}s^z field, and the
// window's base index, come from records built once per Hamiltonian and field.
constexpr int kMaxPassSingles = 4;

template <typename R, bool POW2, int RPT>
struct PassRec {
  // record layout in units of R
  static constexpr int kDq = 0;                                  // POW2: [RPT]  general: [1]
  static constexpr int kPhi = POW2 ? RPT : 1;                    // POW2: [8][RPT]  general: [8]
  static constexpr int kFq = POW2 ? 9 * RPT : 9;                 // Cx [4][2][RPT] / Cx [4][2]
  static constexpr int kLen = POW2 ? 9 * RPT + 16 * RPT : 9 + 16;
  // lane table layout (POW2 only): Cx flane[4][2][256], then R dlane[256]
  static constexpr int kLaneBytes = POW2 ? (int)(sizeof(Cx<R>) * kMaxPassSingles * 2 * 256 + sizeof(R) * 256) : 0;
};

// One block builds the record of window wid (and, for block 0 / wid 0, the lane
// table).  s_min/s_idig/s_tmp: LDS scratch of >= 32, 32 and 32*RPT entries.
template <typename R, bool POW2, int RPT>
__global__ __launch_bounds__(kBlock) void pass_record_kernel(HamGeom g, DevTables<R> tb, PassDesc D,
                                                             R *__restrict__ rec,
                                                             uint32_t *__restrict__ base_out,
                                                             unsigned char *__restrict__ lane) {
  using L = PassRec<R, POW2, RPT>;
  __shared__ R s_min[32];
  __shared__ int s_idig[32];
  __shared__ R s_tmp[32 * RPT];
  const int t = threadIdx.x;
  const int na = D.na, ni = D.ni, n = g.n;
  if (POW2 && blockIdx.x == 0) {
    // lane table: z-field of each single over active sites < 8, diagonal over sites < 8
    Cx<R> *flane = reinterpret_cast<Cx<R> *>(lane);
    R *dlane = reinterpret_cast<R *>(flane + kMaxPassSingles * 2 * 256);
    for (int s2 = 0; s2 < kMaxPassSingles; s2++) {
      Cx<R> f0{0, 0}, f1{0, 0};
      if (s2 < D.nsing && g.has_z) {
        const int a = D.sing[s2], k = D.act[a];
        for (int a2 = 0; a2 < na && a2 < kLowBits; a2++) {
          if (a2 == a) continue;
          const R m2 = ((t >> a2) & 1) ? R(0.5) : R(-0.5);
          const Cx<R> cm = tb.czm[k * n + D.act[a2]], cp = tb.czp[k * n + D.act[a2]];
          f0.re = fma(cm.re, m2, f0.re);
          f0.im = fma(cm.im, m2, f0.im);
          f1.re = fma(cp.re, m2, f1.re);
          f1.im = fma(cp.im, m2, f1.im);
        }
      }
      flane[(s2 * 2 + 0) * 256 + t] = f0;
      flane[(s2 * 2 + 1) * 256 + t] = f1;
    }
    R dl = 0;
    if (D.first)
      for (int a = 0; a < na && a < kLowBits; a++) {
        dl += tb.hdiag[D.act[a] * 16 + ((t >> a) & 1)];
        const R ma = ((t >> a) & 1) ? R(0.5) : R(-0.5);
        for (int a2 = a + 1; a2 < na && a2 < kLowBits; a2++)
          dl = fma(tb.zz[D.act[a] * n + D.act[a2]] * ma, ((t >> a2) & 1) ? R(0.5) : R(-0.5), dl);
      }
    dlane[t] = dl;
  }
  for (uint32_t wid = blockIdx.x; wid < D.nwin; wid += gridDim.x) {
    R *out = rec + (size_t)wid * L::kLen;
    __syncthreads();
    if (t < ni) {
      uint32_t rem = wid, dg = 0;
      for (int i = 0; i <= t; i++) {
        const uint32_t r = (uint32_t)D.irad[i], q = rem / r;
        dg = rem - q * r;
        rem = q;
      }
      s_idig[t] = (int)dg;
      s_min[t] = tb.mval[D.inact[t] * 16 + dg];
    }
    if (t == 0) {
      uint32_t rem = wid, b = 0;
      for (int i = 0; i < ni; i++) {
        const uint32_t r = (uint32_t)D.irad[i], q = rem / r;
        b += (rem - q * r) * D.ist[i];
        rem = q;
      }
      base_out[wid] = b;
    }
    __syncthreads();
    Cx<R> *fq = reinterpret_cast<Cx<R> *>(out + L::kFq);
    if (POW2) {
      for (int e = t; e < kMaxPassSingles * 2 * RPT; e += kBlock) {
        const int s2 = e / (2 * RPT), sel = (e / RPT) & 1, q = e % RPT;
        R fr = 0, fi = 0;
        if (s2 < D.nsing && g.has_z) {
          const int a = D.sing[s2], k = D.act[a];
          const Cx<R> *cz = sel ? tb.czp : tb.czm;
          for (int i = 0; i < ni; i++) {
            const Cx<R> c = cz[k * n + D.inact[i]];
            fr = fma(c.re, s_min[i], fr);
            fi = fma(c.im, s_min[i], fi);
          }
          for (int a2 = kLowBits; a2 < na; a2++) {
            if (a2 == a) continue;
            const R m2 = (((uint32_t)q >> (a2 - kLowBits)) & 1u) ? R(0.5) : R(-0.5);
            const Cx<R> c = cz[k * n + D.act[a2]];
            fr = fma(c.re, m2, fr);
            fi = fma(c.im, m2, fi);
          }
        }
        fq[e] = Cx<R>{fr, fi};
      }
      for (int e = t; e < 8 * RPT; e += kBlock) {
        const int a = e / RPT, q = e % RPT;
        R ph = 0;
        if (D.first && a < na) {
          const int k = D.act[a];
          for (int i = 0; i < ni; i++) ph = fma(tb.zz[k * n + D.inact[i]], s_min[i], ph);
          for (int a2 = kLowBits; a2 < na; a2++)
            ph = fma(tb.zz[k * n + D.act[a2]], (((uint32_t)q >> (a2 - kLowBits)) & 1u) ? R(0.5) : R(-0.5), ph);
        }
        out[L::kPhi + e] = ph;
      }
      const int nq = na > kLowBits ? na - kLowBits : 0;
      for (int e = t; e < 32 * RPT; e += kBlock) {
        const int j = e / RPT, q = e % RPT;
        R term = 0;
        if (D.first && j < nq + ni) {
          int k, dk;
          R mk;
          if (j < nq) {
            k = D.act[kLowBits + j];
            dk = (int)(((uint32_t)q >> j) & 1u);
            mk = dk ? R(0.5) : R(-0.5);
          } else {
            k = D.inact[j - nq];
            dk = s_idig[j - nq];
            mk = s_min[j - nq];
          }
          term = tb.hdiag[k * 16 + dk];
          for (int j2 = j + 1; j2 < nq + ni; j2++) {
            int k2;
            R m2;
            if (j2 < nq) {
              k2 = D.act[kLowBits + j2];
              m2 = (((uint32_t)q >> j2) & 1u) ? R(0.5) : R(-0.5);
            } else {
              k2 = D.inact[j2 - nq];
              m2 = s_min[j2 - nq];
            }
            term = fma(tb.zz[k * n + k2] * mk, m2, term);
          }
        }
        s_tmp[e] = term;
      }
      __syncthreads();
      for (int q = t; q < RPT; q += kBlock) {
        R d = 0;
        for (int j = 0; j < 32; j++) d += s_tmp[j * RPT + q];
        out[L::kDq + q] = d;
      }
    } else {
      for (int a = t; a < 8; a += kBlock) {
        R ph = 0;
        if (D.first && a < na) {
          const int k = D.act[a];
          for (int i = 0; i < ni; i++) ph = fma(tb.zz[k * n + D.inact[i]], s_min[i], ph);
        }
        out[L::kPhi + a] = ph;
      }
      for (int e = t; e < kMaxPassSingles * 2; e += kBlock) {
        R fr = 0, fi = 0;
        if ((e >> 1) < D.nsing && g.has_z) {
          const int a = D.sing[e >> 1], k = D.act[a];
          const Cx<R> *cz = (e & 1) ? tb.czp : tb.czm;
          for (int i = 0; i < ni; i++) {
            const Cx<R> c = cz[k * n + D.inact[i]];
            fr = fma(c.re, s_min[i], fr);
            fi = fma(c.im, s_min[i], fi);
          }
        }
        fq[e] = Cx<R>{fr, fi};
      }
      for (int i = t; i < 32; i += kBlock) {
        R term = 0;
        if (D.first && i < ni) {
          const int k = D.inact[i];
          term = tb.hdiag[k * 16 + s_idig[i]];
          for (int i2 = i + 1; i2 < ni; i2++) term = fma(tb.zz[k * n + D.inact[i2]] * s_min[i], s_min[i2], term);
        }
        s_tmp[i] = term;
      }
      __syncthreads();
      if (t == 0) {
        R d = 0;
        for (int i = 0; i < 32; i++) d += s_tmp[i];
        out[L::kDq] = d;
      }
    }
  }
}

template <typename R, bool POW2, int RPT>
__global__ __launch_bounds__(kBlock) void hv_pass(HamGeom g, DevTables<R> tb, PassDesc D,
                                                  const int4 *__restrict__ pp,
                                                  const R *__restrict__ rec,
                                                  const uint32_t *__restrict__ bases,
                                                  const unsigned char *__restrict__ lane,
                                                  const Cx<R> *__restrict__ czp, const Cx<R> *__restrict__ czm,
                                                  const R *__restrict__ zz, HvParams P) {
  using L = PassRec<R, POW2, RPT>;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t ws = D.wsize;
  const int na = D.na, n = g.n, npp = D.npp;
  Cx<R> *win = reinterpret_cast<Cx<R> *>(smem);        // [ws]
  Cx<R> *s_pc = win + ws;                              // [npp][4]
  Cx<R> *s_hoff = s_pc + 4 * npp;                      // [4 singles][4 D][16]
  R *s_rec = reinterpret_cast<R *>(s_hoff + kMaxPassSingles * 64);  // [kLen]
  R *s_hd = s_rec + L::kLen;                           // [na][16]
  R *s_gp = s_hd + 16 * na;                            // [na][16]
  R *s_gm = s_gp + 16 * na;                            // [na][16]
  R *s_m = s_gm + 16 * na;                             // [na][16]
  int4 *s_pi = reinterpret_cast<int4 *>(s_m + 16 * na);  // [npp]
  // general radix: pair coefficients with the ladder factors and the validity
  // folded in, per pair [d_i][d_j][type] (0 where a digit leaves its range)
  int *s_toff = reinterpret_cast<int *>(s_pi + npp);     // [npp + 1]
  Cx<R> *s_ct = reinterpret_cast<Cx<R> *>(smem + ((reinterpret_cast<unsigned char *>(s_toff + npp + 1) - smem + 15) & ~(size_t)15));
  const int t = threadIdx.x;
  const int K = P.K, c0 = blockIdx.y;

  for (int i = t; i < 4 * npp; i += kBlock) {
    const int p = pp[D.pp_off + i / 4].x;
    s_pc[i] = POW2 ? tb.pc_half[4 * p + (i & 3)] : tb.pc[4 * p + (i & 3)];
  }
  for (int i = t; i < npp; i += kBlock) {
    const int4 e = pp[D.pp_off + i];
    s_pi[i] = POW2 ? make_int4(e.y, e.z, (int)(D.wst[e.y] | D.wst[e.z]), 0)
                   : make_int4(e.y, e.z, (int)D.wst[e.y], (int)D.wst[e.z]);
  }
  for (int i = t; i < 16 * na; i += kBlock) {
    const int k = D.act[i / 16];
    s_hd[i] = tb.hdiag[k * 16 + (i & 15)];
    s_gp[i] = tb.gp[k * 16 + (i & 15)];
    s_gm[i] = tb.gm[k * 16 + (i & 15)];
    s_m[i] = tb.mval[k * 16 + (i & 15)];
  }
  for (int i = t; i < D.nsing * 64; i += kBlock) {
    const int k = D.act[D.sing[i / 64]];
    s_hoff[i] = tb.hoff[k * 64 + (i & 63)];
  }
  // the table pays off at complex128; at complex64 the per-row factors are faster
  const int ctab = (!POW2 && sizeof(R) == 8) ? D.ctab : 0;
  if (ctab > 0) {
    if (t == 0) {
      int o = 0;
      for (int e = 0; e < npp; e++) {
        s_toff[e] = o;
        const int4 pe = pp[D.pp_off + e];
        o += 4 * D.wrad[pe.y] * D.wrad[pe.z];
      }
      s_toff[npp] = o;
    }
    __syncthreads();
    for (int idx = t; idx < ctab; idx += kBlock) {
      int e = 0;
      while (e + 1 < npp && s_toff[e + 1] <= idx) e++;
      const int4 pe = pp[D.pp_off + e];
      const int ai = pe.y, aj = pe.z, ri = D.wrad[ai], rj = D.wrad[aj];
      const int loc = idx - s_toff[e], ty = loc & 3, dd = loc >> 2, di = dd / rj, dj = dd - di * rj;
      const bool im_ = (ty >> 1) != 0, jm = (ty & 1) != 0;
      const bool ok = (im_ ? (di <= ri - 2) : (di >= 1)) && (jm ? (dj <= rj - 2) : (dj >= 1));
      const Cx<R> cq = tb.pc[4 * pe.x + ty];
      const R f = ok ? (im_ ? tb.gm[D.act[ai] * 16 + di] : tb.gp[D.act[ai] * 16 + di]) *
                           (jm ? tb.gm[D.act[aj] * 16 + dj] : tb.gp[D.act[aj] * 16 + dj])
                     : R(0);
      s_ct[idx] = Cx<R>{cq.re * f, cq.im * f};
    }
  }
  // per-thread rows: packed active digits and offset within the full basis
  uint32_t dig[RPT], gof[RPT];
#pragma unroll
  for (int q = 0; q < RPT; q++) {
    const uint32_t r = (uint32_t)(t + kBlock * q);
    uint32_t packed = 0, off = 0;
    if (POW2) {
      for (int a = 0; a < na; a++) off += ((r >> a) & 1u) * D.gst[a];
      packed = r;
    } else {
      uint32_t rem = r;
      for (int a = 0; a < na; a++) {
        const uint32_t rr = (uint32_t)D.wrad[a], qq = rem / rr, d = rem - qq * rr;
        off += d * D.gst[a];
        packed |= d << (4 * a);
        rem = qq;
      }
    }
    dig[q] = packed;
    gof[q] = r < ws ? off : 0u;  // rows past the window read the window's first row (unused)
  }
  auto digit = [&](int q, int a) -> uint32_t {
    return POW2 ? ((dig[q] >> a) & 1u) : ((dig[q] >> (4 * a)) & 15u);
  };
  Cx<R> flane[kMaxPassSingles][2];
  R dlane = 0;
  if (POW2) {
    const Cx<R> *fl = reinterpret_cast<const Cx<R> *>(lane);
#pragma unroll
    for (int s2 = 0; s2 < kMaxPassSingles; s2++) {
      flane[s2][0] = fl[(s2 * 2 + 0) * 256 + t];
      flane[s2][1] = fl[(s2 * 2 + 1) * 256 + t];
    }
    dlane = reinterpret_cast<const R *>(fl + kMaxPassSingles * 2 * 256)[t];
  }
  R mlane[kLowBits];
#pragma unroll
  for (int a = 0; a < kLowBits; a++) mlane[a] = ((t >> a) & 1) ? R(0.5) : R(-0.5);

  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v);
  Cx<R> *wout = reinterpret_cast<Cx<R> *>(P.w);
  double red[3][1] = {{0.0}, {0.0}, {0.0}};

  for (uint32_t wid = blockIdx.x; wid < D.nwin; wid += gridDim.x) {
    const uint32_t base = bases[wid];
    __syncthreads();
    // eight rows' loads in flight before the first LDS store (a load and store
    // per row under the row's bound check would wait out each load in turn)
#pragma unroll
    for (int h = 0; h < RPT; h += 8) {
      Cx<R> tmp[8];
#pragma unroll
      for (int u = 0; u < 8; u++) tmp[u] = v[(size_t)(base + gof[h + u]) * K + c0];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const uint32_t r = (uint32_t)(t + kBlock * (h + u));
        if (r < ws) win[r] = tmp[u];
      }
    }
    for (int i = t; i < L::kLen; i += kBlock) s_rec[i] = rec[(size_t)wid * L::kLen + i];
    __syncthreads();
    const Cx<R> *s_fq = reinterpret_cast<const Cx<R> *>(s_rec + L::kFq);

    Cx<R> acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; q++) acc[q] = Cx<R>{0, 0};
    if (D.first) {
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const uint32_t r = (uint32_t)(t + kBlock * q);
        if (r >= ws) continue;
        R dg;
        if (POW2) {
          dg = dlane + s_rec[L::kDq + q];
          for (int a = 0; a < na && a < kLowBits; a++) dg = fma(mlane[a], s_rec[L::kPhi + a * RPT + q], dg);
        } else {
          dg = s_rec[L::kDq];
          for (int a = 0; a < na; a++) {
            const uint32_t da = digit(q, a);
            dg += s_hd[a * 16 + da];
            R zs = s_rec[L::kPhi + a];
            for (int a2 = a + 1; a2 < na; a2++) zs = fma(zz[D.act[a] * n + D.act[a2]], s_m[a2 * 16 + digit(q, a2)], zs);
            dg = fma(s_m[a * 16 + da], zs, dg);
          }
        }
        const Cx<R> x = win[r];
        acc[q] = Cx<R>{dg * x.re, dg * x.im};
      }
    }
    // single flips
    for (int s2 = 0; s2 < D.nsing; s2++) {
      const int a = D.sing[s2], k = D.act[a];
      const int rk = D.wrad[a];
      const uint32_t st = D.wst[a];
      Cx<R> fl0{0, 0}, fl1{0, 0};
#pragma unroll
      for (int s3 = 0; s3 < kMaxPassSingles; s3++)
        if (s3 == s2) {
          fl0 = flane[s3][0];
          fl1 = flane[s3][1];
        }
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const uint32_t r = (uint32_t)(t + kBlock * q);
        if (r >= ws) continue;
        const int d = (int)digit(q, a);
        R fpr = 0, fpi = 0, fmr = 0, fmi = 0;
        if (g.has_z) {
          if (POW2) {
            const Cx<R> u0 = s_fq[(s2 * 2 + 0) * RPT + q], u1 = s_fq[(s2 * 2 + 1) * RPT + q];
            fmr = fl0.re + u0.re;
            fmi = fl0.im + u0.im;
            fpr = fl1.re + u1.re;
            fpi = fl1.im + u1.im;
          } else {
            fmr = s_fq[s2 * 2].re;
            fmi = s_fq[s2 * 2].im;
            fpr = s_fq[s2 * 2 + 1].re;
            fpi = s_fq[s2 * 2 + 1].im;
            for (int a2 = 0; a2 < na; a2++) {
              if (a2 == a) continue;
              const R m2 = s_m[a2 * 16 + digit(q, a2)];
              const Cx<R> cm = czm[k * n + D.act[a2]], cp = czp[k * n + D.act[a2]];
              fmr = fma(cm.re, m2, fmr);
              fmi = fma(cm.im, m2, fmi);
              fpr = fma(cp.re, m2, fpr);
              fpi = fma(cp.im, m2, fpi);
            }
          }
        }
#pragma unroll
        for (int di = 0; di < 4; di++) {
          const int Dl = (di < 2) ? di - 2 : di - 1;
          const int nd = d + Dl;
          if (nd < 0 || nd >= rk) continue;
          Cx<R> c = s_hoff[(s2 * 4 + di) * 16 + d];
          if (Dl == -1) {
            const R gg = s_gp[a * 16 + d];
            c.re = fma(gg, fpr, c.re);
            c.im = fma(gg, fpi, c.im);
          } else if (Dl == 1) {
            const R gg = s_gm[a * 16 + d];
            c.re = fma(gg, fmr, c.re);
            c.im = fma(gg, fmi, c.im);
          }
          const Cx<R> x = win[r + (uint32_t)Dl * st];
          acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
          acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
        }
      }
    }
    // pair flips
    if (POW2) {
      for (int e = 0; e < npp; e++) {
        const int4 pi = s_pi[e];
        const Cx<R> *cp = s_pc + 4 * e;
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          const uint32_t r = (uint32_t)(t + kBlock * q);
          if (r >= ws) continue;
          const int type = (int)((((r >> pi.x) & 1u) << 1) | ((r >> pi.y) & 1u));
          const Cx<R> c = cp[type];
          const Cx<R> x = win[r ^ (uint32_t)pi.z];
          acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
          acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
        }
      }
    } else {
      for (int e = 0; e < npp && ctab > 0; e++) {
        const int4 pi = s_pi[e];
        const int rj = D.wrad[pi.y];
        const Cx<R> *ct = s_ct + s_toff[e];
        bool live[4];
        uint32_t off[4];
#pragma unroll
        for (int ty = 0; ty < 4; ty++) {
          const Cx<R> cq = s_pc[4 * e + ty];
          live[ty] = !(cq.re == R(0) && cq.im == R(0));  // uniform: a ladder pair absent from the pair
          off[ty] = ((ty >> 1) ? (uint32_t)pi.z : (uint32_t)(-pi.z)) + ((ty & 1) ? (uint32_t)pi.w : (uint32_t)(-pi.w));
        }
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          const uint32_t r = (uint32_t)(t + kBlock * q);
          if (r >= ws) continue;
          const int di = (int)digit(q, pi.x), dj = (int)digit(q, pi.y);
          const Cx<R> *c4 = ct + 4 * (di * rj + dj);
#pragma unroll
          for (int ty = 0; ty < 4; ty++) {
            if (!live[ty]) continue;
            // a digit leaving its range has a zero coefficient; the clamped
            // partner keeps that read inside the window
            const Cx<R> c = c4[ty];
            const uint32_t pr = min(r + off[ty], ws - 1u);
            const Cx<R> x = win[pr];
            acc[q].re = fma(c.re, x.re, fma(-c.im, x.im, acc[q].re));
            acc[q].im = fma(c.re, x.im, fma(c.im, x.re, acc[q].im));
          }
        }
      }
      // without a table (large radices): the ladder factors per row
      for (int e = 0; e < npp && ctab == 0; e++) {
        const int4 pi = s_pi[e];
        const int ri = D.wrad[pi.x], rj = D.wrad[pi.y];
        Cx<R> cq[4];
#pragma unroll
        for (int ty = 0; ty < 4; ty++) cq[ty] = s_pc[4 * e + ty];
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          const uint32_t r = (uint32_t)(t + kBlock * q);
          if (r >= ws) continue;
          const int di = (int)digit(q, pi.x), dj = (int)digit(q, pi.y);
          const R gpi = s_gp[pi.x * 16 + di], gmi = s_gm[pi.x * 16 + di];
          const R gpj = s_gp[pi.y * 16 + dj], gmj = s_gm[pi.y * 16 + dj];
#pragma unroll
          for (int ty = 0; ty < 4; ty++) {
            const bool im_ = (ty >> 1) != 0, jm = (ty & 1) != 0;
            const bool vi = im_ ? (di <= ri - 2) : (di >= 1);
            const bool vj = jm ? (dj <= rj - 2) : (dj >= 1);
            if (!(vi && vj) || (cq[ty].re == R(0) && cq[ty].im == R(0))) continue;
            const R f = (im_ ? gmi : gpi) * (jm ? gmj : gpj);
            const uint32_t pr = r + (im_ ? (uint32_t)pi.z : (uint32_t)(-pi.z)) + (jm ? (uint32_t)pi.w : (uint32_t)(-pi.w));
            const Cx<R> x = win[pr];
            const R cr = cq[ty].re * f, ci = cq[ty].im * f;
            acc[q].re = fma(cr, x.re, fma(-ci, x.im, acc[q].re));
            acc[q].im = fma(cr, x.im, fma(ci, x.re, acc[q].im));
          }
        }
      }
    }
    // four rows at a time: every load of the group (earlier passes' partial
    // sums; on the last pass of a Lanczos step the previous vector and O v_1)
    // is issued before the group's first store
    const Cx<R> *xpv = P.xprev ? reinterpret_cast<const Cx<R> *>(P.xprev) : nullptr;
    const Cx<R> *o1v = P.ov1 ? reinterpret_cast<const Cx<R> *>(P.ov1) : nullptr;
    const bool lz = D.last && P.lanczos;
    const double sx = lz ? P.scale[c0] : 0.0;
    const double bp = (lz && xpv) ? P.beta_prev[c0] * P.sx_prev[c0] : 0.0;
    const R sc = (D.last && !P.lanczos && P.scale) ? (R)P.scale[c0] : R(1);
#pragma unroll
    for (int h = 0; h < RPT; h += 4) {
      Cx<R> wo[4], xo[4], ov[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const size_t gi = (size_t)(base + gof[h + u]) * K + c0;
        wo[u] = D.first ? Cx<R>{0, 0} : wout[gi];
        xo[u] = (lz && xpv) ? xpv[gi] : Cx<R>{0, 0};
        ov[u] = (lz && o1v) ? o1v[gi] : Cx<R>{0, 0};
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int q = h + u;
        const uint32_t r = (uint32_t)(t + kBlock * q);
        if (r >= ws) continue;
        Cx<R> *wp = wout + (size_t)(base + gof[q]) * K + c0;
        const R are = acc[q].re + wo[u].re, aim = acc[q].im + wo[u].im;
        if (!D.last) {
          *wp = Cx<R>{are, aim};
        } else if (!P.lanczos) {
          *wp = Cx<R>{are * sc, aim * sc};
        } else {
          // the Lanczos epilogue of hv_epilogue with its loads hoisted
          const double wr = (double)are * sx - bp * (double)xo[u].re;
          const double wi = (double)aim * sx - bp * (double)xo[u].im;
          const Cx<R> out{(R)wr, (R)wi};
          *wp = out;
          const Cx<R> x = win[r];
          red[0][0] += (double)x.re * (double)out.re + (double)x.im * (double)out.im;
          if (o1v) {
            red[1][0] += (double)ov[u].re * (double)x.re + (double)ov[u].im * (double)x.im;
            red[2][0] += (double)ov[u].re * (double)x.im - (double)ov[u].im * (double)x.re;
          }
        }
      }
    }
  }
  if (D.last) hv_finish<1>(P, red);
}

// General mixed-radix systems (any 2 s_i <= 15, N <= 32).
template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void hv_gen(HamGeom g, DevTables<R> tb, const Cx<R> *__restrict__ pcg,
                                                 const Cx<R> *__restrict__ czp, const Cx<R> *__restrict__ czm,
                                                 const int2 *__restrict__ pij, const R *__restrict__ pzz,
                                                 HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n;
  Cx<R> *s_hoff = reinterpret_cast<Cx<R> *>(smem);  // [n][4][16]
  R *s_hd = reinterpret_cast<R *>(s_hoff + n * 64);  // [n][16]
  R *s_gp = s_hd + n * 16;
  R *s_gm = s_gp + n * 16;
  R *s_m = s_gm + n * 16;
  const int t = threadIdx.x;
  const int c0 = blockIdx.y * KC;
  for (int i = t; i < n * 64; i += kBlock) s_hoff[i] = tb.hoff[i];
  for (int i = t; i < n * 16; i += kBlock) {
    s_hd[i] = tb.hdiag[i];
    s_gp[i] = tb.gp[i];
    s_gm[i] = tb.gm[i];
    s_m[i] = tb.mval[i];
  }
  __syncthreads();
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v) + c0;
  double red[3][KC];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int q = 0; q < KC; q++) red[a][q] = 0.0;

  for (uint32_t tile = blockIdx.x; tile < P.ntile; tile += gridDim.x) {
    const uint32_t row = tile * kBlock + t;
    if (row >= g.dim) continue;
    // digits, 4 bits each: sites 0..15 in dlo, 16..31 in dhi
    uint64_t dlo = 0, dhi = 0;
    {
      uint32_t rem = row;
      for (int k = 0; k < n; k++) {
        const uint32_t r = (uint32_t)g.radix[k];
        const uint32_t q = rem / r;
        const uint64_t dk = rem - q * r;
        rem = q;
        if (k < 16) dlo |= dk << (4 * k);
        else dhi |= dk << (4 * (k - 16));
      }
    }
    auto digit = [&](int k) -> int {
      return (int)(((k < 16) ? (dlo >> (4 * k)) : (dhi >> (4 * (k - 16)))) & 15u);
    };
    R diag = 0;
    for (int k = 0; k < n; k++) diag += s_hd[k * 16 + digit(k)];
    for (int p = 0; p < g.npair; p++) {
      const int2 ij = pij[p];
      diag = fma(pzz[p], s_m[ij.x * 16 + digit(ij.x)] * s_m[ij.y * 16 + digit(ij.y)], diag);
    }
    Acc<R, KC> acc;
    acc_zero(acc);
    const Cx<R> *own = v + (size_t)row * P.K;
    mac_real(acc, diag, own);
    for (int k = 0; k < n; k++) {
      const int dk = digit(k), rk = g.radix[k];
      const uint32_t st = g.stride[k];
      R fpr = 0, fpi = 0, fmr = 0, fmi = 0;
      if (g.has_z) {
        for (int l = 0; l < n; l++) {
          if (l == k) continue;
          const R ml = s_m[l * 16 + digit(l)];
          const Cx<R> cp = czp[k * n + l], cm = czm[k * n + l];
          fpr = fma(cp.re, ml, fpr);
          fpi = fma(cp.im, ml, fpi);
          fmr = fma(cm.re, ml, fmr);
          fmi = fma(cm.im, ml, fmi);
        }
      }
#pragma unroll
      for (int di = 0; di < 4; di++) {
        const int D = (di < 2) ? di - 2 : di - 1;  // -2,-1,+1,+2
        const int nd = dk + D;
        if (nd < 0 || nd >= rk) continue;
        Cx<R> c = s_hoff[(k * 4 + di) * 16 + dk];
        if (D == -1) {
          const R gg = s_gp[k * 16 + dk];
          c.re = fma(gg, fpr, c.re);
          c.im = fma(gg, fpi, c.im);
        } else if (D == 1) {
          const R gg = s_gm[k * 16 + dk];
          c.re = fma(gg, fmr, c.re);
          c.im = fma(gg, fmi, c.im);
        }
        const uint32_t partner = row + (uint32_t)(D * (int)st);
        mac(acc, c, v + (size_t)partner * P.K);
      }
    }
    for (int p = 0; p < g.npair; p++) {
      const int2 ij = pij[p];
      const int di = digit(ij.x), dj = digit(ij.y);
      const int ri = g.radix[ij.x], rj = g.radix[ij.y];
      const uint32_t si = g.stride[ij.x], sj = g.stride[ij.y];
      const R gpi = s_gp[ij.x * 16 + di], gmi = s_gm[ij.x * 16 + di];
      const R gpj = s_gp[ij.y * 16 + dj], gmj = s_gm[ij.y * 16 + dj];
      const Cx<R> *pc = pcg + 4 * p;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const Cx<R> cq = pc[q];
        if (cq.re == R(0) && cq.im == R(0)) continue;
        const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;  // '-' ladder on site i / j
        const bool vi = im_ ? (di <= ri - 2) : (di >= 1);
        const bool vj = jm ? (dj <= rj - 2) : (dj >= 1);
        if (!(vi && vj)) continue;
        const R f = (im_ ? gmi : gpi) * (jm ? gmj : gpj);
        const uint32_t partner = row + (im_ ? si : (uint32_t)(-(int)si)) + (jm ? sj : (uint32_t)(-(int)sj));
        mac(acc, Cx<R>{cq.re * f, cq.im * f}, v + (size_t)partner * P.K);
      }
    }
    hv_epilogue<R, KC>(P, row, c0, acc, own, red);
  }
  hv_finish<KC>(P, red);
}

// ------------------------------------------------------------------ L2-window passes
// Scatters the low bits of x to the set bits of mask (ascending).
__device__ __forceinline__ uint32_t scatter_bits(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    const uint32_t low = mask & (0u - mask);
    if (x & 1u) r |= low;
    x >>= 1;
    mask &= mask - 1u;
  }
  return r;
}

// Work-item walk of one L2-window pass.  With at least 8 windows and a grid that
// is a multiple of 8, block b runs on XCD b % 8 (workgroups are dispatched to the
// XCDs round robin); XCD x owns windows x, x+8, ... and its blocks walk the
// items of those windows in order, so the windows an XCD works on at any time
// are consecutive in its list and their rows stay in that XCD's L2 (as many
// windows are in flight as the XCD's blocks cover: nb / nin).  Otherwise the
// items are walked flat.  body(win, item) is called for every item of the pass.
template <typename F>
__device__ __forceinline__ void win_walk(const WinPass &W, F &&body) {
  const bool xcd = W.nwin >= 8 && (gridDim.x & 7u) == 0;
  const uint32_t x = xcd ? (blockIdx.x & 7u) : 0u;
  const uint64_t nwx = xcd ? (uint64_t)((W.nwin - x + 7u) >> 3) : (uint64_t)W.nwin;
  const uint64_t jn = nwx * W.nin;
  const uint64_t jstart = xcd ? (blockIdx.x >> 3) : blockIdx.x;
  const uint64_t jstep = xcd ? (gridDim.x >> 3) : gridDim.x;
  for (uint64_t j = jstart; j < jn; j += jstep) {
    const uint32_t wl = (uint32_t)(j / W.nin);
    const uint32_t item = (uint32_t)(j - (uint64_t)wl * W.nin);
    body(xcd ? x + 8u * wl : wl, item);
  }
}

// Adds the earlier passes' partial sum, then stores the raw partial (not the
// last pass) or runs the epilogue (last pass).  KC columns from c0.
template <typename R, int KC>
__device__ __forceinline__ void win_store(const WinPass &W, const HvParams &P, uint32_t row, int c0,
                                          Acc<R, KC> &acc, const Cx<R> *own, double (&red)[3][KC]) {
  Cx<R> *wp = reinterpret_cast<Cx<R> *>(P.w) + (size_t)row * P.K + c0;
  if (!W.first) {
#pragma unroll
    for (int q = 0; q < KC; q++) {
      const Cx<R> o = wp[q];
      acc.re[q] += o.re;
      acc.im[q] += o.im;
    }
  }
  if (W.last) {
    hv_epilogue<R, KC>(P, row, c0, acc, own, red);
  } else {
#pragma unroll
    for (int q = 0; q < KC; q++) wp[q] = Cx<R>{acc.re[q], acc.im[q]};
  }
}

// Spin-1/2, N >= 8: one 256-row tile per item (row bits 0..7 over the lanes,
// bits >= 8 from the window and item indices), terms as in hv_half restricted
// to the pass.
template <typename R>
__global__ __launch_bounds__(kBlock) void hv_half_win(HamGeom g, DevTables<R> tb, WinPass W,
                                                      const int4 *__restrict__ plist, HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n, np = W.np;
  Cx<R> *s_pc = reinterpret_cast<Cx<R> *>(smem);   // [np][4]
  Cx<R> *s_hf = s_pc + 4 * np;                     // [n][2]
  Cx<R> *s_fh = s_hf + 2 * n;                      // [n][2] high part of F (per tile)
  R *s_hd = reinterpret_cast<R *>(s_fh + 2 * n);   // [n][2]
  R *s_phi = s_hd + 2 * n;                         // [8]
  R *s_dt = s_phi + 8;                             // [n]
  const int t = threadIdx.x;
  const int c0 = blockIdx.y;
  const int4 *pl = plist + W.p0;
  for (int i = t; i < 4 * np; i += kBlock) s_pc[i] = tb.pc_half[4 * pl[i >> 2].x + (i & 3)];
  for (int i = t; i < 2 * n; i += kBlock) {
    s_hf[i] = tb.hflip[i];
    s_hd[i] = tb.hdiag[(i >> 1) * 16 + (i & 1)];
  }
  __syncthreads();
  R dlow = 0;
  if (W.diag) {
    for (int k = 0; k < kLowBits; k++) dlow += s_hd[2 * k + ((t >> k) & 1)];
    for (int p = 0; p < g.npair; p++) {
      const int2 ij = tb.pij[p];
      if (ij.y >= kLowBits) continue;
      const R mm = (((t >> ij.x) ^ (t >> ij.y)) & 1) ? R(-0.25) : R(0.25);
      dlow = fma(tb.pzz[p], mm, dlow);
    }
  }
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v) + c0;
  double red[3][1] = {{0.0}, {0.0}, {0.0}};
  const bool zf = g.has_z && W.smask != 0u;

  win_walk(W, [&](uint32_t win, uint32_t item) {
    // uniform over the block: keep it (and everything derived) in scalar registers
    const uint32_t hi = __builtin_amdgcn_readfirstlane(scatter_bits(item, W.emask) | scatter_bits(win, W.omask));
    __syncthreads();
    if (t < 2 * n) {
      if (zf) {
        const int k = t >> 1, sel = t & 1;
        R fr = 0, fi = 0;
        for (int l = kLowBits; l < n; l++) {
          if (l == k) continue;
          const R ml = ((hi >> l) & 1) ? R(0.5) : R(-0.5);
          const Cx<R> c = tb.cz_half[(k * n + l) * 2 + sel];
          fr = fma(c.re, ml, fr);
          fi = fma(c.im, ml, fi);
        }
        s_fh[t] = Cx<R>{fr, fi};
      } else {
        s_fh[t] = Cx<R>{0, 0};
      }
    } else if (W.diag && t >= 64 && t < 64 + kLowBits) {
      const int i = t - 64;
      R ph = 0;
      for (int j = kLowBits; j < n; j++) ph = fma(tb.zz[i * n + j], ((hi >> j) & 1) ? R(0.5) : R(-0.5), ph);
      s_phi[i] = ph;
    } else if (W.diag && t >= 128 && t < 128 + n - kLowBits) {
      const int k = kLowBits + (t - 128);
      const R mk = ((hi >> k) & 1) ? R(0.5) : R(-0.5);
      R acc = s_hd[2 * k + ((hi >> k) & 1)];
      for (int j = k + 1; j < n; j++) acc = fma(tb.zz[k * n + j] * mk, ((hi >> j) & 1) ? R(0.5) : R(-0.5), acc);
      s_dt[k - kLowBits] = acc;
    }
    __syncthreads();
    const uint32_t row = hi | (uint32_t)t;
    Acc<R, 1> acc;
    acc_zero(acc);
    const Cx<R> *own = v + (size_t)row * P.K;
    if (W.diag) {
      R diag = dlow;
      for (int k = 0; k < n - kLowBits; k++) diag += s_dt[k];
#pragma unroll
      for (int i = 0; i < kLowBits; i++) diag = fma(((t >> i) & 1) ? R(0.5) : R(-0.5), s_phi[i], diag);
      mac_real(acc, diag, own);
    }
    for (uint32_t sm = W.smask; sm; sm &= sm - 1u) {
      const int k = __builtin_ctz(sm);
      const int b = (row >> k) & 1;
      const Cx<R> a1 = s_hf[2 * k + b], a2 = s_fh[2 * k + b];
      const Cx<R> a3 = tb.lowf[(k * 2 + b) * 256 + t];
      const Cx<R> c{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im};
      mac(acc, c, v + (size_t)(row ^ (1u << k)) * P.K);
    }
    // pairs inside the lanes' bits: coefficient and partner lane from t
    const size_t tk = (size_t)t * P.K;
    const Cx<R> *vt = v + (size_t)hi * P.K;  // this tile (uniform)
#pragma unroll 4
    for (int e = 0; e < W.np_ll; e++) {
      const int4 q = pl[e];
      const int2 ij = make_int2(q.y, q.z);
      const int type = (((t >> ij.x) & 1) << 1) | ((t >> ij.y) & 1);
      mac(acc, s_pc[4 * e + type], vt + (size_t)(t ^ ((1 << ij.x) | (1 << ij.y))) * P.K);
    }
    // one lane bit i, one tile bit j: partner tile hi ^ 2^j (uniform), lane t ^ 2^i
    const int e1 = W.np_ll + W.np_lh;
#pragma unroll 4
    for (int e = W.np_ll; e < e1; e++) {
      const int4 q = pl[e];
      const int2 ij = make_int2(q.y, q.z);
      const uint32_t bj = (hi >> ij.y) & 1u;
      const int type = (((t >> ij.x) & 1) << 1) | (int)bj;
      const Cx<R> *vp = v + (size_t)(hi ^ (1u << ij.y)) * P.K;
      mac(acc, s_pc[4 * e + type], vp + (size_t)(t ^ (1 << ij.x)) * P.K);
    }
    // both tile bits: the coefficient and the partner tile are uniform
#pragma unroll 4
    for (int e = e1; e < np; e++) {
      const int4 q = pl[e];
      const int2 ij = make_int2(q.y, q.z);
      const int type = (int)((((hi >> ij.x) & 1u) << 1) | ((hi >> ij.y) & 1u));
      const Cx<R> c = s_pc[4 * e + type];  // same address in every lane (broadcast)
      const Cx<R> *vp = v + (size_t)(hi ^ ((1u << ij.x) | (1u << ij.y))) * P.K;
      mac(acc, c, vp + tk);
    }
    win_store<R, 1>(W, P, row, c0, acc, own, red);
  });
  if (W.last) hv_finish<1>(P, red);
}

// Spin-1/2, N >= 12: the LDS tile kernel (2048-row tiles) walked window by
// window over the tile bits >= 11, terms restricted to the pass: pairs inside
// the tile (first pass), then for every outer site a of xmask the partner tile
// (tile with bit a flipped) staged once for the single flip of a and the mixed
// pairs (i < 11, a), then pairs of two outer sites read straight from global
// memory (L2-resident: both sites lie in the window).
//
// Thread layout: a block of 256 G threads holds one tile; thread t = 256 g + l
// owns the Q = 8 / G rows q 256 + tq, tq = g Q 256 + l: lane part l (row bits
// 0..7) and slots s = g Q + q (row bits 8..10; g gives the high slot bits).  The
// tile's LDS bounds the blocks per CU, so G > 1 puts more waves on the same LDS.
// g is uniform over a wave.  In the slot-bit terms the flipped slot bit SB is a
// compile-time constant: a flip of a q bit moves to another of the thread's
// rows, a flip of a g bit to the same row of another group.
template <typename R>
__device__ __forceinline__ void fma_cx(Cx<R> &a, const Cx<R> &c, const Cx<R> &x) {
  a.re = fma(c.re, x.re, fma(-c.im, x.im, a.re));
  a.im = fma(c.re, x.im, fma(c.im, x.re, a.im));
}

// For slot bit SB and Q rows per thread: the flip of the row index q, the flip
// of the thread offset tq, and the bit's value for row q of group gg.
template <int SB, int Q>
__device__ __forceinline__ constexpr int slot_qflip() { return (1 << SB) < Q ? (1 << SB) : 0; }
template <int SB, int Q>
__device__ __forceinline__ constexpr int slot_tflip() { return (1 << SB) < Q ? 0 : ((1 << SB) / Q) * Q * kBlock; }
template <int SB, int Q>
__device__ __forceinline__ int slot_bit(int q, int gg) {
  if constexpr ((1 << SB) < Q) return (q >> SB) & 1;
  else return (gg >> (SB - (Q == 8 ? 3 : Q == 4 ? 2 : Q == 2 ? 1 : 0))) & 1;
}

// acc[q] += (bit SB of slot ? c1 : c0) * src[row q of offset tq with slot bit SB flipped]
template <int SB, int G, typename R>
__device__ __forceinline__ void slot_flip(Cx<R> (&acc)[kRowsPerThread / G], const Cx<R> *src, int gg, int tq,
                                          Cx<R> c0, Cx<R> c1) {
  constexpr int Q = kRowsPerThread / G;
  const int tp = tq ^ slot_tflip<SB, Q>();
#pragma unroll
  for (int q = 0; q < Q; q++)
    fma_cx(acc[q], slot_bit<SB, Q>(q, gg) ? c1 : c0, src[(q ^ slot_qflip<SB, Q>()) * kBlock + tp]);
}

// two slot bits A < B: acc[q] += cp[(bit A) << 1 | bit B] * src[row with both flipped]
template <int A, int B, int G, typename R>
__device__ __forceinline__ void slot_pair(Cx<R> (&acc)[kRowsPerThread / G], const Cx<R> *src, int gg, int tq,
                                          const Cx<R> *cp) {
  constexpr int Q = kRowsPerThread / G;
  const Cx<R> c00 = cp[0], c01 = cp[1], c10 = cp[2], c11 = cp[3];
  const int tp = tq ^ slot_tflip<A, Q>() ^ slot_tflip<B, Q>();
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int ba = slot_bit<A, Q>(q, gg), bb = slot_bit<B, Q>(q, gg);  // selects, no indexed array
    fma_cx(acc[q], ba ? (bb ? c11 : c10) : (bb ? c01 : c00),
           src[(q ^ slot_qflip<A, Q>() ^ slot_qflip<B, Q>()) * kBlock + tp]);
  }
}

template <int G, typename R>
__device__ __forceinline__ void slot_flip_any(int sb, Cx<R> (&acc)[kRowsPerThread / G], const Cx<R> *src, int gg,
                                              int tq, Cx<R> c0, Cx<R> c1) {
  if (sb == 0) slot_flip<0, G>(acc, src, gg, tq, c0, c1);
  else if (sb == 1) slot_flip<1, G>(acc, src, gg, tq, c0, c1);
  else slot_flip<2, G>(acc, src, gg, tq, c0, c1);
}

// One mixed pair (i < 11, outer site a) read from the staged partner tile:
// acc[q] += (bit i of the row ? chi : clo) * part[row with bit i flipped].
template <int G, typename R>
__device__ __forceinline__ void mixed_pair(Cx<R> (&acc)[kRowsPerThread / G], const Cx<R> *part, int gg, int tq,
                                           int l, int i, Cx<R> clo, Cx<R> chi) {
  constexpr int Q = kRowsPerThread / G;
  if (i < kLowBits) {
    const Cx<R> c = ((l >> i) & 1) ? chi : clo;
    const int tf = tq ^ (1 << i);
#pragma unroll
    for (int q = 0; q < Q; q++) fma_cx(acc[q], c, part[q * kBlock + tf]);
  } else {
    slot_flip_any<G>(i - kLowBits, acc, part, gg, tq, clo, chi);
  }
}

// NB pairs of two outer sites: every partner tile row is loaded before the
// first FMA, so NB Q loads per lane are in flight at once.  The FMAs run in
// pair order, as a one-at-a-time loop would.
template <int NB, int G, typename R>
__device__ __forceinline__ void outer_pairs(Cx<R> (&acc)[kRowsPerThread / G], const int4 *__restrict__ pe,
                                            uint32_t base, const Cx<R> *__restrict__ pc, const Cx<R> *v,
                                            size_t K, size_t tk) {
  constexpr int Q = kRowsPerThread / G;
  Cx<R> x[NB][Q];
  Cx<R> c[NB];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int4 e = pe[b];
    c[b] = pc[4 * b + ((((base >> e.y) & 1) << 1) | ((base >> e.z) & 1))];
    const Cx<R> *vb = v + (size_t)(base ^ (1u << e.y) ^ (1u << e.z)) * K;
#pragma unroll
    for (int q = 0; q < Q; q++) x[b][q] = vb[(size_t)q * kBlock * K + tk];
  }
#pragma unroll
  for (int b = 0; b < NB; b++)
#pragma unroll
    for (int q = 0; q < Q; q++) fma_cx(acc[q], c[b], x[b][q]);
}

// plist and pcl (the spin-1/2 pair coefficients in plist order: entry e's four
// at pcl[4 e]) are read at wave-uniform addresses; as __restrict__ kernel
// arguments they are known not to be written by the kernel's stores, so these
// reads go through the scalar data cache instead of becoming vector loads with
// a full wait in every trip.  Addressed by list position, an entry's
// coefficients are fetched together with the entry instead of after it.
template <typename R, int G>
__global__ __launch_bounds__(kBlock * G, 2 * G) void hv_tile_win(HamGeom g, DevTables<R> tb, WinPass W,
                                                             const int4 *__restrict__ plist,
                                                             const Cx<R> *__restrict__ pcl, HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = kBlock * G;           // threads per block
  constexpr int S = kRowsPerThread;        // slots per tile (row bits 8..10)
  constexpr int Q = S / G;                 // rows per thread
  constexpr int NB = 2;                    // outer pairs per batch
  const int n = g.n, n_in = W.np_ll, e_out = W.np_ll + W.np_lh, np = W.np;
  Cx<R> *own = reinterpret_cast<Cx<R> *>(smem);   // [2048]
  Cx<R> *part = own + kTileRows;                  // [2048]
  Cx<R> *s_pc = part + kTileRows;                 // [n_in][4]
  Cx<R> *s_fmh = s_pc + 4 * n_in;                 // [n][2][S]
  Cx<R> *s_hf = s_fmh + 2 * S * n;                // [n][2]
  R *s_hd = reinterpret_cast<R *>(s_hf + 2 * n);  // [n][2]
  R *s_dmh = s_hd + 2 * n;                        // [S]
  R *s_phi = s_dmh + S;                           // [8][S]
  R *s_term = s_phi + 8 * S;                      // [32][S]
  const int t = threadIdx.x;
  const int l = t & (kBlock - 1);
  const int gg = G == 1 ? 0 : __builtin_amdgcn_readfirstlane(t >> 8);
  const int tq = gg * Q * kBlock + l;  // the thread's row offset in the tile for q = 0
  const int c0 = blockIdx.y;
  const int K = P.K;
  const int4 *pl = plist + W.p0;
  const Cx<R> *__restrict__ pch = pcl + 4 * (size_t)W.p0;  // the pass's entries
  for (int i = t; i < 4 * n_in; i += NT) s_pc[i] = pch[i];
  for (int i = t; i < 2 * n; i += NT) {
    s_hf[i] = tb.hflip[i];
    s_hd[i] = tb.hdiag[(i >> 1) * 16 + (i & 1)];
  }
  __syncthreads();
  R dlow = 0;
  if (W.diag) {
    for (int k = 0; k < kLowBits; k++) dlow += s_hd[2 * k + ((l >> k) & 1)];
    for (int p = 0; p < g.npair; p++) {
      const int2 ij = tb.pij[p];
      if (ij.y >= kLowBits) continue;
      dlow = fma(tb.pzz[p], (((l >> ij.x) ^ (l >> ij.y)) & 1) ? R(-0.25) : R(0.25), dlow);
    }
  }
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v);
  const bool zf = W.smask != 0u;
  const int nsm = __builtin_popcount(W.smask);
  double red[3][1] = {{0.0}, {0.0}, {0.0}};
  const size_t tk = (size_t)tq * K;  // thread offset; the tile bases below are uniform
  constexpr size_t QS = (size_t)kBlock;  // row step between a thread's rows

  win_walk(W, [&](uint32_t win, uint32_t item) {
    const uint32_t base = __builtin_amdgcn_readfirstlane(scatter_bits(item, W.emask) | scatter_bits(win, W.omask));
    __syncthreads();
    {
      const Cx<R> *vb = v + (size_t)base * K + c0;
#pragma unroll
      for (int q = 0; q < Q; q++) own[q * kBlock + tq] = vb[q * QS * K + tk];
    }
    // per-tile uniform parts: rows of slot s have bits 8..10 = s and bits >= 11 = base;
    // the z-field part only for the sites whose single flips this pass applies
    if (zf)
      for (int e = t; e < 2 * S * nsm; e += NT) {
        const int r = e / (2 * S), sel = (e / S) & 1, sl = e % S;
        uint32_t m = W.smask;
        for (int u = 0; u < r; u++) m &= m - 1u;
        const int k = __builtin_ctz(m);
        const uint32_t rb = base | ((uint32_t)sl << kLowBits);
        R fr = 0, fi = 0;
        // four sites per trip, their loads issued together (a weight of zero
        // stands for j = k and for j >= n)
        for (int j0 = kLowBits; j0 < n; j0 += 4) {
          Cx<R> c[4];
          R mj[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int j = j0 + u < n ? j0 + u : n - 1;
            c[u] = tb.cz_half[(k * n + j) * 2 + sel];
            mj[u] = (j0 + u < n && j != k) ? (((rb >> j) & 1) ? R(0.5) : R(-0.5)) : R(0);
          }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            fr = fma(c[u].re, mj[u], fr);
            fi = fma(c[u].im, mj[u], fi);
          }
        }
        s_fmh[(k * 2 + sel) * S + sl] = Cx<R>{fr, fi};
      }
    if (W.diag) {
      if (t < 24 * S) {
        const int k = kLowBits + t / S, sl = t % S;
        if (k < n) {
          const uint32_t rb = base | ((uint32_t)sl << kLowBits);
          const R mk = ((rb >> k) & 1) ? R(0.5) : R(-0.5);
          R acc = s_hd[2 * k + ((rb >> k) & 1)];
          for (int j0 = k + 1; j0 < n; j0 += 4) {  // loads four at a time; weight 0 past n
            R z[4], mj[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
              const int j = j0 + u < n ? j0 + u : n - 1;
              z[u] = tb.zz[k * n + j];
              mj[u] = j0 + u < n ? (((rb >> j) & 1) ? R(0.5) : R(-0.5)) : R(0);
            }
#pragma unroll
            for (int u = 0; u < 4; u++) acc = fma(z[u] * mk, mj[u], acc);
          }
          s_term[(k - kLowBits) * S + sl] = acc;
        }
      } else if (t < 24 * S + 8 * S) {
        const int i = (t - 24 * S) / S, sl = (t - 24 * S) % S;
        const uint32_t rb = base | ((uint32_t)sl << kLowBits);
        R ph = 0;
        for (int j0 = kLowBits; j0 < n; j0 += 4) {
          R z[4], mj[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int j = j0 + u < n ? j0 + u : n - 1;
            z[u] = tb.zz[i * n + j];
            mj[u] = j0 + u < n ? (((rb >> j) & 1) ? R(0.5) : R(-0.5)) : R(0);
          }
#pragma unroll
          for (int u = 0; u < 4; u++) ph = fma(z[u], mj[u], ph);
        }
        s_phi[i * S + sl] = ph;
      }
    }
    __syncthreads();
    if (W.diag && t < S) {
      R d = 0;
      for (int k = kLowBits; k < n; k++) d += s_term[(k - kLowBits) * S + t];
      s_dmh[t] = d;
    }
    __syncthreads();

    Cx<R> acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      acc[q] = Cx<R>{0, 0};
      if (W.diag) {
        const int sl = gg * Q + q;
        R dg = dlow + s_dmh[sl];
#pragma unroll
        for (int i = 0; i < kLowBits; i++) dg = fma(((l >> i) & 1) ? R(0.5) : R(-0.5), s_phi[i * S + sl], dg);
        const Cx<R> x = own[q * kBlock + tq];
        acc[q] = Cx<R>{dg * x.re, dg * x.im};
      }
    }
    // single flips of tile sites
#pragma unroll 1
    for (uint32_t sm = W.smask & ((1u << kTileBits) - 1u); sm; sm &= sm - 1u) {
      const int k = __builtin_ctz(sm);
      if (k < kLowBits) {  // lane bit: the row bit and the lane part of F do not depend on q
        const int b = (l >> k) & 1;
        const Cx<R> a1 = s_hf[2 * k + b], a2 = tb.lowf[(k * 2 + b) * 256 + l];
        const int tf = tq ^ (1 << k);
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const Cx<R> a3 = s_fmh[(k * 2 + b) * S + gg * Q + q];
          fma_cx(acc[q], Cx<R>{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im}, own[q * kBlock + tf]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const int sl = gg * Q + q;
          const int b = (sl >> (k - kLowBits)) & 1;
          const Cx<R> a1 = s_hf[2 * k + b], a2 = tb.lowf[(k * 2 + b) * 256 + l], a3 = s_fmh[(k * 2 + b) * S + sl];
          fma_cx(acc[q], Cx<R>{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im},
                 own[(sl ^ (1 << (k - kLowBits))) * kBlock + l]);
        }
      }
    }
    // pairs inside the tile (i < j < 11); two consecutive pairs of two lane
    // bits go together, so that the second pair's LDS reads are in flight
    // during the first pair's FMAs (the accumulation order is unchanged)
#pragma unroll 1
    for (int e = 0; e < n_in; e++) {
      const int4 ij = pl[e];
      const int i = ij.y, j = ij.z;
      if (j < kLowBits && e + 1 < n_in && pl[e + 1].z < kLowBits) {
        const int4 ij2 = pl[e + 1];
        const Cx<R> c = s_pc[4 * e + ((((l >> i) & 1) << 1) | ((l >> j) & 1))];
        const Cx<R> c2 = s_pc[4 * (e + 1) + ((((l >> ij2.y) & 1) << 1) | ((l >> ij2.z) & 1))];
        const int tf = tq ^ ((1 << i) | (1 << j)), tf2 = tq ^ ((1 << ij2.y) | (1 << ij2.z));
        Cx<R> x[Q], x2[Q];
#pragma unroll
        for (int q = 0; q < Q; q++) {
          x[q] = own[q * kBlock + tf];
          x2[q] = own[q * kBlock + tf2];
        }
#pragma unroll
        for (int q = 0; q < Q; q++) {
          fma_cx(acc[q], c, x[q]);
          fma_cx(acc[q], c2, x2[q]);
        }
        e++;
      } else if (j < kLowBits) {  // two lane bits: one coefficient per thread, partner t ^ mask
        const Cx<R> c = s_pc[4 * e + ((((l >> i) & 1) << 1) | ((l >> j) & 1))];
        const int tf = tq ^ ((1 << i) | (1 << j));
#pragma unroll
        for (int q = 0; q < Q; q++) fma_cx(acc[q], c, own[q * kBlock + tf]);
      } else if (i < kLowBits) {  // lane bit i, slot bit j
        const int bi = (l >> i) & 1;
        slot_flip_any<G>(j - kLowBits, acc, own, gg, tq ^ (1 << i), s_pc[4 * e + (bi << 1)],
                         s_pc[4 * e + (bi << 1) + 1]);
      } else {  // two slot bits
        const Cx<R> *cp = s_pc + 4 * e;
        if (i == kLowBits && j == kLowBits + 1) slot_pair<0, 1, G>(acc, own, gg, tq, cp);
        else if (i == kLowBits) slot_pair<0, 2, G>(acc, own, gg, tq, cp);
        else slot_pair<1, 2, G>(acc, own, gg, tq, cp);
      }
    }
    // outer sites with work in this pass: partner tile staged once; the next
    // site's tile is loaded into registers while the current one is in use
    int e = n_in;
    uint32_t xm = W.xmask;
    // (with no next site the own tile is loaded instead, so that the prefetch
    // registers are always defined)
    R nre[Q], nim[Q];
    {
      const uint32_t nb = xm ? (base ^ (1u << __builtin_ctz(xm))) : base;
      const Cx<R> *vb = v + (size_t)nb * K + c0;
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const Cx<R> x = vb[q * QS * K + tk];
        nre[q] = x.re;
        nim[q] = x.im;
      }
    }
#pragma unroll 1
    while (xm) {
      const int a = __builtin_ctz(xm);
      xm &= xm - 1u;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; q++) part[q * kBlock + tq] = Cx<R>{nre[q], nim[q]};
      {
        const uint32_t nb = xm ? (base ^ (1u << __builtin_ctz(xm))) : base;
        const Cx<R> *vb = v + (size_t)nb * K + c0;
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const Cx<R> x = vb[q * QS * K + tk];
          nre[q] = x.re;
          nim[q] = x.im;
        }
      }
      __syncthreads();
      const int ba = (base >> a) & 1;
      if ((W.smask >> a) & 1u) {
        const Cx<R> a1 = s_hf[2 * a + ba], a2 = tb.lowf[(a * 2 + ba) * 256 + l];
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const Cx<R> a3 = s_fmh[(a * 2 + ba) * S + gg * Q + q];
          fma_cx(acc[q], Cx<R>{a1.re + a2.re + a3.re, a1.im + a2.im + a3.im}, part[q * kBlock + tq]);
        }
      }
      // the mixed pairs (i < 11, a): a run of entries whose first one gives
      // the run's end, taken two at a time, so that both entries and their
      // coefficients are fetched with no wait in between
      int eend = e;
      if (e < e_out) {
        const int4 p0 = pl[e];
        if (p0.z == a) eend = p0.w;
      }
      eend = __builtin_amdgcn_readfirstlane(eend);
#pragma unroll 1
      for (; e + 1 < eend; e += 2) {
        e = __builtin_amdgcn_readfirstlane(e);
        const int i = pl[e].y, i2 = pl[e + 1].y;
        const Cx<R> clo = pch[4 * e + ba], chi = pch[4 * e + 2 + ba];
        const Cx<R> clo2 = pch[4 * e + 4 + ba], chi2 = pch[4 * e + 6 + ba];
        if (i < kLowBits && i2 < kLowBits) {
          // two lane-bit pairs: the second one's LDS reads go out with the first's
          const Cx<R> c = ((l >> i) & 1) ? chi : clo, c2 = ((l >> i2) & 1) ? chi2 : clo2;
          const int tf = tq ^ (1 << i), tf2 = tq ^ (1 << i2);
          Cx<R> x[Q], x2[Q];
#pragma unroll
          for (int q = 0; q < Q; q++) {
            x[q] = part[q * kBlock + tf];
            x2[q] = part[q * kBlock + tf2];
          }
#pragma unroll
          for (int q = 0; q < Q; q++) {
            fma_cx(acc[q], c, x[q]);
            fma_cx(acc[q], c2, x2[q]);
          }
        } else {
          mixed_pair<G>(acc, part, gg, tq, l, i, clo, chi);
          mixed_pair<G>(acc, part, gg, tq, l, i2, clo2, chi2);
        }
      }
      if (e < eend) {
        e = __builtin_amdgcn_readfirstlane(e);
        mixed_pair<G>(acc, part, gg, tq, l, pl[e].y, pch[4 * e + ba], pch[4 * e + 2 + ba]);
        e++;
      }
    }
    // the earlier passes' partial sums of these rows, loaded now so that they
    // arrive during the outer pairs
    Cx<R> wprev[Q];
    Cx<R> *wt = reinterpret_cast<Cx<R> *>(P.w) + (size_t)base * K + c0;
#pragma unroll
    for (int q = 0; q < Q; q++) wprev[q] = W.first ? Cx<R>{0, 0} : ld_stream(wt + q * QS * K + tk);
    // pairs of two outer sites, NB at a time
    {
      const Cx<R> *vc = v + c0;
      int e2 = e_out;
#pragma unroll 1
      for (; e2 + NB <= np; e2 += NB) outer_pairs<NB, G>(acc, pl + e2, base, pch + 4 * e2, vc, (size_t)K, tk);
      if (e2 < np) outer_pairs<1, G>(acc, pl + e2, base, pch + 4 * e2, vc, (size_t)K, tk);
    }
#pragma unroll
    for (int q = 0; q < Q; q++) {
      Acc<R, 1> a1;
      a1.re[0] = acc[q].re + wprev[q].re;
      a1.im[0] = acc[q].im + wprev[q].im;
      const uint32_t row = base + q * kBlock + tq;
      if (W.last) hv_epilogue<R, 1, true>(P, row, c0, a1, own + q * kBlock + tq, red);
      else st_stream(wt + q * QS * K + tk, Cx<R>{a1.re[0], a1.im[0]});
    }
  });
  if (W.last) hv_finish<1, NT>(P, red);
}

// General mixed radix: one 256-row slice of a window per item; the window's
// rows are enumerated with the window sites' digits (lowest site fastest), the
// outer digits come from the window index.
// The tables read at wave-uniform addresses in loops (pair coefficients, the
// z-field coupling tables, the diagonal pair list) come in as __restrict__
// kernel arguments as well: the kernel's stores cannot alias them, so those
// reads go through the scalar data cache instead of vector loads with a full
// wait each.
template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void hv_gen_win(HamGeom g, DevTables<R> tb, WinPass W,
                                                     const int4 *__restrict__ plist,
                                                     const Cx<R> *__restrict__ pcg, const Cx<R> *__restrict__ czp,
                                                     const Cx<R> *__restrict__ czm, const int2 *__restrict__ pij,
                                                     const R *__restrict__ pzz, HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = g.n;
  Cx<R> *s_hoff = reinterpret_cast<Cx<R> *>(smem);  // [n][4][16]
  R *s_hd = reinterpret_cast<R *>(s_hoff + n * 64);  // [n][16]
  R *s_gp = s_hd + n * 16;
  R *s_gm = s_gp + n * 16;
  R *s_m = s_gm + n * 16;
  const int t = threadIdx.x;
  const int c0 = blockIdx.y * KC;
  for (int i = t; i < n * 64; i += kBlock) s_hoff[i] = tb.hoff[i];
  for (int i = t; i < n * 16; i += kBlock) {
    s_hd[i] = tb.hdiag[i];
    s_gp[i] = tb.gp[i];
    s_gm[i] = tb.gm[i];
    s_m[i] = tb.mval[i];
  }
  __syncthreads();
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v) + c0;
  const int4 *pl = plist + W.p0;
  double red[3][KC];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int q = 0; q < KC; q++) red[a][q] = 0.0;

  win_walk(W, [&](uint32_t win, uint32_t item) {
    const uint32_t iw = item * kBlock + (uint32_t)t;
    if (iw >= W.wsize) return;
    // outer digits from the window index (uniform), window digits from iw
    uint64_t dlo = 0, dhi = 0;
    uint32_t row = 0;
    auto put = [&](int k, uint32_t d) {
      row += d * g.stride[k];
      if (k < 16) dlo |= (uint64_t)d << (4 * k);
      else dhi |= (uint64_t)d << (4 * (k - 16));
    };
    {
      uint32_t rem = win;
      for (int i = 0; i < W.ni; i++) {
        const uint32_t r = (uint32_t)W.irad[i], q = rem / r;
        put(W.inact[i], rem - q * r);
        rem = q;
      }
      rem = iw;
      for (int a = 0; a < W.na; a++) {
        const uint32_t r = (uint32_t)W.wrad[a], q = rem / r;
        put(W.act[a], rem - q * r);
        rem = q;
      }
    }
    auto digit = [&](int k) -> int {
      return (int)(((k < 16) ? (dlo >> (4 * k)) : (dhi >> (4 * (k - 16)))) & 15u);
    };
    Acc<R, KC> acc;
    acc_zero(acc);
    const Cx<R> *own = v + (size_t)row * P.K;
    if (W.diag) {
      R diag = 0;
      for (int k = 0; k < n; k++) diag += s_hd[k * 16 + digit(k)];
      for (int p = 0; p < g.npair; p++) {
        const int2 ij = pij[p];
        diag = fma(pzz[p], s_m[ij.x * 16 + digit(ij.x)] * s_m[ij.y * 16 + digit(ij.y)], diag);
      }
      mac_real(acc, diag, own);
    }
    for (uint32_t sm = W.smask; sm; sm &= sm - 1u) {
      const int k = __builtin_ctz(sm);
      const int dk = digit(k), rk = g.radix[k];
      const uint32_t st = g.stride[k];
      R fpr = 0, fpi = 0, fmr = 0, fmi = 0;
      if (g.has_z) {
        for (int l = 0; l < n; l++) {
          if (l == k) continue;
          const R ml = s_m[l * 16 + digit(l)];
          const Cx<R> cp = czp[k * n + l], cm = czm[k * n + l];
          fpr = fma(cp.re, ml, fpr);
          fpi = fma(cp.im, ml, fpi);
          fmr = fma(cm.re, ml, fmr);
          fmi = fma(cm.im, ml, fmi);
        }
      }
#pragma unroll
      for (int di = 0; di < 4; di++) {
        const int D = (di < 2) ? di - 2 : di - 1;  // -2,-1,+1,+2
        const int nd = dk + D;
        if (nd < 0 || nd >= rk) continue;
        Cx<R> c = s_hoff[(k * 4 + di) * 16 + dk];
        if (D == -1) {
          const R gg = s_gp[k * 16 + dk];
          c.re = fma(gg, fpr, c.re);
          c.im = fma(gg, fpi, c.im);
        } else if (D == 1) {
          const R gg = s_gm[k * 16 + dk];
          c.re = fma(gg, fmr, c.re);
          c.im = fma(gg, fmi, c.im);
        }
        mac(acc, c, v + (size_t)(row + (uint32_t)(D * (int)st)) * P.K);
      }
    }
    for (int e = 0; e < W.np; e++) {
      const int4 pe = pl[e];
      const int pi_ = pe.y, pj_ = pe.z;
      const int di = digit(pi_), dj = digit(pj_);
      const int ri = g.radix[pi_], rj = g.radix[pj_];
      const uint32_t si = g.stride[pi_], sj = g.stride[pj_];
      const R gpi = s_gp[pi_ * 16 + di], gmi = s_gm[pi_ * 16 + di];
      const R gpj = s_gp[pj_ * 16 + dj], gmj = s_gm[pj_ * 16 + dj];
      const Cx<R> *pc = pcg + 4 * pe.x;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const Cx<R> cq = pc[q];
        if (cq.re == R(0) && cq.im == R(0)) continue;
        const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;  // '-' ladder on site i / j
        const bool vi = im_ ? (di <= ri - 2) : (di >= 1);
        const bool vj = jm ? (dj <= rj - 2) : (dj >= 1);
        if (!(vi && vj)) continue;
        const R f = (im_ ? gmi : gpi) * (jm ? gmj : gpj);
        const uint32_t partner = row + (im_ ? si : (uint32_t)(-(int)si)) + (jm ? sj : (uint32_t)(-(int)sj));
        mac(acc, Cx<R>{cq.re * f, cq.im * f}, v + (size_t)partner * P.K);
      }
    }
    win_store<R, KC>(W, P, row, c0, acc, own, red);
  });
  if (W.last) hv_finish<KC>(P, red);
}

static bool tile_ok(const HamGeom &g, int K) { return g.spin_half && g.n >= kTileBits && K == 1; }
static thread_local int g_variant = 0;  // variant of the launch in progress (0 = heuristic)
static bool use_tile(const HamGeom &g, int K) { return tile_ok(g, K) && (g_variant == 0 || g_variant == 3); }

// Windowed passes pay off once the vector leaves the caches.
static bool use_passes(const HamGeom &g, int K, int variant) {
  if (variant == 1 || variant == 3) return false;
  if (variant == 2) return K == 1;
  return K == 1 && g.dim >= (1u << 20) && !tile_ok(g, K);
}

// Rows per thread of a pass: 16 (4096-row windows), or 32 for complex64 windows
// above 4096 rows (a 64 KB LDS window holds 8192 of them).  Windows of general
// radix are usually smaller (5^5 = 3125 rows): with 16 rows per thread most
// lanes stay busy.
template <typename R>
static int pass_rpt(const PassDesc &D) {
  return (sizeof(R) == 4 && D.wsize > 16u * kBlock) ? 32 : 16;
}

static bool pass_pow2(const PassDesc &D) { return D.pow2 && D.na >= kLowBits && D.na - kLowBits <= 5; }

template <typename R>
static size_t pass_rec_len(const PassDesc &D) {
  const bool p2 = pass_pow2(D);
  if (pass_rpt<R>(D) == 32) return p2 ? PassRec<R, true, 32>::kLen : PassRec<R, false, 32>::kLen;
  return p2 ? PassRec<R, true, 16>::kLen : PassRec<R, false, 16>::kLen;
}

template <typename R>
static size_t pass_smem(const PassDesc &D) {
  size_t b = sizeof(Cx<R>) * ((size_t)D.wsize + 4 * (size_t)D.npp + kMaxPassSingles * 64) +
             sizeof(R) * (pass_rec_len<R>(D) + 64 * (size_t)D.na) + sizeof(int4) * (size_t)D.npp;
  b += sizeof(int) * ((size_t)D.npp + 1);
  b = (b + 15) & ~size_t(15);
  if (!pass_pow2(D) && sizeof(R) == 8) b += sizeof(Cx<R>) * (size_t)D.ctab;
  return b;
}

template <typename R, bool POW2, int RPT>
static void launch_pass_t(const DevHam &dh, const DevTables<R> &tb, const PassPlan &plan, size_t ps,
                          const HvParams &P, dim3 grid, size_t sm, hipStream_t s) {
  static size_t granted = 0;
  if (sm > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&hv_pass<R, POW2, RPT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    granted = sm;
  }
  const unsigned char *blk = reinterpret_cast<const unsigned char *>(plan.rec_block);
  hipLaunchKernelGGL((hv_pass<R, POW2, RPT>), grid, dim3(kBlock), sm, s, dh.geom, tb, plan.passes[ps],
                     plan.d_pairs, reinterpret_cast<const R *>(blk + plan.rec_off[ps]),
                     reinterpret_cast<const uint32_t *>(blk + plan.base_off[ps]), blk + plan.lane_off[ps],
                     tb.czp, tb.czm, tb.zz, P);
}

template <typename R>
static int launch_passes(const DevHam &dh, const DevTables<R> &tb, const PassPlan &plan,
                         const HvParams &P, int gy, int cap, unsigned *last_gx, hipStream_t s) {
  if (!plan.rec_block) return FTLM_EINVAL;
  for (size_t ps = 0; ps < plan.passes.size(); ps++) {
    const PassDesc &D = plan.passes[ps];
    const int rpt = pass_rpt<R>(D);
    if (D.wsize > (uint32_t)(kBlock * rpt) || D.nsing > kMaxPassSingles) return FTLM_ERANGE;
    const size_t sm = pass_smem<R>(D);
    if (sm > 160 * 1024) return FTLM_ERANGE;
    const int gx = (int)(D.nwin < (uint32_t)cap ? D.nwin : (uint32_t)cap);
    HvParams Pp = P;
    if (!D.last) Pp.lanczos = 0;
    const dim3 grid(gx, gy);
    if (rpt == 32) {
      if (pass_pow2(D)) launch_pass_t<R, true, 32>(dh, tb, plan, ps, Pp, grid, sm, s);
      else launch_pass_t<R, false, 32>(dh, tb, plan, ps, Pp, grid, sm, s);
    } else {
      if (pass_pow2(D)) launch_pass_t<R, true, 16>(dh, tb, plan, ps, Pp, grid, sm, s);
      else launch_pass_t<R, false, 16>(dh, tb, plan, ps, Pp, grid, sm, s);
    }
    *last_gx = (unsigned)gx;
  }
  return FTLM_OK;
}

template <typename R, int RPT>
static void launch_records(const DevHam &dh, const DevTables<R> &tb, const PassPlan &plan, size_t ps) {
  unsigned char *blk = reinterpret_cast<unsigned char *>(plan.rec_block);
  const PassDesc &D = plan.passes[ps];
  const uint32_t gx = D.nwin < 65536u ? D.nwin : 65536u;
  if (pass_pow2(D))
    hipLaunchKernelGGL((pass_record_kernel<R, true, RPT>), dim3(gx), dim3(kBlock), 0, 0, dh.geom, tb, D,
                       reinterpret_cast<R *>(blk + plan.rec_off[ps]),
                       reinterpret_cast<uint32_t *>(blk + plan.base_off[ps]), blk + plan.lane_off[ps]);
  else
    hipLaunchKernelGGL((pass_record_kernel<R, false, RPT>), dim3(gx), dim3(kBlock), 0, 0, dh.geom, tb, D,
                       reinterpret_cast<R *>(blk + plan.rec_off[ps]),
                       reinterpret_cast<uint32_t *>(blk + plan.base_off[ps]), blk + plan.lane_off[ps]);
}

template <typename R>
static int build_records_t(DevHam &dh, const DevTables<R> &tb, PassPlan &plan) {
  for (size_t ps = 0; ps < plan.passes.size(); ps++) {
    if (pass_rpt<R>(plan.passes[ps]) == 32) launch_records<R, 32>(dh, tb, plan, ps);
    else launch_records<R, 16>(dh, tb, plan, ps);
    if (hipGetLastError() != hipSuccess) return FTLM_EHIP;
  }
  return FTLM_OK;
}

template <typename R>
static size_t layout_records(PassPlan &plan) {
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return o;
  };
  plan.rec_off.assign(plan.passes.size(), 0);
  plan.base_off.assign(plan.passes.size(), 0);
  plan.lane_off.assign(plan.passes.size(), 0);
  for (size_t ps = 0; ps < plan.passes.size(); ps++) {
    const PassDesc &D = plan.passes[ps];
    plan.rec_off[ps] = take(sizeof(R) * pass_rec_len<R>(D) * (size_t)D.nwin);
    plan.base_off[ps] = take(sizeof(uint32_t) * (size_t)D.nwin);
    plan.lane_off[ps] = take(sizeof(Cx<R>) * kMaxPassSingles * 2 * 256 + sizeof(R) * 256);
  }
  return (off + 255) & ~size_t(255);
}

void free_pass_records(DevHam &dh) {
  for (PassPlan *pl : {&dh.plan64, &dh.plan32}) {
    if (pl->rec_block) (void)hipFree(pl->rec_block);
    pl->rec_block = nullptr;
    pl->rec_bytes = 0;
  }
}

int build_pass_records(DevHam &dh, std::string &err) {
  struct Item {
    PassPlan *pl;
    bool f32;
  } items[2] = {{&dh.plan64, false}, {&dh.plan32, true}};
  for (auto &it : items) {
    const size_t bytes = it.f32 ? layout_records<float>(*it.pl) : layout_records<double>(*it.pl);
    if (it.pl->rec_block && it.pl->rec_bytes != bytes) {
      (void)hipFree(it.pl->rec_block);
      it.pl->rec_block = nullptr;
    }
    if (!it.pl->rec_block) {
      if (hipMalloc(&it.pl->rec_block, bytes) != hipSuccess) {
        it.pl->rec_block = nullptr;
        err = "hipMalloc of pass records failed";
        return FTLM_ENOMEM;
      }
      it.pl->rec_bytes = bytes;
    }
    const int rc = it.f32 ? build_records_t<float>(dh, dh.t32, *it.pl) : build_records_t<double>(dh, dh.t64, *it.pl);
    if (rc) {
      err = "pass record kernel launch failed";
      return rc;
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    err = "pass record kernels failed";
    return FTLM_EHIP;
  }
  return FTLM_OK;
}

template <typename R>
static size_t hv_tile_smem(const HamGeom &g) {
  return sizeof(Cx<R>) * (2 * (size_t)kTileRows + 4 * (size_t)g.n_ll + 2 * kRowsPerThread * g.n + 2 * g.n) +
         sizeof(R) * (2 * g.n + kRowsPerThread + 8 * kRowsPerThread + 32 * kRowsPerThread);
}

template <typename R>
static size_t hv_smem(const HamGeom &g) {
  if (g.spin_half && g.n >= kLowBits)
    return sizeof(Cx<R>) * (4 * (size_t)g.npair + 4 * g.n) + sizeof(R) * (3 * g.n + 8);
  return sizeof(Cx<R>) * 64 * (size_t)g.n + sizeof(R) * 64 * g.n;
}

static int pick_kc(int K, int want) {
  const int opts[4] = {8, 4, 2, 1};
  for (int o : opts)
    if (o <= want && K % o == 0) return o;
  return 1;
}

int hv_grid_blocks(const DevHam &dh, const HvLaunch &L, int *gx, int *gy, int *kc) {
  const HamGeom &g = dh.geom;
  int want = L.kc > 0 ? L.kc : 8;
  int k = pick_kc(L.K, want);
  uint32_t ntile = (g.spin_half && g.n >= kLowBits) ? (g.dim >> kLowBits)
                                                     : (uint32_t)(((uint64_t)g.dim + kBlock - 1) / kBlock);
  if (use_tile(g, L.K)) {
    ntile = g.dim >> kTileBits;
    k = 1;
  }
  if (L.variant == 3 && !tile_ok(g, L.K)) return FTLM_EINVAL;
  int cap = L.grid_cap > 0 ? L.grid_cap : 2048;
  if (L.lz) cap = cap < 2048 ? cap : 2048;  // partials buffer holds 2048 slots per column block
  *gx = (int)(ntile < (uint32_t)cap ? ntile : (uint32_t)cap);
  *gy = L.K / k;
  *kc = k;
  return FTLM_OK;
}

template <typename R, int KC>
static void launch_hv_t(const DevHam &dh, const DevTables<R> &tb, const HvParams &P, dim3 grid,
                        hipStream_t s) {
  const HamGeom &g = dh.geom;
  const size_t sm = hv_smem<R>(g);
  const UniformTabs<R> U = uniform_tabs(tb, false);
  if (g.spin_half && g.n >= kLowBits)
    hipLaunchKernelGGL((hv_half<R, KC>), grid, dim3(kBlock), sm, s, g, tb, U.pij, U.pzz, P);
  else
    hipLaunchKernelGGL((hv_gen<R, KC>), grid, dim3(kBlock), sm, s, g, tb, U.pc, U.czp, U.czm, U.pij, U.pzz, P);
}

template <typename R>
static void launch_hv_r(const DevHam &dh, const DevTables<R> &tb, const HvParams &P, dim3 grid,
                        int kc, hipStream_t s) {
  if (use_tile(dh.geom, P.K)) {
    const size_t sm = hv_tile_smem<R>(dh.geom);
    static size_t granted = 0;  // per instantiation: largest dynamic LDS size requested so far
    if (sm > granted) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&hv_tile<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      granted = sm;
    }
    hipLaunchKernelGGL((hv_tile<R>), grid, dim3(kBlock), sm, s, dh.geom, tb, tb.pij, tb.pc_half, tb.pzz, P);
    return;
  }
  switch (kc) {
    case 8: launch_hv_t<R, 8>(dh, tb, P, grid, s); break;
    case 4: launch_hv_t<R, 4>(dh, tb, P, grid, s); break;
    case 2: launch_hv_t<R, 2>(dh, tb, P, grid, s); break;
    default: launch_hv_t<R, 1>(dh, tb, P, grid, s); break;
  }
}

template <typename R>
static int launch_win(const DevHam &dh, const DevTables<R> &tb, const WinPlan &plan, const HvParams &P,
                      int cap, int kc, unsigned *last_gx, hipStream_t s) {
  const HamGeom &g = dh.geom;
  if (!plan.d_plist || plan.passes.empty()) return FTLM_EINVAL;
  for (const WinPass &W : plan.passes) {
    const uint64_t items = (uint64_t)W.nwin * W.nin;
    uint32_t gx = (uint32_t)(items < (uint64_t)cap ? items : (uint64_t)cap);
    if (W.nwin >= 8 && gx >= 8) gx &= ~7u;
    HvParams Pp = P;
    if (!W.last) Pp.lanczos = 0;
    const dim3 grid(gx, P.K);
    if (g.spin_half) {
      const size_t sm = sizeof(Cx<R>) * (4 * (size_t)W.np + 4 * g.n) + sizeof(R) * (3 * g.n + 8);
      if (sm > 64 * 1024) return FTLM_ERANGE;
      hipLaunchKernelGGL((hv_half_win<R>), grid, dim3(kBlock), sm, s, g, tb, W, plan.d_plist, Pp);
    } else {
      const size_t sm = sizeof(Cx<R>) * 64 * (size_t)g.n + sizeof(R) * 64 * g.n;
      const dim3 gk(gx, P.K / kc);
      const UniformTabs<R> U = uniform_tabs(tb, false);
      switch (kc) {
        case 8: hipLaunchKernelGGL((hv_gen_win<R, 8>), gk, dim3(kBlock), sm, s, g, tb, W, plan.d_plist, U.pc, U.czp, U.czm, U.pij, U.pzz, Pp); break;
        case 4: hipLaunchKernelGGL((hv_gen_win<R, 4>), gk, dim3(kBlock), sm, s, g, tb, W, plan.d_plist, U.pc, U.czp, U.czm, U.pij, U.pzz, Pp); break;
        case 2: hipLaunchKernelGGL((hv_gen_win<R, 2>), gk, dim3(kBlock), sm, s, g, tb, W, plan.d_plist, U.pc, U.czp, U.czm, U.pij, U.pzz, Pp); break;
        default: hipLaunchKernelGGL((hv_gen_win<R, 1>), gk, dim3(kBlock), sm, s, g, tb, W, plan.d_plist, U.pc, U.czp, U.czm, U.pij, U.pzz, Pp); break;
      }
    }
    *last_gx = gx;
  }
  return FTLM_OK;
}

template <typename R>
static size_t hv_tile_win_smem(const HamGeom &g, const WinPass &W) {
  return sizeof(Cx<R>) * (2 * (size_t)kTileRows + 4 * (size_t)W.np_ll + 2 * kRowsPerThread * g.n + 2 * g.n) +
         sizeof(R) * (2 * g.n + kRowsPerThread + 8 * kRowsPerThread + 32 * kRowsPerThread);
}

// Threads per tile-window block: 256 G (G groups of rows on one LDS tile).
// want = 1, 2 or 4 (the tuned choice), else 2 for complex128 (the tile's LDS
// allows two blocks per CU, so every doubling of G doubles the resident waves
// up to 8 per SIMD at G = 4) and 1 for complex64 (four 256-thread blocks
// already fit).
static int tile_win_groups(int want, bool f32) {
  if (want == 1 || want == 2 || want == 4) return want;
  return f32 ? 1 : 2;
}

template <typename R, int G>
static void launch_tile_win_g(dim3 grid, size_t sm, hipStream_t s, const HamGeom &g, const DevTables<R> &tb,
                              const WinPass &W, const int4 *plist, const Cx<R> *pcl, const HvParams &P) {
  static size_t granted = 0;  // per instantiation
  if (sm > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&hv_tile_win<R, G>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    granted = sm;
  }
  hipLaunchKernelGGL((hv_tile_win<R, G>), grid, dim3(kBlock * G), sm, s, g, tb, W, plist, pcl, P);
}

template <typename R>
static int launch_tile_win(const DevHam &dh, const DevTables<R> &tb, const WinPlan &plan, const HvParams &P,
                           int cap, int groups, unsigned *last_gx, hipStream_t s) {
  const HamGeom &g = dh.geom;
  if (!plan.d_plist || !plan.d_pcoef || plan.passes.empty() || !g.spin_half || g.n <= kTileBits) return FTLM_EINVAL;
  const Cx<R> *pcl = reinterpret_cast<const Cx<R> *>(plan.d_pcoef);
  const int G = tile_win_groups(groups, sizeof(R) == 4);
  for (const WinPass &W : plan.passes) {
    const uint64_t items = (uint64_t)W.nwin * W.nin;
    uint32_t gx = (uint32_t)(items < (uint64_t)cap ? items : (uint64_t)cap);
    if (W.nwin >= 8 && gx >= 8) gx &= ~7u;
    HvParams Pp = P;
    if (!W.last) Pp.lanczos = 0;
    const size_t sm = hv_tile_win_smem<R>(g, W);
    if (sm > 160 * 1024) return FTLM_ERANGE;
    const dim3 grid(gx, P.K);
    if (G == 4) launch_tile_win_g<R, 4>(grid, sm, s, g, tb, W, plan.d_plist, pcl, Pp);
    else if (G == 2) launch_tile_win_g<R, 2>(grid, sm, s, g, tb, W, plan.d_plist, pcl, Pp);
    else launch_tile_win_g<R, 1>(grid, sm, s, g, tb, W, plan.d_plist, pcl, Pp);
    *last_gx = gx;
  }
  return FTLM_OK;
}

int launch_hv(const DevHam &dh, const HvLaunch &Lin, hipStream_t s) {
  HvLaunch L = Lin;
  if (L.K >= 1 && L.K <= 64 && (L.precision == 0 || L.precision == 1)) {
    const HvTuning &tn = dh.tune[L.precision][L.K];
    if (!L.variant) L.variant = tn.variant;
    if (!L.grid_cap) L.grid_cap = tn.grid_cap;
    if (!L.kc) L.kc = tn.kc;
  }
  // built-in choice for one column of a vector beyond the caches: the
  // single-pass tile kernel wherever its plan exists (no s+- s^z pair pieces);
  // it beat the multi-pass and tile kernels on every such workload measured
  if (!L.variant && L.K == 1 && dh.geom.dim >= (1u << 20) && (L.precision == FTLM_C64 ? dh.sp32 : dh.sp64).ok)
    L.variant = 6;
  g_variant = L.variant;
  int gx, gy, kc;
  const int rcg = hv_grid_blocks(dh, L, &gx, &gy, &kc);
  if (rcg) return rcg;
  HvParams P{};
  P.K = L.K;
  P.ntile = (dh.geom.spin_half && dh.geom.n >= kLowBits)
                ? (dh.geom.dim >> kLowBits)
                : (uint32_t)(((uint64_t)dh.geom.dim + kBlock - 1) / kBlock);
  P.v = L.v;
  P.w = L.w;
  P.scale = L.scale;
  if (L.lz) {
    P.lanczos = 1;
    P.scale = L.lz->sx_cur;
    P.xprev = L.lz->xprev;
    P.ov1 = L.lz->ov1;
    P.sx_prev = L.lz->sx_prev;
    P.beta_prev = L.lz->beta_prev;
    P.part = L.lz->part;
    P.counter = L.lz->counter;
    P.alpha_out = L.lz->alpha_out;
    P.yre_out = L.lz->yre_out;
    P.yim_out = L.lz->yim_out;
  }
  // the grid of the last dispatch and its columns per lane, for the Lanczos
  // finishing kernel (alpha_j, y_j from the per-block partials)
  unsigned fin_gx = (unsigned)gx, fin_gy = (unsigned)gy;
  int fin_kc = kc;
  int rc = FTLM_OK;
  if (L.variant == 6) {
    if (L.K != 1) return FTLM_EINVAL;
    const int cap = L.grid_cap > 0 ? std::min(L.grid_cap, 2048) : 2048;
    rc = launch_stream(dh, L.precision, P, cap, L.kc, &fin_gx, s);
    fin_gy = 1;
    fin_kc = 1;
  } else if (L.variant == 5) {
    const int cap = L.grid_cap > 0 ? std::min(L.grid_cap, 2048) : 2048;
    // (the columns-per-lane field carries the row groups per tile)
    rc = (L.precision == FTLM_C64) ? launch_tile_win<float>(dh, dh.t32, dh.tw32, P, cap, L.kc, &fin_gx, s)
                                   : launch_tile_win<double>(dh, dh.t64, dh.tw64, P, cap, L.kc, &fin_gx, s);
    fin_gy = (unsigned)L.K;
    fin_kc = 1;
  } else if (L.variant == 4) {
    const int cap = L.grid_cap > 0 ? std::min(L.grid_cap, 2048) : 2048;
    // general radix: kc columns per lane (the spin-1/2 window kernel takes one)
    const int wkc = dh.geom.spin_half ? 1 : kc;
    rc = (L.precision == FTLM_C64) ? launch_win<float>(dh, dh.t32, dh.win32, P, cap, wkc, &fin_gx, s)
                                   : launch_win<double>(dh, dh.t64, dh.win64, P, cap, wkc, &fin_gx, s);
    fin_gy = (unsigned)(L.K / wkc);
    fin_kc = wkc;
  } else if (use_passes(dh.geom, L.K, L.variant)) {
    const int cap = L.grid_cap > 0 ? std::min(L.grid_cap, 2048) : 2048;
    rc = (L.precision == FTLM_C64) ? launch_passes<float>(dh, dh.t32, dh.plan32, P, L.K, cap, &fin_gx, s)
                                   : launch_passes<double>(dh, dh.t64, dh.plan64, P, L.K, cap, &fin_gx, s);
    fin_gy = (unsigned)L.K;
    fin_kc = 1;
  } else {
    dim3 grid(gx, gy);
    if (L.precision == FTLM_C64) launch_hv_r<float>(dh, dh.t32, P, grid, kc, s);
    else launch_hv_r<double>(dh, dh.t64, P, grid, kc, s);
    if (use_tile(dh.geom, L.K)) fin_kc = 1;
  }
  if (rc) return rc;
  if (P.lanczos) launch_hv_finish(P, fin_gx, fin_gy, fin_kc, s);
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

// ------------------------------------------------------------------ start vectors
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies with the round constants 0xD2511F53 / 0xCD9E8D57 and Weyl key
// increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void gauss(uint64_t seed, uint32_t nu, uint32_t r, uint32_t f,
                                      uint32_t inst, double &x, double &y) {
  uint32_t c[4] = {nu, r, f, inst};
  philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)(c[0] >> 5) << 26) | (c[1] >> 6);
  const uint64_t b = ((uint64_t)(c[2] >> 5) << 26) | (c[3] >> 6);
  const double u1 = (double)(a + 1) * 0x1.0p-53;
  const double u2 = (double)b * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(2.0 * M_PI * u2, &sn, &cs);
  x = rad * cs;
  y = rad * sn;
}

struct StartParams {
  uint64_t seed;
  uint32_t inst, field, r0;
  int K;
  uint32_t dim;
  void *out;
  const double2 *src;  // copy mode: source [dim][src_cols] c128
  int src_cols, col0;
  double *part;
  unsigned *counter;
  double *sx0;
};

template <typename R, int KC, bool COPY>
__global__ __launch_bounds__(kBlock) void start_kernel(StartParams S) {
  const int c0 = blockIdx.y * KC;
  double red[1][KC];
#pragma unroll
  for (int q = 0; q < KC; q++) red[0][q] = 0.0;
  Cx<R> *out = reinterpret_cast<Cx<R> *>(S.out);
  // 64-bit row counter: near dim = 2^32 a 32-bit row + stride would wrap
  for (uint64_t row = (uint64_t)blockIdx.x * kBlock + threadIdx.x; row < S.dim;
       row += (uint64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int q = 0; q < KC; q++) {
      double x, y;
      if (COPY) {
        const double2 z = S.src[(size_t)row * S.src_cols + S.col0 + c0 + q];
        x = z.x;
        y = z.y;
      } else {
        gauss(S.seed, (uint32_t)row, S.r0 + c0 + q, S.field, S.inst, x, y);
      }
      const Cx<R> z{(R)x, (R)y};
      out[(size_t)row * S.K + c0 + q] = z;
      red[0][q] += (double)z.re * (double)z.re + (double)z.im * (double)z.im;
    }
  }
  block_partials_store<1, KC>(red, S.part, blockIdx.y * gridDim.x + blockIdx.x);
}

// sx0 = 1/|r| of every column from the start kernel's partials, one block per
// column (each summing in block order).
template <int KC>
__global__ __launch_bounds__(kBlock) void start_finish(StartParams S, unsigned gx) {
  const int c = blockIdx.x;
  const int cb = c / KC, q = c % KC;
  const double s = block_sum_strided(S.part + (size_t)cb * gx * KC + q, gx, KC);
  if (threadIdx.x == 0) S.sx0[c] = s > 0 ? 1.0 / sqrt(s) : 0.0;
}

template <typename R, bool COPY>
static void launch_start_r(const StartParams &S, int grid_cap, hipStream_t s) {
  const int kc = pick_kc(S.K, 8);
  uint32_t nb = (uint32_t)(((uint64_t)S.dim + kBlock - 1) / kBlock);
  const uint32_t cap = grid_cap > 0 ? (uint32_t)grid_cap : 2048u;
  dim3 grid(nb < cap ? nb : cap, S.K / kc);
  switch (kc) {
    case 8: hipLaunchKernelGGL((start_kernel<R, 8, COPY>), grid, dim3(kBlock), 0, s, S); break;
    case 4: hipLaunchKernelGGL((start_kernel<R, 4, COPY>), grid, dim3(kBlock), 0, s, S); break;
    case 2: hipLaunchKernelGGL((start_kernel<R, 2, COPY>), grid, dim3(kBlock), 0, s, S); break;
    default: hipLaunchKernelGGL((start_kernel<R, 1, COPY>), grid, dim3(kBlock), 0, s, S); break;
  }
  const dim3 fgrid(grid.y * (unsigned)kc);
  switch (kc) {
    case 8: hipLaunchKernelGGL(start_finish<8>, fgrid, dim3(kBlock), 0, s, S, grid.x); break;
    case 4: hipLaunchKernelGGL(start_finish<4>, fgrid, dim3(kBlock), 0, s, S, grid.x); break;
    case 2: hipLaunchKernelGGL(start_finish<2>, fgrid, dim3(kBlock), 0, s, S, grid.x); break;
    default: hipLaunchKernelGGL(start_finish<1>, fgrid, dim3(kBlock), 0, s, S, grid.x); break;
  }
}

int launch_gaussian(uint64_t seed, uint32_t inst, uint32_t field, uint32_t r0, int K,
                    uint32_t dim, int precision, void *out, double *part, unsigned *counter,
                    double *sx0, int grid_cap, hipStream_t s) {
  StartParams S{};
  S.seed = seed;
  S.inst = inst;
  S.field = field;
  S.r0 = r0;
  S.K = K;
  S.dim = dim;
  S.out = out;
  S.part = part;
  S.counter = counter;
  S.sx0 = sx0;
  if (precision == FTLM_C64) launch_start_r<float, false>(S, grid_cap, s);
  else launch_start_r<double, false>(S, grid_cap, s);
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

int launch_copy_start(const void *src_c128, int src_cols, int col0, int K, uint32_t dim,
                      int precision, void *out, double *part, unsigned *counter, double *sx0,
                      int grid_cap, hipStream_t s) {
  StartParams S{};
  S.K = K;
  S.dim = dim;
  S.out = out;
  S.src = reinterpret_cast<const double2 *>(src_c128);
  S.src_cols = src_cols;
  S.col0 = col0;
  S.part = part;
  S.counter = counter;
  S.sx0 = sx0;
  if (precision == FTLM_C64) launch_start_r<float, true>(S, grid_cap, s);
  else launch_start_r<double, true>(S, grid_cap, s);
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

// ------------------------------------------------------------------ Lanczos update
template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void update_kernel(UpdateArgs A) {
  const int c0 = blockIdx.y * KC;
  double red[1][KC];
  double coef[KC];
#pragma unroll
  for (int q = 0; q < KC; q++) {
    red[0][q] = 0.0;
    coef[q] = A.alpha[c0 + q] * A.sx_cur[c0 + q];
  }
  Cx<R> *w = reinterpret_cast<Cx<R> *>(A.w);
  const Cx<R> *x = reinterpret_cast<const Cx<R> *>(A.x);
  // four rows per thread per trip keep eight loads in flight
  const uint64_t gstride = (uint64_t)gridDim.x * kBlock;
  uint64_t row = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; row + 3 * gstride < A.dim; row += 4 * gstride) {
#pragma unroll
    for (int q = 0; q < KC; q++) {
      Cx<R> a[4], b[4];
#pragma unroll
      for (int u4 = 0; u4 < 4; u4++) {
        const size_t o = (size_t)(row + (uint64_t)u4 * gstride) * A.K + c0 + q;
        a[u4] = w[o];
        b[u4] = x[o];
      }
#pragma unroll
      for (int u4 = 0; u4 < 4; u4++) {
        const size_t o = (size_t)(row + (uint64_t)u4 * gstride) * A.K + c0 + q;
        const double ur = (double)a[u4].re - coef[q] * (double)b[u4].re;
        const double ui = (double)a[u4].im - coef[q] * (double)b[u4].im;
        const Cx<R> u{(R)ur, (R)ui};
        w[o] = u;
        red[0][q] += (double)u.re * (double)u.re + (double)u.im * (double)u.im;
      }
    }
  }
  for (; row < A.dim; row += gstride) {
#pragma unroll
    for (int q = 0; q < KC; q++) {
      const size_t o = (size_t)row * A.K + c0 + q;
      const Cx<R> a = w[o], b = x[o];
      const double ur = (double)a.re - coef[q] * (double)b.re;
      const double ui = (double)a.im - coef[q] * (double)b.im;
      const Cx<R> u{(R)ur, (R)ui};
      w[o] = u;
      red[0][q] += (double)u.re * (double)u.re + (double)u.im * (double)u.im;
    }
  }
  block_partials_store<1, KC>(red, A.part, blockIdx.y * gridDim.x + blockIdx.x);
}

// One block per column: beta_j = |u| from the update kernel's per-block
// partials (layout [cb][bx][KC], summed in block order), the next scale
// 1/beta_j and the breakdown test.
template <int KC>
__global__ __launch_bounds__(kBlock) void update_finish(UpdateArgs A, unsigned gx) {
  const int c = blockIdx.x;  // one block per column
  {
    const int cb = c / KC, q = c % KC;
    const double s = block_sum_strided(A.part + (size_t)cb * gx * KC + q, gx, KC);
    if (threadIdx.x != 0) return;
    double b = sqrt(s);
    const double al = fabs(A.alpha[c]);
    double sm = A.scale_max[c];
    if (al > sm) sm = al;
    if (A.done[c]) {
      A.beta[c] = 0.0;
      A.sx_next[c] = 0.0;
    } else {
      A.n_used[c] = A.step + 1;
      const bool breakdown = (A.step + 1 < A.n_lanczos) && !(b > 1e-12 * sm);
      A.beta[c] = b;
      if (breakdown) {
        A.done[c] = 1;
        A.sx_next[c] = 0.0;
      } else {
        A.sx_next[c] = b > 0 ? 1.0 / b : 0.0;
      }
      if (b > sm) sm = b;
    }
    A.scale_max[c] = sm;
  }
}

int launch_update(const UpdateArgs &a, hipStream_t s) {
  const int kc = pick_kc(a.K, 8);
  uint32_t nb = (uint32_t)(((uint64_t)a.dim + kBlock - 1) / kBlock);
  const uint32_t cap = a.grid_cap > 0 ? (uint32_t)a.grid_cap : 2048u;
  dim3 grid(nb < cap ? nb : cap, a.K / kc);
  const bool f32 = a.precision == FTLM_C64;
  switch (kc) {
    case 8:
      if (f32) hipLaunchKernelGGL((update_kernel<float, 8>), grid, dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((update_kernel<double, 8>), grid, dim3(kBlock), 0, s, a);
      break;
    case 4:
      if (f32) hipLaunchKernelGGL((update_kernel<float, 4>), grid, dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((update_kernel<double, 4>), grid, dim3(kBlock), 0, s, a);
      break;
    case 2:
      if (f32) hipLaunchKernelGGL((update_kernel<float, 2>), grid, dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((update_kernel<double, 2>), grid, dim3(kBlock), 0, s, a);
      break;
    default:
      if (f32) hipLaunchKernelGGL((update_kernel<float, 1>), grid, dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((update_kernel<double, 1>), grid, dim3(kBlock), 0, s, a);
      break;
  }
  const dim3 fgrid(grid.y * (unsigned)kc);
  switch (kc) {
    case 8: hipLaunchKernelGGL(update_finish<8>, fgrid, dim3(kBlock), 0, s, a, grid.x); break;
    case 4: hipLaunchKernelGGL(update_finish<4>, fgrid, dim3(kBlock), 0, s, a, grid.x); break;
    case 2: hipLaunchKernelGGL(update_finish<2>, fgrid, dim3(kBlock), 0, s, a, grid.x); break;
    default: hipLaunchKernelGGL(update_finish<1>, fgrid, dim3(kBlock), 0, s, a, grid.x); break;
  }
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

__global__ void zero_state_kernel(double *scale_max, int *done, int *n_used, unsigned *counters,
                                  int n_counters, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) {
    scale_max[i] = 0.0;
    done[i] = 0;
    n_used[i] = 0;
  }
  if (i < n_counters) counters[i] = 0u;
}

int launch_zero_state(double *scale_max, int *done, int *n_used, unsigned *counters,
                      int n_counters, int K, hipStream_t s) {
  const int n = K > n_counters ? K : n_counters;
  hipLaunchKernelGGL(zero_state_kernel, dim3((n + 255) / 256), dim3(256), 0, s, scale_max, done,
                     n_used, counters, n_counters, K);
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

// ------------------------------------------------------------------ tridiagonal
// Implicit QL with shifts on T = tridiag(alpha, beta) (n <= n_lanczos), one
// thread per column; Z = product of the plane rotations, of which only the rows
// e_1^T Z (-> Q_1n) and y^T Z (-> sum_a y_a Q_an) are carried along.
// Scratch layout [4][n_lanczos][n_cols].
// LDS: the four work arrays of the block's columns live in LDS ([4][nl][blockDim]),
// else in the global scratch ([4][nl][n_cols]).
template <bool LDS>
__global__ void tridiag_kernel(int n_cols, int nl, const int *n_used, int used_stride,
                               int in_stride, const double *alpha, const double *beta, const double *y,
                               double *eps, double *q1, double *qy, int out_stride, int out_col0,
                               double *scratch) {
  extern __shared__ double tri_sh[];
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n_cols) return;
  const int n = n_used ? n_used[col * used_stride] : nl;
  const size_t S = LDS ? (size_t)blockDim.x : (size_t)n_cols;
  double *base = LDS ? tri_sh + threadIdx.x : scratch + col;
  double *d = base;
  double *e = base + (size_t)nl * S;
  double *z1 = base + 2 * (size_t)nl * S;
  double *zy = base + 3 * (size_t)nl * S;
#define AT(p, i) (p)[(size_t)(i)*S]
  for (int i = 0; i < n; i++) {
    AT(d, i) = alpha[(size_t)i * in_stride + col];
    AT(e, i) = (i + 1 < n) ? beta[(size_t)i * in_stride + col] : 0.0;
    AT(z1, i) = (i == 0) ? 1.0 : 0.0;
    AT(zy, i) = y ? y[(size_t)i * in_stride + col] : 0.0;
  }
  for (int l = 0; l < n; l++) {
    int iter = 0;
    while (true) {
      int m = l;
      {
        double dm = AT(d, l);
        for (; m < n - 1; m++) {
          const double dm1 = AT(d, m + 1);
          const double dd = fabs(dm) + fabs(dm1);
          if (fabs(AT(e, m)) <= 2.220446049250313e-16 * dd) break;
          dm = dm1;
        }
      }
      if (m == l || iter++ >= 100) break;
      double gg = (AT(d, l + 1) - AT(d, l)) / (2.0 * AT(e, l));
      double r = hypot(gg, 1.0);
      gg = AT(d, m) - AT(d, l) + AT(e, l) / (gg + copysign(r, gg));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool underflow = false;
      // A step at i reads e[i], d[i], d[i+1] and rows i, i+1 of the tracked Z
      // rows and writes indices i+1 and i only, so the next step's reads (index
      // i-1) are issued one step ahead, d[i+1] is the previous step's d[i], and
      // the rotated Z entries of index i stay in registers for the next step.
      double d_hi = AT(d, m), z1_hi = AT(z1, m), zy_hi = AT(zy, m);
      double e_i = AT(e, m - 1), d_i = AT(d, m - 1), z1_i = AT(z1, m - 1), zy_i = AT(zy, m - 1);
      for (; i >= l; i--) {
        double e_n = 0.0, d_n = 0.0, z1_n = 0.0, zy_n = 0.0;
        if (i > l) {
          e_n = AT(e, i - 1);
          d_n = AT(d, i - 1);
          z1_n = AT(z1, i - 1);
          zy_n = AT(zy, i - 1);
        }
        const double f = s * e_i, b = c * e_i;
        r = hypot(f, gg);
        AT(e, i + 1) = r;
        if (r == 0.0) {
          AT(d, i + 1) = d_hi - p;
          AT(e, m) = 0.0;
          AT(z1, i + 1) = z1_hi;
          AT(zy, i + 1) = zy_hi;
          underflow = true;
          break;
        }
        s = f / r;
        c = gg / r;
        gg = d_hi - p;
        r = (d_i - gg) * s + 2.0 * c * b;
        p = s * r;
        AT(d, i + 1) = gg + p;
        gg = c * r - b;
        // rotate columns i, i+1 of Z in the two tracked rows
        const double z1_lo = c * z1_i - s * z1_hi;
        AT(z1, i + 1) = s * z1_i + c * z1_hi;
        z1_hi = z1_lo;
        const double zy_lo = c * zy_i - s * zy_hi;
        AT(zy, i + 1) = s * zy_i + c * zy_hi;
        zy_hi = zy_lo;
        d_hi = d_i;
        e_i = e_n;
        d_i = d_n;
        z1_i = z1_n;
        zy_i = zy_n;
      }
      if (underflow) continue;
      AT(z1, l) = z1_hi;
      AT(zy, l) = zy_hi;
      AT(d, l) -= p;
      AT(e, l) = gg;
      AT(e, m) = 0.0;
    }
  }
  const size_t os = (size_t)out_stride;
  for (int i = 0; i < nl; i++) {
    const bool ok = i < n;
    eps[(size_t)i * os + out_col0 + col] = ok ? AT(d, i) : 0.0;
    q1[(size_t)i * os + out_col0 + col] = ok ? AT(z1, i) : 0.0;
    qy[(size_t)i * os + out_col0 + col] = ok ? AT(zy, i) : 0.0;
  }
#undef AT
}

int launch_tridiag(int n_cols, int n_lanczos, const int *n_used, int used_stride, int in_stride,
                   const double *alpha, const double *beta, const double *y, double *eps,
                   double *q1, double *qy, int out_stride, int out_col0, double *scratch,
                   hipStream_t s) {
  // 64 KB of LDS per block: as many columns as fit (at most 64), else global scratch
  const int per_col = 32 * n_lanczos;  // bytes of the four work arrays
  int cpb = per_col > 0 ? 65536 / per_col : 0;
  if (cpb > 64) cpb = 64;
  if (cpb >= 1) {
    hipLaunchKernelGGL(tridiag_kernel<true>, dim3((n_cols + cpb - 1) / cpb), dim3(cpb),
                       (size_t)cpb * per_col, s, n_cols, n_lanczos, n_used, used_stride, in_stride,
                       alpha, beta, y, eps, q1, qy, out_stride, out_col0, scratch);
  } else {
    hipLaunchKernelGGL(tridiag_kernel<false>, dim3((n_cols + 63) / 64), dim3(64), 0, s, n_cols,
                       n_lanczos, n_used, used_stride, in_stride, alpha, beta, y, eps, q1, qy,
                       out_stride, out_col0, scratch);
  }
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

// ------------------------------------------------------------------ Boltzmann sums
// One block of kBz threads per (curve, temperature).  Columns f*R .. f*R+R-1 of
// the [n_lanczos][n_curves*R] arrays belong to curve f; the curve's terms
// k = i R + r (Ritz value i of vector r) are dealt to the threads in a fixed
// stride and every sum and extremum meets in a fixed LDS tree, so the results
// do not depend on scheduling.  With
//   l_{rn} = ln Q_1n^2 - (eps_n - E_min)/T,  lmax = max l:
//   ln Z = ln(dim/R) - E_min/T + lmax + ln sum exp(l - lmax)        (Eq. E-2-D)
//   <A>  = sum exp(l - lmax) A(eps) / sum exp(l - lmax)
//   M    = sum exp(-(eps-E_min)/T - lmax) Q_1n (sum_a Q_an y_a) / sum exp(l - lmax)
constexpr int kBz = 256;

template <int OP>  // 0: sum, 1: max, 2: min
__device__ __forceinline__ double bz_tree(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBz / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + w];
      sh[threadIdx.x] = OP == 0 ? a + b : OP == 1 ? fmax(a, b) : fmin(a, b);
    }
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBz) void boltzmann_kernel(int n_curves, int R, int nl, const int *n_used,
                                                        const double *eps, const double *q1, const double *qy,
                                                        const double *dims, const double *T, int n_T,
                                                        double *lnZ, double *E, double *C, double *M,
                                                        double *E_min) {
  __shared__ double sh[kBz];
  const int f = blockIdx.x / n_T, it = blockIdx.x % n_T;
  const int ncol = n_curves * R, nterm = nl * R;
  const double temp = T[it];
  double loc = INFINITY;
  for (int k = threadIdx.x; k < nterm; k += kBz) {
    const int i = k / R, c = f * R + k % R;
    if (i < n_used[c]) loc = fmin(loc, eps[(size_t)i * ncol + c]);
  }
  const double emin = bz_tree<2>(loc, sh);
  loc = -INFINITY;
  for (int k = threadIdx.x; k < nterm; k += kBz) {
    const int i = k / R, c = f * R + k % R;
    if (i >= n_used[c]) continue;
    const size_t o = (size_t)i * ncol + c;
    const double qq = q1[o];
    if (qq == 0.0) continue;
    loc = fmax(loc, log(qq * qq) - (eps[o] - emin) / temp);
  }
  const double lmax = bz_tree<1>(loc, sh);
  double z = 0, ez = 0, mz = 0;
  for (int k = threadIdx.x; k < nterm; k += kBz) {
    const int i = k / R, c = f * R + k % R;
    if (i >= n_used[c]) continue;
    const size_t o = (size_t)i * ncol + c;
    const double w = exp(-(eps[o] - emin) / temp - lmax);
    const double qq = q1[o];
    z += w * qq * qq;
    ez += w * qq * qq * eps[o];
    mz += w * qq * qy[o];
  }
  z = bz_tree<0>(z, sh);
  ez = bz_tree<0>(ez, sh);
  mz = bz_tree<0>(mz, sh);
  const double em = ez / z;
  double cz = 0;
  for (int k = threadIdx.x; k < nterm; k += kBz) {
    const int i = k / R, c = f * R + k % R;
    if (i >= n_used[c]) continue;
    const size_t o = (size_t)i * ncol + c;
    const double w = exp(-(eps[o] - emin) / temp - lmax);
    const double qq = q1[o];
    const double de = eps[o] - em;
    cz += w * qq * qq * de * de;
  }
  cz = bz_tree<0>(cz, sh);
  if (threadIdx.x != 0) return;
  const size_t out = (size_t)f * n_T + it;
  lnZ[out] = log(dims[f] / R) - emin / temp + lmax + log(z);
  E[out] = em;
  C[out] = cz / z / (temp * temp);
  M[out] = mz / z;
  if (it == 0 && E_min) E_min[f] = emin;
}

int launch_boltzmann(int n_curves, int R, int n_lanczos, const int *n_used, const double *eps,
                     const double *q1, const double *qy, const double *dims, const double *T,
                     int n_T, double *lnZ, double *E, double *C, double *M, double *E_min,
                     hipStream_t s) {
  const unsigned n = (unsigned)n_curves * (unsigned)n_T;
  if (n == 0) return FTLM_OK;
  hipLaunchKernelGGL(boltzmann_kernel, dim3(n), dim3(kBz), 0, s, n_curves, R, n_lanczos, n_used, eps,
                     q1, qy, dims, T, n_T, lnZ, E, C, M, E_min);
  return hipGetLastError() == hipSuccess ? FTLM_OK : FTLM_EHIP;
}

}  // namespace ftlm
