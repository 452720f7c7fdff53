// Batched FTLM (ftlm_run_batched): many Hamiltonian instances of uneven
// dimension and their field directions run together.  A wave holds items =
// (instance, field, group of K random vectors); every Lanczos step is ONE
// persistent H*v launch over a work queue of (item, row chunk) units for all
// items of the wave, followed by one persistent update launch; both are
// replayed from a captured HIP graph.  Reductions are per item and fixed-order:
// each unit stores its partial sums, and a finishing launch (one block per
// item) sums the item's partials in unit order.
//
// Vectors of an item are column-interleaved [dim][K], so a gather of one partner
// row reads K contiguous complex numbers and every coefficient serves K columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "device_reduce.hpp"
#include "ftlm_internal.hpp"

namespace ftlm {

// Rows per work unit: 2^ubits with ubits = 11 (2048 rows, 8 tiles of 256) or
// 12, a tuning choice.  Units are laid out item by item and the grid is kept
// small enough that the units in flight at any time cover a few large items, so
// the partners an item's gathers touch stay in the caches.  The spin-1/2 z-field
// tables split a row into bits 0..7 (two nibbles), 8..ubits-1 (the unit table's
// index) and >= ubits (the unit's).
constexpr uint32_t kUnitRows = 2048;  // smallest unit: sizes the workspace's unit arrays
constexpr int kMaxUnitSub = 16;       // unit-table entries per (site, ladder) at ubits = 12
// Launch choices of the batched run (the batched autotuner sets them): grid
// cap, unit size, the order in which a wave's items take their units (0: curve
// order, 1: largest instance first) and the threads of the H*v step's blocks.
// A block works on one unit at a time, so the block size sets how many of a
// CU's resident waves share a unit's rows, partner rows and staged tables.
struct BatchTuning {
  int grid_cap = 1024;
  int ubits = 11;
  int order = 0;
  int block = 512;
};
static thread_local BatchTuning g_btune;

template <typename R>
struct BItem {
  DevTables<R> tb;   // instance pair tables + this field's one-site tables
  DevTables<R> tbo;  // moment operator (one-site tables only)
  int n, npair, has_z, half;
  int pow2r;              // every radix a power of two: digits are bit fields
  uint32_t dim;
  uint32_t unit0, nunit;  // work units [unit0, unit0 + nunit)
  int col0;               // first column of the item in the wave's scalar arrays
  uint32_t rng_inst, rng_field, rng_r0;
  Cx<R> *x[3];            // rotating Lanczos buffers [dim][K]
  Cx<R> *ov1;             // O v_1
  R *diag;                // H's diagonal [dim]: written by the first Lanczos step, read by the rest
  int radix[kMaxSites];
  uint32_t stride[kMaxSites];
};

// the host packs the item array at the stride of BItem<double> for both precisions
static_assert(sizeof(BItem<float>) == sizeof(BItem<double>), "BItem must not depend on R in size");

struct BStep {
  int K, step, n_lanczos, mode;  // mode 0: O v_1 (plain, scaled); 1: Lanczos H*v
  uint32_t n_units;
  uint64_t seed;
  double *alpha, *beta, *yre, *yim;   // [K*n_items] slices for this step
  double *sx_cur, *sx_prev, *beta_prev, *sx_next;
  double *smax;
  int *done, *nused;
  double *part;                        // [n_units][3][K]
  uint32_t n_items;                    // items of the wave (blocks of the finishing launch)
  uint32_t lds;                        // dynamic LDS of the H*v launch (largest item's tables)
  int ubits;                           // log2 of the rows per work unit (11 or 12)
  int block;                           // threads per block of the H*v launch (256, 512, 1024)
  const int *unit_item;                // [n_units]
};

template <typename R, int KC>
struct BAcc {
  R re[KC], im[KC];
};

// a += c x for KC loaded columns
template <typename R, int KC>
__device__ __forceinline__ void bfma(BAcc<R, KC> &a, R cr, R ci, const Cx<R> (&xv)[KC]) {
#pragma unroll
  for (int q = 0; q < KC; q++) {
    a.re[q] = fma(cr, xv[q].re, fma(-ci, xv[q].im, a.re[q]));
    a.im[q] = fma(cr, xv[q].im, fma(ci, xv[q].re, a.im[q]));
  }
}

// a vector in global memory, for loads that the compiler would otherwise issue
// as generic (flat) loads (the host pass of the compiler only parses device
// code, and has no such address space)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename R>
using GPtr = const __attribute__((address_space(1))) Cx<R> *;
template <typename R>
using GPtrW = __attribute__((address_space(1))) Cx<R> *;
#else
template <typename R>
using GPtr = const Cx<R> *;
template <typename R>
using GPtrW = Cx<R> *;
#endif

// a += c x[0..KC), x a row of a Lanczos vector (device memory: read as global)
template <typename R, int KC>
__device__ __forceinline__ void bmac(BAcc<R, KC> &a, R cr, R ci, const Cx<R> *__restrict__ x) {
  const GPtr<R> gx = (GPtr<R>)x;
  Cx<R> xv[KC];
#pragma unroll
  for (int q = 0; q < KC; q++) xv[q] = gx[q];
  bfma<R, KC>(a, cr, ci, xv);
}

// LDS bytes of one item's staged tables (see stage_tables).
__host__ __device__ inline size_t staged_bytes(int n, int npair, bool half, size_t rs) {
  const size_t cs = 2 * rs;
  auto a16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  size_t b = a16((size_t)n * 16 * rs) + 2 * a16((size_t)n * n * cs) + a16((size_t)npair * 8) +
             a16((size_t)npair * rs) + a16((size_t)npair * 4 * cs);
  // hflip; lane-bit z-field tables [2 nibbles][k][b][16]; unit table [k][b][<= 16]
  if (half) b += a16((size_t)n * 2 * cs) + a16((size_t)2 * n * 2 * 16 * cs) + a16((size_t)n * 2 * kMaxUnitSub * cs);
  else b += 3 * a16((size_t)n * 16 * rs) + a16((size_t)n * 64 * cs);
  return b;
}

// LDS layout of one item's staged tables (operator H, or O for the moment
// product): the tables brow reads, at offsets that depend only on the item's
// sizes.  Recomputed from the LDS base wherever it is used, so that the
// compiler sees LDS pointers (not generic ones) in brow.
template <typename R>
__device__ __forceinline__ DevTables<R> table_layout(const BItem<R> &it, bool moment, unsigned char *lds) {
  const int n = it.n, np = moment ? 0 : it.npair;
  const size_t rs = sizeof(R), cs = sizeof(Cx<R>);
  auto a16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  DevTables<R> d{};
  size_t off = 0;
  d.hdiag = reinterpret_cast<const R *>(lds + off);
  off += a16((size_t)n * 16 * rs);
  d.czp = reinterpret_cast<const Cx<R> *>(lds + off);
  off += a16((size_t)n * n * cs);
  d.czm = reinterpret_cast<const Cx<R> *>(lds + off);
  off += a16((size_t)n * n * cs);
  d.pij = reinterpret_cast<const int2 *>(lds + off);
  off += a16((size_t)np * 8);
  d.pzz = reinterpret_cast<const R *>(lds + off);
  off += a16((size_t)np * rs);
  if (it.half) {
    d.pc_half = reinterpret_cast<const Cx<R> *>(lds + off);
    off += a16((size_t)np * 4 * cs);
    d.hflip = reinterpret_cast<const Cx<R> *>(lds + off);
    off += a16((size_t)n * 2 * cs);
    // z-field F_k^b(row) = sum_{l != k} C^b_kl m_l(row) split by row bits:
    // cz_half [nibble j < 2][k][b][v]: the sites 4j..4j+3 (lane bits) for
    // nibble value v (staged per item); lowf [k][b][i]: the sites >= 8 for row
    // bits 8..ubits-1 = i and the current unit's bits >= ubits (filled per unit)
    d.cz_half = reinterpret_cast<const Cx<R> *>(lds + off);
    off += a16((size_t)2 * n * 2 * 16 * cs);
    d.lowf = reinterpret_cast<const Cx<R> *>(lds + off);
  } else {
    d.pc = reinterpret_cast<const Cx<R> *>(lds + off);
    off += a16((size_t)np * 4 * cs);
    d.mval = reinterpret_cast<const R *>(lds + off);
    off += a16((size_t)n * 16 * rs);
    d.gp = reinterpret_cast<const R *>(lds + off);
    off += a16((size_t)n * 16 * rs);
    d.gm = reinterpret_cast<const R *>(lds + off);
    off += a16((size_t)n * 16 * rs);
    d.hoff = reinterpret_cast<const Cx<R> *>(lds + off);
  }
  return d;
}

template <typename T>
__device__ __forceinline__ void stage_copy(const T *dst, const T *src, size_t cnt) {
  T *d = const_cast<T *>(dst);
  if (src)
    for (size_t i = threadIdx.x; i < cnt; i += blockDim.x) d[i] = src[i];
}

// Copies the tables brow reads for item it into LDS (layout table_layout).
// brow walks the pairs and sites at wave-uniform indices; read from global
// memory those reads are vector loads that each wait out their latency, read
// from LDS they are broadcasts.  The caller synchronises before and after.
template <typename R>
__device__ void stage_tables(const BItem<R> &it, bool moment, unsigned char *lds) {
  const DevTables<R> &src = moment ? it.tbo : it.tb;
  const DevTables<R> d = table_layout(it, moment, lds);
  const int n = it.n, np = moment ? 0 : it.npair;
  const bool hz = !moment && it.has_z;
  stage_copy(d.hdiag, src.hdiag, (size_t)n * 16);
  stage_copy(d.czp, hz ? src.czp : nullptr, (size_t)n * n);
  stage_copy(d.czm, hz ? src.czm : nullptr, (size_t)n * n);
  stage_copy(d.pij, src.pij, (size_t)np);
  stage_copy(d.pzz, src.pzz, (size_t)np);
  if (it.half) {
    stage_copy(d.pc_half, src.pc_half, (size_t)np * 4);
    stage_copy(d.hflip, src.hflip, (size_t)n * 2);
    if (hz) {
      Cx<R> *T = const_cast<Cx<R> *>(d.cz_half);
      for (int e = threadIdx.x; e < 2 * n * 32; e += (int)blockDim.x) {
        const int v = e & 15, b = (e >> 4) & 1, k = (e >> 5) % n, j = (e >> 5) / n;
        R fr = 0, fi = 0;
        for (int l = 4 * j; l < 4 * j + 4 && l < n; l++) {
          if (l == k) continue;
          const R ml = ((v >> (l - 4 * j)) & 1) ? R(0.5) : R(-0.5);
          const Cx<R> c = b ? src.czp[k * n + l] : src.czm[k * n + l];
          fr = fma(c.re, ml, fr);
          fi = fma(c.im, ml, fi);
        }
        T[e] = Cx<R>{fr, fi};
      }
    }
  } else {
    stage_copy(d.pc, src.pc, (size_t)np * 4);
    stage_copy(d.mval, src.mval, (size_t)n * 16);
    stage_copy(d.gp, src.gp, (size_t)n * 16);
    stage_copy(d.gm, src.gm, (size_t)n * 16);
    stage_copy(d.hoff, src.hoff, (size_t)n * 64);
  }
}

// One row of H v (or O v) for KC columns; tb holds the operator's tables.
// dmode: 0 computes the diagonal element, 1 computes and stores it in dcache[row],
// 2 reads it from there (H does not change between the steps of a run).
template <typename R, int KC>
__device__ __forceinline__ void brow(const BItem<R> &it, const DevTables<R> &tb, bool moment, uint32_t row,
                                     const Cx<R> *__restrict__ v, BAcc<R, KC> &acc, R *dcache, int dmode,
                                     int usb) {
  const int n = it.n;
  const int npair = moment ? 0 : it.npair;
  const bool has_z = !moment && it.has_z;
#pragma unroll
  for (int q = 0; q < KC; q++) acc.re[q] = acc.im[q] = R(0);
  if (it.half) {
    R diag = 0;
    if (dmode == 2) {
      diag = dcache[row];
    } else {
      for (int k = 0; k < n; k++) diag += tb.hdiag[k * 16 + ((row >> k) & 1)];
      for (int p = 0; p < npair; p++) {
        const int2 ij = tb.pij[p];
        diag = fma(tb.pzz[p], (((row >> ij.x) ^ (row >> ij.y)) & 1) ? R(-0.25) : R(0.25), diag);
      }
      if (dmode == 1) dcache[row] = diag;
    }
    {
      const Cx<R> *x = v + (size_t)row * KC;
#pragma unroll
      for (int q = 0; q < KC; q++) {
        acc.re[q] = diag * x[q].re;
        acc.im[q] = diag * x[q].im;
      }
    }
    for (int k = 0; k < n; k++) {
      const int b = (row >> k) & 1;
      Cx<R> c = tb.hflip[2 * k + b];
      if (has_z) {  // three table reads: row bits 0..3, 4..7, and 8.. (unit table)
        const Cx<R> f0 = tb.cz_half[((size_t)k * 2 + b) * 16 + (row & 15u)];
        const Cx<R> f1 = tb.cz_half[((size_t)(n + k) * 2 + b) * 16 + ((row >> 4) & 15u)];
        const Cx<R> f2 = tb.lowf[(((size_t)k * 2 + b) << usb) + ((row >> 8) & ((1u << usb) - 1u))];
        c.re += f0.re + f1.re + f2.re;
        c.im += f0.im + f1.im + f2.im;
      }
      bmac<R, KC>(acc, c.re, c.im, v + (size_t)(row ^ (1u << k)) * KC);
    }
    // two pairs per trip: both partner rows are loaded before the first FMA
    // (the accumulation order is that of one pair at a time); the vectors are
    // read through global (not generic) pointers, so that waiting for an LDS
    // table read does not also wait for the gathers in flight
    const GPtr<R> gv = (GPtr<R>)v;  // generic -> global: the vectors are device memory
    int p = 0;
    for (; p + 1 < npair; p += 2) {
      const int2 ij0 = tb.pij[p], ij1 = tb.pij[p + 1];
      const GPtr<R> p0 = gv + (size_t)(row ^ ((1u << ij0.x) | (1u << ij0.y))) * KC;
      const GPtr<R> p1 = gv + (size_t)(row ^ ((1u << ij1.x) | (1u << ij1.y))) * KC;
      Cx<R> x0[KC], x1[KC];
#pragma unroll
      for (int q = 0; q < KC; q++) {
        x0[q] = p0[q];
        x1[q] = p1[q];
      }
      const Cx<R> c0 = tb.pc_half[4 * p + ((((row >> ij0.x) & 1) << 1) | ((row >> ij0.y) & 1))];
      const Cx<R> c1 = tb.pc_half[4 * (p + 1) + ((((row >> ij1.x) & 1) << 1) | ((row >> ij1.y) & 1))];
      bfma<R, KC>(acc, c0.re, c0.im, x0);
      bfma<R, KC>(acc, c1.re, c1.im, x1);
    }
    if (p < npair) {
      const int2 ij = tb.pij[p];
      const int type = (((row >> ij.x) & 1) << 1) | ((row >> ij.y) & 1);
      const Cx<R> c = tb.pc_half[4 * p + type];
      bmac<R, KC>(acc, c.re, c.im, v + (size_t)(row ^ ((1u << ij.x) | (1u << ij.y))) * KC);
    }
    return;
  }
  uint64_t dlo = 0, dhi = 0;
  if (it.pow2r) {  // digit k = bits log2(stride_k) .. of the row
    for (int k = 0; k < n; k++) {
      const uint64_t dk = (row >> __builtin_ctz(it.stride[k])) & (uint32_t)(it.radix[k] - 1);
      if (k < 16) dlo |= dk << (4 * k);
      else dhi |= dk << (4 * (k - 16));
    }
  } else {
    uint32_t rem = row;
    for (int k = 0; k < n; k++) {
      const uint32_t r = (uint32_t)it.radix[k], qq = rem / r;
      const uint64_t dk = rem - qq * r;
      rem = qq;
      if (k < 16) dlo |= dk << (4 * k);
      else dhi |= dk << (4 * (k - 16));
    }
  }
  auto digit = [&](int k) -> int {
    return (int)(((k < 16) ? (dlo >> (4 * k)) : (dhi >> (4 * (k - 16)))) & 15u);
  };
  R diag = 0;
  if (dmode == 2) {
    diag = dcache[row];
  } else {
    for (int k = 0; k < n; k++) diag += tb.hdiag[k * 16 + digit(k)];
    for (int p = 0; p < npair; p++) {
      const int2 ij = tb.pij[p];
      diag = fma(tb.pzz[p], tb.mval[ij.x * 16 + digit(ij.x)] * tb.mval[ij.y * 16 + digit(ij.y)], diag);
    }
    if (dmode == 1) dcache[row] = diag;
  }
  {
    const Cx<R> *x = v + (size_t)row * KC;
#pragma unroll
    for (int q = 0; q < KC; q++) {
      acc.re[q] = diag * x[q].re;
      acc.im[q] = diag * x[q].im;
    }
  }
  for (int k = 0; k < n; k++) {
    const int dk = digit(k), rk = it.radix[k];
    const uint32_t st = it.stride[k];
    R fpr = 0, fpi = 0, fmr = 0, fmi = 0;
    if (has_z)
      for (int l = 0; l < n; l++) {
        if (l == k) continue;
        const R ml = tb.mval[l * 16 + digit(l)];
        const Cx<R> cp = tb.czp[k * n + l], cm = tb.czm[k * n + l];
        fpr = fma(cp.re, ml, fpr);
        fpi = fma(cp.im, ml, fpi);
        fmr = fma(cm.re, ml, fmr);
        fmi = fma(cm.im, ml, fmi);
      }
#pragma unroll
    for (int di = 0; di < 4; di++) {
      const int D = (di < 2) ? di - 2 : di - 1;
      const int nd = dk + D;
      if (nd < 0 || nd >= rk) continue;
      Cx<R> c = tb.hoff[(k * 4 + di) * 16 + dk];
      if (D == -1) {
        const R gg = tb.gp[k * 16 + dk];
        c.re = fma(gg, fpr, c.re);
        c.im = fma(gg, fpi, c.im);
      } else if (D == 1) {
        const R gg = tb.gm[k * 16 + dk];
        c.re = fma(gg, fmr, c.re);
        c.im = fma(gg, fmi, c.im);
      }
      bmac<R, KC>(acc, c.re, c.im, v + (size_t)(row + (uint32_t)(D * (int)st)) * KC);
    }
  }
  for (int p = 0; p < npair; p++) {
    const int2 ij = tb.pij[p];
    const int di = digit(ij.x), dj = digit(ij.y);
    const int ri = it.radix[ij.x], rj = it.radix[ij.y];
    const uint32_t si = it.stride[ij.x], sj = it.stride[ij.y];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const Cx<R> cq = tb.pc[4 * p + q];
      if (cq.re == R(0) && cq.im == R(0)) continue;
      const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;
      const bool vi = im_ ? (di <= ri - 2) : (di >= 1);
      const bool vj = jm ? (dj <= rj - 2) : (dj >= 1);
      if (!(vi && vj)) continue;
      const R f = (im_ ? tb.gm[ij.x * 16 + di] : tb.gp[ij.x * 16 + di]) *
                  (jm ? tb.gm[ij.y * 16 + dj] : tb.gp[ij.y * 16 + dj]);
      const uint32_t partner = row + (im_ ? si : (uint32_t)(-(int)si)) + (jm ? sj : (uint32_t)(-(int)sj));
      bmac<R, KC>(acc, cq.re * f, cq.im * f, v + (size_t)partner * KC);
    }
  }
}

// ------------------------------------------------------------------ kernels
template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void bstart_kernel(const BItem<R> *__restrict__ items, BStep S) {
  for (uint32_t u = blockIdx.x; u < S.n_units; u += gridDim.x) {
    const int ii = S.unit_item[u];
    const BItem<R> &it = items[ii];
    const uint32_t r0 = (u - it.unit0) << S.ubits, r1 = min(it.dim, r0 + (1u << S.ubits));
    double red[1][KC];
#pragma unroll
    for (int q = 0; q < KC; q++) red[0][q] = 0.0;
    Cx<R> *x = it.x[0];
    for (uint32_t row = r0 + threadIdx.x; row < r1; row += kBlock) {
#pragma unroll
      for (int q = 0; q < KC; q++) {
        uint32_t c[4] = {row, it.rng_r0 + (uint32_t)q, it.rng_field, it.rng_inst};
        // Philox4x32-10 + Box-Muller, as in the plain start-vector kernel
        uint32_t k0 = (uint32_t)S.seed, k1 = (uint32_t)(S.seed >> 32);
#pragma unroll
        for (int rr = 0; rr < 10; rr++) {
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
        const uint64_t a = ((uint64_t)(c[0] >> 5) << 26) | (c[1] >> 6);
        const uint64_t b = ((uint64_t)(c[2] >> 5) << 26) | (c[3] >> 6);
        const double u1 = (double)(a + 1) * 0x1.0p-53, u2 = (double)b * 0x1.0p-53;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos(2.0 * M_PI * u2, &sn, &cs);
        const Cx<R> z{(R)(rad * cs), (R)(rad * sn)};
        x[(size_t)row * KC + q] = z;
        red[0][q] += (double)z.re * (double)z.re + (double)z.im * (double)z.im;
      }
    }
    block_partials_store<1, KC>(red, S.part, u);
    __syncthreads();  // the block's LDS partials are reused by the next unit
  }
}

template <typename R, int KC, int NT>
__global__ __launch_bounds__(NT) void bhv_kernel(const BItem<R> *__restrict__ items, BStep S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = S.step;
  int staged = -1;  // item whose tables are in LDS (a block's units are mostly of one item)
  for (uint32_t u = blockIdx.x; u < S.n_units; u += gridDim.x) {
    const int ii = S.unit_item[u];
    const BItem<R> &it = items[ii];
    if (ii != staged) {
      __syncthreads();
      stage_tables(it, S.mode == 0, smem);
      __syncthreads();
      staged = ii;
    }
    const DevTables<R> lt = table_layout(it, S.mode == 0, smem);
    const uint32_t r0 = (u - it.unit0) << S.ubits, r1 = min(it.dim, r0 + (1u << S.ubits));
    const int usb = S.ubits - 8;
    if (it.half && it.has_z && S.mode != 0) {
      // z-field of the sites >= 8 for the unit's rows with bits 8..ubits-1 = i:
      // F_k^b(i) = sum_{l >= 8, l != k} C^b_kl m_l
      const int n = it.n;
      for (int e = threadIdx.x; e < (n * 2) << usb; e += NT) {
        const int i = e & ((1 << usb) - 1), b = (e >> usb) & 1, k = e >> (usb + 1);
        const uint32_t rb = r0 | ((uint32_t)i << 8);
        R fr = 0, fi = 0;
        for (int l = 8; l < n; l++) {
          if (l == k) continue;
          const R ml = ((rb >> l) & 1) ? R(0.5) : R(-0.5);
          const Cx<R> c = b ? lt.czp[k * n + l] : lt.czm[k * n + l];
          fr = fma(c.re, ml, fr);
          fi = fma(c.im, ml, fi);
        }
        const_cast<Cx<R> *>(lt.lowf)[e] = Cx<R>{fr, fi};
      }
      __syncthreads();
    }
    const bool moment = S.mode == 0;
    const int dmode = (moment || !it.diag) ? 0 : (j == 0 ? 1 : 2);  // uniform
    const Cx<R> *v = moment ? it.x[0] : it.x[j % 3];
    Cx<R> *w = moment ? it.ov1 : it.x[(j + 1) % 3];
    const Cx<R> *xp = (!moment && j > 0) ? it.x[(j + 2) % 3] : nullptr;
    double sx[KC], bp[KC];
#pragma unroll
    for (int q = 0; q < KC; q++) {
      sx[q] = S.sx_cur[it.col0 + q];
      bp[q] = xp ? S.beta_prev[it.col0 + q] * S.sx_prev[it.col0 + q] : 0.0;
    }
    double red[3][KC];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int q = 0; q < KC; q++) red[a][q] = 0.0;
    for (uint32_t row = r0 + threadIdx.x; row < r1; row += NT) {
      BAcc<R, KC> acc;
      brow<R, KC>(it, lt, moment, row, v, acc, it.diag, dmode, usb);
      const size_t o = (size_t)row * KC;
      // the item's vectors are device memory: global (not generic) accesses
      const GPtr<R> gxp = (GPtr<R>)xp, gv = (GPtr<R>)v, gov = (GPtr<R>)it.ov1;
      const GPtrW<R> gw = (GPtrW<R>)w;
#pragma unroll
      for (int q = 0; q < KC; q++) {
        double wr = (double)acc.re[q] * sx[q], wi = (double)acc.im[q] * sx[q];
        if (xp) {
          const Cx<R> a = gxp[o + q];
          wr -= bp[q] * (double)a.re;
          wi -= bp[q] * (double)a.im;
        }
        const Cx<R> out{(R)wr, (R)wi};
        gw[o + q].re = out.re;
        gw[o + q].im = out.im;
        if (!moment) {
          const Cx<R> xo = gv[o + q];
          const Cx<R> ov = gov[o + q];
          red[0][q] += (double)xo.re * (double)out.re + (double)xo.im * (double)out.im;
          red[1][q] += (double)ov.re * (double)xo.re + (double)ov.im * (double)xo.im;
          red[2][q] += (double)ov.re * (double)xo.im - (double)ov.im * (double)xo.re;
        }
      }
    }
    if (moment) continue;  // uniform over the launch
    block_partials_store<3, KC, NT>(red, S.part, u);
    __syncthreads();  // the block's LDS partials are reused by the next unit
  }
}

template <typename R, int KC>
__global__ __launch_bounds__(kBlock) void bupdate_kernel(const BItem<R> *__restrict__ items, BStep S) {
  const int j = S.step;
  for (uint32_t u = blockIdx.x; u < S.n_units; u += gridDim.x) {
    const int ii = S.unit_item[u];
    const BItem<R> &it = items[ii];
    const uint32_t r0 = (u - it.unit0) << S.ubits, r1 = min(it.dim, r0 + (1u << S.ubits));
    Cx<R> *w = it.x[(j + 1) % 3];
    const Cx<R> *x = it.x[j % 3];
    double coef[KC], red[1][KC];
#pragma unroll
    for (int q = 0; q < KC; q++) {
      coef[q] = S.alpha[it.col0 + q] * S.sx_cur[it.col0 + q];
      red[0][q] = 0.0;
    }
    for (uint32_t row = r0 + threadIdx.x; row < r1; row += kBlock) {
      const size_t o = (size_t)row * KC;
#pragma unroll
      for (int q = 0; q < KC; q++) {
        const Cx<R> a = w[o + q], b = x[o + q];
        const Cx<R> uu{(R)((double)a.re - coef[q] * (double)b.re), (R)((double)a.im - coef[q] * (double)b.im)};
        w[o + q] = uu;
        red[0][q] += (double)uu.re * (double)uu.re + (double)uu.im * (double)uu.im;
      }
    }
    block_partials_store<1, KC>(red, S.part, u);
    __syncthreads();  // the block's LDS partials are reused by the next unit
  }
}

// One block per item: the item's per-unit partials summed in unit order, then
// the step's per-column scalars.  kind 0: start-vector norms -> sx; 1: alpha
// and <O v_1, v_j> (already scaled by sx); 2: beta, breakdown and the next
// scale.
template <typename R>
__global__ __launch_bounds__(kBlock) void bfinish_kernel(const BItem<R> *__restrict__ items, BStep S, int kind) {
  const BItem<R> &it = items[blockIdx.x];
  const int K = S.K, j = S.step;
  const int nv = kind == 1 ? 3 : 1;
  for (int idx = 0; idx < nv * K; idx++) {  // whole block, fixed order over the item's units
    const int a = idx / K, q = idx % K, c = it.col0 + q;
    const double s = block_sum_strided(S.part + ((size_t)it.unit0 * nv + a) * K + q, it.nunit, (size_t)nv * K);
    if (threadIdx.x != 0) continue;
    if (kind == 0) {
      S.sx_cur[c] = s > 0 ? 1.0 / sqrt(s) : 0.0;
    } else if (kind == 1) {
      const double v = s * S.sx_cur[c];
      if (a == 0) S.alpha[c] = v;
      else if (a == 1) S.yre[c] = v;
      else S.yim[c] = v;
    } else {
      const double b = sqrt(s);
      double sm = S.smax[c];
      const double al = fabs(S.alpha[c]);
      if (al > sm) sm = al;
      if (S.done[c]) {
        S.beta[c] = 0.0;
        S.sx_next[c] = 0.0;
      } else {
        S.nused[c] = j + 1;
        const bool breakdown = (j + 1 < S.n_lanczos) && !(b > 1e-12 * sm);
        S.beta[c] = b;
        if (breakdown) {
          S.done[c] = 1;
          S.sx_next[c] = 0.0;
        } else {
          S.sx_next[c] = b > 0 ? 1.0 / b : 0.0;
        }
        if (b > sm) sm = b;
      }
      S.smax[c] = sm;
    }
  }
}

__global__ void bzero_kernel(double *smax, int *done, int *nused, int ncol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncol) {
    smax[i] = 0.0;
    done[i] = 0;
    nused[i] = 0;
  }
}

// ------------------------------------------------------------------ host driver
namespace {

struct Carve {
  size_t off = 0;
  size_t take(size_t n) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return o;
  }
};

// Columns per item: the requested count if it is one of 16, 8, 4, 2, 1 and
// divides R; automatic: 4 once the largest instance has 2^17 rows or more (the
// gathers of 16 interleaved columns then miss the caches), else the widest of
// 16, 8, 4, 2, 1 dividing R.
int pick_batch_k(int R, int requested, uint64_t max_dim) {
  const int opts[5] = {16, 8, 4, 2, 1};
  if (requested > 0) {
    for (int o : opts)
      if (o == requested && R % o == 0) return o;
    return -1;
  }
  if (max_dim >= (1ull << 17))
    for (int o : {4, 2, 1})
      if (R % o == 0) return o;
  for (int o : opts)
    if (R % o == 0) return o;
  return 1;
}

template <typename R>
size_t site_block_bytes(int maxn) {
  return (((size_t)maxn * 16 * sizeof(R) + (size_t)maxn * 66 * sizeof(Cx<R>)) + 255) & ~size_t(255);
}

struct CurveInfo {
  int inst, field;
  double B[3];
};

struct PlanB {
  int K, R, NL, nT, prec, n_inst;
  size_t es;
  std::vector<CurveInfo> curves;
  std::vector<int> curve0;       // first curve of each instance
  size_t fixed = 0;              // bytes of the fixed part
  // fixed-part offsets
  size_t site_tabs, eps, q1, qy, nused_all, T, dims, lnZ, E, C, M, emin, tri;
  size_t site_bytes_per_curve = 0;
  size_t max_vec_bytes = 0;      // largest single item
  size_t all_vec_bytes = 0;      // every item at once
};

int validate_batched(const ftlm_hamiltonian *const *hs, int n_inst, const ftlm_run_params *pp,
                     std::string &err) {
  if (!hs || !pp || n_inst < 1) {
    err = "hs, per_inst and n_inst >= 1 are required";
    return FTLM_EINVAL;
  }
  for (int k = 0; k < n_inst; k++) {
    if (!hs[k]) {
      err = "NULL Hamiltonian";
      return FTLM_EINVAL;
    }
    const ftlm_run_params &p = pp[k];
    if (p.R < 1 || p.n_lanczos < 1 || p.n_lanczos > 1024 || p.n_T < 1 || !p.T) {
      err = "bad R, n_lanczos or temperature grid";
      return FTLM_EINVAL;
    }
    if (p.precision != FTLM_C128 && p.precision != FTLM_C64) {
      err = "bad precision";
      return FTLM_EINVAL;
    }
    if (p.r_init) {
      err = "r_init is not supported by the batched run";
      return FTLM_EINVAL;
    }
    if (p.fields && p.n_fields < 1) {
      err = "n_fields must be >= 1";
      return FTLM_EINVAL;
    }
    if (!p.fields && p.n_fields > 1) {
      err = "n_fields > 1 needs a fields array";
      return FTLM_EINVAL;
    }
    for (int i = 0; i < p.n_T; i++)
      if (!(p.T[i] > 0)) {
        err = "temperatures must be positive";
        return FTLM_EINVAL;
      }
    if (p.R != pp[0].R || p.n_lanczos != pp[0].n_lanczos || p.n_T != pp[0].n_T ||
        p.precision != pp[0].precision || p.columns != pp[0].columns) {
      err = "R, n_lanczos, n_T, precision and columns must agree across instances";
      return FTLM_EINVAL;
    }
    for (int i = 0; i < p.n_T; i++)
      if (p.T[i] != pp[0].T[i]) {
        err = "temperature grids must agree across instances";
        return FTLM_EINVAL;
      }
  }
  if (pick_batch_k(pp[0].R, pp[0].columns, 0) < 0) {
    err = "columns must be one of 1, 2, 4, 8, 16 and divide R";
    return FTLM_EINVAL;
  }
  return FTLM_OK;
}

void make_plan_b(const ftlm_hamiltonian *const *hs, int n_inst, const ftlm_run_params *pp, PlanB &pl) {
  uint64_t max_dim = 0;
  for (int k = 0; k < n_inst; k++) max_dim = std::max<uint64_t>(max_dim, hs[k]->host.dim);
  pl.K = pick_batch_k(pp[0].R, pp[0].columns, max_dim);
  pl.R = pp[0].R;
  pl.NL = pp[0].n_lanczos;
  pl.nT = pp[0].n_T;
  pl.prec = pp[0].precision;
  pl.es = pl.prec == FTLM_C64 ? 8 : 16;
  pl.n_inst = n_inst;
  pl.curves.clear();
  pl.curve0.assign(n_inst, 0);
  int maxn = 1;
  for (int k = 0; k < n_inst; k++) {
    pl.curve0[k] = (int)pl.curves.size();
    const int nf = pp[k].fields ? pp[k].n_fields : 1;
    for (int f = 0; f < nf; f++) {
      CurveInfo c;
      c.inst = k;
      c.field = f;
      for (int a = 0; a < 3; a++) c.B[a] = pp[k].fields ? pp[k].fields[3 * f + a] : hs[k]->host.B[a];
      pl.curves.push_back(c);
    }
    maxn = std::max(maxn, hs[k]->host.n);
  }
  // one-site tables per curve: for each precision hdiag [n][16] R, hoff [n][64] Cx,
  // hflip [n][2] Cx -- for H and for O
  pl.site_bytes_per_curve = 2 * site_block_bytes<double>(maxn) + 2 * site_block_bytes<float>(maxn);
  const size_t ncurve = pl.curves.size(), ncol_all = ncurve * pl.R;
  Carve c;
  pl.site_tabs = c.take(pl.site_bytes_per_curve * ncurve);
  pl.eps = c.take(sizeof(double) * pl.NL * ncol_all);
  pl.q1 = c.take(sizeof(double) * pl.NL * ncol_all);
  pl.qy = c.take(sizeof(double) * pl.NL * ncol_all);
  pl.nused_all = c.take(sizeof(int) * ncol_all);
  pl.T = c.take(sizeof(double) * pl.nT);
  pl.dims = c.take(sizeof(double) * ncurve);
  pl.lnZ = c.take(sizeof(double) * pl.nT * ncurve);
  pl.E = c.take(sizeof(double) * pl.nT * ncurve);
  pl.C = c.take(sizeof(double) * pl.nT * ncurve);
  pl.M = c.take(sizeof(double) * pl.nT * ncurve);
  pl.emin = c.take(sizeof(double) * ncurve);
  pl.fixed = (c.off + 255) & ~size_t(255);
  pl.max_vec_bytes = 0;
  pl.all_vec_bytes = 0;
  for (size_t ci = 0; ci < ncurve; ci++) {
    const uint64_t dim = hs[pl.curves[ci].inst]->host.dim;
    // four vectors [dim][K] and the diagonal of H [dim], each 256-byte aligned
    const size_t per_item = 4 * (size_t)dim * pl.K * pl.es + (size_t)dim * (pl.es / 2) + 5 * 256;
    pl.max_vec_bytes = std::max(pl.max_vec_bytes, per_item);
    pl.all_vec_bytes += per_item * (size_t)(pl.R / pl.K);
  }
}

// per-wave dynamic part: item array, unit map, scalars, partials, tridiag scratch
size_t wave_meta_bytes(size_t n_items, size_t n_units, int K, int NL) {
  const size_t ncol = n_items * (size_t)K;
  Carve c;
  c.take(sizeof(BItem<double>) * n_items);
  c.take(sizeof(int) * n_units);
  c.take(sizeof(double) * ncol * NL * 4);       // alpha, beta, yre, yim
  c.take(sizeof(double) * ncol * (NL + 1));     // sx
  c.take(sizeof(double) * ncol);                // smax
  c.take(sizeof(int) * ncol * 2);               // done, nused
  c.take(sizeof(double) * n_units * 3 * K);     // partials
  c.take(sizeof(double) * 4 * NL * ncol);       // tridiagonal scratch
  return (c.off + 255) & ~size_t(255);
}

template <typename R>
void pack_site(const HostHam &hh, unsigned char *dst, int maxn, DevTables<R> &tb_rel) {
  // layout: hdiag [maxn][16] R, hoff [maxn][64] Cx, hflip [maxn][2] Cx
  R *hd = reinterpret_cast<R *>(dst);
  Cx<R> *ho = reinterpret_cast<Cx<R> *>(hd + (size_t)maxn * 16);
  Cx<R> *hf = ho + (size_t)maxn * 64;
  std::memset(dst, 0, (size_t)maxn * 16 * sizeof(R) + (size_t)maxn * 66 * sizeof(Cx<R>));
  for (int k = 0; k < hh.n; k++) {
    const int r = hh.radix[k];
    for (int d = 0; d < r; d++) {
      hd[k * 16 + d] = (R)hh.h[(size_t)k * 256 + d * 16 + d].re;
      const int Ds[4] = {-2, -1, 1, 2};
      for (int di = 0; di < 4; di++) {
        const int nd = d + Ds[di];
        if (nd < 0 || nd >= r) continue;
        const Cx<double> c = hh.h[(size_t)k * 256 + d * 16 + nd];
        ho[(k * 4 + di) * 16 + d] = Cx<R>{(R)c.re, (R)c.im};
      }
    }
    if (r == 2) {
      const Cx<double> a = hh.h[(size_t)k * 256 + 1], c = hh.h[(size_t)k * 256 + 16];
      hf[2 * k] = Cx<R>{(R)a.re, (R)a.im};
      hf[2 * k + 1] = Cx<R>{(R)c.re, (R)c.im};
    }
  }
  // offsets relative to dst, resolved against the device address later
  tb_rel.hdiag = reinterpret_cast<const R *>((uintptr_t)0);
  tb_rel.hoff = reinterpret_cast<const Cx<R> *>((uintptr_t)((unsigned char *)ho - dst));
  tb_rel.hflip = reinterpret_cast<const Cx<R> *>((uintptr_t)((unsigned char *)hf - dst));
}

template <typename R, int KC, int NT>
void launch_bhv(dim3 grid, const BItem<R> *items, const BStep &S, hipStream_t s) {
  static uint32_t granted = 64 * 1024;  // per instantiation
  if (S.lds > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&bhv_kernel<R, KC, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)S.lds);
    granted = S.lds;
  }
  hipLaunchKernelGGL((bhv_kernel<R, KC, NT>), grid, dim3(NT), S.lds, s, items, S);
}

template <typename R, int KC>
void launch_b(int kind, dim3 grid, const BItem<R> *items, const BStep &S, hipStream_t s) {
  if (kind == 0) hipLaunchKernelGGL((bstart_kernel<R, KC>), grid, dim3(kBlock), 0, s, items, S);
  else if (kind == 1) {
    if (S.block == 256) launch_bhv<R, KC, 256>(grid, items, S, s);
    else if (S.block == 1024) launch_bhv<R, KC, 1024>(grid, items, S, s);
    else launch_bhv<R, KC, 512>(grid, items, S, s);
  }
  else hipLaunchKernelGGL((bupdate_kernel<R, KC>), grid, dim3(kBlock), 0, s, items, S);
  if (kind != 1 || S.mode == 1)  // O v_1 has no reductions
    hipLaunchKernelGGL((bfinish_kernel<R>), dim3(S.n_items), dim3(kBlock), 0, s, items, S, kind);
}

template <typename R>
void launch_bk(int kind, int K, dim3 grid, const void *items, const BStep &S, hipStream_t s) {
  const BItem<R> *it = reinterpret_cast<const BItem<R> *>(items);
  switch (K) {
    case 16: launch_b<R, 16>(kind, grid, it, S, s); break;
    case 8: launch_b<R, 8>(kind, grid, it, S, s); break;
    case 4: launch_b<R, 4>(kind, grid, it, S, s); break;
    case 2: launch_b<R, 2>(kind, grid, it, S, s); break;
    default: launch_b<R, 1>(kind, grid, it, S, s); break;
  }
}

}  // namespace

}  // namespace ftlm

using namespace ftlm;

extern "C" {

int ftlm_run_batched_workspace_size(const ftlm_hamiltonian *const *hs, int32_t n_inst,
                                    const ftlm_run_params *per_inst, size_t *bytes) {
  std::string err;
  if (!bytes) {
    set_error("bytes is NULL");
    return FTLM_EINVAL;
  }
  int rc = validate_batched(hs, n_inst, per_inst, err);
  if (rc) {
    set_error(err);
    return rc;
  }
  PlanB pl;
  make_plan_b(hs, n_inst, per_inst, pl);
  // all items at once if that is below 160 GiB, else a budget of 160 GiB of vectors
  const size_t budget = (size_t)160 << 30;
  size_t vec = std::min(pl.all_vec_bytes, std::max(budget, pl.max_vec_bytes));
  size_t n_items = 0, n_units = 0;
  for (const CurveInfo &c : pl.curves) {
    n_items += pl.R / pl.K;
    n_units += (size_t)(pl.R / pl.K) * ((hs[c.inst]->host.dim + kUnitRows - 1) / kUnitRows);
  }
  *bytes = pl.fixed + vec + wave_meta_bytes(n_items, n_units, pl.K, pl.NL);
  return FTLM_OK;
}

int ftlm_run_batched(const ftlm_hamiltonian *const *hs, int32_t n_inst, const ftlm_run_params *pp,
                     void *ws, size_t bytes, void *stream_, ftlm_result *out) {
  std::string err;
  if (!ws || !out) {
    set_error("NULL argument");
    return FTLM_EINVAL;
  }
  int rc = validate_batched(hs, n_inst, pp, err);
  if (rc) {
    set_error(err);
    return rc;
  }
  PlanB pl;
  make_plan_b(hs, n_inst, pp, pl);
  if (bytes < pl.fixed + pl.max_vec_bytes) {
    set_error("workspace too small");
    return FTLM_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream_;
  unsigned char *base = reinterpret_cast<unsigned char *>(ws);
  const int K = pl.K, NL = pl.NL, R = pl.R;
  const size_t ncurve = pl.curves.size();
  const bool f32 = pl.prec == FTLM_C64;
  int maxn = 1;
  for (int k = 0; k < n_inst; k++) maxn = std::max(maxn, hs[k]->host.n);

  // one-site tables of H and O for every curve, both precisions
  const size_t sb64 = site_block_bytes<double>(maxn), sb32 = site_block_bytes<float>(maxn);
  std::vector<unsigned char> host_sites(pl.site_bytes_per_curve * ncurve, 0);
  std::vector<double> dims(ncurve);
  for (size_t ci = 0; ci < ncurve; ci++) {
    const CurveInfo &c = pl.curves[ci];
    HostHam hh = hs[c.inst]->host;
    for (int a = 0; a < 3; a++) hh.B[a] = c.B[a];
    compile_site_terms(hh);
    HostHam ho;
    {
      double bh[3], beff[3];
      const double nb = std::sqrt(c.B[0] * c.B[0] + c.B[1] * c.B[1] + c.B[2] * c.B[2]);
      for (int a = 0; a < 3; a++) bh[a] = nb > 0 ? c.B[a] / nb : (a == 2 ? 1.0 : 0.0);
      for (int a = 0; a < 3; a++) beff[a] = -bh[a] / kMuB;
      ftlm_system so{};
      so.n_sites = hh.n;
      so.two_s = hh.two_s;
      so.g = hh.g.data();
      so.B = beff;
      if (compile_hamiltonian(&so, ho, err)) {
        set_error(err);
        return FTLM_EINVAL;
      }
    }
    unsigned char *dst = host_sites.data() + pl.site_bytes_per_curve * ci;
    DevTables<double> d64;
    DevTables<float> d32;
    pack_site<double>(hh, dst, maxn, d64);
    pack_site<double>(ho, dst + sb64, maxn, d64);
    pack_site<float>(hh, dst + 2 * sb64, maxn, d32);
    pack_site<float>(ho, dst + 2 * sb64 + sb32, maxn, d32);
    dims[ci] = (double)hh.dim;
  }
  if (hipMemcpy(base + pl.site_tabs, host_sites.data(), host_sites.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + pl.T, pp[0].T, sizeof(double) * pl.nT, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + pl.dims, dims.data(), sizeof(double) * ncurve, hipMemcpyHostToDevice) != hipSuccess) {
    set_error("copy of batched inputs failed");
    return FTLM_EHIP;
  }
  // device pointers of one curve's one-site tables (precision R, operator H or O)
  auto site_ptrs = [&](size_t ci, bool single, bool moment, const void **hd, const void **ho, const void **hf) {
    unsigned char *blk = base + pl.site_tabs + pl.site_bytes_per_curve * ci;
    size_t off = single ? 2 * sb64 + (moment ? sb32 : 0) : (moment ? sb64 : 0);
    const size_t rs = single ? 4 : 8;
    *hd = blk + off;
    *ho = blk + off + (size_t)maxn * 16 * rs;
    *hf = blk + off + (size_t)maxn * 16 * rs + (size_t)maxn * 64 * 2 * rs;
  };

  // items in curve order: (curve, group)
  struct Item {
    size_t curve;
    int group;
  };
  std::vector<Item> items;
  for (size_t ci = 0; ci < ncurve; ci++)
    for (int g = 0; g < R / K; g++) items.push_back({ci, g});
  const size_t avail = bytes - pl.fixed;
  const bool timing = out[0].hv_ms != nullptr;
  const bool use_graph = true;
  const BatchTuning bt = g_btune;
  const uint32_t urows = 1u << bt.ubits;
  hipEvent_t tev[2] = {nullptr, nullptr};
  double step_ms = 0.0;
  int step_launches = 0;
  if (timing && (hipEventCreate(&tev[0]) != hipSuccess || hipEventCreate(&tev[1]) != hipSuccess)) {
    set_error("hipEventCreate failed");
    return FTLM_EHIP;
  }
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 2; i++)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{tev};
  size_t next = 0;
  while (next < items.size()) {
    // greedy wave: as many items as fit with their metadata
    size_t end = next, vec = 0, units = 0;
    while (end < items.size()) {
      const uint64_t dim = hs[pl.curves[items[end].curve].inst]->host.dim;
      const size_t iv = 4 * (((size_t)dim * K * pl.es + 255) & ~size_t(255)) +
                        (((size_t)dim * (pl.es / 2) + 255) & ~size_t(255));
      const size_t iu = (dim + urows - 1) / urows;
      const size_t meta = wave_meta_bytes(end + 1 - next, units + iu, K, NL);
      if (vec + iv + meta > avail && end > next) break;
      vec += iv;
      units += iu;
      end++;
    }
    const size_t nit = end - next, ncol = nit * K;
    Carve c;
    const size_t o_items = c.take(sizeof(BItem<double>) * nit);
    const size_t o_umap = c.take(sizeof(int) * units);
    const size_t o_alpha = c.take(sizeof(double) * ncol * NL);
    const size_t o_beta = c.take(sizeof(double) * ncol * NL);
    const size_t o_yre = c.take(sizeof(double) * ncol * NL);
    const size_t o_yim = c.take(sizeof(double) * ncol * NL);
    const size_t o_sx = c.take(sizeof(double) * ncol * (NL + 1));
    const size_t o_smax = c.take(sizeof(double) * ncol);
    const size_t o_done = c.take(sizeof(int) * ncol);
    const size_t o_nused = c.take(sizeof(int) * ncol);
    const size_t o_part = c.take(sizeof(double) * units * 3 * K);
    const size_t o_tri = c.take(sizeof(double) * 4 * NL * ncol);
    const size_t meta_end = (c.off + 255) & ~size_t(255);
    unsigned char *wbase = base + pl.fixed;
    unsigned char *vbase = wbase + meta_end;
    // item descriptors (curve order); their units are laid out in the tuned
    // order: curve order, or largest instance first (the long items start
    // first and the small ones fill the launch's tail)
    std::vector<unsigned char> hitems(sizeof(BItem<double>) * nit);
    std::vector<int> umap(units);
    std::vector<uint32_t> unit0_of(nit, 0);
    {
      std::vector<size_t> uord(nit);
      for (size_t i = 0; i < nit; i++) uord[i] = i;
      if (bt.order == 1)
        std::stable_sort(uord.begin(), uord.end(), [&](size_t a, size_t b) {
          return hs[pl.curves[items[next + a].curve].inst]->host.dim > hs[pl.curves[items[next + b].curve].inst]->host.dim;
        });
      uint32_t uu = 0;
      for (size_t i : uord) {
        const uint32_t dim = (uint32_t)hs[pl.curves[items[next + i].curve].inst]->host.dim;
        const uint32_t nunit = (dim + urows - 1) / urows;
        unit0_of[i] = uu;
        for (uint32_t v2 = 0; v2 < nunit; v2++) umap[uu + v2] = (int)i;
        uu += nunit;
      }
    }
    size_t voff = 0;
    for (size_t i = 0; i < nit; i++) {
      const Item &itm = items[next + i];
      const CurveInfo &cv = pl.curves[itm.curve];
      const ftlm_hamiltonian *h = hs[cv.inst];
      const uint32_t dim = (uint32_t)h->host.dim;
      const uint32_t nunit = (dim + urows - 1) / urows;
      const size_t vb = ((size_t)dim * K * pl.es + 255) & ~size_t(255);
      const size_t vbd = ((size_t)dim * (pl.es / 2) + 255) & ~size_t(255);
      auto fill = [&](auto tag) {
        using R = decltype(tag);
        BItem<R> bi;
        std::memset(&bi, 0, sizeof(bi));
        const DevTables<R> &src = f32 ? *reinterpret_cast<const DevTables<R> *>(&h->dev.t32)
                                      : *reinterpret_cast<const DevTables<R> *>(&h->dev.t64);
        bi.tb = src;
        bi.tbo = src;
        const void *hd, *ho, *hf;
        site_ptrs(itm.curve, f32, false, &hd, &ho, &hf);
        bi.tb.hdiag = reinterpret_cast<const R *>(hd);
        bi.tb.hoff = reinterpret_cast<const Cx<R> *>(ho);
        bi.tb.hflip = reinterpret_cast<const Cx<R> *>(hf);
        site_ptrs(itm.curve, f32, true, &hd, &ho, &hf);
        bi.tbo.hdiag = reinterpret_cast<const R *>(hd);
        bi.tbo.hoff = reinterpret_cast<const Cx<R> *>(ho);
        bi.tbo.hflip = reinterpret_cast<const Cx<R> *>(hf);
        bi.n = h->host.n;
        bi.npair = h->host.npair;
        bi.has_z = h->host.has_z;
        bi.half = h->host.spin_half;
        bi.pow2r = 1;
        for (int k = 0; k < h->host.n; k++)
          if (h->host.radix[k] & (h->host.radix[k] - 1)) bi.pow2r = 0;
        bi.dim = dim;
        bi.unit0 = unit0_of[i];
        bi.nunit = nunit;
        bi.col0 = (int)(i * K);
        bi.rng_inst = pp[cv.inst].instance;
        bi.rng_field = (uint32_t)cv.field;
        bi.rng_r0 = (uint32_t)(itm.group * K);
        for (int q = 0; q < 3; q++) bi.x[q] = reinterpret_cast<Cx<R> *>(vbase + voff + q * vb);
        bi.ov1 = reinterpret_cast<Cx<R> *>(vbase + voff + 3 * vb);
        bi.diag = reinterpret_cast<R *>(vbase + voff + 4 * vb);
        for (int k = 0; k < h->host.n; k++) {
          bi.radix[k] = h->host.radix[k];
          bi.stride[k] = h->host.stride[k];
        }
        std::memcpy(hitems.data() + i * sizeof(BItem<double>), &bi, sizeof(bi));
      };
      if (f32) fill(float(0));
      else fill(double(0));
      voff += 4 * vb + vbd;
    }
    if (hipMemcpy(wbase + o_items, hitems.data(), hitems.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(wbase + o_umap, umap.data(), sizeof(int) * units, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("copy of wave descriptors failed");
      return FTLM_EHIP;
    }
    const uint32_t gx = (uint32_t)std::min<size_t>(units, (size_t)bt.grid_cap);
    BStep S{};
    S.K = K;
    S.n_lanczos = NL;
    S.n_units = (uint32_t)units;
    S.seed = pp[0].seed;
    S.part = reinterpret_cast<double *>(wbase + o_part);
    S.n_items = (uint32_t)nit;
    S.ubits = bt.ubits;
    S.block = bt.block;
    {
      size_t lds = 16;
      for (size_t i = 0; i < nit; i++) {
        const HostHam &hh = hs[pl.curves[items[next + i].curve].inst]->host;
        lds = std::max(lds, staged_bytes(hh.n, hh.npair, hh.spin_half, pl.es / 2));
      }
      // with the block's static partial-sum array (block_partials_store)
      const size_t stat = (size_t)(bt.block / 64) * 3 * (size_t)K * sizeof(double);
      if (lds + stat > 160 * 1024) {
        set_error("batched item tables exceed the LDS");
        return FTLM_ERANGE;
      }
      S.lds = (uint32_t)lds;
    }
    S.unit_item = reinterpret_cast<const int *>(wbase + o_umap);
    S.smax = reinterpret_cast<double *>(wbase + o_smax);
    S.done = reinterpret_cast<int *>(wbase + o_done);
    S.nused = reinterpret_cast<int *>(wbase + o_nused);
    double *alpha = reinterpret_cast<double *>(wbase + o_alpha);
    double *beta = reinterpret_cast<double *>(wbase + o_beta);
    double *yre = reinterpret_cast<double *>(wbase + o_yre);
    double *yim = reinterpret_cast<double *>(wbase + o_yim);
    double *sx = reinterpret_cast<double *>(wbase + o_sx);
    const void *ditems = wbase + o_items;
    hipLaunchKernelGGL(bzero_kernel, dim3((ncol + 255) / 256), dim3(256), 0, s, S.smax, S.done, S.nused,
                       (int)ncol);
    // start vectors (norms -> sx[0]) and O v_1
    BStep S0 = S;
    S0.sx_cur = sx;
    S0.step = 0;
    S0.mode = 0;
    if (f32) {
      launch_bk<float>(0, K, dim3(gx), ditems, S0, s);
      launch_bk<float>(1, K, dim3(gx), ditems, S0, s);
    } else {
      launch_bk<double>(0, K, dim3(gx), ditems, S0, s);
      launch_bk<double>(1, K, dim3(gx), ditems, S0, s);
    }
    if (hipGetLastError() != hipSuccess) {
      set_error("batched start launch failed");
      return FTLM_EHIP;
    }
    auto issue = [&](hipStream_t st) {
      for (int j = 0; j < NL; j++) {
        BStep Sj = S;
        Sj.step = j;
        Sj.mode = 1;
        Sj.alpha = alpha + (size_t)j * ncol;
        Sj.beta = beta + (size_t)j * ncol;
        Sj.yre = yre + (size_t)j * ncol;
        Sj.yim = yim + (size_t)j * ncol;
        Sj.sx_cur = sx + (size_t)j * ncol;
        Sj.sx_prev = j > 0 ? sx + (size_t)(j - 1) * ncol : nullptr;
        Sj.beta_prev = j > 0 ? beta + (size_t)(j - 1) * ncol : nullptr;
        Sj.sx_next = sx + (size_t)(j + 1) * ncol;
        if (f32) {
          launch_bk<float>(1, K, dim3(gx), ditems, Sj, st);
          launch_bk<float>(2, K, dim3(gx), ditems, Sj, st);
        } else {
          launch_bk<double>(1, K, dim3(gx), ditems, Sj, st);
          launch_bk<double>(2, K, dim3(gx), ditems, Sj, st);
        }
      }
      return hipGetLastError() == hipSuccess;
    };
    if (use_graph) {
      hipStream_t cap = nullptr;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess &&
                hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
      bool issued = ok && issue(cap);
      if (ok) ok = hipStreamEndCapture(cap, &graph) == hipSuccess && issued;
      if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (ok && timing) ok = hipEventRecord(tev[0], s) == hipSuccess;
      if (ok) ok = hipGraphLaunch(exec, s) == hipSuccess;
      if (ok && timing) ok = hipEventRecord(tev[1], s) == hipSuccess;
      if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
      if (ok && timing) {
        float ms = 0;
        ok = hipEventElapsedTime(&ms, tev[0], tev[1]) == hipSuccess;
        step_ms += ms;
        step_launches += NL;
      }
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      if (cap) (void)hipStreamDestroy(cap);
      if (!ok) {
        set_error("batched graph capture or launch failed");
        return FTLM_EHIP;
      }
    } else if (!issue(s)) {
      set_error("batched Lanczos launch failed");
      return FTLM_EHIP;
    }
    // Krylov eigenpairs of every column of the wave in one launch: items are in
    // (curve, group) order, so item j's columns sit at global positions
    // curve * R + group * K + c = j * K + c and the wave's columns are contiguous
    {
      const int gcol = (int)(next * K);
      rc = launch_tridiag((int)ncol, NL, S.nused, 1, (int)ncol, alpha, beta, yre,
                          reinterpret_cast<double *>(base + pl.eps), reinterpret_cast<double *>(base + pl.q1),
                          reinterpret_cast<double *>(base + pl.qy), (int)(ncurve * R), gcol,
                          reinterpret_cast<double *>(wbase + o_tri), s);
      if (rc) {
        set_error("tridiagonal launch failed");
        return rc;
      }
      if (hipMemcpyAsync(reinterpret_cast<int *>(base + pl.nused_all) + gcol, S.nused, sizeof(int) * ncol,
                         hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("copy of n_used failed");
        return FTLM_EHIP;
      }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
      set_error("batched wave failed");
      return FTLM_EHIP;
    }
    next = end;
  }
  rc = launch_boltzmann((int)ncurve, R, NL, reinterpret_cast<int *>(base + pl.nused_all),
                        reinterpret_cast<double *>(base + pl.eps), reinterpret_cast<double *>(base + pl.q1),
                        reinterpret_cast<double *>(base + pl.qy), reinterpret_cast<double *>(base + pl.dims),
                        reinterpret_cast<double *>(base + pl.T), pl.nT, reinterpret_cast<double *>(base + pl.lnZ),
                        reinterpret_cast<double *>(base + pl.E), reinterpret_cast<double *>(base + pl.C),
                        reinterpret_cast<double *>(base + pl.M), reinterpret_cast<double *>(base + pl.emin), s);
  if (rc) {
    set_error("Boltzmann launch failed");
    return rc;
  }
  // results per instance
  std::vector<double> hres(pl.nT * ncurve);
  std::vector<int> hn(ncurve * R);
  std::vector<double> hemin(ncurve);
  struct { size_t off; int which; } outs[4] = {{pl.lnZ, 0}, {pl.E, 1}, {pl.C, 2}, {pl.M, 3}};
  for (auto &o : outs) {
    if (hipMemcpy(hres.data(), base + o.off, sizeof(double) * hres.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("copy of results failed");
      return FTLM_EHIP;
    }
    for (int k = 0; k < n_inst; k++) {
      double *dst = o.which == 0 ? out[k].lnZ : o.which == 1 ? out[k].E : o.which == 2 ? out[k].C : out[k].M;
      if (!dst) continue;
      const int nf = pp[k].fields ? pp[k].n_fields : 1;
      std::memcpy(dst, hres.data() + (size_t)pl.curve0[k] * pl.nT, sizeof(double) * nf * pl.nT);
    }
  }
  if (hipMemcpy(hn.data(), base + pl.nused_all, sizeof(int) * hn.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hemin.data(), base + pl.emin, sizeof(double) * ncurve, hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("copy of results failed");
    return FTLM_EHIP;
  }
  for (int k = 0; k < n_inst; k++) {
    const int nf = pp[k].fields ? pp[k].n_fields : 1;
    if (out[k].n_lanczos_used)
      std::memcpy(out[k].n_lanczos_used, hn.data() + (size_t)pl.curve0[k] * R, sizeof(int) * nf * R);
    if (out[k].E_min) std::memcpy(out[k].E_min, hemin.data() + pl.curve0[k], sizeof(double) * nf);
  }
  if (timing) {
    *out[0].hv_ms = step_ms;
    if (out[0].hv_launches) *out[0].hv_launches = step_launches;
  }
  return FTLM_OK;
}

int ftlm_batched_set_tuning(int32_t grid_cap, int32_t unit_bits, int32_t order, int32_t block) {
  if (grid_cap != 0 && (grid_cap < 64 || grid_cap > 65536)) {
    set_error("grid_cap must be 0 or in [64, 65536]");
    return FTLM_EINVAL;
  }
  if (unit_bits != 0 && unit_bits != 11 && unit_bits != 12) {
    set_error("unit_bits must be 0, 11 or 12");
    return FTLM_EINVAL;
  }
  if (order < 0 || order > 1) {
    set_error("order must be 0 (curve order) or 1 (largest first)");
    return FTLM_EINVAL;
  }
  if (block != 0 && block != 256 && block != 512 && block != 1024) {
    set_error("block must be 0, 256, 512 or 1024");
    return FTLM_EINVAL;
  }
  g_btune.grid_cap = grid_cap ? grid_cap : 1024;
  g_btune.ubits = unit_bits ? unit_bits : 11;
  g_btune.order = order;
  g_btune.block = block ? block : 512;
  return FTLM_OK;
}

}  // extern "C"
