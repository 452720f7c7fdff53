// Single-pass H*v for one column (variant 6): w = H v in gather form (Sec. 2.1,
// Eq. mce-hamop, in the ladder form of ftlm_internal.hpp), one launch, every
// row of w written once.
//
// Rows are walked in tiles of the low digits (sites 0..t-1, T = st_t rows,
// contiguous in memory).  A block stages its tile of v in LDS with coalesced
// loads, then for each of its rows
//   - the diagonal: a per-row table over the tile sites, plus the tile-uniform
//     part of the outer sites and the z-z couplings between tile and outer sites
//     (phi_i = sum_j zz_ij m_j over outer j, per tile);
//   - single flips and pair flips whose sites are all tile sites: partner rows
//     from LDS;
//   - terms that move an outer digit: partner rows read straight from v.  For a
//     given term the partner rows of a tile are the tile's rows shifted by one
//     offset (plus, for a pair with one tile site, a shift inside the tile), so
//     the loads are coalesced; their validity and coefficient are uniform over
//     the tile except for the tile site's ladder factor.  Optionally (a launch
//     choice) the pairs with one tile site are grouped by their outer site and
//     move: each group's partner tile is staged in LDS once and all the group's
//     pairs (every tile site, both of its ladder moves) read it from there.
// Coefficients of invalid moves are zero in the site tables (the ladder factor
// of a digit that would leave its range is 0), and such a move reads the row's
// own element instead of an out-of-range one.
//
// Tile walk: with a grid that is a multiple of 8, block b runs on XCD b % 8
// (workgroups are dispatched to the XCDs round robin).  Chunks of consecutive
// tiles go to the XCDs in turn and each XCD's blocks walk its chunks in order:
// inside a chunk a partner tile a few tiles away is in the XCD's L2, and since
// all XCDs sweep the vector together, partner tiles further away were read
// recently by some XCD and are found in the last-level cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "device_reduce.hpp"
#include "ftlm_internal.hpp"
#include "hv_common.hpp"

namespace ftlm {

namespace {

template <typename R, bool CPLX>
__device__ __forceinline__ void cfma(R &ar, R &ai, const Cx<R> c, const Cx<R> x) {
  ar = fma(c.re, x.re, ar);
  ai = fma(c.re, x.im, ai);
  if (CPLX) {
    ar = fma(-c.im, x.im, ar);
    ai = fma(c.im, x.re, ai);
  }
}

// LDS layout of the stream kernel (sizes from the plan, offsets 16-byte aligned).
template <typename R>
struct StreamLds {
  size_t tile, hoff, pc, gp, gm, hd, pzz, phi, pij, ooff, oc, moff, mg, mc0, mc1, mi, cnt, ptile, total;
  __host__ __device__ StreamLds(const StreamGeom &g, bool stage) {
    const size_t np = (size_t)(g.np_in + g.np_mx + g.np_out), cs = sizeof(Cx<R>), rs = sizeof(R);
    const size_t no = 4 * ((size_t)g.np_out + (size_t)(g.n - g.t)), nm = (g.half ? 1 : 4) * (size_t)g.np_mx;
    size_t o = 0;
    auto take = [&](size_t b) {
      const size_t r = o;
      o += (b + 15) & ~size_t(15);
      return r;
    };
    tile = take(cs * g.T);
    hoff = take(cs * 64 * g.t);
    pc = take(cs * 4 * np);
    gp = take(rs * 16 * g.n);
    gm = take(rs * 16 * g.n);
    hd = take(rs * 16 * g.n);
    pzz = take(rs * np);
    phi = take(rs * (g.t + 1));
    pij = take(sizeof(int2) * np);
    ooff = take(sizeof(int64_t) * no);
    oc = take(cs * no);
    moff = take(sizeof(int64_t) * nm);
    mg = take(sizeof(int64_t) * nm);
    mc0 = take(cs * nm);
    mc1 = take(cs * nm);
    mi = take(sizeof(int) * nm);
    cnt = take(sizeof(int) * 2);
    ptile = stage ? take(cs * g.T) : o;  // partner tile of the staged mixed pairs
    total = o;
  }
};

// A value every lane holds alike (read from one LDS address), moved to scalar
// registers so that the compiler treats it as wave-uniform.
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint64_t u = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float uniform_r(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform_r(double x) {
  return __longlong_as_double(uniform_i64(__double_as_longlong(x)));
}
template <typename R>
__device__ __forceinline__ Cx<R> uniform_cx(const Cx<R> &c) {
  return Cx<R>{uniform_r(c.re), uniform_r(c.im)};
}

// Appends the lane's candidate to an LDS list if valid: wave-wide ballot and
// prefix count (called by all 64 lanes of one wave).
__device__ __forceinline__ int wave_append(bool valid, int count, int *pos) {
  const unsigned long long m = __ballot(valid);
  const int lane = threadIdx.x & 63;
  *pos = count + __popcll(m & ((1ull << lane) - 1ull));
  return count + __popcll(m);
}

template <typename R, bool POW2, bool HALF, bool CPLX, int RPT, int NT, bool STAGE>
__global__ __launch_bounds__(NT) void hv_stream(StreamGeom G, DevTables<R> tb, const int2 *__restrict__ pij,
                                                const Cx<R> *__restrict__ pcs, const R *__restrict__ pzz,
                                                const R *__restrict__ tdiag, const Cx<R> *__restrict__ hoffg,
                                                uint32_t chunk, HvParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = G.t, n = G.n, tid = threadIdx.x;
  const int np = G.np_in + G.np_mx + G.np_out;
  const uint32_t T = G.T;
  const StreamLds<R> L(G, STAGE);
  Cx<R> *tile = reinterpret_cast<Cx<R> *>(smem + L.tile);  // [T]
  Cx<R> *s_hoff = reinterpret_cast<Cx<R> *>(smem + L.hoff); // [t][4][16] single flips of tile sites
  Cx<R> *s_pc = reinterpret_cast<Cx<R> *>(smem + L.pc);     // [np][4]
  R *s_gp = reinterpret_cast<R *>(smem + L.gp);             // [n][16]
  R *s_gm = reinterpret_cast<R *>(smem + L.gm);             // [n][16]
  R *s_hd = reinterpret_cast<R *>(smem + L.hd);             // [n][16]
  R *s_pzz = reinterpret_cast<R *>(smem + L.pzz);           // [np]
  R *s_phi = reinterpret_cast<R *>(smem + L.phi);           // [t] phi_i, then the outer diagonal part
  int2 *s_pij = reinterpret_cast<int2 *>(smem + L.pij);     // [np]
  // per tile: the valid terms that move an outer digit
  int64_t *s_ooff = reinterpret_cast<int64_t *>(smem + L.ooff);  // uniform terms: row offset
  Cx<R> *s_oc = reinterpret_cast<Cx<R> *>(smem + L.oc);          //   and coefficient
  int64_t *s_moff = reinterpret_cast<int64_t *>(smem + L.moff);  // mixed pairs: outer offset (+ tile shift)
  int64_t *s_mg = reinterpret_cast<int64_t *>(smem + L.mg);      //   outer offset alone (the partner tile)
  Cx<R> *s_mc0 = reinterpret_cast<Cx<R> *>(smem + L.mc0);        //   uniform coefficient part
  Cx<R> *s_mc1 = reinterpret_cast<Cx<R> *>(smem + L.mc1);        //   (spin 1/2: for tile bit 0 / 1)
  int *s_mi = reinterpret_cast<int *>(smem + L.mi);              //   tile site | ladder << 8 | partner tile << 9
  int *s_cnt = reinterpret_cast<int *>(smem + L.cnt);
  for (int i = tid; i < 64 * t; i += NT) s_hoff[i] = tb.hoff[i];
  for (int i = tid; i < 4 * np; i += NT) s_pc[i] = pcs[i];
  for (int i = tid; i < 16 * n; i += NT) {
    s_gp[i] = tb.gp[i];
    s_gm[i] = tb.gm[i];
    s_hd[i] = tb.hdiag[i];
  }
  for (int i = tid; i < np; i += NT) {
    s_pzz[i] = pzz[i];
    s_pij[i] = pij[i];
  }
  // digits of the thread's rows inside a tile (the same in every tile): bit
  // fields of the row when every radix is a power of two, else 4-bit digits
  // packed here once
  uint32_t dig[RPT];
#pragma unroll
  for (int k = 0; k < RPT; k++) {
    const uint32_t r = tid + (uint32_t)k * NT;
    uint32_t pk = 0;
    if (!POW2 && r < T) {
      uint32_t rem = r;
      for (int i = 0; i < t; i++) {
        const uint32_t rd = (uint32_t)G.radix[i], q = rem / rd;
        pk |= (rem - q * rd) << (4 * i);
        rem = q;
      }
    }
    dig[k] = POW2 ? r : pk;
  }
  auto digit = [&](int k, int i) -> int {
    return POW2 ? (int)((dig[k] >> G.lg[i]) & (uint32_t)(G.radix[i] - 1)) : (int)((dig[k] >> (4 * i)) & 15u);
  };
  const Cx<R> *__restrict__ v = reinterpret_cast<const Cx<R> *>(P.v);
  double red[3][1] = {{0.0}, {0.0}, {0.0}};
  __syncthreads();

  // tile walk: chunks of `chunk` consecutive tiles are dealt to the XCDs in
  // turn (chunk c to XCD c % 8), and the blocks of an XCD walk its chunks in
  // order, so all XCDs sweep the vector together
  const bool xcd = gridDim.x >= 8 && (gridDim.x & 7u) == 0;
  const uint32_t nbx = xcd ? gridDim.x >> 3 : gridDim.x, x = xcd ? blockIdx.x & 7u : 0u;
  const uint32_t stride_c = xcd ? 8u : 1u;
  for (uint32_t l = xcd ? blockIdx.x >> 3 : blockIdx.x;; l += nbx) {
    const uint64_t tl64 = ((uint64_t)(l / chunk) * stride_c + x) * chunk + l % chunk;
    if (tl64 >= G.ntile) break;
    const uint32_t tl = (uint32_t)tl64;
    const uint32_t base = tl * T;
    // outer digits of this tile: bit fields of the row when every radix is a
    // power of two, else 4 bits each (sites t..n-1 at bit 4 (k - t), n - t <= 16)
    uint64_t od = 0;
    if (!POW2) {
      uint32_t rem = tl;
      for (int k = t; k < n; k++) {
        const uint32_t rd = (uint32_t)G.radix[k], q = rem / rd;
        od |= (uint64_t)(rem - q * rd) << (4 * (k - t));
        rem = q;
      }
    }
    auto odig = [&](int k) -> int {
      return POW2 ? (int)((base >> G.lg[k]) & (uint32_t)(G.radix[k] - 1)) : (int)((od >> (4 * (k - t))) & 15u);
    };
    auto om = [&](int k) -> R { return (R)odig(k) - (R)G.s[k]; };
    // stage the tile
#pragma unroll
    for (int k = 0; k < RPT; k++) {
      const uint32_t r = tid + (uint32_t)k * NT;
      if (r < T) tile[r] = v[base + r];
    }
    if (tid < 64) {
      // wave 0: lists of the valid terms that move an outer digit
      int no = 0, nm = 0, pos;
      const int nso = 4 * (n - t);
      for (int c0 = 0; c0 < nso; c0 += 64) {  // single flips of outer sites
        const int c = c0 + tid, j = t + c / 4, di = c & 3;
        const int D = (di < 2) ? di - 2 : di - 1;
        bool ok = c < nso && ((G.smask >> j) & 1u);
        // staged: a move by one step whose partner tile a staged group reads
        // (same outer site and move) is applied with that group instead
        if (STAGE && (D == 1 || D == -1) && ((G.gmask >> (2 * j + (D > 0))) & 1ull)) ok = false;
        int d = 0;
        if (ok) {
          d = odig(j);
          ok = (unsigned)(d + D) < (unsigned)G.radix[j];
        }
        no = wave_append(ok, no, &pos);
        if (ok) {
          s_ooff[pos] = (int64_t)D * (int64_t)G.st[j];
          s_oc[pos] = hoffg[(j * 4 + di) * 16 + d];
        }
      }
      const int p0 = G.np_in + G.np_mx;
      for (int c0 = 0; c0 < 4 * G.np_out; c0 += 64) {  // pairs of two outer sites
        const int c = c0 + tid, p = p0 + c / 4, q = c & 3;
        bool ok = c < 4 * G.np_out;
        Cx<R> cf{0, 0};
        int64_t off = 0;
        if (ok) {
          const int2 ij = s_pij[p];
          const int di = odig(ij.x), dj = odig(ij.y);
          const Cx<R> cc = s_pc[4 * p + q];
          const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;  // '-' ladder on site i / j
          ok = (cc.re != R(0) || cc.im != R(0)) && (im_ ? di <= G.radix[ij.x] - 2 : di >= 1) &&
               (jm ? dj <= G.radix[ij.y] - 2 : dj >= 1);
          if (ok) {
            const R f = (im_ ? s_gm[ij.x * 16 + di] : s_gp[ij.x * 16 + di]) *
                        (jm ? s_gm[ij.y * 16 + dj] : s_gp[ij.y * 16 + dj]);
            cf = Cx<R>{cc.re * f, cc.im * f};
            off = (im_ ? (int64_t)G.st[ij.x] : -(int64_t)G.st[ij.x]) + (jm ? (int64_t)G.st[ij.y] : -(int64_t)G.st[ij.y]);
          }
        }
        no = wave_append(ok, no, &pos);
        if (ok) {
          s_ooff[pos] = off;
          s_oc[pos] = cf;
        }
      }
      // pairs with one tile site: spin 1/2 -- one entry per pair (the move of the
      // outer bit is fixed by the tile; the tile bit picks the coefficient);
      // general -- one per (pair, ladder pair) whose outer move is valid.  The
      // mixed pairs are sorted by outer site, and the candidates are taken in
      // the order (outer ladder, pair, tile ladder), so that the entries that
      // read the same partner tile (same outer site and move) are consecutive
      const int ncm = HALF ? G.np_mx : 4 * G.np_mx;
      for (int c0 = 0; c0 < ncm; c0 += 64) {
        const int c = c0 + tid;
        const int rem = HALF ? c : c % (2 * G.np_mx);
        const int p = G.np_in + (HALF ? c : rem / 2);
        const int q = HALF ? 0 : (((rem & 1) << 1) | (c / (2 * G.np_mx)));
        bool ok = c < ncm;
        Cx<R> c0v{0, 0}, c1v{0, 0};
        int64_t off = 0, goff = 0;
        int mi = 0;
        if (ok) {
          const int2 ij = s_pij[p];
          const int dj = odig(ij.y);
          const int64_t sj = (int64_t)G.st[ij.y];
          if (HALF) {
            // row bits (b_i, b_j) -> ladder pair (b_i ? '+' : '-', b_j ? '+' : '-')
            c0v = s_pc[4 * p + 3 - (0 | dj)];
            c1v = s_pc[4 * p + 3 - (2 | dj)];
            ok = (c0v.re != R(0) || c0v.im != R(0) || c1v.re != R(0) || c1v.im != R(0));
            off = dj ? -sj : sj;
            goff = off;
            mi = ij.x | (ij.y << 9);
          } else {
            const Cx<R> cc = s_pc[4 * p + q];
            const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;
            ok = (cc.re != R(0) || cc.im != R(0)) && (jm ? dj <= G.radix[ij.y] - 2 : dj >= 1);
            if (ok) {
              const R fj = jm ? s_gm[ij.y * 16 + dj] : s_gp[ij.y * 16 + dj];
              c0v = Cx<R>{cc.re * fj, cc.im * fj};
              const int64_t si = (int64_t)G.st[ij.x];
              goff = jm ? sj : -sj;
              off = goff + (im_ ? si : -si);
              mi = ij.x | ((int)im_ << 8) | (ij.y << 9) | ((int)jm << 15);
            }
          }
        }
        nm = wave_append(ok, nm, &pos);
        if (ok) {
          s_moff[pos] = off;
          s_mg[pos] = goff;
          s_mc0[pos] = c0v;
          s_mc1[pos] = c1v;
          s_mi[pos] = mi;
        }
      }
      if (tid == 0) {
        s_cnt[0] = no;
        s_cnt[1] = nm;
      }
    } else if (tid < 64 + t) {
      // wave 1: phi_i = sum over mixed pairs (i, j) of zz m_j (lane 64 + i)
      const int i = tid - 64;
      R ph = 0;
      for (int p = G.np_in; p < G.np_in + G.np_mx; p++) {
        const int2 ij = s_pij[p];
        if (ij.x == i) ph = fma(s_pzz[p], om(ij.y), ph);
      }
      s_phi[i] = ph;
    } else if (tid == 64 + t) {
      // the outer sites' own and mutual diagonal terms
      R d0 = 0;
      for (int k = t; k < n; k++) d0 += s_hd[k * 16 + odig(k)];
      for (int p = G.np_in + G.np_mx; p < np; p++) {
        const int2 ij = s_pij[p];
        d0 = fma(s_pzz[p] * om(ij.x), om(ij.y), d0);
      }
      s_phi[t] = d0;
    }
    __syncthreads();
    R ar[RPT], ai[RPT];
    const R d0 = s_phi[t];
    // diagonal and the terms inside the tile (LDS)
#pragma unroll
    for (int k = 0; k < RPT; k++) {
      ar[k] = ai[k] = 0;
      const uint32_t r = tid + (uint32_t)k * NT;
      if (r >= T) continue;
      R dg = tdiag[r] + d0;
      for (int i = 0; i < t; i++) dg = fma((R)digit(k, i) - (R)G.s[i], s_phi[i], dg);
      const Cx<R> xo = tile[r];
      ar[k] = dg * xo.re;
      ai[k] = dg * xo.im;
      uint32_t sm = G.smask & ((t < 32) ? ((1u << t) - 1u) : 0xffffffffu);
      while (sm) {
        const int i = __builtin_ctz(sm);
        sm &= sm - 1u;
        const int d = digit(k, i), rd = G.radix[i];
        const int st = (int)G.st[i];
#pragma unroll
        for (int di = 0; di < 4; di++) {
          const int D = (di < 2) ? di - 2 : di - 1;
          if (HALF && (D == -2 || D == 2)) continue;
          const bool ok = (unsigned)(d + D) < (unsigned)rd;
          const Cx<R> c = s_hoff[(i * 4 + di) * 16 + d];
          const uint32_t pr = ok ? (uint32_t)((int)r + D * st) : r;
          cfma<R, CPLX>(ar[k], ai[k], c, tile[pr]);
        }
      }
      for (int p = 0; p < G.np_in; p++) {
        const int2 ij = s_pij[p];
        if (HALF) {
          // one move per row: both bits flip; row bits pick the ladder pair
          const uint32_t bi = (r >> ij.x) & 1u, bj = (r >> ij.y) & 1u;
          const Cx<R> c = s_pc[4 * p + 3 - (int)((bi << 1) | bj)];
          cfma<R, CPLX>(ar[k], ai[k], c, tile[r ^ ((1u << ij.x) | (1u << ij.y))]);
          continue;
        }
        const int di = digit(k, ij.x), dj = digit(k, ij.y);
        const int si = (int)G.st[ij.x], sj = (int)G.st[ij.y];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const Cx<R> c = s_pc[4 * p + q];
          if (c.re == R(0) && c.im == R(0)) continue;
          const bool im_ = (q >> 1) != 0, jm = (q & 1) != 0;
          const R f = (im_ ? s_gm[ij.x * 16 + di] : s_gp[ij.x * 16 + di]) *
                      (jm ? s_gm[ij.y * 16 + dj] : s_gp[ij.y * 16 + dj]);
          const uint32_t pr = (f != R(0)) ? (uint32_t)((int)r + (im_ ? si : -si) + (jm ? sj : -sj)) : r;
          cfma<R, CPLX>(ar[k], ai[k], Cx<R>{c.re * f, c.im * f}, tile[pr]);
        }
      }
    }
    // terms with a uniform coefficient (single flips of outer sites, pairs of
    // two outer sites): the tile's rows shifted by one offset.  The term's base
    // address and coefficient are made wave-uniform (scalar registers), so a
    // load takes the lane's 32-bit row offset only; four terms' loads are in
    // flight at a time
    const int no = s_cnt[0], nm = s_cnt[1];
    for (int e = 0; e < no; e += 4) {
      const Cx<R> *src[4];
      Cx<R> c[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int eu = e + u < no ? e + u : e;
        src[u] = v + ((int64_t)base + uniform_i64(s_ooff[eu]));
        c[u] = e + u < no ? uniform_cx(s_oc[eu]) : Cx<R>{0, 0};
      }
      Cx<R> y[4][RPT];
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int k = 0; k < RPT; k++) {
          const uint32_t r = tid + (uint32_t)k * NT;
          y[u][k] = Cx<R>{0, 0};
          if (r < T) y[u][k] = src[u][r];
        }
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int k = 0; k < RPT; k++) cfma<R, CPLX>(ar[k], ai[k], c[u], y[u][k]);
    }
    // pairs with one tile site i: the outer move is uniform; the tile site's
    // digit gives the ladder factor (or, spin 1/2, the coefficient) and validity.
    if constexpr (STAGE) {
      // staged: the entries that share a partner tile (same outer site and
      // move) read it from LDS, staged once with coalesced loads
      Cx<R> *ptile = reinterpret_cast<Cx<R> *>(smem + L.ptile);
      for (int e = 0; e < nm;) {
        const int key = __builtin_amdgcn_readfirstlane(s_mi[e] >> 9);
        int eend = e + 1;
        while (eend < nm && (s_mi[eend] >> 9) == key) eend++;
        eend = __builtin_amdgcn_readfirstlane(eend);
        const Cx<R> *src = v + ((int64_t)base + uniform_i64(s_mg[e]));
        __syncthreads();  // the previous partner tile has been read
#pragma unroll
        for (int k = 0; k < RPT; k++) {
          const uint32_t r = tid + (uint32_t)k * NT;
          if (r < T) ptile[r] = src[r];
        }
        __syncthreads();
        {
          // the single flip of the group's outer site by the same move (a step of
          // +1 for a move of +stride), if the site has single flips: left out of
          // the uniform list, it reads the staged tile's own rows
          const int j = key & 63, m = (key >> 6) & 1;
          if ((G.smask >> j) & 1u) {
            const Cx<R> cs1 = uniform_cx(hoffg[(j * 4 + (m ? 2 : 1)) * 16 + odig(j)]);
#pragma unroll
            for (int k = 0; k < RPT; k++) {
              const uint32_t r = tid + (uint32_t)k * NT;
              if (r < T) cfma<R, CPLX>(ar[k], ai[k], cs1, ptile[r]);
            }
          }
        }
        for (; e < eend; e++) {
          const Cx<R> c0v = uniform_cx(s_mc0[e]), c1v = uniform_cx(s_mc1[e]);
          const int mi = __builtin_amdgcn_readfirstlane(s_mi[e]);
          const int i = mi & 255, im_ = (mi >> 8) & 1;
          const R *gi = (im_ ? s_gm : s_gp) + i * 16;
          const int sh = im_ ? (int)G.st[i] : -(int)G.st[i];
#pragma unroll
          for (int k = 0; k < RPT; k++) {
            const uint32_t r = tid + (uint32_t)k * NT;
            if (r >= T) continue;
            Cx<R> cc;
            uint32_t idx;
            if (HALF) {
              cc = ((r >> i) & 1u) ? c1v : c0v;
              idx = r ^ (1u << i);
            } else {
              // a ladder factor of 0 marks a digit move out of range: read the row itself
              const R fi = gi[digit(k, i)];
              cc = Cx<R>{c0v.re * fi, c0v.im * fi};
              idx = fi != R(0) ? (uint32_t)((int)r + sh) : r;
            }
            cfma<R, CPLX>(ar[k], ai[k], cc, ptile[idx]);
          }
        }
      }
    }
    // direct: rows whose move is invalid load nothing (coefficient 0, value 0)
    if constexpr (!STAGE)
    for (int e = 0; e < nm; e += 2) {
      Cx<R> y[2][RPT], cr[2][RPT];
#pragma unroll
      for (int u = 0; u < 2; u++) {
        const bool oku = e + u < nm;
        const int eu = oku ? e + u : e;
        const Cx<R> *src = v + ((int64_t)base + uniform_i64(s_moff[eu]));
        const Cx<R> c0v = uniform_cx(s_mc0[eu]), c1v = uniform_cx(s_mc1[eu]);
        const int mi = __builtin_amdgcn_readfirstlane(s_mi[eu]);
        const int i = mi & 255, im_ = (mi >> 8) & 1;
        const R *gi = (im_ ? s_gm : s_gp) + i * 16;
#pragma unroll
        for (int k = 0; k < RPT; k++) {
          const uint32_t r = tid + (uint32_t)k * NT;
          Cx<R> cc{0, 0};
          uint32_t row = r;
          if (oku && r < T) {
            if (HALF) {
              cc = ((r >> i) & 1u) ? c1v : c0v;
              row = r ^ (1u << i);
            } else {
              const R fi = gi[digit(k, i)];
              cc = Cx<R>{c0v.re * fi, c0v.im * fi};
            }
          }
          cr[u][k] = cc;
          y[u][k] = Cx<R>{0, 0};
          if (cc.re != R(0) || cc.im != R(0)) y[u][k] = src[row];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; u++)
#pragma unroll
        for (int k = 0; k < RPT; k++) cfma<R, CPLX>(ar[k], ai[k], cr[u][k], y[u][k]);
    }
#pragma unroll
    for (int k = 0; k < RPT; k++) {
      const uint32_t r = tid + (uint32_t)k * NT;
      if (r >= T) continue;
      Acc<R, 1> a;
      a.re[0] = ar[k];
      a.im[0] = ai[k];
      hv_epilogue<R, 1, true>(P, base + r, 0, a, tile + r, red);
    }
    __syncthreads();  // the next tile overwrites the LDS
  }
  hv_finish<1, NT>(P, red);
}

template <typename R>
size_t stream_smem(const StreamGeom &g, bool stage) {
  return StreamLds<R>(g, stage).total;
}

// kc of the tuning: bits 0..3 select the block (1: 256 threads, else 1024),
// bits 4..7 the log2 of the tiles per XCD chunk, bit 8 stages the partner
// tiles of the pairs with one tile site in LDS
inline int stream_threads(int kc) { return (kc & 15) == 1 ? 256 : 1024; }
inline uint32_t stream_chunk(int kc) { return 1u << ((kc >> 4) & 15); }
inline bool stream_stage(int kc) { return ((kc >> 8) & 1) != 0; }

template <typename R, bool POW2, bool HALF, bool CPLX, int RPT, int NT, bool STAGE>
void launch_stream_t(const StreamPlan &sp, const DevTables<R> &tb, const HvParams &P, unsigned gx, uint32_t chunk,
                     hipStream_t s) {
  static size_t granted = 0;  // per instantiation
  const size_t sm = stream_smem<R>(sp.geom, STAGE);
  if (sm > granted) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&hv_stream<R, POW2, HALF, CPLX, RPT, NT, STAGE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    granted = sm;
  }
  hipLaunchKernelGGL((hv_stream<R, POW2, HALF, CPLX, RPT, NT, STAGE>), dim3(gx), dim3(NT), sm, s, sp.geom, tb,
                     sp.d_pij, reinterpret_cast<const Cx<R> *>(sp.d_pc), reinterpret_cast<const R *>(sp.d_pzz),
                     reinterpret_cast<const R *>(sp.d_tdiag), tb.hoff, chunk, P);
}

template <typename R, bool POW2, bool HALF, bool CPLX, int NT, bool STAGE>
void launch_stream_rpt(const StreamPlan &sp, const DevTables<R> &tb, const HvParams &P, unsigned gx, uint32_t chunk,
                       hipStream_t s) {
  // rows per thread: 4 or 8 at 1024 threads (tiles up to 8192 rows), 4, 8 or 16
  // at 256 (tiles up to 4096 rows; the caller checks)
  const uint32_t rpt = (sp.geom.T + NT - 1) / NT;
  if (rpt <= 4) launch_stream_t<R, POW2, HALF, CPLX, 4, NT, STAGE>(sp, tb, P, gx, chunk, s);
  else if (rpt <= 8) launch_stream_t<R, POW2, HALF, CPLX, 8, NT, STAGE>(sp, tb, P, gx, chunk, s);
  else if constexpr (NT <= 256) launch_stream_t<R, POW2, HALF, CPLX, 16, NT, STAGE>(sp, tb, P, gx, chunk, s);
}

// spin-1/2 systems take the direct mixed-pair reads only (the caller checks)
template <typename R, int NT>
void launch_stream_nt(const StreamPlan &sp, const DevTables<R> &tb, const HvParams &P, unsigned gx, uint32_t chunk,
                      bool stage, hipStream_t s) {
  if (sp.half) {
    if (sp.cplx) launch_stream_rpt<R, true, true, true, NT, false>(sp, tb, P, gx, chunk, s);
    else launch_stream_rpt<R, true, true, false, NT, false>(sp, tb, P, gx, chunk, s);
  } else if (sp.pow2) {
    if (stage) {
      if (sp.cplx) launch_stream_rpt<R, true, false, true, NT, true>(sp, tb, P, gx, chunk, s);
      else launch_stream_rpt<R, true, false, false, NT, true>(sp, tb, P, gx, chunk, s);
    } else {
      if (sp.cplx) launch_stream_rpt<R, true, false, true, NT, false>(sp, tb, P, gx, chunk, s);
      else launch_stream_rpt<R, true, false, false, NT, false>(sp, tb, P, gx, chunk, s);
    }
  } else {
    if (stage) {
      if (sp.cplx) launch_stream_rpt<R, false, false, true, NT, true>(sp, tb, P, gx, chunk, s);
      else launch_stream_rpt<R, false, false, false, NT, true>(sp, tb, P, gx, chunk, s);
    } else {
      if (sp.cplx) launch_stream_rpt<R, false, false, true, NT, false>(sp, tb, P, gx, chunk, s);
      else launch_stream_rpt<R, false, false, false, NT, false>(sp, tb, P, gx, chunk, s);
    }
  }
}

template <typename R>
int launch_stream_r(const StreamPlan &sp, const DevTables<R> &tb, const HvParams &P, int cap, int kc,
                    unsigned *gx_out, hipStream_t s) {
  if (!sp.ok || !sp.d_pij || !sp.d_tdiag) return FTLM_EINVAL;
  // 256 threads take tiles of up to 4096 rows (16 rows per thread); larger tiles take 1024
  const int nt = (stream_threads(kc) == 256 && sp.geom.T <= 4096u) ? 256 : 1024;
  if (sp.geom.T > 8192u) return FTLM_ERANGE;
  // staging serves several pairs per partner tile; spin-1/2 systems have one
  // move per mixed pair and row and are not staged
  const bool stage = stream_stage(kc);
  if (stage && sp.half) return FTLM_EINVAL;
  if (stream_smem<R>(sp.geom, stage) > 159 * 1024) return FTLM_ERANGE;  // 1 KB for static LDS
  uint32_t gx = sp.geom.ntile < (uint32_t)cap ? sp.geom.ntile : (uint32_t)cap;
  if (gx >= 8) gx &= ~7u;
  const uint32_t chunk = stream_chunk(kc);
  if (nt == 256) launch_stream_nt<R, 256>(sp, tb, P, gx, chunk, stage, s);
  else launch_stream_nt<R, 1024>(sp, tb, P, gx, chunk, stage, s);
  *gx_out = gx;
  return FTLM_OK;
}

}  // namespace

int launch_stream(const DevHam &dh, int precision, const HvParams &P, int cap, int kc, unsigned *gx, hipStream_t s) {
  if (P.K != 1) return FTLM_EINVAL;
  return precision == FTLM_C64 ? launch_stream_r<float>(dh.sp32, dh.t32, P, cap, kc, gx, s)
                               : launch_stream_r<double>(dh.sp64, dh.t64, P, cap, kc, gx, s);
}

// Host plan: the tile takes the low sites while their rows fit tile_rows (and,
// unless every tile radix is a power of two, at most 8 sites so that a row's
// tile digits pack into 32 bits); pairs are ordered inside | mixed | outer.
void plan_stream(const HostHam &hh, uint32_t tile_rows, StreamPlan &pl) {
  pl = StreamPlan();
  const int n = hh.n;
  if (hh.has_z || n < 1) return;
  bool pow2 = true;
  for (int k = 0; k < n; k++) pow2 = pow2 && (hh.radix[k] & (hh.radix[k] - 1)) == 0;
  uint64_t T = 1;
  int t = 0;
  while (t < n && T * (uint64_t)hh.radix[t] <= tile_rows && (pow2 || t < 8)) T *= (uint64_t)hh.radix[t++];
  // digits of rows and tiles are bit fields when every radix is a power of two,
  // else 4-bit fields packed in 32 (tile) and 64 (outer) bits
  if (t < 1 || (!pow2 && n - t > 16)) return;
  StreamGeom &g = pl.geom;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.t = t;
  g.T = (uint32_t)T;
  g.dim = (uint32_t)hh.dim;
  g.ntile = (uint32_t)(hh.dim / T);
  for (int k = 0; k < n; k++) {
    g.radix[k] = hh.radix[k];
    g.st[k] = hh.stride[k];
    g.s[k] = 0.5f * (float)hh.two_s[k];
    int lg = 0;
    while ((1u << lg) < hh.stride[k]) lg++;
    g.lg[k] = lg;
    if (site_has_singles(hh, k)) g.smask |= 1u << k;
  }
  auto cls = [&](int p) { return (hh.pi[p] >= t) + (hh.pj[p] >= t); };
  pl.order.resize(hh.npair);
  for (int p = 0; p < hh.npair; p++) pl.order[p] = p;
  // classes in the order inside | mixed | outer; the mixed pairs (tile site i <
  // outer site j) by outer site, so that the pairs sharing a partner tile are
  // consecutive
  std::stable_sort(pl.order.begin(), pl.order.end(), [&](int a, int b) {
    const int ca = cls(a), cb = cls(b);
    if (ca != cb) return ca < cb;
    if (ca == 1 && hh.pj[a] != hh.pj[b]) return hh.pj[a] < hh.pj[b];
    return false;
  });
  for (int p = 0; p < hh.npair; p++) {
    const int c = cls(p);
    (c == 0 ? g.np_in : c == 1 ? g.np_mx : g.np_out)++;
  }
  bool cplx = false;
  for (int p = 0; p < hh.npair; p++)
    for (int a = 0; a < 4; a++) cplx = cplx || hh.pc[4 * p + a].im != 0.0;
  for (int k = 0; k < n; k++)
    for (int a = 0; a < hh.radix[k]; a++)
      for (int b = 0; b < hh.radix[k]; b++)
        if (a != b) cplx = cplx || hh.h[(size_t)k * 256 + a * 16 + b].im != 0.0;
  pl.cplx = cplx;
  pl.pow2 = pow2;
  pl.half = hh.spin_half;
  g.half = hh.spin_half ? 1 : 0;
  g.gmask = 0;
  for (int p = 0; p < hh.npair; p++)
    if (cls(p) == 1)
      for (int q = 0; q < 4; q++)
        if (hh.pc[4 * p + q].re != 0.0 || hh.pc[4 * p + q].im != 0.0) g.gmask |= 1ull << (2 * hh.pj[p] + (q & 1));
  // diagonal over the tile sites, per tile row
  pl.tdiag.assign(T, 0.0);
  for (uint32_t r = 0; r < T; r++) {
    int d[kMaxSites];
    uint32_t rem = r;
    for (int k = 0; k < t; k++) {
      d[k] = (int)(rem % (uint32_t)hh.radix[k]);
      rem /= (uint32_t)hh.radix[k];
    }
    double s = 0;
    for (int k = 0; k < t; k++) s += hh.h[(size_t)k * 256 + d[k] * 16 + d[k]].re;
    for (int p = 0; p < hh.npair; p++)
      if (hh.pi[p] < t && hh.pj[p] < t)
        s += hh.pzz[p] * (d[hh.pi[p]] - 0.5 * hh.two_s[hh.pi[p]]) * (d[hh.pj[p]] - 0.5 * hh.two_s[hh.pj[p]]);
    pl.tdiag[r] = s;
  }
  pl.ok = true;
}

}  // namespace ftlm
