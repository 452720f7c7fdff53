// C ABI of the FTLM library (include/ftlm.h): handle lifetime, device tables,
// H*v, start vectors and the plain (one Hamiltonian) FTLM run driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ftlm_internal.hpp"

namespace ftlm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

#define HIP_OK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return FTLM_EHIP;                                                       \
    }                                                                         \
  } while (0)

// ---------------------------------------------------------------- table upload
namespace {

struct Blob {
  std::vector<unsigned char> bytes;
  size_t add(const void *src, size_t n) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
};

template <typename R>
struct TableOffsets {
  size_t hdiag, hoff, gp, gm, mval, pij, pc, pzz, zz, czp, czm, pc_half, hflip, cz_half, lowf;
};

template <typename R>
static TableOffsets<R> pack_tables(const HostHam &hh, const std::vector<int> &perm, Blob &b) {
  const int n = hh.n, np = hh.npair;
  TableOffsets<R> o{};
  std::vector<R> hdiag(n * 16, 0), gp(n * 16, 0), gm(n * 16, 0), mval(n * 16, 0);
  std::vector<Cx<R>> hoff(n * 64, Cx<R>{0, 0});
  for (int k = 0; k < n; k++) {
    const int r = hh.radix[k];
    const double s = 0.5 * hh.two_s[k];
    for (int dk = 0; dk < r; dk++) {
      const double m = dk - s;
      hdiag[k * 16 + dk] = (R)hh.h[(size_t)k * 256 + dk * 16 + dk].re;
      mval[k * 16 + dk] = (R)m;
      if (dk >= 1) gp[k * 16 + dk] = (R)std::sqrt(s * (s + 1) - m * (m - 1));
      if (dk <= r - 2) gm[k * 16 + dk] = (R)std::sqrt(s * (s + 1) - m * (m + 1));
      const int Ds[4] = {-2, -1, 1, 2};
      for (int di = 0; di < 4; di++) {
        const int nd = dk + Ds[di];
        if (nd < 0 || nd >= r) continue;
        const Cx<double> c = hh.h[(size_t)k * 256 + dk * 16 + nd];
        hoff[(k * 4 + di) * 16 + dk] = Cx<R>{(R)c.re, (R)c.im};
      }
    }
  }
  std::vector<int2> pij(std::max(np, 1));
  std::vector<Cx<R>> pc(4 * std::max(np, 1), Cx<R>{0, 0}), pch(4 * std::max(np, 1), Cx<R>{0, 0});
  std::vector<R> pzz(std::max(np, 1), 0);
  for (int q = 0; q < np; q++) {
    const int p = perm[q];
    pij[q] = make_int2(hh.pi[p], hh.pj[p]);
    for (int a = 0; a < 4; a++) pc[4 * q + a] = Cx<R>{(R)hh.pc[4 * p + a].re, (R)hh.pc[4 * p + a].im};
    // row bits (b_i, b_j) -> ladder pair: (0,0) --, (0,1) -+, (1,0) +-, (1,1) ++
    pch[4 * q + 0] = pc[4 * q + 3];
    pch[4 * q + 1] = pc[4 * q + 2];
    pch[4 * q + 2] = pc[4 * q + 1];
    pch[4 * q + 3] = pc[4 * q + 0];
    pzz[q] = (R)hh.pzz[p];
  }
  std::vector<R> zz(n * n);
  std::vector<Cx<R>> czp(n * n), czm(n * n), czh(n * n * 2);
  for (int k = 0; k < n * n; k++) {
    zz[k] = (R)hh.zz[k];
    czp[k] = Cx<R>{(R)hh.czp[k].re, (R)hh.czp[k].im};
    czm[k] = Cx<R>{(R)hh.czm[k].re, (R)hh.czm[k].im};
    czh[2 * k + 0] = czm[k];
    czh[2 * k + 1] = czp[k];
  }
  std::vector<Cx<R>> hflip(2 * n, Cx<R>{0, 0});
  for (int k = 0; k < n; k++)
    if (hh.radix[k] == 2) {
      const Cx<double> a = hh.h[(size_t)k * 256 + 0 * 16 + 1], c = hh.h[(size_t)k * 256 + 1 * 16 + 0];
      hflip[2 * k + 0] = Cx<R>{(R)a.re, (R)a.im};
      hflip[2 * k + 1] = Cx<R>{(R)c.re, (R)c.im};
    }
  std::vector<Cx<R>> lowf;
  if (hh.spin_half && n >= kLowBits) {
    lowf.assign((size_t)n * 2 * 256, Cx<R>{0, 0});
    for (int k = 0; k < n; k++)
      for (int sel = 0; sel < 2; sel++)
        for (int t = 0; t < 256; t++) {
          double fr = 0, fi = 0;
          for (int l = 0; l < kLowBits; l++) {
            if (l == k) continue;
            const double ml = ((t >> l) & 1) ? 0.5 : -0.5;
            const Cx<double> c = sel ? hh.czp[k * n + l] : hh.czm[k * n + l];
            fr += c.re * ml;
            fi += c.im * ml;
          }
          lowf[((size_t)k * 2 + sel) * 256 + t] = Cx<R>{(R)fr, (R)fi};
        }
  } else {
    lowf.assign(1, Cx<R>{0, 0});
  }
  o.hdiag = b.add(hdiag.data(), hdiag.size() * sizeof(R));
  o.hoff = b.add(hoff.data(), hoff.size() * sizeof(Cx<R>));
  o.gp = b.add(gp.data(), gp.size() * sizeof(R));
  o.gm = b.add(gm.data(), gm.size() * sizeof(R));
  o.mval = b.add(mval.data(), mval.size() * sizeof(R));
  o.pij = b.add(pij.data(), pij.size() * sizeof(int2));
  o.pc = b.add(pc.data(), pc.size() * sizeof(Cx<R>));
  o.pzz = b.add(pzz.data(), pzz.size() * sizeof(R));
  o.zz = b.add(zz.data(), zz.size() * sizeof(R));
  o.czp = b.add(czp.data(), czp.size() * sizeof(Cx<R>));
  o.czm = b.add(czm.data(), czm.size() * sizeof(Cx<R>));
  o.pc_half = b.add(pch.data(), pch.size() * sizeof(Cx<R>));
  o.hflip = b.add(hflip.data(), hflip.size() * sizeof(Cx<R>));
  o.cz_half = b.add(czh.data(), czh.size() * sizeof(Cx<R>));
  o.lowf = b.add(lowf.data(), lowf.size() * sizeof(Cx<R>));
  return o;
}

// The spin-1/2 pair coefficients of a window plan's pair list, in list order:
// entry e holds the four coefficients of device pair plist[e].x (the same
// values as the pc_half table).
template <typename R>
static std::vector<Cx<R>> plist_coefs(const HostHam &hh, const std::vector<int> &perm, const std::vector<int4> &plist) {
  std::vector<Cx<R>> c(4 * std::max<size_t>(plist.size(), 1), Cx<R>{0, 0});
  for (size_t e = 0; e < plist.size(); e++) {
    const int q = plist[e].x;
    if (q < 0 || q >= (int)perm.size()) continue;
    const int p = perm[q];
    for (int a = 0; a < 4; a++) {
      const Cx<double> v = hh.pc[4 * p + 3 - a];  // row bits (b_i, b_j) -> ladder pair, as in pc_half
      c[4 * e + a] = Cx<R>{(R)v.re, (R)v.im};
    }
  }
  return c;
}

template <typename R>
static DevTables<R> resolve(const TableOffsets<R> &o, unsigned char *base) {
  DevTables<R> t;
  t.hdiag = reinterpret_cast<const R *>(base + o.hdiag);
  t.hoff = reinterpret_cast<const Cx<R> *>(base + o.hoff);
  t.gp = reinterpret_cast<const R *>(base + o.gp);
  t.gm = reinterpret_cast<const R *>(base + o.gm);
  t.mval = reinterpret_cast<const R *>(base + o.mval);
  t.pij = reinterpret_cast<const int2 *>(base + o.pij);
  t.pc = reinterpret_cast<const Cx<R> *>(base + o.pc);
  t.pzz = reinterpret_cast<const R *>(base + o.pzz);
  t.zz = reinterpret_cast<const R *>(base + o.zz);
  t.czp = reinterpret_cast<const Cx<R> *>(base + o.czp);
  t.czm = reinterpret_cast<const Cx<R> *>(base + o.czm);
  t.pc_half = reinterpret_cast<const Cx<R> *>(base + o.pc_half);
  t.hflip = reinterpret_cast<const Cx<R> *>(base + o.hflip);
  t.cz_half = reinterpret_cast<const Cx<R> *>(base + o.cz_half);
  t.lowf = reinterpret_cast<const Cx<R> *>(base + o.lowf);
  return t;
}

}  // namespace

// Pair order: inside the 11-bit tile | mixed (i inside, j outside), by j then i |
// outside.  Every kernel that walks the pair list sees this order.
void sort_pairs(const HostHam &hh, std::vector<int> &perm, int &n_ll, int &n_lh,
                int mx_off[kMaxSites + 1]) {
  const int n = hh.n, np = hh.npair;
  perm.resize(np);
  for (int p = 0; p < np; p++) perm[p] = p;
  auto cls = [&](int p) { return (hh.pi[p] >= kTileBits) + (hh.pj[p] >= kTileBits); };
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
    if (cls(a) != cls(b)) return cls(a) < cls(b);
    if (cls(a) == 1 && hh.pj[a] != hh.pj[b]) return hh.pj[a] < hh.pj[b];
    return false;
  });
  n_ll = n_lh = 0;
  for (int p = 0; p < np; p++) {
    n_ll += cls(p) == 0;
    n_lh += cls(p) == 1;
  }
  int q = n_ll;
  for (int a = 0; a < n; a++) {
    mx_off[a] = q;
    while (q < n_ll + n_lh && hh.pj[perm[q]] == a) q++;
  }
  for (int a = n; a <= kMaxSites; a++) mx_off[a] = q;
}

namespace {
// FNV-1a over the bytes an H*v launch takes by value.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void *p, size_t n) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
  }
  template <typename T>
  void pod(const T &x) { add(&x, sizeof(T)); }
  template <typename T>
  void vec(const std::vector<T> &v) {
    pod(v.size());
    if (!v.empty()) add(v.data(), v.size() * sizeof(T));
  }
};

uint64_t launch_signature(const DevHam &dh) {
  Fnv f;
  f.pod(dh.geom);
  f.pod(dh.t64);
  f.pod(dh.t32);
  for (const PassPlan *pl : {&dh.plan64, &dh.plan32}) {
    f.vec(pl->passes);
    f.pod(pl->d_pairs);
    f.pod(pl->rec_block);
    f.vec(pl->rec_off);
    f.vec(pl->base_off);
    f.vec(pl->lane_off);
  }
  for (const WinPlan *pl : {&dh.win64, &dh.win32, &dh.tw64, &dh.tw32}) {
    f.vec(pl->passes);
    f.pod(pl->d_plist);
    f.pod(pl->d_pcoef);
  }
  for (const StreamPlan *sp : {&dh.sp64, &dh.sp32}) {
    f.pod(sp->ok);
    f.pod(sp->pow2);
    f.pod(sp->half);
    f.pod(sp->cplx);
    f.pod(sp->geom);
    f.pod(sp->d_pij);
    f.pod(sp->d_pc);
    f.pod(sp->d_pzz);
    f.pod(sp->d_tdiag);
  }
  f.pod(dh.block);
  return f.h;
}
}  // namespace

// Packs every table of hh for both precisions and copies it to the device.
// Reuses dh.block when its size matches (so captured graphs stay valid).
int upload_tables(const HostHam &hh, DevHam &dh, std::string &err) {
  // the pass plans are rebuilt below; keep their record allocations for reuse
  void *rec64 = dh.plan64.rec_block, *rec32 = dh.plan32.rec_block;
  const size_t rb64 = dh.plan64.rec_bytes, rb32 = dh.plan32.rec_bytes;
  const int n = hh.n, np = hh.npair;
  std::vector<int> perm;
  int n_ll = 0, n_lh = 0;
  int mx_off[kMaxSites + 1];
  sort_pairs(hh, perm, n_ll, n_lh, mx_off);
  std::vector<int> spi(np), spj(np);
  for (int q = 0; q < np; q++) {
    spi[q] = hh.pi[perm[q]];
    spj[q] = hh.pj[perm[q]];
  }
  const size_t wb = window_bytes_setting();
  const size_t l2b = l2_window_bytes_setting();
  // the plans depend on the pair structure (fixed per handle), on which sites
  // have single flips (field dependent) and on the window sizes
  uint32_t smask = 0;
  for (int k = 0; k < n; k++)
    if (site_has_singles(hh, k)) smask |= 1u << k;
  const size_t tbytes = tile_window_bytes_setting((uint64_t)hh.dim * 16);
  const size_t tbytes32 = tile_window_bytes_setting((uint64_t)hh.dim * 8);
  const bool replan = !dh.plan_valid || dh.plan_smask != smask || dh.plan_wb != wb || dh.plan_l2b != l2b ||
                      dh.plan_tb != tbytes || dh.plan_tb32 != tbytes32;
  if (replan) {
    int prc = plan_passes_sorted(hh, spi, spj, wb / 16, dh.plan64);
    if (!prc) prc = plan_passes_sorted(hh, spi, spj, wb / 8, dh.plan32);
    if (prc) {
      err = "no windowed-pass plan fits the window size";
      return prc;
    }
    const bool half = hh.spin_half && n >= kLowBits;
    prc = plan_l2_windows(hh, spi, spj, l2b / 16, half ? kLowBits : 0, dh.win64);
    if (!prc) prc = plan_l2_windows(hh, spi, spj, l2b / 8, half ? kLowBits : 0, dh.win32);
    if (prc) {
      err = "no L2-window plan fits the window size";
      return prc;
    }
    dh.tw64 = WinPlan();
    dh.tw32 = WinPlan();
    if (hh.spin_half && n > kTileBits) {
      if (plan_l2_windows(hh, spi, spj, tbytes / 16, kTileBits, dh.tw64) ||
          plan_l2_windows(hh, spi, spj, tbytes32 / 8, kTileBits, dh.tw32)) {
        dh.tw64 = WinPlan();
        dh.tw32 = WinPlan();
      }
    }
    dh.plan_valid = true;
    dh.plan_smask = smask;
    dh.plan_wb = wb;
    dh.plan_l2b = l2b;
    dh.plan_tb = tbytes;
    dh.plan_tb32 = tbytes32;
  }
  dh.plan64.window_bytes = wb;
  dh.plan32.window_bytes = wb;
  dh.plan64.rec_block = rec64;
  dh.plan64.rec_bytes = rb64;
  dh.plan32.rec_block = rec32;
  dh.plan32.rec_bytes = rb32;
  Blob b;
  TableOffsets<double> o64 = pack_tables<double>(hh, perm, b);
  TableOffsets<float> o32 = pack_tables<float>(hh, perm, b);
  const size_t off_p64 = b.add(dh.plan64.pairs.data(), dh.plan64.pairs.size() * sizeof(int4));
  const size_t off_p32 = b.add(dh.plan32.pairs.data(), dh.plan32.pairs.size() * sizeof(int4));
  const size_t off_w64 = b.add(dh.win64.plist.data(), dh.win64.plist.size() * sizeof(int4));
  const size_t off_w32 = b.add(dh.win32.plist.data(), dh.win32.plist.size() * sizeof(int4));
  const size_t off_t64 = b.add(dh.tw64.plist.data(), dh.tw64.plist.size() * sizeof(int4));
  const size_t off_t32 = b.add(dh.tw32.plist.data(), dh.tw32.plist.size() * sizeof(int4));
  const std::vector<Cx<double>> tc64 = plist_coefs<double>(hh, perm, dh.tw64.plist);
  const std::vector<Cx<float>> tc32 = plist_coefs<float>(hh, perm, dh.tw32.plist);
  const size_t off_c64 = b.add(tc64.data(), tc64.size() * sizeof(Cx<double>));
  const size_t off_c32 = b.add(tc32.data(), tc32.size() * sizeof(Cx<float>));
  // single-pass tile plans (64 KB tiles); field dependent (single flips,
  // complex coefficients, the tile diagonal)
  plan_stream(hh, 65536 / sizeof(Cx<double>), dh.sp64);
  plan_stream(hh, 65536 / sizeof(Cx<float>), dh.sp32);
  size_t off_s[2][4] = {{0}};
  {
    StreamPlan *sps[2] = {&dh.sp64, &dh.sp32};
    for (int q = 0; q < 2; q++) {
      const StreamPlan &sp = *sps[q];
      const size_t npq = std::max<size_t>(sp.order.size(), 1);
      std::vector<int2> sij(npq, make_int2(0, 0));
      std::vector<Cx<double>> sc(4 * npq, Cx<double>{0, 0});
      std::vector<double> sz(npq, 0.0);
      for (size_t e = 0; e < sp.order.size(); e++) {
        const int p = sp.order[e];
        sij[e] = make_int2(hh.pi[p], hh.pj[p]);
        for (int a = 0; a < 4; a++) sc[4 * e + a] = hh.pc[4 * p + a];
        sz[e] = hh.pzz[p];
      }
      const std::vector<double> td = sp.tdiag.empty() ? std::vector<double>(1, 0.0) : sp.tdiag;
      off_s[q][0] = b.add(sij.data(), sij.size() * sizeof(int2));
      if (q == 0) {
        off_s[q][1] = b.add(sc.data(), sc.size() * sizeof(Cx<double>));
        off_s[q][2] = b.add(sz.data(), sz.size() * sizeof(double));
        off_s[q][3] = b.add(td.data(), td.size() * sizeof(double));
      } else {
        std::vector<Cx<float>> sc32(sc.size());
        for (size_t e = 0; e < sc.size(); e++) sc32[e] = Cx<float>{(float)sc[e].re, (float)sc[e].im};
        std::vector<float> sz32(sz.begin(), sz.end()), td32(td.begin(), td.end());
        off_s[q][1] = b.add(sc32.data(), sc32.size() * sizeof(Cx<float>));
        off_s[q][2] = b.add(sz32.data(), sz32.size() * sizeof(float));
        off_s[q][3] = b.add(td32.data(), td32.size() * sizeof(float));
      }
    }
  }
  const size_t bytes = (b.bytes.size() + 255) & ~size_t(255);
  if (dh.block && dh.block_bytes != bytes) {
    (void)hipFree(dh.block);
    dh.block = nullptr;
  }
  if (!dh.block) {
    if (hipMalloc(&dh.block, bytes) != hipSuccess) {
      err = "hipMalloc of Hamiltonian tables failed";
      dh.block = nullptr;
      return FTLM_ENOMEM;
    }
    dh.block_bytes = bytes;
  }
  if (hipMemcpy(dh.block, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
    err = "hipMemcpy of Hamiltonian tables failed";
    return FTLM_EHIP;
  }
  unsigned char *base = reinterpret_cast<unsigned char *>(dh.block);
  dh.t64 = resolve<double>(o64, base);
  dh.t32 = resolve<float>(o32, base);
  dh.plan64.d_pairs = reinterpret_cast<const int4 *>(base + off_p64);
  dh.plan32.d_pairs = reinterpret_cast<const int4 *>(base + off_p32);
  dh.win64.d_plist = reinterpret_cast<const int4 *>(base + off_w64);
  dh.win32.d_plist = reinterpret_cast<const int4 *>(base + off_w32);
  dh.tw64.d_plist = dh.tw64.plist.empty() ? nullptr : reinterpret_cast<const int4 *>(base + off_t64);
  dh.tw32.d_plist = dh.tw32.plist.empty() ? nullptr : reinterpret_cast<const int4 *>(base + off_t32);
  dh.tw64.d_pcoef = dh.tw64.plist.empty() ? nullptr : base + off_c64;
  dh.tw32.d_pcoef = dh.tw32.plist.empty() ? nullptr : base + off_c32;
  {
    StreamPlan *sps[2] = {&dh.sp64, &dh.sp32};
    for (int q = 0; q < 2; q++) {
      sps[q]->d_pij = reinterpret_cast<const int2 *>(base + off_s[q][0]);
      sps[q]->d_pc = base + off_s[q][1];
      sps[q]->d_pzz = base + off_s[q][2];
      sps[q]->d_tdiag = base + off_s[q][3];
    }
  }
  HamGeom &g = dh.geom;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.npair = np;
  g.has_z = hh.has_z;
  g.spin_half = hh.spin_half && n >= kLowBits;
  g.n_ll = n_ll;
  g.n_lh = n_lh;
  for (int a = 0; a <= kMaxSites; a++) g.mx_off[a] = mx_off[a];
  g.single_mask = 0;
  for (int k = 0; k < n; k++)
    if (site_has_singles(hh, k)) g.single_mask |= 1u << k;
  g.dim = (uint32_t)hh.dim;
  for (int k = 0; k < n; k++) {
    g.radix[k] = hh.radix[k];
    g.stride[k] = hh.stride[k];
    g.s[k] = 0.5f * hh.two_s[k];
  }
  const int rc = build_pass_records(dh, err);
  const uint64_t sig = launch_signature(dh);
  if (sig != dh.launch_sig) {
    dh.launch_sig = sig;
    dh.generation++;
  }
  return rc;
}

size_t window_bytes_setting() {
  const int kb = g_windows.pass_kb.load();
  return (size_t)(kb ? kb : 64) * 1024;
}

static void field_direction(const double B[3], double out[3]) {
  const double nb = std::sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  if (nb > 0) {
    for (int a = 0; a < 3; a++) out[a] = B[a] / nb;
  } else {
    out[0] = out[1] = 0;
    out[2] = 1;
  }
}

// O = -sum_i g_i s_i.B_hat, built as a site-only Hamiltonian whose Zeeman field
// is -B_hat/mu_B.
int build_moment(ftlm_hamiltonian *h, std::string &err) {
  const HostHam &hh = h->host;
  double bh[3], beff[3];
  field_direction(hh.B, bh);
  for (int a = 0; a < 3; a++) beff[a] = -bh[a] / kMuB;
  ftlm_system s{};
  s.n_sites = hh.n;
  s.two_s = hh.two_s;
  s.g = hh.g.data();
  s.B = beff;
  int rc = compile_hamiltonian(&s, h->mom_host, err);
  if (rc) return rc;
  return upload_tables(h->mom_host, h->mom_dev, err);
}

}  // namespace ftlm

using namespace ftlm;

extern "C" {

const char *ftlm_last_error(void) { return g_last_error.c_str(); }
int ftlm_version(void) { return 10000; }

int ftlm_hamiltonian_create(const ftlm_system *sys, ftlm_hamiltonian **out) {
  if (!out) { set_error("out is NULL"); return FTLM_EINVAL; }
  ftlm_hamiltonian *h = new (std::nothrow) ftlm_hamiltonian();
  if (!h) { set_error("out of host memory"); return FTLM_ENOMEM; }
  std::string err;
  int rc = compile_hamiltonian(sys, h->host, err);
  if (!rc) {
    if (hipGetDevice(&h->device) != hipSuccess) { err = "no HIP device"; rc = FTLM_EHIP; }
  }
  if (!rc) rc = upload_tables(h->host, h->dev, err);
  if (!rc) rc = build_moment(h, err);
  if (rc) {
    set_error(err);
    ftlm_hamiltonian_destroy(h);
    return rc;
  }
  *out = h;
  return FTLM_OK;
}

void ftlm_hamiltonian_destroy(ftlm_hamiltonian *h) {
  if (!h) return;
  if (h->dev.block) (void)hipFree(h->dev.block);
  if (h->mom_dev.block) (void)hipFree(h->mom_dev.block);
  free_pass_records(h->dev);
  free_pass_records(h->mom_dev);
  delete h;
}

int ftlm_hamiltonian_dim(const ftlm_hamiltonian *h, uint64_t *dim) {
  if (!h || !dim) { set_error("NULL argument"); return FTLM_EINVAL; }
  *dim = h->host.dim;
  return FTLM_OK;
}

int ftlm_hamiltonian_nnz_per_row(const ftlm_hamiltonian *h, double *nnz) {
  if (!h || !nnz) { set_error("NULL argument"); return FTLM_EINVAL; }
  *nnz = h->host.nnz_per_row;
  return FTLM_OK;
}

int ftlm_hamiltonian_set_field(ftlm_hamiltonian *h, const double B[3]) {
  if (!h || !B) { set_error("NULL argument"); return FTLM_EINVAL; }
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(B[a])) { set_error("B must be finite"); return FTLM_EINVAL; }
  HIP_OK(hipDeviceSynchronize());
  for (int a = 0; a < 3; a++) h->host.B[a] = B[a];
  compile_site_terms(h->host);
  h->host.nnz_per_row = count_nnz_per_row(h->host);
  std::string err;
  int rc = upload_tables(h->host, h->dev, err);
  if (!rc) rc = build_moment(h, err);
  if (rc) set_error(err);
  return rc;
}

int ftlm_apply(const ftlm_hamiltonian *h, int32_t precision, int32_t n_cols, const void *v,
               void *w, void *stream) {
  if (!h || !v || !w) { set_error("NULL argument"); return FTLM_EINVAL; }
  if (precision != FTLM_C128 && precision != FTLM_C64) { set_error("bad precision"); return FTLM_EINVAL; }
  if (n_cols < 1 || n_cols > 64) { set_error("n_cols must be in [1, 64]"); return FTLM_ERANGE; }
  if (v == w) { set_error("v and w must differ"); return FTLM_EINVAL; }
  const size_t es = precision == FTLM_C64 ? 8 : 16;
  const size_t span = (size_t)h->host.dim * n_cols * es;
  const char *pv = (const char *)v, *pw = (const char *)w;
  if (pv < pw + span && pw < pv + span) { set_error("v and w overlap"); return FTLM_EINVAL; }
  if (((uintptr_t)v | (uintptr_t)w) & 15) { set_error("v and w must be 16-byte aligned"); return FTLM_EINVAL; }
  HvLaunch L{};
  L.precision = precision;
  L.K = n_cols;
  L.v = v;
  L.w = w;
  int rc = launch_hv(h->dev, L, (hipStream_t)stream);
  if (rc) set_error(std::string("H*v launch failed: ") + hipGetErrorString(hipGetLastError()));
  return rc;
}

int ftlm_gaussian_vectors(uint64_t seed, uint32_t instance, uint32_t field, uint32_t r0,
                          int32_t n_cols, uint64_t dim, void *out, void *stream) {
  if (!out) { set_error("out is NULL"); return FTLM_EINVAL; }
  if (n_cols < 1 || n_cols > 64) { set_error("n_cols must be in [1, 64]"); return FTLM_ERANGE; }
  if (dim < 1 || dim >= (1ull << 32)) { set_error("dim out of range"); return FTLM_ERANGE; }
  // the start kernel also writes norm partials, which are not returned here:
  // a private buffer per device (and host thread), kept until the process ends
  constexpr int kMaxDev = 64;
  static thread_local double *scratch_by_dev[kMaxDev] = {};
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) { set_error("device index out of range"); return FTLM_ERANGE; }
  const size_t need = sizeof(double) * (2048 * 64 + 64) + sizeof(unsigned) * kCounterWords;
  double *&scratch = scratch_by_dev[dev];
  if (!scratch) {
    HIP_OK(hipMalloc(&scratch, need));
    HIP_OK(hipMemset(scratch, 0, need));
  }
  unsigned *counter = reinterpret_cast<unsigned *>(scratch + 2048 * 64 + 64);
  int rc = launch_gaussian(seed, instance, field, r0, n_cols, (uint32_t)dim, FTLM_C128, out,
                           scratch, counter, scratch + 2048 * 64, 0, (hipStream_t)stream);
  if (rc) set_error("gaussian launch failed");
  return rc;
}

}  // extern "C"
