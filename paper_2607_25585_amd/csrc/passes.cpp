// Planner of the windowed H*v passes.
//
// The Hamiltonian of Sec. 2.1 couples every pair of sites (all-to-all dipolar
// term), so a matrix-free product gathers partners that differ in any two
// digits.  On a vector far larger than the caches those gathers come from HBM.
// Instead, each pass fixes all digits except those of a small set of "active"
// sites: the rows that share the fixed digits form a window of prod(radix)
// rows that is staged once in LDS, and every term acting only on active sites
// is applied from there.  The planner covers all interacting pairs with as few
// windows as it can (greedy set cover).  The lowest sites are active in every
// pass ("chunk"), so each window is read as contiguous runs of
// prod_{k<c} radix_k rows.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#include "ftlm_internal.hpp"

namespace ftlm {

bool site_has_singles(const HostHam &hh, int k) {
  const int r = hh.radix[k];
  for (int a = 0; a < r; a++)
    for (int b = 0; b < r; b++) {
      if (a == b) continue;
      const Cx<double> c = hh.h[(size_t)k * 256 + a * 16 + b];
      if (c.re != 0.0 || c.im != 0.0) return true;
    }
  if (hh.has_z)
    for (int l = 0; l < hh.n; l++) {
      const Cx<double> p = hh.czp[k * hh.n + l], m = hh.czm[k * hh.n + l];
      if (p.re != 0.0 || p.im != 0.0 || m.re != 0.0 || m.im != 0.0) return true;
    }
  return false;
}

namespace {

struct Cover {
  std::vector<std::vector<int>> extra;  // extra active sites of each pass
  std::vector<std::vector<int>> pairs;  // pairs (device order) of each pass
};

// Greedy cover for chunk size c; returns false if some pair cannot be placed.
// With rng, the seed pair and ties between equal gains are drawn at random
// (restarts of the greedy search); without it the lowest index wins.
bool greedy_cover(const HostHam &hh, const std::vector<int> &pi, const std::vector<int> &pj, int c,
                  uint64_t cap_extra, int max_extra, Cover &out, std::mt19937 *rng = nullptr) {
  const int n = hh.n, np = (int)pi.size();
  std::vector<char> covered(np, 0);
  int left = np;
  out = Cover();
  auto inC = [&](int k) { return k < c; };
  while (left > 0 || out.extra.empty()) {
    std::vector<int> S;
    uint64_t prod = 1;
    std::vector<char> inS(n, 0);
    auto add = [&](int k) {
      if (inC(k) || inS[k]) return true;
      if (prod * (uint64_t)hh.radix[k] > cap_extra || (int)S.size() >= max_extra) return false;
      prod *= hh.radix[k];
      inS[k] = 1;
      S.push_back(k);
      return true;
    };
    int seed = -1;
    if (rng && left > 0) {
      int pick = (int)((*rng)() % (uint32_t)left);
      for (int p = 0; p < np; p++)
        if (!covered[p] && pick-- == 0) { seed = p; break; }
    } else {
      for (int p = 0; p < np; p++)
        if (!covered[p]) { seed = p; break; }
    }
    if (seed >= 0) {
      if (!add(pi[seed]) || !add(pj[seed])) return false;
    }
    while (true) {
      int best = -1, best_gain = 0, n_tie = 0;
      for (int k = c; k < n; k++) {
        if (inS[k] || prod * (uint64_t)hh.radix[k] > cap_extra || (int)S.size() >= max_extra) continue;
        int gain = 0;
        for (int p = 0; p < np; p++) {
          if (covered[p]) continue;
          const int a = pi[p], b = pj[p];
          if ((a == k && (inC(b) || inS[b])) || (b == k && (inC(a) || inS[a]))) gain++;
        }
        if (gain > best_gain) {
          best_gain = gain;
          best = k;
          n_tie = 1;
        } else if (rng && gain == best_gain && gain > 0 && ((*rng)() % (uint32_t)(++n_tie)) == 0) {
          best = k;  // reservoir choice among equal gains
        }
      }
      if (best < 0) break;
      add(best);
    }
    // fill the window: more active sites cost nothing and make later passes lighter
    for (int k = c; k < n; k++)
      if (!inS[k] && prod * (uint64_t)hh.radix[k] <= cap_extra && (int)S.size() < max_extra) add(k);
    std::vector<int> mine;
    for (int p = 0; p < np; p++) {
      if (covered[p]) continue;
      if ((inC(pi[p]) || inS[pi[p]]) && (inC(pj[p]) || inS[pj[p]])) {
        covered[p] = 1;
        left--;
        mine.push_back(p);
      }
    }
    std::sort(S.begin(), S.end());
    out.extra.push_back(S);
    out.pairs.push_back(mine);
    if (seed < 0) break;  // no pairs at all: one pass for diagonal and singles
  }
  return true;
}

}  // namespace

constexpr int kPassRestarts = 256;  // randomised greedy restarts of the LDS-window cover

int plan_passes_sorted(const HostHam &hh, const std::vector<int> &pi, const std::vector<int> &pj,
                       size_t window_rows, PassPlan &plan) {
  plan.passes.clear();
  plan.pairs.clear();
  const int n = hh.n;
  std::vector<char> need_single(n);
  for (int k = 0; k < n; k++) need_single[k] = site_has_singles(hh, k);

  // windows with other spins than 1/2 keep their digits packed in 32 bits
  bool all_two = true;
  for (int k = 0; k < n; k++) all_two = all_two && hh.radix[k] == 2;
  const int max_active = all_two ? kMaxSites : 8;
  Cover best;
  int best_c = -1;
  double best_cost = 1e300;
  if (hh.dim <= window_rows && n <= max_active) {
    best_c = n;  // one window holds everything
    best.extra.assign(1, {});
    std::vector<int> all(pi.size());
    for (size_t p = 0; p < pi.size(); p++) all[p] = (int)p;
    best.pairs.assign(1, all);
  } else {
    for (int c = 0; c < n && c <= max_active; c++) {
      const uint64_t chunk = hh.stride[c];  // prod_{k<c} radix
      if (chunk > window_rows) break;
      Cover cv;
      if (!greedy_cover(hh, pi, pj, c, window_rows / chunk, max_active - c, cv)) continue;
      // randomised restarts (fixed seed: the plan is reproducible); every pass
      // saved is one read of v and one read and write of w
      {
        std::mt19937 rng(1234567u + (unsigned)c);
        for (int r = 0; r < kPassRestarts && cv.extra.size() > 1; r++) {
          Cover alt;
          if (greedy_cover(hh, pi, pj, c, window_rows / chunk, max_active - c, alt, &rng) &&
              alt.extra.size() < cv.extra.size())
            cv = alt;
        }
      }
      // place sites with single flips that no pass holds yet
      for (int k = c; k < n; k++) {
        if (!need_single[k]) continue;
        bool found = false;
        for (auto &S : cv.extra)
          if (std::find(S.begin(), S.end(), k) != S.end()) found = true;
        if (found) continue;
        bool placed = false;
        for (auto &S : cv.extra) {
          uint64_t prod = 1;
          for (int x : S) prod *= hh.radix[x];
          if (prod * hh.radix[k] * chunk <= window_rows && c + (int)S.size() < max_active) {
            S.push_back(k);
            std::sort(S.begin(), S.end());
            placed = true;
            break;
          }
        }
        if (!placed) {
          cv.extra.push_back({k});
          cv.pairs.push_back({});
        }
      }
      const double bytes = (double)chunk * 16.0;
      const double eff = bytes >= 128.0 ? 1.0 : bytes / 128.0;
      const double cost = (double)cv.extra.size() * (32.0 + 16.0 / eff);
      if (cost < best_cost) {
        best_cost = cost;
        best = cv;
        best_c = c;
      }
    }
    if (best_c < 0) return FTLM_ERANGE;
  }

  // single flips of site k go to the pass holding k that has the fewest singles so
  // far, at most kMaxSinglesPerPass per pass (a new pass is opened when all are full)
  constexpr int kMaxSinglesPerPass = 4;
  std::vector<int> owner(n, -1), load(best.extra.size(), 0);
  auto holds = [&](size_t ps, int k) {
    return k < best_c || std::find(best.extra[ps].begin(), best.extra[ps].end(), k) != best.extra[ps].end();
  };
  for (int k = 0; k < n; k++) {
    if (!need_single[k]) continue;
    int bp = -1;
    for (size_t ps = 0; ps < best.extra.size(); ps++)
      if (holds(ps, k) && load[ps] < kMaxSinglesPerPass && (bp < 0 || load[ps] < load[bp])) bp = (int)ps;
    if (bp < 0) {
      std::vector<int> S;
      uint64_t prod = 1;
      const uint64_t chunk = best_c < n ? hh.stride[best_c] : hh.dim;
      const int max_extra = max_active - std::min(best_c, n);
      if (k >= best_c) {
        S.push_back(k);
        prod = hh.radix[k];
      }
      for (int x = best_c; x < n; x++)
        if (x != k && prod * hh.radix[x] * chunk <= window_rows && (int)S.size() < max_extra) {
          S.push_back(x);
          prod *= hh.radix[x];
        }
      std::sort(S.begin(), S.end());
      best.extra.push_back(S);
      best.pairs.push_back({});
      load.push_back(0);
      bp = (int)best.extra.size() - 1;
    }
    owner[k] = bp;
    load[bp]++;
  }
  const int npass = (int)best.extra.size();
  for (int ps = 0; ps < npass; ps++) {
    PassDesc D;
    std::memset(&D, 0, sizeof(D));
    std::vector<int> act;
    for (int k = 0; k < std::min(best_c, n); k++) act.push_back(k);
    for (int k : best.extra[ps]) act.push_back(k);
    D.na = (int)act.size();
    uint32_t ws = 1;
    bool pow2 = true;
    std::vector<int> pos(n, -1);
    for (int a = 0; a < D.na; a++) {
      D.act[a] = act[a];
      D.wrad[a] = hh.radix[act[a]];
      D.wst[a] = ws;
      D.gst[a] = hh.stride[act[a]];
      ws *= (uint32_t)hh.radix[act[a]];
      pow2 = pow2 && hh.radix[act[a]] == 2;
      pos[act[a]] = a;
    }
    D.wsize = ws;
    D.nwin = (uint32_t)(hh.dim / ws);
    D.pow2 = pow2 ? 1 : 0;
    int ni = 0;
    for (int k = 0; k < n; k++)
      if (pos[k] < 0) {
        D.inact[ni] = k;
        D.irad[ni] = hh.radix[k];
        D.ist[ni] = hh.stride[k];
        ni++;
      }
    D.ni = ni;
    D.first = ps == 0;
    D.last = ps == npass - 1;
    int ns = 0;
    for (int a = 0; a < D.na; a++)
      if (owner[act[a]] == ps) D.sing[ns++] = a;
    D.nsing = ns;
    D.pp_off = (int)plan.pairs.size();
    for (int p : best.pairs[ps]) plan.pairs.push_back(make_int4(p, pos[pi[p]], pos[pj[p]], 0));
    D.npp = (int)plan.pairs.size() - D.pp_off;
    // the pair-coefficient table of a general-radix pass, if it fits 48 KB of
    // LDS at complex128 (else 0: the kernel evaluates the factors per row)
    D.ctab = 0;
    for (int p : best.pairs[ps]) D.ctab += 4 * hh.radix[pi[p]] * hh.radix[pj[p]];
    if ((size_t)D.ctab * 16 > 48 * 1024) D.ctab = 0;
    plan.passes.push_back(D);
  }
  if (plan.pairs.empty()) plan.pairs.push_back(make_int4(0, 0, 0, 0));
  return FTLM_OK;
}

// L2-window plan.  The window budget is an XCD's share of L2 (a few MB), three
// orders of magnitude above the LDS windows, so a pass covers far more pairs:
// the lowest sites are always in the window (contiguous runs), the greedy
// cover picks the others.
constexpr int kRestarts = 64;  // randomised greedy restarts of the L2-window cover

int plan_l2_windows(const HostHam &hh, const std::vector<int> &pi, const std::vector<int> &pj,
                    size_t window_rows, int lane_bits, WinPlan &plan) {
  const bool spin_half = lane_bits > 0;
  const int lb = spin_half ? lane_bits : kLowBits;
  plan = WinPlan();
  plan.window_rows = window_rows;
  const int n = hh.n, np = (int)pi.size();
  std::vector<char> need_single(n);
  for (int k = 0; k < n; k++) need_single[k] = site_has_singles(hh, k);
  Cover best;
  int best_c = -1;
  if (hh.dim <= window_rows) {
    best_c = n;
    best.extra.assign(1, {});
    std::vector<int> all(np);
    for (int p = 0; p < np; p++) all[p] = p;
    best.pairs.assign(1, all);
  } else if (spin_half) {
    int ebits = 0;
    while (((uint64_t)1 << (lb + ebits + 1)) <= window_rows) ebits++;
    if (ebits < 1 && n > lb) return FTLM_ERANGE;
    if (!greedy_cover(hh, pi, pj, lb, (uint64_t)1 << ebits, ebits, best)) return FTLM_ERANGE;
    best_c = lb;
    std::mt19937 rng(12345u);
    for (int rs = 0; rs < kRestarts; rs++) {
      Cover cv;
      if (greedy_cover(hh, pi, pj, lb, (uint64_t)1 << ebits, ebits, cv, &rng) &&
          cv.extra.size() < best.extra.size())
        best = cv;
    }
  } else {
    double best_cost = 1e300;
    std::mt19937 rng(12345u);
    for (int c = 1; c < n; c++) {
      const uint64_t chunk = hh.stride[c];
      if (chunk > window_rows) break;
      const double bytes = (double)chunk * 16.0;
      const double eff = bytes >= 128.0 ? 1.0 : bytes / 128.0;
      for (int rs = 0; rs <= kRestarts; rs++) {
        Cover cv;
        if (!greedy_cover(hh, pi, pj, c, window_rows / chunk, n, cv, rs ? &rng : nullptr)) break;
        const double cost = (double)cv.extra.size() * (32.0 + 16.0 / eff);
        if (cost < best_cost) {
          best_cost = cost;
          best = cv;
          best_c = c;
        }
      }
    }
    if (best_c < 0) return FTLM_ERANGE;
  }
  const int c = std::min(best_c, n);
  const uint64_t chunk = c < n ? hh.stride[c] : hh.dim;
  auto holds = [&](size_t ps, int k) {
    return k < c || std::find(best.extra[ps].begin(), best.extra[ps].end(), k) != best.extra[ps].end();
  };
  // single flips of site k: the first pass whose window holds k (else a new pass)
  std::vector<int> owner(n, -1);
  for (int k = 0; k < n; k++) {
    if (!need_single[k]) continue;
    for (size_t ps = 0; ps < best.extra.size() && owner[k] < 0; ps++)
      if (holds(ps, k)) owner[k] = (int)ps;
    if (owner[k] >= 0) continue;
    std::vector<int> S{k};
    uint64_t prod = hh.radix[k];
    const uint64_t cap = window_rows / chunk;
    for (int x = c; x < n; x++) {
      const int max_extra = spin_half ? 31 : n;
      if (x != k && prod * (uint64_t)hh.radix[x] <= cap && (int)S.size() < max_extra) {
        S.push_back(x);
        prod *= hh.radix[x];
      }
    }
    std::sort(S.begin(), S.end());
    best.extra.push_back(S);
    best.pairs.push_back({});
    owner[k] = (int)best.extra.size() - 1;
  }
  const int npass = (int)best.extra.size();
  for (int ps = 0; ps < npass; ps++) {
    WinPass W;
    std::memset(&W, 0, sizeof(W));
    W.first = ps == 0;
    W.last = ps == npass - 1;
    W.diag = ps == 0;
    W.p0 = (int)plan.plist.size();
    {
      // order by the number of sites outside the lane / tile bits (spin-1/2
      // kernels); pairs with one such site by that site
      std::vector<int> prs = best.pairs[ps];
      auto cls = [&](int p) { return (pi[p] >= lb) + (pj[p] >= lb); };
      std::stable_sort(prs.begin(), prs.end(), [&](int a, int b) {
        if (cls(a) != cls(b)) return cls(a) < cls(b);
        if (cls(a) == 1) return pj[a] < pj[b];
        return false;
      });
      for (int p : prs) {
        plan.plist.push_back(make_int4(p, pi[p], pj[p], 0));
        if (cls(p) == 0) W.np_ll++;
        else if (cls(p) == 1) {
          W.np_lh++;
          W.xmask |= 1u << pj[p];
        }
      }
      // entries with one site outside the low bits come in runs of the same
      // outer site: .w = the end of the entry's run, counted from the pass's
      // first entry, so that a kernel knows a run's length from its first entry
      const int q0 = W.p0 + W.np_ll, q1 = q0 + W.np_lh;
      for (int q = q0; q < q1;) {
        int r = q;
        while (r < q1 && plan.plist[r].z == plan.plist[q].z) r++;
        for (int u = q; u < r; u++) plan.plist[u].w = r - W.p0;
        q = r;
      }
    }
    W.np = (int)plan.plist.size() - W.p0;
    for (int k = 0; k < n; k++)
      if (owner[k] == ps) W.smask |= 1u << k;
    std::vector<char> inw(n, 0);
    for (int k = 0; k < c; k++) inw[k] = 1;
    for (int k : best.extra[ps]) inw[k] = 1;
    uint64_t ws = 1;
    for (int k = 0; k < n; k++) {
      if (inw[k]) {
        W.act[W.na] = k;
        W.wrad[W.na] = hh.radix[k];
        W.na++;
        ws *= (uint64_t)hh.radix[k];
      } else {
        W.inact[W.ni] = k;
        W.irad[W.ni] = hh.radix[k];
        W.ni++;
      }
    }
    W.wsize = (uint32_t)ws;
    W.nwin = (uint32_t)(hh.dim / ws);
    if (spin_half) {
      for (int k = lb; k < n; k++) {
        if (inw[k]) W.emask |= 1u << k;
        else W.omask |= 1u << k;
        if ((W.smask >> k) & 1u) W.xmask |= 1u << k;
      }
      W.nin = (uint32_t)(ws >> lb);
    } else {
      W.nin = (uint32_t)((ws + kBlock - 1) / kBlock);
    }
    plan.passes.push_back(W);
  }
  if (plan.plist.empty()) plan.plist.push_back(make_int4(0, 0, 0, 0));
  return FTLM_OK;
}

PlanWindows g_windows;

size_t tile_window_bytes_setting(uint64_t vec_bytes) {
  // default: 2 MB windows (two in flight per XCD fill its 4 MB L2); a vector of
  // at most 160 MB stays in the 256 MB last-level cache, where one window over
  // everything (a single pass) is faster
  const int kb = g_windows.tile_kb.load();
  return (size_t)(kb ? kb : (vec_bytes <= (160ull << 20) ? 65536 : 2048)) * 1024;
}

size_t l2_window_bytes_setting() {
  const int kb = g_windows.l2_kb.load();
  return (size_t)(kb ? kb : 1024) * 1024;
}

}  // namespace ftlm

using namespace ftlm;

extern "C" int ftlm_set_plan_windows(int32_t pass_kb, int32_t l2_kb, int32_t tile_kb) {
  auto ok = [](int32_t v, int32_t hi) { return v == 0 || (v >= 4 && v <= hi); };
  if (!ok(pass_kb, 128) || !ok(l2_kb, 65536) || !ok(tile_kb, 65536)) {
    set_error("plan windows out of range (pass 4..128 KiB, L2 and tile 4..65536 KiB, or 0)");
    return FTLM_EINVAL;
  }
  g_windows.pass_kb = pass_kb;
  g_windows.l2_kb = l2_kb;
  g_windows.tile_kb = tile_kb;
  return FTLM_OK;
}

extern "C" int ftlm_describe_passes(const ftlm_system *sys, int32_t precision, int32_t max_pass,
                                    int32_t *n_pass, uint32_t *window_rows, int32_t *n_active,
                                    int32_t *n_pairs, int32_t *n_singles, int32_t *pair_sites,
                                    double *nnz_per_row) {
  if (!n_pass || (max_pass > 0 && (!window_rows || !n_active || !n_pairs || !n_singles))) {
    set_error("NULL argument");
    return FTLM_EINVAL;
  }
  if (precision != FTLM_C128 && precision != FTLM_C64) {
    set_error("bad precision");
    return FTLM_EINVAL;
  }
  HostHam hh;
  std::string err;
  int rc = compile_hamiltonian(sys, hh, err);
  if (rc) {
    set_error(err);
    return rc;
  }
  std::vector<int> perm;
  int n_ll, n_lh, mx_off[kMaxSites + 1];
  sort_pairs(hh, perm, n_ll, n_lh, mx_off);
  std::vector<int> spi(hh.npair), spj(hh.npair);
  for (int q = 0; q < hh.npair; q++) {
    spi[q] = hh.pi[perm[q]];
    spj[q] = hh.pj[perm[q]];
  }
  PassPlan plan;
  rc = plan_passes_sorted(hh, spi, spj, window_bytes_setting() / (precision == FTLM_C64 ? 8 : 16),
                          plan);
  if (rc) {
    set_error("no windowed-pass plan fits the window size");
    return rc;
  }
  *n_pass = (int32_t)plan.passes.size();
  if (nnz_per_row) *nnz_per_row = hh.nnz_per_row;
  int w = 0;
  for (int ps = 0; ps < (int)plan.passes.size() && ps < max_pass; ps++) {
    const PassDesc &D = plan.passes[ps];
    window_rows[ps] = D.wsize;
    n_active[ps] = D.na;
    n_pairs[ps] = D.npp;
    n_singles[ps] = D.nsing;
    if (pair_sites)
      for (int q = 0; q < D.npp; q++) {
        const int4 e = plan.pairs[D.pp_off + q];
        pair_sites[w++] = D.act[e.y];
        pair_sites[w++] = D.act[e.z];
      }
  }
  return FTLM_OK;
}

extern "C" int ftlm_describe_windows(const ftlm_system *sys, int32_t precision, int64_t window_bytes,
                                     int32_t max_pass, int32_t *n_pass, uint32_t *window_rows,
                                     uint32_t *window_sites, int32_t *n_pairs, uint32_t *single_sites,
                                     int32_t *pair_sites) {
  if (!n_pass || (max_pass > 0 && (!window_rows || !window_sites || !n_pairs || !single_sites))) {
    set_error("NULL argument");
    return FTLM_EINVAL;
  }
  if (precision != FTLM_C128 && precision != FTLM_C64) {
    set_error("bad precision");
    return FTLM_EINVAL;
  }
  HostHam hh;
  std::string err;
  int rc = compile_hamiltonian(sys, hh, err);
  if (rc) {
    set_error(err);
    return rc;
  }
  std::vector<int> perm;
  int n_ll, n_lh, mx_off[kMaxSites + 1];
  sort_pairs(hh, perm, n_ll, n_lh, mx_off);
  std::vector<int> spi(hh.npair), spj(hh.npair);
  for (int q = 0; q < hh.npair; q++) {
    spi[q] = hh.pi[perm[q]];
    spj[q] = hh.pj[perm[q]];
  }
  const size_t wb = window_bytes > 0 ? (size_t)window_bytes : l2_window_bytes_setting();
  WinPlan plan;
  rc = plan_l2_windows(hh, spi, spj, wb / (precision == FTLM_C64 ? 8 : 16),
                       (hh.spin_half && hh.n >= kLowBits) ? kLowBits : 0, plan);
  if (rc) {
    set_error("no L2-window plan fits the window size");
    return rc;
  }
  *n_pass = (int32_t)plan.passes.size();
  int w = 0;
  for (int ps = 0; ps < (int)plan.passes.size() && ps < max_pass; ps++) {
    const WinPass &W = plan.passes[ps];
    window_rows[ps] = W.wsize;
    uint32_t m = 0;
    for (int a = 0; a < W.na; a++) m |= 1u << W.act[a];
    window_sites[ps] = m;
    n_pairs[ps] = W.np;
    single_sites[ps] = W.smask;
    if (pair_sites)
      for (int q = 0; q < W.np; q++) {
        const int4 e = plan.plist[W.p0 + q];
        pair_sites[w++] = e.y;
        pair_sites[w++] = e.z;
      }
  }
  return FTLM_OK;
}
