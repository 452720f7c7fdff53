// Internal declarations shared by the host runtime and the HIP kernels of the
// FTLM library.  Not part of the public ABI (include/ftlm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ftlm.h"

namespace ftlm {

constexpr double kMuB = 0.67171381563;    // mu_B / k_B in K/T (CODATA 2018)
constexpr double kCDip = 6.2294807e-4;    // mu0 mu_B^2 / (4 pi k_B) in K nm^3
constexpr int kMaxSites = FTLM_MAX_SITES;
constexpr int kMaxRadix = FTLM_MAX_TWO_S + 1;  // 16
constexpr int kLowBits = 8;                    // spin-1/2 tile: 256 rows, sites 0..7 vary
constexpr int kBlock = 256;
constexpr int kTileBits = 11;                  // spin-1/2 LDS tile: 2048 rows, sites 0..10 vary
constexpr int kTileRows = 1 << kTileBits;
constexpr int kRowsPerThread = kTileRows / kBlock;  // 8
constexpr int kCtrGroups = 64;                 // arrival counters of the grid reductions
constexpr int kCounterWords = 1 + kCtrGroups;  // words of one reduction counter array

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R re, im;
};

// ---------------------------------------------------------------------------
// Host-side compiled Hamiltonian (Sec. 2.1, Eq. mce-hamop, in ladder form).
//
// Row nu with digits d_k (m_k = d_k - s_k) couples to partner pi through
//   diagonal   sum_k h_k[d,d] + sum_{i<j} c^zz_ij m_i m_j
//   site flip  pi = nu + D st_k, D in {-2,-1,1,2}:
//              h_k[d_k][d_k+D] + (D=-1: gp_k(m_k) F^+_k) + (D=+1: gm_k(m_k) F^-_k)
//              with F^{+-}_k = sum_{l != k} C^{+-z}_{kl} m_l
//   pair flip  pi = nu + Di st_i + Dj st_j, Di,Dj in {-1,+1}:
//              c^{ab}_ij g_a(m_i) g_b(m_j), a = '+' for Di = -1, '-' for Di = +1
// where gp(m) = <m|s+|m-1> and gm(m) = <m|s-|m+1>.
// ---------------------------------------------------------------------------
struct HostHam {
  int n = 0;
  int two_s[kMaxSites] = {0};
  int radix[kMaxSites] = {0};
  uint32_t stride[kMaxSites] = {0};
  uint64_t dim = 0;
  // inputs kept for set_field
  std::vector<double> J, d, e, g, pos;
  bool has_J = false, has_d = false, has_pos = false;
  double B[3] = {0, 0, 0};
  // one-site matrices h_k, [k][a*16+b] (a = row digit)
  std::vector<Cx<double>> h;  // n * 256
  // interacting pairs
  int npair = 0;
  std::vector<int> pi, pj;
  std::vector<Cx<double>> pc;   // [p][4]: c^{++}, c^{+-}, c^{-+}, c^{--}
  std::vector<double> pzz;      // [p]
  std::vector<double> zz;       // [n*n] symmetric c^zz matrix (0 off-pairs)
  // C^{+z}_{kl} (site k raised with s^+, times s^z of l) and C^{-z}_{kl}; [k*n+l]
  std::vector<Cx<double>> czp, czm;
  bool has_z = false;
  double nnz_per_row = 0;
  bool spin_half = false;  // every site s = 1/2
};

// Builds everything field-independent plus the one-site matrices for hh.B.
int compile_hamiltonian(const ftlm_system *sys, HostHam &hh, std::string &err);
void compile_site_terms(HostHam &hh);
double count_nnz_per_row(const HostHam &hh);

// ---------------------------------------------------------------------------
// Device tables.  All pointers refer to one contiguous device allocation
// owned by the handle.  Real = double for the complex128 path, float for the
// complex64 path.
// ---------------------------------------------------------------------------
template <typename R>
struct DevTables {
  // site tables, [k][16]
  const R *hdiag;          // h_k[d][d]
  const Cx<R> *hoff;       // [k][4][16]: h_k[d][d+D] for D = -2,-1,+1,+2
  const R *gp;             // <m|s+|m-1>
  const R *gm;             // <m|s-|m+1>
  const R *mval;           // m = d - s
  // pairs
  const int2 *pij;         // [p] (i, j)
  const Cx<R> *pc;         // [p][4] ordered (++, +-, -+, --)
  const R *pzz;            // [p]
  const R *zz;             // [n*n]
  const Cx<R> *czp, *czm;  // [n*n]
  // spin-1/2 tables
  const Cx<R> *pc_half;    // [p][4] indexed by row bits (b_i<<1 | b_j)
  const Cx<R> *hflip;      // [k][2]: h_k[b][1-b]
  const Cx<R> *cz_half;    // [k][l][2]: row bit b_k selects C^{-z} (b=0) or C^{+z} (b=1)
  const Cx<R> *lowf;       // [k][2][256]: sum_{l<8, l!=k} cz_half[k][l][sel] m_l(t)
};

struct HamGeom {
  int n, npair, has_z, spin_half;
  int n_ll, n_lh;          // spin-1/2: pairs sorted inside | mixed | outside the 11-bit tile
  int mx_off[kMaxSites + 1];  // mixed pairs with outer site a occupy [mx_off[a], mx_off[a+1])
  uint32_t single_mask;       // bit k: site k has non-zero single-site flip elements
  uint32_t dim;
  int radix[kMaxSites];
  uint32_t stride[kMaxSites];
  float s[kMaxSites];
};

// One pass of the windowed H*v: the "active" sites span a window of rows that
// fits in LDS (all other digits fixed); the pass applies the single flips of
// sites sing[] and the pairs listed at pass_pairs[pp_off .. pp_off+npp), all of
// whose sites are active.  Pass 0 also applies the diagonal; the last pass adds
// the partial sums of the earlier passes and runs the epilogue.
struct PassDesc {
  int na, ni, first, last, pow2, nsing, npp, pp_off;
  uint32_t wsize, nwin;
  int act[kMaxSites];       // active position a -> site
  int wrad[kMaxSites];      // radix of active position a
  uint32_t wst[kMaxSites];  // stride of a inside the window
  uint32_t gst[kMaxSites];  // stride of a in the full basis
  int inact[kMaxSites];     // inactive sites (ascending)
  int irad[kMaxSites];
  uint32_t ist[kMaxSites];
  int sing[kMaxSites];      // active positions whose single flips this pass applies
  int ctab;                 // general radix: entries of the pass's pair-coefficient table
                            // (sum over its pairs of 4 radix_i radix_j)
};

struct PassPlan {
  std::vector<PassDesc> passes;
  std::vector<int4> pairs;   // (pair index, active pos of i, active pos of j, 0)
  const int4 *d_pairs = nullptr;  // device copy (inside the handle's table block)
  size_t window_bytes = 0;
  // Per-window records (uniform diagonal / z-field parts and window base index)
  // and per-lane tables, computed on the device once per Hamiltonian and field.
  std::vector<size_t> rec_off, base_off, lane_off;  // byte offsets into rec_block, per pass
  void *rec_block = nullptr;
  size_t rec_bytes = 0;
};

struct HvTuning {
  int variant = 0;   // 0 = heuristic, 1 = direct gather, 2 = windowed passes, 3 = LDS tile, 4 = L2 windows,
                     // 5 = LDS tile over L2 windows, 6 = single-pass tiles (stream)
  int grid_cap = 0;  // 0 = default
  int kc = 0;        // columns per lane of the direct kernels (0 = widest dividing K)
};

// One pass of the L2-window H*v.  The rows are walked window by window: a
// window is the set of rows that share the digits of every "outer" site; its
// size is chosen to fit an XCD's L2, and all blocks of one XCD work on the same
// window, so every gather of a term acting only on window sites hits L2.  The
// pass applies the diagonal (if diag), the single flips of the sites in smask
// and the pairs [p0, p0 + np) of the plan's pair list; passes after the first
// add to w, the last one runs the Lanczos epilogue.
struct WinPass {
  int first, last, diag;
  int p0, np;
  int np_ll, np_lh;  // spin-1/2: the pass's pairs are ordered (both sites < 8),
                     // (one site < 8), (both >= 8); counts of the first two classes
  uint32_t smask;
  uint32_t nwin;   // windows
  uint32_t nin;    // 256-row work items per window
  // spin-1/2 kernel: row bits 0..7 run over the lanes; emask / omask are the
  // row bits >= 8 that vary inside a window / index the windows
  uint32_t emask, omask;
  uint32_t xmask;  // tile kernel: outer sites whose partner tile this pass stages
  // general kernel: window sites (ascending) and outer sites with radix and stride
  uint32_t wsize;  // rows per window
  int na, ni;
  int act[kMaxSites], wrad[kMaxSites];
  int inact[kMaxSites], irad[kMaxSites];
};

struct WinPlan {
  std::vector<WinPass> passes;
  std::vector<int4> plist;        // (pair index in device order, i, j, w), pass by pass; w = 0, or
                                  // for a pair with one site outside the low bits the end of
                                  // its run of pairs with that site (from the pass's first entry)
  const int4 *d_plist = nullptr;  // device copy (inside the handle's table block)
  size_t window_rows = 0;
  // tile plans: the spin-1/2 pair coefficients (four per pair, indexed by the
  // row bits b_i << 1 | b_j) in plist order, in the plan's precision, so that
  // an entry's coefficients are addressed by its position alone
  const void *d_pcoef = nullptr;
};

// Single-pass H*v for one column ("stream" kernel, variant 6).  Rows are walked
// in tiles of the low digits: a tile is the T = st_t consecutive rows that share
// the digits of every site >= t, so it is contiguous in memory and is staged in
// LDS once.  Terms on tile sites only read the tile from LDS; terms that move an
// outer digit read their partner rows straight from the vector (coalesced: the
// partner rows of a tile are contiguous up to a shift within the tile), so v is
// read from HBM about once and w written once, with the partner reads served by
// L2 and the last-level cache.  Needs has_z == 0 (no row-dependent single-flip
// coefficients).
struct StreamGeom {
  int n, t;                 // sites, tile sites (0..t-1)
  int np_in, np_mx, np_out;  // pairs in stream order: both sites < t | i < t <= j | t <= i
  uint32_t T, ntile, dim;   // rows per tile, tiles
  uint32_t smask;           // sites with single-site flips
  int half;                 // every spin 1/2: one list entry per mixed pair (else four)
  uint64_t gmask;           // bit 2 j + m: a mixed pair (i, j) has a nonzero coefficient whose
                            // move of j is +stride (m = 1) or -stride (m = 0)
  int radix[kMaxSites];
  uint32_t st[kMaxSites];
  int lg[kMaxSites];        // log2 of the stride of a tile site (tile radices all powers of two)
  float s[kMaxSites];
};

struct StreamPlan {
  bool ok = false;          // the kernel applies (has_z == 0)
  bool pow2 = false;        // every radix is a power of two (digits are bit fields of the row)
  bool half = false;        // every site has spin 1/2 (one pair move per row and pair)
  bool cplx = true;         // some pair or single-site coefficient is complex
  StreamGeom geom{};
  std::vector<int> order;   // stream order -> host pair index
  std::vector<double> tdiag;  // [T] diagonal of H restricted to the tile sites
  // device copies (inside the handle's table block), in the plan's precision
  const int2 *d_pij = nullptr;   // [np] (i, j), i < j
  const void *d_pc = nullptr;    // [np][4] (++, +-, -+, --)
  const void *d_pzz = nullptr;   // [np]
  const void *d_tdiag = nullptr; // [T]
};

// Host part of the stream plan for tiles of at most tile_rows rows.
void plan_stream(const HostHam &hh, uint32_t tile_rows, StreamPlan &pl);

struct DevHam {
  HamGeom geom;
  HvTuning tune[2][65];  // [precision][columns]
  DevTables<double> t64;
  DevTables<float> t32;
  PassPlan plan64, plan32;  // windowed-pass plans for complex128 / complex64
  WinPlan win64, win32;     // L2-window plans for complex128 / complex64
  WinPlan tw64, tw32;       // L2-window plans of the LDS tile kernel (spin 1/2, N >= 12)
  StreamPlan sp64, sp32;    // single-pass tile plans (complex128 / complex64)
  // key of the plans above (recomputed only when it changes)
  bool plan_valid = false;
  uint32_t plan_smask = 0;
  size_t plan_wb = 0, plan_l2b = 0, plan_tb = 0, plan_tb32 = 0;
  void *block = nullptr;  // device allocation holding every table
  size_t block_bytes = 0;
  // Launch layout: everything an H*v launch copies by value (geometry, table
  // addresses, pass and window plans).  A captured graph replays these values,
  // so a field change that alters any of them bumps the generation and the run
  // drivers capture again.
  uint64_t launch_sig = 0;
  uint64_t generation = 0;
};

// pi/pj: pair sites in the device (sorted) order.
bool site_has_singles(const HostHam &hh, int k);
int plan_passes_sorted(const HostHam &hh, const std::vector<int> &pi, const std::vector<int> &pj,
                       size_t window_rows, PassPlan &plan);
// window sizes of the planners in KiB (0: default), set by ftlm_set_plan_windows
struct PlanWindows {
  std::atomic<int> pass_kb{0}, l2_kb{0}, tile_kb{0};
};
extern PlanWindows g_windows;
size_t window_bytes_setting();
// L2-window plan for windows of at most window_rows rows (spin_half: the
// kernel's lanes run over row bits 0..7, which every window holds).
// lane_bits: 0 = general kernel; spin-1/2 kernels: the low row bits that every
// window holds (8 for the lane kernel, 11 for the LDS tile kernel).
int plan_l2_windows(const HostHam &hh, const std::vector<int> &pi, const std::vector<int> &pj,
                    size_t window_rows, int lane_bits, WinPlan &plan);
size_t l2_window_bytes_setting();
size_t tile_window_bytes_setting(uint64_t vec_bytes);  // window of the tile kernel for a vector of vec_bytes
void sort_pairs(const HostHam &hh, std::vector<int> &perm, int &n_ll, int &n_lh,
                int mx_off[kMaxSites + 1]);

}  // namespace ftlm

// Opaque handle of the public ABI.
struct ftlm_hamiltonian {
  ftlm::HostHam host;
  ftlm::DevHam dev;
  // moment operator O = -sum g_i s_i.B_hat as a site-only Hamiltonian
  ftlm::HostHam mom_host;
  ftlm::DevHam mom_dev;
  int device = 0;
};

namespace ftlm {

void set_error(const std::string &msg);
int upload_tables(const HostHam &hh, DevHam &dh, std::string &err);
int build_moment(ftlm_hamiltonian *h, std::string &err);

// ---- kernel launchers (kernels.hip) ----
struct EpiLanczos {
  // w = sx[j] * (H X_j) - beta[j-1] * sx[j-1] * X_{j-1}; alpha/y partials
  const void *xprev;       // X_{j-1} (nullptr at j = 0)
  const void *ov1;         // O v_1 (nullptr: no y)
  const double *sx_cur;    // [K] scale of X_j
  const double *sx_prev;   // [K]
  const double *beta_prev; // [K] (nullptr at j = 0)
  double *part;            // [grid][3][K] partials (alpha, y.re, y.im)
  unsigned *counter;
  double *alpha_out;       // [K]
  double *yre_out, *yim_out;  // [K]
};

struct HvLaunch {
  int precision;       // 0 c128, 1 c64
  int K;               // columns (row stride)
  const void *v;
  void *w;
  const double *scale; // optional per-column scale of v (nullptr = 1)
  const EpiLanczos *lz;  // nullptr = plain product
  int grid_cap;        // max blocks along x (0 = default)
  int kc;              // columns per lane (0 = auto)
  int variant;         // 0 auto, 1 direct kernels, 2 windowed passes, 3 LDS tile, 4 L2 windows
};

int launch_hv(const DevHam &dh, const HvLaunch &L, hipStream_t s);
struct HvParams;
// Variant 6 (stream.hip): one launch of grid <= cap blocks; *gx receives its grid.
// kc: bits 0..3 the block size (1: 256 threads, else 1024), bits 4..7 the log2 of
// the tiles per XCD chunk, bit 8 the LDS staging of the mixed pairs' partner tiles.
int launch_stream(const DevHam &dh, int precision, const HvParams &P, int cap, int kc, unsigned *gx,
                  hipStream_t s);
// (Re)computes the per-window records of both pass plans (allocates rec_block on
// first use).  Synchronous.
int build_pass_records(DevHam &dh, std::string &err);
void free_pass_records(DevHam &dh);
int hv_grid_blocks(const DevHam &dh, const HvLaunch &L, int *gx, int *gy, int *kc);

int launch_gaussian(uint64_t seed, uint32_t inst, uint32_t field, uint32_t r0, int K,
                    uint32_t dim, int precision, void *out, double *part, unsigned *counter,
                    double *sx0, int grid_cap, hipStream_t s);
int launch_copy_start(const void *src_c128, int src_cols, int col0, int K, uint32_t dim,
                      int precision, void *out, double *part, unsigned *counter, double *sx0,
                      int grid_cap, hipStream_t s);
struct UpdateArgs {
  int precision, K, step, n_lanczos;
  uint32_t dim;
  void *w;               // in: w, out: u = w - alpha sx X_j
  const void *x;         // X_j
  const double *sx_cur;  // [K]
  const double *alpha;   // [K] alpha_j
  double *beta;          // [K] beta_j (out)
  double *sx_next;       // [K] (out)
  double *scale_max;     // [K] running max(|alpha|, beta)
  int *done;             // [K]
  int *n_used;           // [K]
  double *part;          // [grid][K]
  unsigned *counter;
  int grid_cap;
};
int launch_update(const UpdateArgs &a, hipStream_t s);
int launch_zero_state(double *scale_max, int *done, int *n_used, unsigned *counters,
                      int n_counters, int K, hipStream_t s);
int launch_tridiag(int n_cols, int n_lanczos, const int *n_used, int used_stride, int in_stride,
                   const double *alpha, const double *beta, const double *y, double *eps,
                   double *q1, double *qy, int out_stride, int out_col0, double *scratch,
                   hipStream_t s);
int launch_boltzmann(int n_curves, int R, int n_lanczos, const int *n_used, const double *eps,
                     const double *q1, const double *qy, const double *dims, const double *T,
                     int n_T, double *lnZ, double *E, double *C, double *M, double *E_min,
                     hipStream_t s);

}  // namespace ftlm
