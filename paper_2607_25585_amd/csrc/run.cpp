// Plain FTLM run driver (ftlm_run): Sec. 2.2 for one Hamiltonian and a list of
// fields.  Per field, the R random vectors are processed in waves of K columns;
// each wave is: start vectors -> O v_1 -> N_L Lanczos steps (two kernels per
// step, replayed from a captured HIP graph) -> implicit-QL Krylov eigenpairs.
// The Boltzmann sums run once per field.  No device memory is allocated: all
// buffers are carved from the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ftlm_internal.hpp"

namespace ftlm {

namespace {

struct Carve {
  size_t off = 0;
  size_t take(size_t n) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return o;
  }
};

struct RunPlan {
  int K = 0, R = 0, NL = 0, nT = 0, nF = 0, prec = 0;
  size_t es = 16;
  uint64_t dim = 0;
  size_t buf[3], ov1, alpha, beta, yre, yim, sx, smax, done, nused, part, counter;
  size_t eps, q1, qy, nused_all, tri, T, dims, lnZ, E, C, M, emin;
  // two staging slots of a wave's (alpha, beta, y_re, n_used) for the
  // eigenpairs, which run on a second stream while the next wave iterates
  size_t st_ab[2], st_nu[2], st_tri[2];
  size_t total = 0;
};

int validate_params(const ftlm_run_params *p, std::string &err) {
  if (!p) { err = "params is NULL"; return FTLM_EINVAL; }
  if (p->R < 1) { err = "R must be >= 1"; return FTLM_EINVAL; }
  if (p->n_lanczos < 1 || p->n_lanczos > 1024) { err = "n_lanczos must be in [1, 1024]"; return FTLM_ERANGE; }
  if (p->n_T < 1 || !p->T) { err = "a temperature grid is required"; return FTLM_EINVAL; }
  for (int i = 0; i < p->n_T; i++)
    if (!(p->T[i] > 0) || !std::isfinite(p->T[i])) { err = "temperatures must be positive"; return FTLM_EINVAL; }
  if (p->precision != FTLM_C128 && p->precision != FTLM_C64) { err = "bad precision"; return FTLM_EINVAL; }
  if (p->columns < 0 || p->columns > 64) { err = "columns must be in [0, 64]"; return FTLM_ERANGE; }
  if (p->fields) {
    if (p->n_fields < 1) { err = "n_fields must be >= 1"; return FTLM_EINVAL; }
    for (int i = 0; i < 3 * p->n_fields; i++)
      if (!std::isfinite(p->fields[i])) { err = "fields must be finite"; return FTLM_EINVAL; }
  } else if (p->n_fields > 1) {
    err = "n_fields > 1 needs a fields array";
    return FTLM_EINVAL;
  }
  return FTLM_OK;
}

void make_plan(const ftlm_hamiltonian *h, const ftlm_run_params *p, RunPlan &pl) {
  pl.R = p->R;
  pl.NL = p->n_lanczos;
  pl.nT = p->n_T;
  pl.nF = p->fields ? p->n_fields : 1;
  pl.prec = p->precision;
  pl.es = p->precision == FTLM_C64 ? 8 : 16;
  // columns = 0: one vector per wave once the vectors leave the caches (the tile
  // and pass kernels stage one column), four between 2^17 and 2^20 rows, up to
  // 16 columns per gather from 2^14 rows (measured on the s=1/2 dipolar rings of
  // 14..20 sites), and below 2^14 rows every vector in one wave (at most 64):
  // there a Lanczos step costs its launch latency more than its columns
  pl.K = p->columns > 0 ? p->columns
                        : (h->host.dim >= (1ull << 20)   ? 1
                           : h->host.dim >= (1ull << 17) ? 4
                           : h->host.dim >= (1ull << 14) ? std::min(p->R, 16)
                                                         : std::min(p->R, 64));
  pl.K = std::min(pl.K, p->R);
  pl.dim = h->host.dim;
  Carve c;
  const size_t vec = (size_t)pl.dim * pl.K * pl.es;
  for (int i = 0; i < 3; i++) pl.buf[i] = c.take(vec);
  pl.ov1 = c.take(vec);
  const size_t sK = sizeof(double) * pl.K;
  pl.alpha = c.take(sK * pl.NL);
  pl.beta = c.take(sK * pl.NL);
  pl.yre = c.take(sK * pl.NL);
  pl.yim = c.take(sK * pl.NL);
  pl.sx = c.take(sK * (pl.NL + 1));
  pl.smax = c.take(sK);
  pl.done = c.take(sizeof(int) * pl.K);
  pl.nused = c.take(sizeof(int) * pl.K);
  pl.part = c.take(sizeof(double) * 2048 * 3 * pl.K);
  pl.counter = c.take(sizeof(unsigned) * kCounterWords);
  const size_t sR = sizeof(double) * pl.R;
  pl.eps = c.take(sR * pl.NL);
  pl.q1 = c.take(sR * pl.NL);
  pl.qy = c.take(sR * pl.NL);
  pl.nused_all = c.take(sizeof(int) * pl.R * pl.nF);
  pl.tri = c.take(sizeof(double) * 4 * pl.NL * pl.K);
  for (int k = 0; k < 2; k++) {
    pl.st_ab[k] = c.take(sK * pl.NL * 3);
    pl.st_nu[k] = c.take(sizeof(int) * pl.K);
    pl.st_tri[k] = c.take(sizeof(double) * 4 * pl.NL * pl.K);
  }
  pl.T = c.take(sizeof(double) * pl.nT);
  pl.dims = c.take(sizeof(double));
  const size_t res = sizeof(double) * pl.nT * pl.nF;
  pl.lnZ = c.take(res);
  pl.E = c.take(res);
  pl.C = c.take(res);
  pl.M = c.take(res);
  pl.emin = c.take(sizeof(double) * pl.nF);
  pl.total = (c.off + 255) & ~size_t(255);
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off);
}

// Issues the N_L Lanczos steps for a wave of K columns on stream s.
int issue_lanczos(const ftlm_hamiltonian *h, const RunPlan &pl, void *ws, int K, hipStream_t s,
                  hipEvent_t *ev = nullptr) {
  for (int j = 0; j < pl.NL; j++) {
    EpiLanczos lz{};
    void *cur = at<char>(ws, pl.buf[j % 3]);
    void *w = at<char>(ws, pl.buf[(j + 1) % 3]);
    lz.xprev = j > 0 ? at<char>(ws, pl.buf[(j + 2) % 3]) : nullptr;
    lz.ov1 = at<char>(ws, pl.ov1);
    lz.sx_cur = at<double>(ws, pl.sx) + (size_t)j * pl.K;
    lz.sx_prev = j > 0 ? at<double>(ws, pl.sx) + (size_t)(j - 1) * pl.K : nullptr;
    lz.beta_prev = j > 0 ? at<double>(ws, pl.beta) + (size_t)(j - 1) * pl.K : nullptr;
    lz.part = at<double>(ws, pl.part);
    lz.counter = at<unsigned>(ws, pl.counter);
    lz.alpha_out = at<double>(ws, pl.alpha) + (size_t)j * pl.K;
    lz.yre_out = at<double>(ws, pl.yre) + (size_t)j * pl.K;
    lz.yim_out = at<double>(ws, pl.yim) + (size_t)j * pl.K;
    HvLaunch L{};
    L.precision = pl.prec;
    L.K = K;
    L.v = cur;
    L.w = w;
    L.lz = &lz;
    if (ev && hipEventRecord(ev[2 * j], s) != hipSuccess) return FTLM_EHIP;
    int rc = launch_hv(h->dev, L, s);
    if (rc) return rc;
    if (ev && hipEventRecord(ev[2 * j + 1], s) != hipSuccess) return FTLM_EHIP;
    UpdateArgs u{};
    u.precision = pl.prec;
    u.K = K;
    u.step = j;
    u.n_lanczos = pl.NL;
    u.dim = (uint32_t)pl.dim;
    u.w = w;
    u.x = cur;
    u.sx_cur = lz.sx_cur;
    u.alpha = lz.alpha_out;
    u.beta = at<double>(ws, pl.beta) + (size_t)j * pl.K;
    u.sx_next = at<double>(ws, pl.sx) + (size_t)(j + 1) * pl.K;
    u.scale_max = at<double>(ws, pl.smax);
    u.done = at<int>(ws, pl.done);
    u.n_used = at<int>(ws, pl.nused);
    u.part = at<double>(ws, pl.part);
    u.counter = at<unsigned>(ws, pl.counter);
    rc = launch_update(u, s);
    if (rc) return rc;
  }
  return FTLM_OK;
}

}  // namespace

// Exposed for the batched driver and the tests of the workspace layout.
size_t plain_workspace_bytes(const ftlm_hamiltonian *h, const ftlm_run_params *p) {
  RunPlan pl;
  make_plan(h, p, pl);
  return pl.total;
}

}  // namespace ftlm

using namespace ftlm;

extern "C" {

int ftlm_run_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, size_t *bytes) {
  std::string err;
  if (!h || !bytes) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_params(p, err);
  if (rc) { set_error(err); return rc; }
  *bytes = plain_workspace_bytes(h, p);
  return FTLM_OK;
}

int ftlm_run(const ftlm_hamiltonian *hc, const ftlm_run_params *p, void *ws, size_t bytes,
             void *stream_, ftlm_result *out) {
  std::string err;
  if (!hc || !ws || !out) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_params(p, err);
  if (rc) { set_error(err); return rc; }
  ftlm_hamiltonian *h = const_cast<ftlm_hamiltonian *>(hc);
  RunPlan pl;
  make_plan(h, p, pl);
  if (bytes < pl.total) { set_error("workspace too small"); return FTLM_ENOMEM; }
  hipStream_t s = (hipStream_t)stream_;
  const double saved_B[3] = {h->host.B[0], h->host.B[1], h->host.B[2]};
  const double dimd = (double)pl.dim;
  if (hipMemcpyAsync(at<double>(ws, pl.T), p->T, sizeof(double) * pl.nT, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(at<double>(ws, pl.dims), &dimd, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("copy of run inputs failed");
    return FTLM_EHIP;
  }
  const bool timing = out->hv_ms != nullptr;
  const bool use_graph = !timing;  // timed runs launch step by step, with events around each H*v
  std::vector<hipEvent_t> events;
  double hv_ms = 0.0;
  int hv_launches = 0;
  if (timing) {
    events.resize(2 * (size_t)pl.NL, nullptr);
    for (auto &e : events)
      if (hipEventCreate(&e) != hipSuccess) {
        set_error("hipEventCreate failed");
        for (auto &x : events) if (x) (void)hipEventDestroy(x);
        return FTLM_EHIP;
      }
  }
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  int exec_K = 0;
  uint64_t exec_gen = 0;  // launch-layout generation the graph was captured with
  // eigenpairs of a finished wave run on s2 (default priority) while the next
  // wave iterates on s; ev[0..1]: slot's inputs staged, ev[2..3]: slot's
  // eigenpairs done, ev[4]: join before the Boltzmann sums
  hipStream_t s2 = nullptr;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  auto cleanup = [&]() {
    for (auto &x : events) if (x) (void)hipEventDestroy(x);
    events.clear();
    if (s2) (void)hipStreamSynchronize(s2);
    for (auto &x : ev) {
      if (x) (void)hipEventDestroy(x);
      x = nullptr;
    }
    if (s2) (void)hipStreamDestroy(s2);
    s2 = nullptr;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    exec = nullptr;
    graph = nullptr;
    cap = nullptr;
  };
  auto fail = [&](int code, const std::string &m) {
    cleanup();
    set_error(m);
    if (p->fields) (void)ftlm_hamiltonian_set_field(h, saved_B);
    return code;
  };
  std::vector<double> host_ab;
  if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) return fail(FTLM_EHIP, "stream create failed");
  for (auto &x : ev)
    if (hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) return fail(FTLM_EHIP, "event create failed");
  int wave = 0;
  for (int f = 0; f < pl.nF; f++) {
    if (p->fields) {
      rc = ftlm_hamiltonian_set_field(h, p->fields + 3 * f);
      if (rc) return fail(rc, std::string("set_field: ") + ftlm_last_error());
    }
    for (int c0 = 0; c0 < pl.R; c0 += pl.K) {
      const int K = std::min(pl.K, pl.R - c0);
      if (launch_zero_state(at<double>(ws, pl.smax), at<int>(ws, pl.done), at<int>(ws, pl.nused),
                            at<unsigned>(ws, pl.counter), kCounterWords, K, s))
        return fail(FTLM_EHIP, "zero_state launch failed");
      void *x0 = at<char>(ws, pl.buf[0]);
      if (p->r_init) {
        const char *src = reinterpret_cast<const char *>(p->r_init) + (size_t)f * pl.dim * pl.R * 16;
        rc = launch_copy_start(src, pl.R, c0, K, (uint32_t)pl.dim, pl.prec, x0, at<double>(ws, pl.part),
                               at<unsigned>(ws, pl.counter), at<double>(ws, pl.sx), 0, s);
      } else {
        rc = launch_gaussian(p->seed, p->instance, (uint32_t)f, (uint32_t)c0, K, (uint32_t)pl.dim,
                             pl.prec, x0, at<double>(ws, pl.part), at<unsigned>(ws, pl.counter),
                             at<double>(ws, pl.sx), 0, s);
      }
      if (rc) return fail(rc, "start-vector launch failed");
      HvLaunch L{};
      L.precision = pl.prec;
      L.K = K;
      L.v = x0;
      L.w = at<char>(ws, pl.ov1);
      L.scale = at<double>(ws, pl.sx);
      if (launch_hv(h->mom_dev, L, s)) return fail(FTLM_EHIP, "O v1 launch failed");
      if (use_graph && K == pl.K) {
        if (exec && exec_gen != h->dev.generation) {
          // the field change re-planned the H*v launches or moved their tables:
          // the captured graph holds the old values
          (void)hipGraphExecDestroy(exec);
          (void)hipGraphDestroy(graph);
          exec = nullptr;
          graph = nullptr;
        }
        if (!exec) {
          if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
            return fail(FTLM_EHIP, "stream create failed");
          if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(FTLM_EHIP, "begin capture failed");
          rc = issue_lanczos(h, pl, ws, K, cap);
          hipError_t e2 = hipStreamEndCapture(cap, &graph);
          if (rc || e2 != hipSuccess) return fail(FTLM_EHIP, "graph capture failed");
          if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
            return fail(FTLM_EHIP, "graph instantiate failed");
          exec_K = K;
          exec_gen = h->dev.generation;
        }
        if (hipGraphLaunch(exec, s) != hipSuccess) return fail(FTLM_EHIP, "graph launch failed");
      } else {
        rc = issue_lanczos(h, pl, ws, K, s, timing ? events.data() : nullptr);
        if (rc) return fail(rc, "Lanczos launch failed");
        if (timing) {
          if (hipStreamSynchronize(s) != hipSuccess) return fail(FTLM_EHIP, "synchronise failed");
          for (int j = 0; j < pl.NL; j++) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, events[2 * j], events[2 * j + 1]) != hipSuccess)
              return fail(FTLM_EHIP, "event timing failed");
            hv_ms += ms;
            hv_launches++;
          }
        }
      }
      (void)exec_K;
      {
        // stage (alpha, beta, y_re, n_used) in this wave's slot once the slot's
        // previous eigenpairs are done, then solve them on s2
        const int slot = wave & 1;
        const size_t ab = sizeof(double) * pl.K * pl.NL;
        double *st = at<double>(ws, pl.st_ab[slot]);
        int *snu = at<int>(ws, pl.st_nu[slot]);
        if ((wave >= 2 && hipStreamWaitEvent(s, ev[2 + slot], 0) != hipSuccess) ||
            hipMemcpyAsync(st, at<double>(ws, pl.alpha), ab, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(st + (size_t)pl.K * pl.NL, at<double>(ws, pl.beta), ab, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(st + 2 * (size_t)pl.K * pl.NL, at<double>(ws, pl.yre), ab, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(snu, at<int>(ws, pl.nused), sizeof(int) * K, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipEventRecord(ev[slot], s) != hipSuccess || hipStreamWaitEvent(s2, ev[slot], 0) != hipSuccess)
          return fail(FTLM_EHIP, "staging of the tridiagonals failed");
        rc = launch_tridiag(K, pl.NL, snu, 1, pl.K, st, st + (size_t)pl.K * pl.NL, st + 2 * (size_t)pl.K * pl.NL,
                            at<double>(ws, pl.eps), at<double>(ws, pl.q1), at<double>(ws, pl.qy), pl.R, c0,
                            at<double>(ws, pl.st_tri[slot]), s2);
        if (rc) return fail(rc, "tridiagonal launch failed");
        if (hipEventRecord(ev[2 + slot], s2) != hipSuccess) return fail(FTLM_EHIP, "event record failed");
        wave++;
      }
      if (hipMemcpyAsync(at<int>(ws, pl.nused_all) + (size_t)f * pl.R + c0, at<int>(ws, pl.nused),
                         sizeof(int) * K, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(FTLM_EHIP, "copy of n_used failed");
      if (out->alpha || out->beta) {
        host_ab.resize((size_t)pl.NL * K * 2);
        if (hipMemcpy2DAsync(host_ab.data(), sizeof(double) * K, at<double>(ws, pl.alpha),
                             sizeof(double) * pl.K, sizeof(double) * K, pl.NL, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpy2DAsync(host_ab.data() + (size_t)pl.NL * K, sizeof(double) * K, at<double>(ws, pl.beta),
                             sizeof(double) * pl.K, sizeof(double) * K, pl.NL, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return fail(FTLM_EHIP, "copy of tridiagonals failed");
        for (int c = 0; c < K; c++)
          for (int j = 0; j < pl.NL; j++) {
            const size_t o = ((size_t)f * pl.R + c0 + c) * pl.NL + j;
            if (out->alpha) out->alpha[o] = host_ab[(size_t)j * K + c];
            if (out->beta) out->beta[o] = host_ab[(size_t)pl.NL * K + (size_t)j * K + c];
          }
      }
    }
    const size_t ro = (size_t)f * pl.nT;
    if (hipEventRecord(ev[4], s2) != hipSuccess || hipStreamWaitEvent(s, ev[4], 0) != hipSuccess)
      return fail(FTLM_EHIP, "join of the eigenpair stream failed");
    rc = launch_boltzmann(1, pl.R, pl.NL, at<int>(ws, pl.nused_all) + (size_t)f * pl.R,
                          at<double>(ws, pl.eps), at<double>(ws, pl.q1), at<double>(ws, pl.qy),
                          at<double>(ws, pl.dims), at<double>(ws, pl.T), pl.nT,
                          at<double>(ws, pl.lnZ) + ro, at<double>(ws, pl.E) + ro,
                          at<double>(ws, pl.C) + ro, at<double>(ws, pl.M) + ro,
                          at<double>(ws, pl.emin) + f, s);
    if (rc) return fail(rc, "Boltzmann launch failed");
  }
  const size_t res = sizeof(double) * pl.nT * pl.nF;
  struct { double *dst; size_t off; size_t n; } outs[] = {
      {out->lnZ, pl.lnZ, res}, {out->E, pl.E, res}, {out->C, pl.C, res}, {out->M, pl.M, res},
      {out->E_min, pl.emin, sizeof(double) * pl.nF}};
  for (auto &o : outs)
    if (o.dst && hipMemcpyAsync(o.dst, at<char>(ws, o.off), o.n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(FTLM_EHIP, "copy of results failed");
  if (out->n_lanczos_used &&
      hipMemcpyAsync(out->n_lanczos_used, at<int>(ws, pl.nused_all), sizeof(int) * pl.R * pl.nF,
                     hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(FTLM_EHIP, "copy of n_used failed");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FTLM_EHIP, "stream synchronise failed");
  if (timing) {
    *out->hv_ms = hv_ms;
    if (out->hv_launches) *out->hv_launches = hv_launches;
  }
  cleanup();
  if (p->fields) {
    rc = ftlm_hamiltonian_set_field(h, saved_B);
    if (rc) return rc;
  }
  return FTLM_OK;
}

int ftlm_tridiag_eigen(int32_t n_cols, int32_t n_lanczos, const int32_t *n_used,
                       const double *alpha, const double *beta, const double *y, double *eps,
                       double *q1, double *qy, double *scratch, void *stream) {
  if (n_cols < 1 || n_lanczos < 1) { set_error("bad sizes"); return FTLM_EINVAL; }
  if (!alpha || !beta || !eps || !q1 || !qy || !scratch) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = launch_tridiag(n_cols, n_lanczos, n_used, 1, n_cols, alpha, beta, y, eps, q1, qy, n_cols, 0,
                          scratch, (hipStream_t)stream);
  if (rc) set_error("tridiagonal launch failed");
  return rc;
}

int ftlm_boltzmann(int32_t n_curves, int32_t R, int32_t n_lanczos, const int32_t *n_used,
                   const double *eps, const double *q1, const double *qy, const double *dims,
                   const double *T, int32_t n_T, double *lnZ, double *E, double *C, double *M,
                   double *E_min, void *stream) {
  if (n_curves < 1 || R < 1 || n_lanczos < 1 || n_T < 1) { set_error("bad sizes"); return FTLM_EINVAL; }
  if (!n_used || !eps || !q1 || !qy || !dims || !T || !lnZ || !E || !C || !M) {
    set_error("NULL argument");
    return FTLM_EINVAL;
  }
  int rc = launch_boltzmann(n_curves, R, n_lanczos, n_used, eps, q1, qy, dims, T, n_T, lnZ, E, C, M,
                            E_min, (hipStream_t)stream);
  if (rc) set_error("Boltzmann launch failed");
  return rc;
}

}  // extern "C"
