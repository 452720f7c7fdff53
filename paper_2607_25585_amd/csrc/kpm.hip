// Chebyshev (kernel polynomial) expansion of the thermal traces without a
// smoothing kernel -- the alternative to the Lanczos recursion named in Sec. 4
// for densities of states with pronounced bunching.  The H*v product is the
// same launch as in the Lanczos driver; only the recursion around it changes.
//
// Per field:
//   1. spectral bounds: N_B Lanczos steps from the first random vector, Krylov
//      eigenvalues (implicit QL), [lo, hi] = [min, max] widened by 2 % of the
//      spread; a = (hi - lo)/2, b = (hi + lo)/2, H~ = (H - b)/a;
//   2. per random vector (normalised Gaussian r): t_0 = r, t_1 = H~ t_0,
//      t_{n+1} = 2 H~ t_n - t_{n-1}; moments mu_n = Re<r|t_n>, nu_n = Re<O r|t_n>
//      (n <= N + 2), accumulated in the kernel that forms t_{n+1};
//   3. exp(-H/T) = exp(-lo/T) sum_{n<=N} c_n(a/T) T_n(H~) with
//      c_n(x) = (2 - delta_n0) (-1)^n exp(-x) I_n(x), the Bessel functions from
//      Miller's backward recurrence normalised by exp(x) = I_0 + 2 sum I_n;
//   4. ln Z, E, C, M from the moments with H = a H~ + b and
//      2 T_1 T_n = T_{n+1} + T_{|n-1|}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "device_reduce.hpp"
#include "ftlm_internal.hpp"

namespace ftlm {

namespace {

constexpr double kMargin = 0.02;

// out = mode 0: x;  1: (w - b x)/a;  2: 2 (w - b x)/a - y.   ab = {a, b} on the device.
// Moments of out: mom[0] = Re<t0|out>, mom[1] = Re<ov|out>.
template <typename R>
__global__ __launch_bounds__(kBlock) void cheb_kernel(int mode, uint32_t dim, const Cx<R> *__restrict__ w,
                                                      const Cx<R> *__restrict__ x, const Cx<R> *__restrict__ y,
                                                      Cx<R> *__restrict__ out, const Cx<R> *__restrict__ t0,
                                                      const Cx<R> *__restrict__ ov, const double *__restrict__ ab,
                                                      double *part, unsigned *counter, double *mom) {
  const double a = ab[0], b = ab[1];
  const double c1 = mode == 2 ? 2.0 / a : 1.0 / a;
  double red[2][1] = {{0.0}, {0.0}};
  for (uint64_t nu = (uint64_t)blockIdx.x * kBlock + threadIdx.x; nu < dim; nu += (uint64_t)gridDim.x * kBlock) {
    const Cx<R> xv = x[nu];
    double orr = xv.re, oi = xv.im;
    if (mode > 0) {
      const Cx<R> wv = w[nu];
      orr = c1 * ((double)wv.re - b * (double)xv.re);
      oi = c1 * ((double)wv.im - b * (double)xv.im);
      if (mode == 2) {
        const Cx<R> yv = y[nu];
        orr -= (double)yv.re;
        oi -= (double)yv.im;
      }
      out[nu] = Cx<R>{(R)orr, (R)oi};
      orr = (double)(R)orr;  // moments of the stored numbers
      oi = (double)(R)oi;
    }
    const Cx<R> tv = t0[nu], o = ov[nu];
    red[0][0] += (double)tv.re * orr + (double)tv.im * oi;
    red[1][0] += (double)o.re * orr + (double)o.im * oi;
  }
  block_partials_store<2, 1>(red, part, blockIdx.x);
}

// One block: the two moments from the Chebyshev kernel's per-block partials.
__global__ __launch_bounds__(kBlock) void cheb_finish(const double *part, unsigned gx, double *mom) {
  for (int k = 0; k < 2; k++) {
    const double s = block_sum_strided(part + k, gx, 2);
    if (threadIdx.x == 0) mom[k] = s;
  }
}

// x *= s[0] (normalises the start vector)
template <typename R>
__global__ __launch_bounds__(kBlock) void scale_kernel(uint32_t dim, Cx<R> *x, const double *s) {
  const double f = s[0];
  for (uint64_t nu = (uint64_t)blockIdx.x * kBlock + threadIdx.x; nu < dim; nu += (uint64_t)gridDim.x * kBlock) {
    const Cx<R> v = x[nu];
    x[nu] = Cx<R>{(R)((double)v.re * f), (R)((double)v.im * f)};
  }
}

// ab = {a, b} from the Ritz values eps[0..n_used)
__global__ void bounds_kernel(const double *eps, const int *n_used, double *ab, double *lohi) {
  if (threadIdx.x != 0) return;
  const int n = *n_used;
  double lo = eps[0], hi = eps[0];
  for (int i = 1; i < n; i++) {
    lo = fmin(lo, eps[i]);
    hi = fmax(hi, eps[i]);
  }
  const double pad = kMargin * (hi - lo) + 1e-12 * fmax(1.0, fmax(fabs(lo), fabs(hi)));
  lo -= pad;
  hi += pad;
  ab[0] = 0.5 * (hi - lo);
  ab[1] = 0.5 * (hi + lo);
  lohi[0] = lo;
  lohi[1] = hi;
}

// c[k][n] = (2 - delta_n0) (-1)^n exp(-x) I_n(x), x = a / T_k, n <= N (one thread
// per temperature).  Miller: backward recurrence I_{n-1} = (2n/x) I_n + I_{n+1}
// from m well above max(N, x), rescaled when large, normalised by
// exp(x) = I_0 + 2 sum_{n>=1} I_n.
__global__ void bessel_kernel(int nT, int N, const double *T, const double *ab, double *c) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nT) return;
  const double x = ab[0] / T[k];
  double *ck = c + (size_t)k * (N + 1);
  if (x < 1e-300) {
    for (int n = 0; n <= N; n++) ck[n] = n == 0 ? 1.0 : 0.0;
    return;
  }
  const double top = fmax((double)N, x);
  const int m = (int)(top + 30.0 + 6.0 * sqrt(top)) + 2;
  double ip = 0.0, i1 = 1e-300, sum = 0.0;  // I_{n+1}, I_n (unnormalised)
  for (int n = m; n >= 1; n--) {
    const double im = (2.0 * n / x) * i1 + ip;  // I_{n-1}
    ip = i1;
    i1 = im;
    // now i1 = I_{n-1}, ip = I_n
    sum += 2.0 * ip;
    if (n <= N) ck[n] = ip;
    if (i1 > 1e250) {
      const double s = 1e-250;
      i1 *= s;
      ip *= s;
      sum *= s;
      for (int q = n; q <= N; q++) ck[q] *= s;
    }
  }
  sum += i1;  // I_0
  ck[0] = i1 / sum;
  for (int n = 1; n <= N; n++) ck[n] = 2.0 * ((n & 1) ? -1.0 : 1.0) * ck[n] / sum;
}

// One thread per temperature: sums over the R vectors' moments of one field.
// mu, nu: [R][N+3]; lohi: {lo, hi}.
__global__ void kpm_thermo_kernel(int nT, int R, int N, const double *T, const double *ab, const double *lohi,
                                  const double *c, const double *mu, const double *nu, const double *dims,
                                  double *lnZ, double *E, double *C, double *M) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nT) return;
  const double a = ab[0], b = ab[1], t = T[k];
  const double *ck = c + (size_t)k * (N + 1);
  const int S = N + 3;
  double z = 0, h1 = 0, h2 = 0, mm = 0;
  for (int r = 0; r < R; r++) {
    const double *m = mu + (size_t)r * S, *v = nu + (size_t)r * S;
    for (int n = 0; n <= N; n++) {
      const int n1 = n > 0 ? n - 1 : 1, n2 = n > 1 ? n - 2 : 2 - n;
      const double ht = 0.5 * (m[n + 1] + m[n1]);                      // <r|H~ T_n|r>
      const double hht = 0.25 * (m[n + 2] + 2.0 * m[n] + m[n2]);       // <r|H~^2 T_n|r>
      z = fma(ck[n], m[n], z);
      h1 = fma(ck[n], a * ht + b * m[n], h1);
      h2 = fma(ck[n], a * a * hht + 2.0 * a * b * ht + b * b * m[n], h2);
      mm = fma(ck[n], v[n], mm);
    }
  }
  const double e1 = h1 / z, e2 = h2 / z;
  lnZ[k] = log(dims[0] / R) - lohi[0] / t + log(z);
  E[k] = e1;
  C[k] = (e2 - e1 * e1) / (t * t);
  M[k] = mm / z;
}

struct KPlan {
  int R = 0, NB = 0, N = 0, nT = 0, nF = 0, prec = 0;
  size_t es = 16;
  uint64_t dim = 0;
  size_t buf[3], W, T0, OV, alpha, beta, yre, yim, sx, smax, done, nused, part, counter;
  size_t eps, q1, qy, tri, ab, lohi, mstage, mu, nu, coef, T, dims, lnZ, E, C, M, emin;
  size_t total = 0;
};

struct Carve3 {
  size_t off = 0;
  size_t take(size_t n) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return o;
  }
};

void make_kplan(const ftlm_hamiltonian *h, const ftlm_run_params *p, int n_moments, KPlan &pl) {
  pl.R = p->R;
  pl.NB = p->n_lanczos;
  pl.N = n_moments;
  pl.nT = p->n_T;
  pl.nF = p->fields ? p->n_fields : 1;
  pl.prec = p->precision;
  pl.es = p->precision == FTLM_C64 ? 8 : 16;
  pl.dim = h->host.dim;
  Carve3 c;
  const size_t vec = (size_t)pl.dim * pl.es;
  for (int i = 0; i < 3; i++) pl.buf[i] = c.take(vec);
  pl.W = c.take(vec);
  pl.T0 = c.take(vec);
  pl.OV = c.take(vec);
  const size_t sd = sizeof(double);
  pl.alpha = c.take(sd * pl.NB);
  pl.beta = c.take(sd * pl.NB);
  pl.yre = c.take(sd * pl.NB);
  pl.yim = c.take(sd * pl.NB);
  pl.sx = c.take(sd * (pl.NB + 1));
  pl.smax = c.take(sd);
  pl.done = c.take(sizeof(int));
  pl.nused = c.take(sizeof(int));
  pl.part = c.take(sd * 2048 * 3);
  pl.counter = c.take(sizeof(unsigned) * kCounterWords);
  pl.eps = c.take(sd * pl.NB);
  pl.q1 = c.take(sd * pl.NB);
  pl.qy = c.take(sd * pl.NB);
  pl.tri = c.take(sd * 4 * pl.NB);
  pl.ab = c.take(sd * 2);
  pl.lohi = c.take(sd * 2 * pl.nF);
  pl.mstage = c.take(sd * 2 * (size_t)(pl.N + 3));
  pl.mu = c.take(sd * (size_t)pl.R * (pl.N + 3));
  pl.nu = c.take(sd * (size_t)pl.R * (pl.N + 3));
  pl.coef = c.take(sd * (size_t)pl.nT * (pl.N + 1));
  pl.T = c.take(sd * pl.nT);
  pl.dims = c.take(sd);
  const size_t res = sd * pl.nT * pl.nF;
  pl.lnZ = c.take(res);
  pl.E = c.take(res);
  pl.C = c.take(res);
  pl.M = c.take(res);
  pl.emin = c.take(sd * pl.nF);
  pl.total = (c.off + 255) & ~size_t(255);
}

template <typename T>
T *at3(void *ws, size_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off);
}

int validate_kpm(const ftlm_hamiltonian *h, const ftlm_run_params *p, int n_moments, std::string &err) {
  if (!p) { err = "params is NULL"; return FTLM_EINVAL; }
  if (p->R < 1) { err = "R must be >= 1"; return FTLM_EINVAL; }
  if (p->n_lanczos < 2 || p->n_lanczos > 1024) { err = "n_lanczos (bound steps) must be in [2, 1024]"; return FTLM_ERANGE; }
  if (n_moments < 2 || n_moments > 1000000) { err = "n_moments must be in [2, 1e6]"; return FTLM_ERANGE; }
  if (p->n_T < 1 || !p->T) { err = "a temperature grid is required"; return FTLM_EINVAL; }
  for (int i = 0; i < p->n_T; i++)
    if (!(p->T[i] > 0) || !std::isfinite(p->T[i])) { err = "temperatures must be positive"; return FTLM_EINVAL; }
  if (p->precision != FTLM_C128 && p->precision != FTLM_C64) { err = "bad precision"; return FTLM_EINVAL; }
  if (p->r_init) { err = "r_init is not supported by the Chebyshev driver"; return FTLM_EINVAL; }
  if (p->fields) {
    if (p->n_fields < 1) { err = "n_fields must be >= 1"; return FTLM_EINVAL; }
    for (int i = 0; i < 3 * p->n_fields; i++)
      if (!std::isfinite(p->fields[i])) { err = "fields must be finite"; return FTLM_EINVAL; }
  } else if (p->n_fields > 1) {
    err = "n_fields > 1 needs a fields array";
    return FTLM_EINVAL;
  }
  if (h->host.dim > 0xFFFFFFFFull) { err = "dimension too large"; return FTLM_ERANGE; }
  return FTLM_OK;
}

}  // namespace
}  // namespace ftlm

using namespace ftlm;

extern "C" {

int ftlm_run_kpm_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, int32_t n_moments,
                                size_t *bytes) {
  std::string err;
  if (!h || !bytes) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_kpm(h, p, n_moments, err);
  if (rc) { set_error(err); return rc; }
  KPlan pl;
  make_kplan(h, p, n_moments, pl);
  *bytes = pl.total;
  return FTLM_OK;
}

int ftlm_run_kpm(const ftlm_hamiltonian *hc, const ftlm_run_params *p, int32_t n_moments, void *ws,
                 size_t bytes, void *stream_, ftlm_result *out, double *bounds) {
  std::string err;
  if (!hc || !ws || !out) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_kpm(hc, p, n_moments, err);
  if (rc) { set_error(err); return rc; }
  ftlm_hamiltonian *h = const_cast<ftlm_hamiltonian *>(hc);
  KPlan pl;
  make_kplan(h, p, n_moments, pl);
  if (bytes < pl.total) { set_error("workspace too small"); return FTLM_ENOMEM; }
  hipStream_t s = (hipStream_t)stream_;
  const double saved_B[3] = {h->host.B[0], h->host.B[1], h->host.B[2]};
  const double dimd = (double)pl.dim;
  if (hipMemcpyAsync(at3<double>(ws, pl.T), p->T, sizeof(double) * pl.nT, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(at3<double>(ws, pl.dims), &dimd, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("copy of run inputs failed");
    return FTLM_EHIP;
  }
  auto fail = [&](int code, const std::string &m) {
    set_error(m);
    if (p->fields) (void)ftlm_hamiltonian_set_field(h, saved_B);
    return code;
  };
  const size_t vbytes = (size_t)pl.dim * pl.es;
  const uint32_t dim = (uint32_t)pl.dim;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(2048, (pl.dim + kBlock - 1) / kBlock);
  char *B3[3] = {at3<char>(ws, pl.buf[0]), at3<char>(ws, pl.buf[1]), at3<char>(ws, pl.buf[2])};
  char *Wv = at3<char>(ws, pl.W), *T0 = at3<char>(ws, pl.T0), *OV = at3<char>(ws, pl.OV);
  double *part = at3<double>(ws, pl.part);
  unsigned *counter = at3<unsigned>(ws, pl.counter);
  double *ab = at3<double>(ws, pl.ab);
  double *ms = at3<double>(ws, pl.mstage);  // (mu_n, nu_n) pairs of the current vector
  const int S = pl.N + 3;
  auto cheb = [&](int mode, const char *w, const char *x, const char *y, char *o, double *mom) {
    if (pl.prec == FTLM_C64)
      hipLaunchKernelGGL(cheb_kernel<float>, dim3(grid), dim3(kBlock), 0, s, mode, dim,
                         reinterpret_cast<const Cx<float> *>(w), reinterpret_cast<const Cx<float> *>(x),
                         reinterpret_cast<const Cx<float> *>(y), reinterpret_cast<Cx<float> *>(o),
                         reinterpret_cast<const Cx<float> *>(T0), reinterpret_cast<const Cx<float> *>(OV), ab,
                         part, counter, mom);
    else
      hipLaunchKernelGGL(cheb_kernel<double>, dim3(grid), dim3(kBlock), 0, s, mode, dim,
                         reinterpret_cast<const Cx<double> *>(w), reinterpret_cast<const Cx<double> *>(x),
                         reinterpret_cast<const Cx<double> *>(y), reinterpret_cast<Cx<double> *>(o),
                         reinterpret_cast<const Cx<double> *>(T0), reinterpret_cast<const Cx<double> *>(OV), ab,
                         part, counter, mom);
    hipLaunchKernelGGL(cheb_finish, dim3(1), dim3(kBlock), 0, s, part, grid, mom);
    return hipGetLastError() == hipSuccess;
  };
  auto hv = [&](const char *x, char *w) {
    HvLaunch L{};
    L.precision = pl.prec;
    L.K = 1;
    L.v = x;
    L.w = w;
    return launch_hv(h->dev, L, s);
  };
  for (int f = 0; f < pl.nF; f++) {
    if (p->fields) {
      rc = ftlm_hamiltonian_set_field(h, p->fields + 3 * f);
      if (rc) return fail(rc, std::string("set_field: ") + ftlm_last_error());
    }
    // 1. spectral bounds from N_B Lanczos steps on the first random vector
    if (launch_zero_state(at3<double>(ws, pl.smax), at3<int>(ws, pl.done), at3<int>(ws, pl.nused), counter, kCounterWords, 1, s))
      return fail(FTLM_EHIP, "zero_state launch failed");
    rc = launch_gaussian(p->seed, p->instance, (uint32_t)f, 0, 1, dim, pl.prec, B3[0], part, counter,
                         at3<double>(ws, pl.sx), 0, s);
    if (rc) return fail(rc, "start-vector launch failed");
    for (int j = 0; j < pl.NB; j++) {
      EpiLanczos lz{};
      lz.xprev = j > 0 ? B3[(j + 2) % 3] : nullptr;
      lz.sx_cur = at3<double>(ws, pl.sx) + j;
      lz.sx_prev = j > 0 ? at3<double>(ws, pl.sx) + (j - 1) : nullptr;
      lz.beta_prev = j > 0 ? at3<double>(ws, pl.beta) + (j - 1) : nullptr;
      lz.part = part;
      lz.counter = counter;
      lz.alpha_out = at3<double>(ws, pl.alpha) + j;
      lz.yre_out = at3<double>(ws, pl.yre) + j;
      lz.yim_out = at3<double>(ws, pl.yim) + j;
      HvLaunch L{};
      L.precision = pl.prec;
      L.K = 1;
      L.v = B3[j % 3];
      L.w = B3[(j + 1) % 3];
      L.lz = &lz;
      rc = launch_hv(h->dev, L, s);
      if (rc) return fail(rc, "H*v launch failed");
      UpdateArgs u{};
      u.precision = pl.prec;
      u.K = 1;
      u.step = j;
      u.n_lanczos = pl.NB;
      u.dim = dim;
      u.w = L.w;
      u.x = L.v;
      u.sx_cur = lz.sx_cur;
      u.alpha = lz.alpha_out;
      u.beta = at3<double>(ws, pl.beta) + j;
      u.sx_next = at3<double>(ws, pl.sx) + (j + 1);
      u.scale_max = at3<double>(ws, pl.smax);
      u.done = at3<int>(ws, pl.done);
      u.n_used = at3<int>(ws, pl.nused);
      u.part = part;
      u.counter = counter;
      rc = launch_update(u, s);
      if (rc) return fail(rc, "update launch failed");
    }
    rc = launch_tridiag(1, pl.NB, at3<int>(ws, pl.nused), 1, 1, at3<double>(ws, pl.alpha), at3<double>(ws, pl.beta),
                        nullptr, at3<double>(ws, pl.eps), at3<double>(ws, pl.q1), at3<double>(ws, pl.qy), 1, 0,
                        at3<double>(ws, pl.tri), s);
    if (rc) return fail(rc, "tridiagonal launch failed");
    hipLaunchKernelGGL(bounds_kernel, dim3(1), dim3(64), 0, s, at3<double>(ws, pl.eps), at3<int>(ws, pl.nused), ab,
                       at3<double>(ws, pl.lohi) + 2 * f);
    // 2. Chebyshev moments of every random vector
    for (int r = 0; r < pl.R; r++) {
      double *mu = at3<double>(ws, pl.mu) + (size_t)r * S, *nu = at3<double>(ws, pl.nu) + (size_t)r * S;
      rc = launch_gaussian(p->seed, p->instance, (uint32_t)f, (uint32_t)r, 1, dim, pl.prec, T0, part, counter,
                           at3<double>(ws, pl.sx), 0, s);
      if (rc) return fail(rc, "start-vector launch failed");
      if (pl.prec == FTLM_C64)
        hipLaunchKernelGGL(scale_kernel<float>, dim3(grid), dim3(kBlock), 0, s, dim, reinterpret_cast<Cx<float> *>(T0),
                           at3<double>(ws, pl.sx));
      else
        hipLaunchKernelGGL(scale_kernel<double>, dim3(grid), dim3(kBlock), 0, s, dim,
                           reinterpret_cast<Cx<double> *>(T0), at3<double>(ws, pl.sx));
      HvLaunch L{};
      L.precision = pl.prec;
      L.K = 1;
      L.v = T0;
      L.w = OV;
      if (launch_hv(h->mom_dev, L, s)) return fail(FTLM_EHIP, "O r launch failed");
      // moments of t_0 (two entries, one launch)
      if (!cheb(0, nullptr, T0, nullptr, nullptr, ms)) return fail(FTLM_EHIP, "moment launch failed");
      // t_0 = T0, t_1 -> B3[1]; then t_{n+1} into the buffer of t_{n-1}
      if (hv(T0, Wv)) return fail(FTLM_EHIP, "H*v launch failed");
      if (!cheb(1, Wv, T0, nullptr, B3[1], ms + 2)) return fail(FTLM_EHIP, "Chebyshev launch failed");
      const char *tm = T0;
      char *tc = B3[1];
      for (int n = 1; n < pl.N + 2; n++) {
        char *tn = B3[(n + 1) % 3];
        if (tn == tc) tn = B3[(n + 2) % 3];
        if (hv(tc, Wv)) return fail(FTLM_EHIP, "H*v launch failed");
        if (!cheb(2, Wv, tc, tm, tn, ms + 2 * (n + 1))) return fail(FTLM_EHIP, "Chebyshev launch failed");
        tm = tc;
        tc = tn;
      }
      // scatter the (mu_n, nu_n) pairs into mu, nu
      if (hipMemcpy2DAsync(mu, sizeof(double), ms, 2 * sizeof(double), sizeof(double), S,
                           hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipMemcpy2DAsync(nu, sizeof(double), ms + 1, 2 * sizeof(double), sizeof(double), S,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(FTLM_EHIP, "moment copy failed");
    }
    // 3./4. expansion coefficients and thermodynamics
    const size_t ro = (size_t)f * pl.nT;
    hipLaunchKernelGGL(bessel_kernel, dim3((pl.nT + 63) / 64), dim3(64), 0, s, pl.nT, pl.N, at3<double>(ws, pl.T), ab,
                       at3<double>(ws, pl.coef));
    hipLaunchKernelGGL(kpm_thermo_kernel, dim3((pl.nT + 63) / 64), dim3(64), 0, s, pl.nT, pl.R, pl.N,
                       at3<double>(ws, pl.T), ab, at3<double>(ws, pl.lohi) + 2 * f, at3<double>(ws, pl.coef),
                       at3<double>(ws, pl.mu), at3<double>(ws, pl.nu), at3<double>(ws, pl.dims),
                       at3<double>(ws, pl.lnZ) + ro, at3<double>(ws, pl.E) + ro, at3<double>(ws, pl.C) + ro,
                       at3<double>(ws, pl.M) + ro);
    if (hipGetLastError() != hipSuccess) return fail(FTLM_EHIP, "thermodynamics launch failed");
    if (hipMemcpyAsync(at3<double>(ws, pl.emin) + f, at3<double>(ws, pl.lohi) + 2 * f, sizeof(double),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(FTLM_EHIP, "copy failed");
  }
  const size_t res = sizeof(double) * pl.nT * pl.nF;
  struct { double *dst; size_t off; size_t n; } outs[] = {
      {out->lnZ, pl.lnZ, res}, {out->E, pl.E, res}, {out->C, pl.C, res}, {out->M, pl.M, res},
      {out->E_min, pl.emin, sizeof(double) * pl.nF}, {bounds, pl.lohi, sizeof(double) * 2 * pl.nF}};
  for (auto &o : outs)
    if (o.dst && hipMemcpyAsync(o.dst, at3<char>(ws, o.off), o.n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(FTLM_EHIP, "copy of results failed");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FTLM_EHIP, "stream synchronise failed");
  if (out->n_lanczos_used)
    for (int i = 0; i < pl.R * pl.nF; i++) out->n_lanczos_used[i] = pl.N;
  if (p->fields) {
    rc = ftlm_hamiltonian_set_field(h, saved_B);
    if (rc) return rc;
  }
  return FTLM_OK;
}

}  // extern "C"
