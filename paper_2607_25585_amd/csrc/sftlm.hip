// Symmetric FTLM (sFTLM) with pairs of mutually time-reversed random vectors,
// Sec. 2.2, Eqs. (E-2-G), (E-2-H).
//
// For each random vector r (the R vectors are R/2 Gaussian vectors and their
// time reverses) the host code runs N_L Lanczos steps keeping every Krylov vector
// (slot j of the workspace holds the unnormalised X_j with scale sx_j), applies
// O = -sum_i g_i s_i.B_hat to every slot, forms O_K = V^H O V (Gram kernel),
// and diagonalises the tridiagonal with the full eigenvector matrix Q.  The
// Boltzmann kernel then evaluates, per temperature,
//   den_r = sum_n exp(-(eps_n - E_min)/T) Q_1n^2                      (Eq. E-2-D)
//   num_r = z^T Re(O_K) z,  z_a = sum_n Q_an exp(-(eps_n - E_min)/2T) Q_1n
// (the double sum of Eq. E-2-H written as a quadratic form), and
//   M = sum_r num_r / sum_r den_r.
// ln Z, E and C come from the Ritz values exactly as in the plain driver.
//
// Time reversal in the product basis (Condon-Shortley phases, site 0 fastest):
//   (Theta x)[dim-1-nu] = (-1)^{sum_i (2 s_i - d_i(nu))} conj(x[nu]).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ftlm_internal.hpp"

namespace ftlm {

namespace {

struct ThetaGeom {
  int n;
  uint32_t dim;
  int radix[kMaxSites];
  int two_s_sum_parity;
};

template <typename R>
__global__ __launch_bounds__(256) void theta_kernel(ThetaGeom g, const Cx<R> *__restrict__ src,
                                                    Cx<R> *__restrict__ dst) {
  for (uint64_t nu = (uint64_t)blockIdx.x * 256 + threadIdx.x; nu < g.dim; nu += (uint64_t)gridDim.x * 256) {
    uint32_t rem = (uint32_t)nu, dsum = 0;
    for (int k = 0; k < g.n; k++) {
      const uint32_t r = (uint32_t)g.radix[k], q = rem / r;
      dsum += rem - q * r;
      rem = q;
    }
    const bool neg = ((uint32_t)g.two_s_sum_parity + dsum) & 1u;  // parity of sum(2 s_i - d_i)
    const Cx<R> x = src[nu];
    dst[g.dim - 1 - nu] = neg ? Cx<R>{-x.re, x.im} : Cx<R>{x.re, -x.im};
  }
}

// Partial Gram sums: part[split][a][b] = sx_a sum_{nu in split} conj(X_a[nu]) W_b[nu]
// for a 16 x 16 tile of (a, b) per block.  X slots at X + a*xstride, W at W + b*xstride.
constexpr int kGT = 16, kGC = 32;

template <typename R>
__global__ __launch_bounds__(256) void gram_kernel(const Cx<R> *__restrict__ X, const Cx<R> *__restrict__ Wv,
                                                   size_t xstride, int nl, uint32_t dim, uint32_t chunk,
                                                   const double *__restrict__ sx, double2 *__restrict__ part) {
  __shared__ Cx<R> xs[kGT][kGC + 1];
  __shared__ Cx<R> wsh[kGT][kGC + 1];
  const int t = threadIdx.x, ta = t / kGT, tb = t % kGT;
  const int a0 = blockIdx.x * kGT, b0 = blockIdx.y * kGT;
  // 64-bit bounds: lo + chunk and r0 + kGC may pass 2^32 when dim is near it
  const uint64_t lo = (uint64_t)blockIdx.z * chunk, hi = min((uint64_t)dim, lo + chunk);
  double ar = 0, ai = 0;
  for (uint64_t r0 = lo; r0 < hi; r0 += kGC) {
    __syncthreads();
    for (int idx = t; idx < kGT * kGC; idx += 256) {
      const int q = idx / kGC, k = idx % kGC;
      const uint64_t row = r0 + k;
      const bool ok = row < hi;
      xs[q][k] = (ok && a0 + q < nl) ? X[(size_t)(a0 + q) * xstride + row] : Cx<R>{0, 0};
      wsh[q][k] = (ok && b0 + q < nl) ? Wv[(size_t)(b0 + q) * xstride + row] : Cx<R>{0, 0};
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kGC; k++) {
      const Cx<R> x = xs[ta][k], w = wsh[tb][k];
      ar = fma((double)x.re, (double)w.re, fma((double)x.im, (double)w.im, ar));
      ai = fma((double)x.re, (double)w.im, fma(-(double)x.im, (double)w.re, ai));
    }
  }
  const int a = a0 + ta, b = b0 + tb;
  if (a < nl && b < nl) {
    const double s = sx[a];
    part[((size_t)blockIdx.z * nl + a) * nl + b] = make_double2(ar * s, ai * s);
  }
}

// Sums the partials over the splits in split order.
__global__ void gram_reduce_kernel(const double2 *__restrict__ part, int nsplit, int nl, double2 *__restrict__ ok) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nl * nl) return;
  double r = 0, i = 0;
  for (int s = 0; s < nsplit; s++) {
    const double2 v = part[(size_t)s * nl * nl + idx];
    r += v.x;
    i += v.y;
  }
  ok[idx] = make_double2(r, i);
}

// Implicit QL with shifts (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math.
// 11 (1968)) on T = tridiag(alpha[0..n), beta[0..n-1)), one block per column;
// thread 0 runs each sweep's scalar recurrence and records its plane rotations,
// then every thread applies them to its rows of the full eigenvector matrix Z
// (LDS, column-major Z[i][a]).  Output: eps[n], Q[a][m] = Z (row-major, nl x nl),
// zero beyond n.
__global__ void tridiag_full_kernel(int nl, const int *__restrict__ n_used, const double *__restrict__ alpha,
                                    const double *__restrict__ beta, double *__restrict__ eps,
                                    double *__restrict__ Qout) {
  extern __shared__ double sh[];
  double *d = sh, *e = d + nl, *rc = e + nl, *rs = rc + nl, *Z = rs + nl;  // Z: [nl][nl]
  __shared__ int s_lo, s_hi, s_done;
  const int t = threadIdx.x;
  const int n = n_used ? *n_used : nl;
  for (int i = t; i < nl; i += blockDim.x) {
    d[i] = i < n ? alpha[i] : 0.0;
    e[i] = (i + 1 < n) ? beta[i] : 0.0;
  }
  for (int idx = t; idx < nl * nl; idx += blockDim.x) Z[idx] = (idx / nl == idx % nl) ? 1.0 : 0.0;
  __syncthreads();
  for (int l = 0; l < n; l++) {
    int iter = 0;
    while (true) {
      if (t == 0) {
        s_done = 0;
        int m = l;
        for (; m < n - 1; m++) {
          const double dd = fabs(d[m]) + fabs(d[m + 1]);
          if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;
        }
        if (m == l || iter >= 100) {
          s_done = 1;
        } else {
          double gg = (d[l + 1] - d[l]) / (2.0 * e[l]);
          double r = hypot(gg, 1.0);
          gg = d[m] - d[l] + e[l] / (gg + copysign(r, gg));
          double s = 1.0, c = 1.0, p = 0.0;
          int i = m - 1;
          bool underflow = false;
          for (; i >= l; i--) {
            const double f = s * e[i], b = c * e[i];
            r = hypot(f, gg);
            e[i + 1] = r;
            if (r == 0.0) {
              d[i + 1] -= p;
              e[m] = 0.0;
              underflow = true;
              break;
            }
            s = f / r;
            c = gg / r;
            gg = d[i + 1] - p;
            r = (d[i] - gg) * s + 2.0 * c * b;
            p = s * r;
            d[i + 1] = gg + p;
            gg = c * r - b;
            rc[i] = c;
            rs[i] = s;
          }
          s_hi = m - 1;
          s_lo = underflow ? i + 1 : l;
          if (!underflow) {
            d[l] -= p;
            e[l] = gg;
            e[m] = 0.0;
          }
        }
      }
      __syncthreads();
      if (s_done) break;
      iter++;
      const int lo = s_lo, hi = s_hi;
      for (int a = t; a < nl; a += blockDim.x)
        for (int i = hi; i >= lo; i--) {
          const double c = rc[i], s = rs[i];
          const double fz = Z[(i + 1) * nl + a];
          Z[(i + 1) * nl + a] = s * Z[i * nl + a] + c * fz;
          Z[i * nl + a] = c * Z[i * nl + a] - s * fz;
        }
      __syncthreads();
    }
    __syncthreads();
  }
  for (int i = t; i < nl; i += blockDim.x) eps[i] = i < n ? d[i] : 0.0;
  for (int idx = t; idx < nl * nl; idx += blockDim.x) {
    const int a = idx / nl, m = idx % nl;  // Q[a][m] = Z column m, row a
    Qout[idx] = (a < n && m < n) ? Z[m * nl + a] : 0.0;
  }
}

// One block per temperature: ln Z, E, C and the symmetric M over the R vectors
// of one field.  eps [R][nl], Q [R][nl][nl], OK [R][nl][nl] (complex), n_used [R].
__global__ __launch_bounds__(256) void sftlm_boltzmann_kernel(int R, int nl, const int *__restrict__ n_used,
                                                              const double *__restrict__ eps,
                                                              const double *__restrict__ Q,
                                                              const double2 *__restrict__ OK,
                                                              const double *__restrict__ dims,
                                                              const double *__restrict__ T, double *lnZ,
                                                              double *E, double *C, double *M,
                                                              double *E_min) {
  extern __shared__ double sh[];
  double *h = sh, *z = h + nl;
  __shared__ double red[256 / 64];
  const int t = threadIdx.x;
  const double temp = T[blockIdx.x];
  auto block_sum = [&](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < 4; w++) s += red[w];
    __syncthreads();
    return s;
  };
  double emin = 1e300;  // lowest Ritz value over all vectors (the QL output is unsorted)
  for (int r = 0; r < R; r++)
    for (int m = 0; m < n_used[r]; m++) emin = fmin(emin, eps[(size_t)r * nl + m]);
  // pass 1: den and the first moment
  double den = 0, e1 = 0;
  for (int r = 0; r < R; r++) {
    const int n = n_used[r];
    for (int m = t; m < n; m += 256) {
      const double q = Q[((size_t)r * nl) * nl + m];  // Q[r][0][m]
      const double ev = eps[(size_t)r * nl + m];
      const double w = exp(-(ev - emin) / temp) * q * q;
      den += w;
      e1 += w * ev;
    }
  }
  den = block_sum(den);
  e1 = block_sum(e1);
  const double em = e1 / den;
  double e2 = 0, num = 0;
  for (int r = 0; r < R; r++) {
    const int n = n_used[r];
    const double *Qr = Q + (size_t)r * nl * nl;
    const double2 *Or = OK + (size_t)r * nl * nl;
    for (int m = t; m < nl; m += 256) {
      double hm = 0;
      if (m < n) {
        const double ev = eps[(size_t)r * nl + m];
        const double q = Qr[m];
        hm = exp(-(ev - emin) / (2.0 * temp)) * q;
        e2 += exp(-(ev - emin) / temp) * q * q * (ev - em) * (ev - em);
      }
      h[m] = hm;
    }
    __syncthreads();
    for (int a = t; a < nl; a += 256) {
      double s = 0;
      for (int m = 0; m < n; m++) s = fma(Qr[(size_t)a * nl + m], h[m], s);
      z[a] = s;
    }
    __syncthreads();
    for (int a = t; a < n; a += 256) {
      double s = 0;
      for (int b = 0; b < n; b++) s = fma(Or[(size_t)a * nl + b].x, z[b], s);
      num = fma(z[a], s, num);
    }
    __syncthreads();
  }
  e2 = block_sum(e2);
  num = block_sum(num);
  if (t == 0) {
    const int k = blockIdx.x;
    lnZ[k] = log(dims[0] / R) - emin / temp + log(den);
    E[k] = em;
    C[k] = e2 / den / (temp * temp);
    M[k] = num / den;
    if (k == 0 && E_min) *E_min = emin;
  }
}

struct SPlan {
  int R = 0, NL = 0, nT = 0, nF = 0, prec = 0, nsplit = 0;
  size_t es = 16;
  uint64_t dim = 0;
  size_t V, W, alpha, beta, yre, yim, sx, smax, done, nused, part, counter;
  size_t gpart, eps, Q, OK, nused_all, T, dims, lnZ, E, C, M, emin;
  size_t total = 0;
};

struct Carve2 {
  size_t off = 0;
  size_t take(size_t n) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return o;
  }
};

void make_splan(const ftlm_hamiltonian *h, const ftlm_run_params *p, SPlan &pl) {
  pl.R = p->R;
  pl.NL = p->n_lanczos;
  pl.nT = p->n_T;
  pl.nF = p->fields ? p->n_fields : 1;
  pl.prec = p->precision;
  pl.es = p->precision == FTLM_C64 ? 8 : 16;
  pl.dim = h->host.dim;
  const uint64_t chunk = 4096;
  pl.nsplit = (int)std::min<uint64_t>(1024, (pl.dim + chunk - 1) / chunk);
  Carve2 c;
  const size_t vec = (size_t)pl.dim * pl.es;
  pl.V = c.take(vec * (pl.NL + 1));
  pl.W = c.take(vec * pl.NL);
  const size_t sd = sizeof(double);
  pl.alpha = c.take(sd * pl.NL);
  pl.beta = c.take(sd * pl.NL);
  pl.yre = c.take(sd * pl.NL);
  pl.yim = c.take(sd * pl.NL);
  pl.sx = c.take(sd * (pl.NL + 1));
  pl.smax = c.take(sd);
  pl.done = c.take(sizeof(int));
  pl.nused = c.take(sizeof(int));
  pl.part = c.take(sd * 2048 * 3);
  pl.counter = c.take(sizeof(unsigned) * kCounterWords);
  pl.gpart = c.take(sizeof(double2) * (size_t)pl.nsplit * pl.NL * pl.NL);
  pl.eps = c.take(sd * (size_t)pl.R * pl.NL);
  pl.Q = c.take(sd * (size_t)pl.R * pl.NL * pl.NL);
  pl.OK = c.take(sizeof(double2) * (size_t)pl.R * pl.NL * pl.NL);
  pl.nused_all = c.take(sizeof(int) * (size_t)pl.R * pl.nF);
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
T *at2(void *ws, size_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off);
}

size_t tridiag_full_smem(int nl) { return sizeof(double) * ((size_t)4 * nl + (size_t)nl * nl); }

int validate_sftlm(const ftlm_hamiltonian *h, const ftlm_run_params *p, std::string &err) {
  if (!p) { err = "params is NULL"; return FTLM_EINVAL; }
  if (p->R < 2 || (p->R & 1)) { err = "R must be even and >= 2 (time-reversed pairs)"; return FTLM_EINVAL; }
  if (p->n_lanczos < 1) { err = "n_lanczos must be >= 1"; return FTLM_ERANGE; }
  if (tridiag_full_smem(p->n_lanczos) > 160 * 1024) { err = "n_lanczos too large for the sFTLM eigensolver (<= 140)"; return FTLM_ERANGE; }
  if (p->n_T < 1 || !p->T) { err = "a temperature grid is required"; return FTLM_EINVAL; }
  for (int i = 0; i < p->n_T; i++)
    if (!(p->T[i] > 0) || !std::isfinite(p->T[i])) { err = "temperatures must be positive"; return FTLM_EINVAL; }
  if (p->precision != FTLM_C128 && p->precision != FTLM_C64) { err = "bad precision"; return FTLM_EINVAL; }
  if (p->r_init) { err = "r_init is not supported by the sFTLM driver"; return FTLM_EINVAL; }
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

int ftlm_run_sftlm_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, size_t *bytes) {
  std::string err;
  if (!h || !bytes) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_sftlm(h, p, err);
  if (rc) { set_error(err); return rc; }
  SPlan pl;
  make_splan(h, p, pl);
  *bytes = pl.total;
  return FTLM_OK;
}

int ftlm_run_sftlm(const ftlm_hamiltonian *hc, const ftlm_run_params *p, void *ws, size_t bytes,
                   void *stream_, ftlm_result *out) {
  std::string err;
  if (!hc || !ws || !out) { set_error("NULL argument"); return FTLM_EINVAL; }
  int rc = validate_sftlm(hc, p, err);
  if (rc) { set_error(err); return rc; }
  ftlm_hamiltonian *h = const_cast<ftlm_hamiltonian *>(hc);
  SPlan pl;
  make_splan(h, p, pl);
  if (bytes < pl.total) { set_error("workspace too small"); return FTLM_ENOMEM; }
  hipStream_t s = (hipStream_t)stream_;
  const double saved_B[3] = {h->host.B[0], h->host.B[1], h->host.B[2]};
  const double dimd = (double)pl.dim;
  if (hipMemcpyAsync(at2<double>(ws, pl.T), p->T, sizeof(double) * pl.nT, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(at2<double>(ws, pl.dims), &dimd, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("copy of run inputs failed");
    return FTLM_EHIP;
  }
  auto fail = [&](int code, const std::string &m) {
    set_error(m);
    if (p->fields) (void)ftlm_hamiltonian_set_field(h, saved_B);
    return code;
  };
  ThetaGeom tg{};
  tg.n = h->host.n;
  tg.dim = (uint32_t)pl.dim;
  int ts = 0;
  for (int k = 0; k < tg.n; k++) {
    tg.radix[k] = h->host.radix[k];
    ts += h->host.two_s[k];
  }
  tg.two_s_sum_parity = ts & 1;
  const size_t vbytes = (size_t)pl.dim * pl.es;
  char *V = at2<char>(ws, pl.V), *Wb = at2<char>(ws, pl.W);
  const int NL = pl.NL;
  const size_t tsm = tridiag_full_smem(NL);
  {
    static size_t granted = 0;
    if (tsm > granted) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&tridiag_full_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)tsm);
      granted = tsm;
    }
  }
  const uint32_t tgrid = (uint32_t)std::min<uint64_t>(4096, (pl.dim + 255) / 256);
  for (int f = 0; f < pl.nF; f++) {
    if (p->fields) {
      rc = ftlm_hamiltonian_set_field(h, p->fields + 3 * f);
      if (rc) return fail(rc, std::string("set_field: ") + ftlm_last_error());
    }
    for (int r = 0; r < pl.R; r++) {
      const int pair = r >> 1, rev = r & 1;
      if (launch_zero_state(at2<double>(ws, pl.smax), at2<int>(ws, pl.done), at2<int>(ws, pl.nused),
                            at2<unsigned>(ws, pl.counter), kCounterWords, 1, s))
        return fail(FTLM_EHIP, "zero_state launch failed");
      // start vector: Gaussian (pair index as the vector index) or its time reverse
      char *dst0 = rev ? V + vbytes : V;
      rc = launch_gaussian(p->seed, p->instance, (uint32_t)f, (uint32_t)pair, 1, (uint32_t)pl.dim, pl.prec,
                           dst0, at2<double>(ws, pl.part), at2<unsigned>(ws, pl.counter),
                           at2<double>(ws, pl.sx), 0, s);
      if (rc) return fail(rc, "start-vector launch failed");
      if (rev) {
        if (pl.prec == FTLM_C64)
          hipLaunchKernelGGL(theta_kernel<float>, dim3(tgrid), dim3(256), 0, s, tg,
                             reinterpret_cast<const Cx<float> *>(V + vbytes), reinterpret_cast<Cx<float> *>(V));
        else
          hipLaunchKernelGGL(theta_kernel<double>, dim3(tgrid), dim3(256), 0, s, tg,
                             reinterpret_cast<const Cx<double> *>(V + vbytes), reinterpret_cast<Cx<double> *>(V));
        if (hipGetLastError() != hipSuccess) return fail(FTLM_EHIP, "theta launch failed");
      }
      // Lanczos: X_j in slot j, u_j written into slot j+1
      for (int j = 0; j < NL; j++) {
        EpiLanczos lz{};
        lz.xprev = j > 0 ? V + (size_t)(j - 1) * vbytes : nullptr;
        lz.ov1 = nullptr;
        lz.sx_cur = at2<double>(ws, pl.sx) + j;
        lz.sx_prev = j > 0 ? at2<double>(ws, pl.sx) + (j - 1) : nullptr;
        lz.beta_prev = j > 0 ? at2<double>(ws, pl.beta) + (j - 1) : nullptr;
        lz.part = at2<double>(ws, pl.part);
        lz.counter = at2<unsigned>(ws, pl.counter);
        lz.alpha_out = at2<double>(ws, pl.alpha) + j;
        lz.yre_out = at2<double>(ws, pl.yre) + j;
        lz.yim_out = at2<double>(ws, pl.yim) + j;
        HvLaunch L{};
        L.precision = pl.prec;
        L.K = 1;
        L.v = V + (size_t)j * vbytes;
        L.w = V + (size_t)(j + 1) * vbytes;
        L.lz = &lz;
        rc = launch_hv(h->dev, L, s);
        if (rc) return fail(rc, "H*v launch failed");
        UpdateArgs u{};
        u.precision = pl.prec;
        u.K = 1;
        u.step = j;
        u.n_lanczos = NL;
        u.dim = (uint32_t)pl.dim;
        u.w = L.w;
        u.x = L.v;
        u.sx_cur = lz.sx_cur;
        u.alpha = lz.alpha_out;
        u.beta = at2<double>(ws, pl.beta) + j;
        u.sx_next = at2<double>(ws, pl.sx) + (j + 1);
        u.scale_max = at2<double>(ws, pl.smax);
        u.done = at2<int>(ws, pl.done);
        u.n_used = at2<int>(ws, pl.nused);
        u.part = at2<double>(ws, pl.part);
        u.counter = at2<unsigned>(ws, pl.counter);
        rc = launch_update(u, s);
        if (rc) return fail(rc, "update launch failed");
      }
      // W_b = O (sx_b X_b)
      for (int b = 0; b < NL; b++) {
        HvLaunch L{};
        L.precision = pl.prec;
        L.K = 1;
        L.v = V + (size_t)b * vbytes;
        L.w = Wb + (size_t)b * vbytes;
        L.scale = at2<double>(ws, pl.sx) + b;
        if (launch_hv(h->mom_dev, L, s)) return fail(FTLM_EHIP, "O V launch failed");
      }
      // O_K = V^H W
      const uint32_t chunk = (uint32_t)((pl.dim + pl.nsplit - 1) / pl.nsplit);
      const dim3 gg((NL + kGT - 1) / kGT, (NL + kGT - 1) / kGT, pl.nsplit);
      double2 *gpart = at2<double2>(ws, pl.gpart);
      if (pl.prec == FTLM_C64)
        hipLaunchKernelGGL(gram_kernel<float>, gg, dim3(256), 0, s, reinterpret_cast<const Cx<float> *>(V),
                           reinterpret_cast<const Cx<float> *>(Wb), (size_t)pl.dim, NL, (uint32_t)pl.dim, chunk,
                           at2<double>(ws, pl.sx), gpart);
      else
        hipLaunchKernelGGL(gram_kernel<double>, gg, dim3(256), 0, s, reinterpret_cast<const Cx<double> *>(V),
                           reinterpret_cast<const Cx<double> *>(Wb), (size_t)pl.dim, NL, (uint32_t)pl.dim, chunk,
                           at2<double>(ws, pl.sx), gpart);
      double2 *okr = at2<double2>(ws, pl.OK) + (size_t)r * NL * NL;
      hipLaunchKernelGGL(gram_reduce_kernel, dim3((NL * NL + 255) / 256), dim3(256), 0, s, gpart, pl.nsplit, NL, okr);
      // full eigenpairs of the tridiagonal
      hipLaunchKernelGGL(tridiag_full_kernel, dim3(1), dim3(std::min(256, ((NL + 63) / 64) * 64)), tsm, s, NL,
                         at2<int>(ws, pl.nused), at2<double>(ws, pl.alpha), at2<double>(ws, pl.beta),
                         at2<double>(ws, pl.eps) + (size_t)r * NL, at2<double>(ws, pl.Q) + (size_t)r * NL * NL);
      if (hipGetLastError() != hipSuccess) return fail(FTLM_EHIP, "sFTLM kernel launch failed");
      if (hipMemcpyAsync(at2<int>(ws, pl.nused_all) + (size_t)f * pl.R + r, at2<int>(ws, pl.nused), sizeof(int),
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(FTLM_EHIP, "copy of n_used failed");
    }
    const size_t ro = (size_t)f * pl.nT;
    const size_t bsm = sizeof(double) * 2 * (size_t)NL;
    hipLaunchKernelGGL(sftlm_boltzmann_kernel, dim3(pl.nT), dim3(256), bsm, s, pl.R, NL,
                       at2<int>(ws, pl.nused_all) + (size_t)f * pl.R, at2<double>(ws, pl.eps),
                       at2<double>(ws, pl.Q), at2<double2>(ws, pl.OK), at2<double>(ws, pl.dims),
                       at2<double>(ws, pl.T), at2<double>(ws, pl.lnZ) + ro, at2<double>(ws, pl.E) + ro,
                       at2<double>(ws, pl.C) + ro, at2<double>(ws, pl.M) + ro, at2<double>(ws, pl.emin) + f);
    if (hipGetLastError() != hipSuccess) return fail(FTLM_EHIP, "sFTLM Boltzmann launch failed");
  }
  const size_t res = sizeof(double) * pl.nT * pl.nF;
  struct { double *dst; size_t off; size_t n; } outs[] = {
      {out->lnZ, pl.lnZ, res}, {out->E, pl.E, res}, {out->C, pl.C, res}, {out->M, pl.M, res},
      {out->E_min, pl.emin, sizeof(double) * pl.nF}};
  for (auto &o : outs)
    if (o.dst && hipMemcpyAsync(o.dst, at2<char>(ws, o.off), o.n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(FTLM_EHIP, "copy of results failed");
  if (out->n_lanczos_used &&
      hipMemcpyAsync(out->n_lanczos_used, at2<int>(ws, pl.nused_all), sizeof(int) * pl.R * pl.nF,
                     hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(FTLM_EHIP, "copy of n_used failed");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FTLM_EHIP, "stream synchronise failed");
  if (p->fields) {
    rc = ftlm_hamiltonian_set_field(h, saved_B);
    if (rc) return rc;
  }
  return FTLM_OK;
}

}  // extern "C"
