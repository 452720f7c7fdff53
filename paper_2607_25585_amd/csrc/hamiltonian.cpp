// Host-side compile of the spin Hamiltonian of Sec. 2.1, Eq. (mce-hamop), into the
// ladder-operator coefficient tables the H*v kernels read.
//
// Pair terms: s_i^T A_ij s_j with A_ij = 2 J_ij 1 + D_ij (1 - 3 e_ij e_ij^T),
// D_ij = C_dip g_i g_j / r_ij^3 (dipolar prefactor with g_i g_j), is rewritten in
// the ladder basis s^x = (s+ + s-)/2, s^y = (s+ - s-)/(2i):
//   sum_{a,b in x,y,z} A_ab s_i^a s_j^b = sum_{mu,nu in +,-,z} c^{mu nu} s_i^mu s_j^nu
// with c^{mu nu} = sum_ab A_ab U_{a mu} U_{b nu}, U_{x+} = U_{x-} = 1/2,
// U_{y+} = -i/2, U_{y-} = +i/2, U_{zz} = 1.
#include <cmath>
#include <complex>
#include <cstring>

#include "ftlm_internal.hpp"

namespace ftlm {

using cd = std::complex<double>;

static Cx<double> to_cx(cd z) { return Cx<double>{z.real(), z.imag()}; }

int compile_hamiltonian(const ftlm_system *sys, HostHam &hh, std::string &err) {
  if (!sys) { err = "system is NULL"; return FTLM_EINVAL; }
  const int n = sys->n_sites;
  if (n < 1 || n > kMaxSites) { err = "n_sites must be in [1, 32]"; return FTLM_ERANGE; }
  if (!sys->two_s || !sys->g || !sys->B) { err = "two_s, g and B are required"; return FTLM_EINVAL; }
  if (sys->d && !sys->e) { err = "anisotropy axes e are required when d is given"; return FTLM_EINVAL; }
  hh = HostHam();
  hh.n = n;
  uint64_t dim = 1;
  bool half = true;
  for (int k = 0; k < n; k++) {
    int t = sys->two_s[k];
    if (t < 1 || t > FTLM_MAX_TWO_S) { err = "two_s[i] must be in [1, 15]"; return FTLM_ERANGE; }
    hh.two_s[k] = t;
    hh.radix[k] = t + 1;
    hh.stride[k] = (uint32_t)dim;
    dim *= (uint64_t)(t + 1);
    if (dim >= (1ull << 32)) { err = "dimension must be below 2^32"; return FTLM_ERANGE; }
    half = half && (t == 1);
    if (!std::isfinite(sys->g[k])) { err = "g must be finite"; return FTLM_EINVAL; }
  }
  hh.dim = dim;
  hh.spin_half = half;
  hh.has_J = sys->J != nullptr;
  hh.has_d = sys->d != nullptr;
  hh.has_pos = sys->pos != nullptr;
  if (hh.has_J) hh.J.assign(sys->J, sys->J + n * n);
  hh.g.assign(sys->g, sys->g + n);
  hh.e.assign(3 * n, 0.0);
  if (hh.has_d) {
    hh.d.assign(sys->d, sys->d + n);
    for (int k = 0; k < n; k++) {
      const double *ek = sys->e + 3 * k;
      double nr = std::sqrt(ek[0] * ek[0] + ek[1] * ek[1] + ek[2] * ek[2]);
      if (!(nr > 0) || !std::isfinite(nr)) {
        if (hh.d[k] != 0.0) { err = "anisotropy axis of zero length"; return FTLM_EINVAL; }
        continue;
      }
      for (int a = 0; a < 3; a++) hh.e[3 * k + a] = ek[a] / nr;
    }
  }
  if (hh.has_pos) hh.pos.assign(sys->pos, sys->pos + 3 * n);
  for (int a = 0; a < 3; a++) {
    if (!std::isfinite(sys->B[a])) { err = "B must be finite"; return FTLM_EINVAL; }
    hh.B[a] = sys->B[a];
  }

  // pairs
  hh.zz.assign(n * n, 0.0);
  hh.czp.assign(n * n, Cx<double>{0, 0});
  hh.czm.assign(n * n, Cx<double>{0, 0});
  const cd I(0.0, 1.0);
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++) {
      double A[3][3] = {{0}};
      double Jij = hh.has_J ? hh.J[i * n + j] : 0.0;
      if (!std::isfinite(Jij)) { err = "J must be finite"; return FTLM_EINVAL; }
      for (int a = 0; a < 3; a++) A[a][a] = 2.0 * Jij;
      if (hh.has_pos) {
        double rv[3];
        for (int a = 0; a < 3; a++) rv[a] = hh.pos[3 * j + a] - hh.pos[3 * i + a];
        double r = std::sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
        if (!(r > 0) || !std::isfinite(r)) { err = "coincident or invalid site positions"; return FTLM_EINVAL; }
        double D = kCDip * hh.g[i] * hh.g[j] / (r * r * r);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) A[a][b] += D * ((a == b ? 1.0 : 0.0) - 3.0 * rv[a] * rv[b] / (r * r));
      }
      bool any = false;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) any = any || (A[a][b] != 0.0);
      if (!any) continue;
      const double xx = A[0][0], xy = A[0][1], xz = A[0][2];
      const double yx = A[1][0], yy = A[1][1], yz = A[1][2];
      const double zx = A[2][0], zy = A[2][1], zzv = A[2][2];
      cd cpp = 0.25 * (xx - yy - I * (xy + yx));
      cd cpm = 0.25 * (xx + yy + I * (xy - yx));
      cd cmp = 0.25 * (xx + yy - I * (xy - yx));
      cd cmm = 0.25 * (xx - yy + I * (xy + yx));
      cd cpz = 0.5 * (xz - I * yz), cmz = 0.5 * (xz + I * yz);
      cd czpl = 0.5 * (zx - I * zy), czmi = 0.5 * (zx + I * zy);
      hh.pi.push_back(i);
      hh.pj.push_back(j);
      hh.pc.push_back(to_cx(cpp));
      hh.pc.push_back(to_cx(cpm));
      hh.pc.push_back(to_cx(cmp));
      hh.pc.push_back(to_cx(cmm));
      hh.pzz.push_back(zzv);
      hh.zz[i * n + j] = hh.zz[j * n + i] = zzv;
      // s_i^+ s_j^z and s_j^+ s_i^z pieces, seen from the flipped site
      hh.czp[i * n + j] = to_cx(cpz);
      hh.czm[i * n + j] = to_cx(cmz);
      hh.czp[j * n + i] = to_cx(czpl);
      hh.czm[j * n + i] = to_cx(czmi);
    }
  hh.npair = (int)hh.pi.size();
  hh.has_z = false;
  for (int k = 0; k < n * n; k++)
    hh.has_z = hh.has_z || hh.czp[k].re != 0 || hh.czp[k].im != 0 || hh.czm[k].re != 0 ||
               hh.czm[k].im != 0;
  compile_site_terms(hh);
  hh.nnz_per_row = count_nnz_per_row(hh);
  return FTLM_OK;
}

// h_k = d_k (s.e_k)^2 + mu_B g_k B.s  (Sec. 2.1) on the ladder basis
// s.e = (e_x - i e_y)/2 s+ + (e_x + i e_y)/2 s- + e_z s^z.
void compile_site_terms(HostHam &hh) {
  const int n = hh.n;
  hh.h.assign((size_t)n * 256, Cx<double>{0, 0});
  const cd I(0.0, 1.0);
  for (int k = 0; k < n; k++) {
    const int r = hh.radix[k];
    const double s = 0.5 * hh.two_s[k];
    cd sp[16][16] = {}, sm[16][16] = {}, sz[16][16] = {};
    for (int b = 0; b < r; b++) {
      double m = b - s;
      sz[b][b] = m;
      if (b + 1 < r) {
        double f = std::sqrt(s * (s + 1) - m * (m + 1));  // <m+1|s+|m>
        sp[b + 1][b] = f;
        sm[b][b + 1] = f;
      }
    }
    auto project = [&](const double *v, cd out[16][16]) {
      cd cp = 0.5 * (v[0] - I * v[1]), cm = 0.5 * (v[0] + I * v[1]);
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) out[a][b] = cp * sp[a][b] + cm * sm[a][b] + v[2] * sz[a][b];
    };
    cd hk[16][16] = {};
    if (hh.has_d && hh.d[k] != 0.0) {
      cd se[16][16];
      project(&hh.e[3 * k], se);
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) {
          cd acc = 0;
          for (int c = 0; c < r; c++) acc += se[a][c] * se[c][b];
          hk[a][b] += hh.d[k] * acc;
        }
    }
    cd sb[16][16];
    project(hh.B, sb);
    for (int a = 0; a < r; a++)
      for (int b = 0; b < r; b++) hk[a][b] += kMuB * hh.g[k] * sb[a][b];
    for (int a = 0; a < r; a++)
      for (int b = 0; b < r; b++) hh.h[(size_t)k * 256 + a * 16 + b] = to_cx(hk[a][b]);
  }
}

static bool nz(Cx<double> c) { return c.re != 0.0 || c.im != 0.0; }

double count_nnz_per_row(const HostHam &hh) {
  double total = 1.0;  // diagonal
  const int n = hh.n;
  for (int k = 0; k < n; k++) {
    const int r = hh.radix[k];
    bool zflip = false;
    for (int l = 0; l < n; l++) zflip = zflip || nz(hh.czp[k * n + l]) || nz(hh.czm[k * n + l]);
    for (int D : {-2, -1, 1, 2}) {
      int cnt = 0;
      for (int dk = 0; dk < r; dk++) {
        int nd = dk + D;
        if (nd < 0 || nd >= r) continue;
        bool val = nz(hh.h[(size_t)k * 256 + dk * 16 + nd]) || ((D == 1 || D == -1) && zflip);
        cnt += val;
      }
      total += (double)cnt / r;
    }
  }
  for (int p = 0; p < hh.npair; p++) {
    const int ri = hh.radix[hh.pi[p]], rj = hh.radix[hh.pj[p]];
    for (int q = 0; q < 4; q++)
      if (nz(hh.pc[4 * p + q])) total += (double)(ri - 1) / ri * (double)(rj - 1) / rj;
  }
  return total;
}

}  // namespace ftlm
