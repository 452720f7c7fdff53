/*
 * ftlm_oracle.c -- plain FP64 CPU oracle for the finite-temperature Lanczos
 * method (FTLM).  TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * What it computes, and where the paper defines it:
 *   - The Hamiltonian of Sec. 2.1, Eq. (mce-hamop), written as a sum of one-site
 *     matrices h_i and two-site matrices P_ij.  Both are formed from textbook
 *     Cartesian spin matrices (s^x, s^y, s^z), never from ladder-operator
 *     coefficients:  h_i = d_i (s_i.e_i)^2 + mu_B g_i B.s_i  and
 *     P_ij = sum_{a,b} A_ij^{ab} s_i^a (x) s_j^b  with
 *     A_ij = 2 J_ij 1 + D_ij (1 - 3 e_ij e_ij^T),  D_ij = C_dip g_i g_j / r_ij^3.
 *   - H*v on the product basis (dimension prod_i (2 s_i + 1), Sec. 2.1) by the
 *     definition: w[nu] = sum_mu <nu|H|mu> v[mu], with every matrix element read
 *     from h_i or P_ij.  Site 0 is the fastest basis digit (a reading).
 *   - Gaussian random vectors, Eqs. (E-1-1), (E-1-2): complex components with
 *     independent N(0,1) real and imaginary parts.  Random bits come from
 *     Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed, with
 *     counter (nu, r, field, instance); Box-Muller turns them into Gaussians.
 *   - The Lanczos recursion of Sec. 2.3 (two predecessor vectors; full
 *     re-orthogonalisation optional), in Paige's order, plus the overlaps
 *     y_j = <O v_1 | v_j> that the asymmetric estimator Eq. (E-2-C) needs for M.
 *
 * Parity status: H*v pinned (closed forms, dense Kronecker construction);
 * Philox pinned to the published known-answer vectors; Lanczos pinned by the
 * moment identity and the invariant-subspace case.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORACLE_MU_B 0.67171381563   /* mu_B / k_B, K/T (CODATA 2018) */
#define ORACLE_C_DIP 6.2294807e-4   /* mu0 mu_B^2 / (4 pi k_B), K nm^3 (CODATA 2018) */
#define ORACLE_MAX_SITES 64

typedef struct {
  int n;          /* number of sites */
  int ns[ORACLE_MAX_SITES];       /* local dimension 2 s_i + 1 */
  int64_t st[ORACLE_MAX_SITES];   /* stride of site i in the basis index */
  int64_t dim;
  cplx *h[ORACLE_MAX_SITES];      /* h[i][a*n_i + b] = <a|h_i|b> */
  int npair;
  int *pi, *pj;                   /* pair sites, i < j */
  cplx **P;                       /* P[p][(ai + ni*aj)*(ni*nj) + (bi + ni*bj)] */
} oracle_ham;

/* ---- textbook spin matrices, basis |m>, m = -s..s ascending (digit d = m+s) ---- */
static void spin_cartesian(int two_s, cplx *sx, cplx *sy, cplx *sz) {
  int n = two_s + 1;
  double s = 0.5 * two_s;
  cplx *splus = calloc((size_t)n * n, sizeof(cplx));
  for (int k = 0; k < n - 1; k++) {
    double m = -s + k;
    splus[(k + 1) * n + k] = sqrt(s * (s + 1) - m * (m + 1)); /* <m+1|s+|m> */
  }
  for (int a = 0; a < n; a++)
    for (int b = 0; b < n; b++) {
      cplx up = splus[a * n + b];
      cplx dn = conj(splus[b * n + a]); /* s- = (s+)^dagger */
      sx[a * n + b] = 0.5 * (up + dn);
      sy[a * n + b] = (up - dn) / (2.0 * I);
      sz[a * n + b] = (a == b) ? (-s + a) : 0.0;
    }
  free(splus);
}

void oracle_spin_matrices(int two_s, double *sx_ri, double *sy_ri, double *sz_ri) {
  int n = two_s + 1;
  cplx *m[3];
  for (int a = 0; a < 3; a++) m[a] = malloc((size_t)n * n * sizeof(cplx));
  spin_cartesian(two_s, m[0], m[1], m[2]);
  double *out[3] = {sx_ri, sy_ri, sz_ri};
  for (int a = 0; a < 3; a++) {
    for (int k = 0; k < n * n; k++) {
      out[a][2 * k] = creal(m[a][k]);
      out[a][2 * k + 1] = cimag(m[a][k]);
    }
    free(m[a]);
  }
}

static void ham_init_basis(oracle_ham *H, int n, const int *two_s) {
  memset(H, 0, sizeof(*H));
  H->n = n;
  int64_t st = 1;
  for (int i = 0; i < n; i++) {
    H->ns[i] = two_s[i] + 1;
    H->st[i] = st;
    st *= H->ns[i];
  }
  H->dim = st;
}

/* Builds the Hamiltonian of Eq. (mce-hamop).  J: [n*n] (J[i*n+j], i<j) or NULL;
 * d: [n] or NULL; e: [n*3]; g: [n]; B: [3]; pos: [n*3] or NULL. */
oracle_ham *oracle_build(int n, const int *two_s, const double *J, const double *d,
                         const double *e, const double *g, const double *B,
                         const double *pos) {
  if (n < 1 || n > ORACLE_MAX_SITES) return NULL;
  oracle_ham *H = malloc(sizeof(oracle_ham));
  ham_init_basis(H, n, two_s);
  cplx *S[ORACLE_MAX_SITES][3];
  for (int i = 0; i < n; i++) {
    int ni = H->ns[i];
    for (int a = 0; a < 3; a++) S[i][a] = malloc((size_t)ni * ni * sizeof(cplx));
    spin_cartesian(two_s[i], S[i][0], S[i][1], S[i][2]);
  }
  /* one-site terms */
  for (int i = 0; i < n; i++) {
    int ni = H->ns[i];
    cplx *h = calloc((size_t)ni * ni, sizeof(cplx));
    cplx *se = calloc((size_t)ni * ni, sizeof(cplx));
    if (d) {
      double en = sqrt(e[3 * i] * e[3 * i] + e[3 * i + 1] * e[3 * i + 1] + e[3 * i + 2] * e[3 * i + 2]);
      for (int k = 0; k < ni * ni; k++)
        for (int a = 0; a < 3; a++) se[k] += (e[3 * i + a] / en) * S[i][a][k];
      for (int r = 0; r < ni; r++)
        for (int c = 0; c < ni; c++) {
          cplx acc = 0;
          for (int k = 0; k < ni; k++) acc += se[r * ni + k] * se[k * ni + c];
          h[r * ni + c] += d[i] * acc;
        }
    }
    for (int k = 0; k < ni * ni; k++)
      for (int a = 0; a < 3; a++) h[k] += ORACLE_MU_B * g[i] * B[a] * S[i][a][k];
    H->h[i] = h;
    free(se);
  }
  /* two-site terms: A_ij (3x3) then P_ij = sum_ab A^{ab} s_i^a (x) s_j^b */
  int maxp = n * (n - 1) / 2;
  H->pi = malloc(sizeof(int) * (maxp > 0 ? maxp : 1));
  H->pj = malloc(sizeof(int) * (maxp > 0 ? maxp : 1));
  H->P = malloc(sizeof(cplx *) * (maxp > 0 ? maxp : 1));
  H->npair = 0;
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++) {
      double A[3][3] = {{0}};
      double Jij = J ? J[i * n + j] : 0.0;
      for (int a = 0; a < 3; a++) A[a][a] += 2.0 * Jij;
      if (pos) {
        double rv[3], r2 = 0;
        for (int a = 0; a < 3; a++) {
          rv[a] = pos[3 * j + a] - pos[3 * i + a];
          r2 += rv[a] * rv[a];
        }
        double r = sqrt(r2);
        double D = ORACLE_C_DIP * g[i] * g[j] / (r * r * r);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++)
            A[a][b] += D * ((a == b ? 1.0 : 0.0) - 3.0 * (rv[a] / r) * (rv[b] / r));
      }
      int nz = 0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) nz |= (A[a][b] != 0.0);
      if (!nz) continue;
      int ni = H->ns[i], nj = H->ns[j], nn = ni * nj;
      cplx *P = calloc((size_t)nn * nn, sizeof(cplx));
      for (int ai = 0; ai < ni; ai++)
        for (int aj = 0; aj < nj; aj++)
          for (int bi = 0; bi < ni; bi++)
            for (int bj = 0; bj < nj; bj++) {
              cplx acc = 0;
              for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                  acc += A[a][b] * S[i][a][ai * ni + bi] * S[j][b][aj * nj + bj];
              P[(ai + ni * aj) * nn + (bi + ni * bj)] = acc;
            }
      H->pi[H->npair] = i;
      H->pj[H->npair] = j;
      H->P[H->npair] = P;
      H->npair++;
    }
  for (int i = 0; i < n; i++)
    for (int a = 0; a < 3; a++) free(S[i][a]);
  return H;
}

/* O = -sum_i g_i s_i . bhat: the moment along the field (units of mu_B). */
oracle_ham *oracle_build_moment(int n, const int *two_s, const double *g, const double *bhat) {
  if (n < 1 || n > ORACLE_MAX_SITES) return NULL;
  oracle_ham *H = malloc(sizeof(oracle_ham));
  ham_init_basis(H, n, two_s);
  for (int i = 0; i < n; i++) {
    int ni = H->ns[i];
    cplx *S[3];
    for (int a = 0; a < 3; a++) S[a] = malloc((size_t)ni * ni * sizeof(cplx));
    spin_cartesian(two_s[i], S[0], S[1], S[2]);
    cplx *h = calloc((size_t)ni * ni, sizeof(cplx));
    for (int k = 0; k < ni * ni; k++)
      for (int a = 0; a < 3; a++) h[k] -= g[i] * bhat[a] * S[a][k];
    for (int a = 0; a < 3; a++) free(S[a]);
    H->h[i] = h;
  }
  H->npair = 0;
  H->pi = H->pj = NULL;
  H->P = NULL;
  return H;
}

void oracle_free(oracle_ham *H) {
  if (!H) return;
  for (int i = 0; i < H->n; i++) free(H->h[i]);
  for (int p = 0; p < H->npair; p++) free(H->P[p]);
  free(H->P);
  free(H->pi);
  free(H->pj);
  free(H);
}

int64_t oracle_dim(const oracle_ham *H) { return H->dim; }
int oracle_npairs(const oracle_ham *H) { return H->npair; }

/* w = H v, straight from the definition of the matrix elements. */
static void hv(const oracle_ham *H, const cplx *v, cplx *w) {
  const int64_t dim = H->dim;
#pragma omp parallel for schedule(static)
  for (int64_t nu = 0; nu < dim; nu++) {
    int dig[ORACLE_MAX_SITES];
    int64_t x = nu;
    for (int i = 0; i < H->n; i++) {
      dig[i] = (int)(x % H->ns[i]);
      x /= H->ns[i];
    }
    cplx acc = 0;
    for (int i = 0; i < H->n; i++) {
      int ni = H->ns[i];
      const cplx *row = H->h[i] + (size_t)dig[i] * ni;
      for (int b = 0; b < ni; b++) {
        cplx c = row[b];
        if (c != 0) acc += c * v[nu + (int64_t)(b - dig[i]) * H->st[i]];
      }
    }
    for (int p = 0; p < H->npair; p++) {
      int i = H->pi[p], j = H->pj[p];
      int ni = H->ns[i], nj = H->ns[j], nn = ni * nj;
      const cplx *row = H->P[p] + (size_t)(dig[i] + ni * dig[j]) * nn;
      for (int bj = 0; bj < nj; bj++)
        for (int bi = 0; bi < ni; bi++) {
          cplx c = row[bi + ni * bj];
          if (c != 0)
            acc += c * v[nu + (int64_t)(bi - dig[i]) * H->st[i] + (int64_t)(bj - dig[j]) * H->st[j]];
        }
    }
    w[nu] = acc;
  }
}

void oracle_hv(const oracle_ham *H, const double *v_ri, double *w_ri) {
  hv(H, (const cplx *)v_ri, (cplx *)w_ri);
}

/* Selected rows of H v: out[k] = (H v)[rows[k]], by the same definition. */
void oracle_hv_rows(const oracle_ham *H, const double *v_ri, const int64_t *rows, int64_t nrows,
                    double *out_ri) {
  const cplx *v = (const cplx *)v_ri;
  cplx *out = (cplx *)out_ri;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nrows; k++) {
    const int64_t nu = rows[k];
    int dig[ORACLE_MAX_SITES];
    int64_t x = nu;
    for (int i = 0; i < H->n; i++) {
      dig[i] = (int)(x % H->ns[i]);
      x /= H->ns[i];
    }
    cplx acc = 0;
    for (int i = 0; i < H->n; i++) {
      int ni = H->ns[i];
      const cplx *row = H->h[i] + (size_t)dig[i] * ni;
      for (int b = 0; b < ni; b++)
        if (row[b] != 0) acc += row[b] * v[nu + (int64_t)(b - dig[i]) * H->st[i]];
    }
    for (int p = 0; p < H->npair; p++) {
      int i = H->pi[p], j = H->pj[p];
      int ni = H->ns[i], nj = H->ns[j], nn = ni * nj;
      const cplx *row = H->P[p] + (size_t)(dig[i] + ni * dig[j]) * nn;
      for (int bj = 0; bj < nj; bj++)
        for (int bi = 0; bi < ni; bi++) {
          cplx c = row[bi + ni * bj];
          if (c != 0)
            acc += c * v[nu + (int64_t)(bi - dig[i]) * H->st[i] + (int64_t)(bj - dig[j]) * H->st[j]];
        }
    }
    out[k] = acc;
  }
}

/* ---- Philox4x32-10 (Salmon et al., SC'11) ---- */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

/* Component nu of the random vector keyed by (seed; r, field, instance):
 * two 53-bit uniforms u1 in (0,1], u2 in [0,1) -> Box-Muller. */
static cplx gaussian_component(uint64_t seed, uint32_t r, uint32_t field, uint32_t inst,
                               uint32_t nu) {
  uint32_t ctr[4] = {nu, r, field, inst};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  uint64_t k1 = ((uint64_t)(x[0] >> 5) << 26) | (x[1] >> 6);
  uint64_t k2 = ((uint64_t)(x[2] >> 5) << 26) | (x[3] >> 6);
  double u1 = (double)(k1 + 1) * 0x1.0p-53;
  double u2 = (double)k2 * 0x1.0p-53;
  double rad = sqrt(-2.0 * log(u1));
  double ang = 2.0 * M_PI * u2;
  return rad * cos(ang) + I * (rad * sin(ang));
}

void oracle_gaussian_vector(uint64_t seed, uint32_t r, uint32_t field, uint32_t inst,
                            int64_t dim, double *out_ri) {
  cplx *out = (cplx *)out_ri;
#pragma omp parallel for schedule(static)
  for (int64_t nu = 0; nu < dim; nu++) out[nu] = gaussian_component(seed, r, field, inst, (uint32_t)nu);
}

/* The same components at the listed indices only (each below 2^32). */
void oracle_gaussian_entries(uint64_t seed, uint32_t r, uint32_t field, uint32_t inst,
                             const int64_t *idx, int64_t n, double *out_ri) {
  cplx *out = (cplx *)out_ri;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++) out[k] = gaussian_component(seed, r, field, inst, (uint32_t)idx[k]);
}

/* ---- Lanczos (Paige order) ---- */
static double dot_re(const cplx *a, const cplx *b, int64_t n) {
  double s = 0;
  for (int64_t k = 0; k < n; k++) s += creal(conj(a[k]) * b[k]);
  return s;
}

static cplx dot(const cplx *a, const cplx *b, int64_t n) {
  cplx s = 0;
  for (int64_t k = 0; k < n; k++) s += conj(a[k]) * b[k];
  return s;
}

/* Runs n_lanczos steps from the start vector r (normalised here).
 *   alpha[j], beta[j]  tridiagonal entries (beta[j] couples v_j and v_{j+1});
 *   y[j] = <O v_1 | v_j> (complex, interleaved re/im) when O != NULL;
 *   *n_used < n_lanczos after a breakdown beta_j <= 1e-12 max(|alpha|, beta).
 * reorth != 0 stores every Lanczos vector and re-orthogonalises u against all of
 * them (twice), for tiny test systems only. */
int oracle_lanczos(const oracle_ham *H, const oracle_ham *O, const double *r_ri, int n_lanczos,
                   int reorth, double *alpha, double *beta, double *y_ri, int *n_used) {
  const int64_t dim = H->dim;
  const cplx *r = (const cplx *)r_ri;
  cplx *y = (cplx *)y_ri;
  cplx *vprev = calloc((size_t)dim, sizeof(cplx));
  cplx *v = malloc((size_t)dim * sizeof(cplx));
  cplx *u = malloc((size_t)dim * sizeof(cplx));
  cplx *ov1 = NULL;
  cplx *basis = NULL;
  if (!vprev || !v || !u) return -2;
  if (reorth) {
    basis = malloc((size_t)dim * n_lanczos * sizeof(cplx));
    if (!basis) return -2;
  }
  double nr = sqrt(dot_re(r, r, dim));
  for (int64_t k = 0; k < dim; k++) v[k] = r[k] / nr;
  if (O) {
    ov1 = malloc((size_t)dim * sizeof(cplx));
    hv(O, v, ov1);
  }
  double beta_prev = 0.0, scale = 0.0;
  *n_used = 0;
  for (int j = 0; j < n_lanczos; j++) {
    if (reorth) memcpy(basis + (size_t)j * dim, v, (size_t)dim * sizeof(cplx));
    if (O) {
      cplx yj = dot(ov1, v, dim);
      y[j] = yj;
    }
    hv(H, v, u);
    for (int64_t k = 0; k < dim; k++) u[k] -= beta_prev * vprev[k];
    double a = dot_re(v, u, dim);
    for (int64_t k = 0; k < dim; k++) u[k] -= a * v[k];
    if (reorth) {
      for (int pass = 0; pass < 2; pass++)
        for (int q = 0; q <= j; q++) {
          cplx *bq = basis + (size_t)q * dim;
          cplx c = dot(bq, u, dim);
          for (int64_t k = 0; k < dim; k++) u[k] -= c * bq[k];
        }
    }
    double b = sqrt(dot_re(u, u, dim));
    alpha[j] = a;
    beta[j] = b;
    *n_used = j + 1;
    if (fabs(a) > scale) scale = fabs(a);
    if (j + 1 == n_lanczos) break;
    if (b <= 1e-12 * scale) break; /* breakdown: invariant subspace reached */
    if (b > scale) scale = b;
    cplx *t = vprev;
    vprev = v;
    v = t;
    for (int64_t k = 0; k < dim; k++) v[k] = u[k] / b;
    beta_prev = b;
  }
  free(vprev);
  free(v);
  free(u);
  free(ov1);
  free(basis);
  return 0;
}
