/*
 * ftlm.h -- C ABI of the MI355X (gfx950) finite-temperature Lanczos library.
 *
 * The library evaluates the finite-temperature Lanczos method (FTLM) for the
 * anisotropic spin Hamiltonian of Sec. 2.1, Eq. (mce-hamop):
 *
 *   H = 2 sum_{i<j} J_ij s_i.s_j + sum_i d_i (s_i.e_i)^2 + mu_B B.sum_i g_i s_i
 *       + mu0 mu_B^2/(4 pi) sum_{i<j} g_i g_j / r_ij^3 (s_i.s_j - 3 (s_i.e_ij)(e_ij.s_j))
 *
 * on the full product basis of dimension prod_i (2 s_i + 1) (Sec. 2.1), with no
 * symmetry reduction.  Thermal averages follow Sec. 2.2: Gaussian random vectors
 * (Eqs. E-1-1, E-1-2), Lanczos recursions, Krylov eigenpairs and the Boltzmann
 * sums of Eqs. (E-2-C) and (E-2-D).
 *
 * Units: J_ij and d_i in kelvin; B in tesla; positions in nm; g dimensionless.
 * Energies are in kelvin (k_B = 1), mu_B/k_B = 0.67171381563 K/T and
 * mu0 mu_B^2/(4 pi k_B) = 6.2294807e-4 K nm^3.  Outputs: T in K, ln Z, E in K,
 * C in units of k_B, M in units of mu_B as the moment along the field,
 * M = -sum_i g_i <s_i . B_hat> (B_hat = z when B = 0).
 *
 * Basis order: index nu = sum_i d_i * st_i with digit d_i = m_i + s_i and
 * st_i = prod_{k<i} (2 s_k + 1): site 0 is the fastest digit, nu = 0 is the
 * state with every m_i = -s_i.  Complex vectors are interleaved (re, im) pairs:
 * complex128 (16 B) or complex64 (8 B).  A block of K column vectors is stored
 * column-interleaved, element (nu, c) at offset nu*K + c.
 *
 * Conventions for every entry point:
 *   - return FTLM_OK (0) or a negative status; ftlm_last_error() then holds a
 *     thread-local message.  No C++ exception crosses this boundary.
 *   - device pointers are HIP device addresses on the current device; "stream"
 *     is a hipStream_t (NULL = the null stream).  Calls are asynchronous on the
 *     stream unless stated otherwise.
 *   - the library never allocates device memory inside ftlm_apply, ftlm_run or
 *     ftlm_run_batched: scratch space comes from the caller's workspace, sized by
 *     the *_workspace_size queries.  Hamiltonian handles own small device tables.
 */
#ifndef FTLM_H
#define FTLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FTLM_OK 0
#define FTLM_EINVAL (-1)  /* invalid argument */
#define FTLM_ENOMEM (-2)  /* host or device allocation failed / workspace too small */
#define FTLM_EHIP (-3)    /* a HIP runtime call failed */
#define FTLM_ERANGE (-4)  /* size out of range (dimension, sites, spin, columns) */

#define FTLM_MAX_SITES 32     /* N <= 32 */
#define FTLM_MAX_TWO_S 15     /* 2 s_i <= 15 */

typedef enum {
  FTLM_C128 = 0, /* complex128 vectors, FP64 arithmetic */
  FTLM_C64 = 1   /* complex64 vectors and H*v arithmetic; FP64 dot products,
                    recurrence scalars, tridiagonal solve and Boltzmann sums */
} ftlm_precision;

/* Parameters of the Hamiltonian of Sec. 2.1, Eq. (mce-hamop).  Host arrays;
 * ftlm_hamiltonian_create copies all of them. */
typedef struct {
  int32_t n_sites;       /* N, 1 <= N <= FTLM_MAX_SITES */
  const int32_t *two_s;  /* [N] 2 s_i in [1, FTLM_MAX_TWO_S]; dim must be < 2^32 */
  const double *J;       /* [N*N] row-major, J[i*N+j] read for i<j; NULL = none */
  const double *d;       /* [N] single-ion strengths; NULL = none */
  const double *e;       /* [N*3] anisotropy axes, normalised on copy; a zero
                            axis with d_i != 0 is FTLM_EINVAL; NULL if d is NULL */
  const double *g;       /* [N] g-factors */
  const double *B;       /* [3] field in tesla */
  const double *pos;     /* [N*3] positions (nm), r_ij = pos_j - pos_i; NULL = no
                            dipolar term; coincident sites are FTLM_EINVAL */
} ftlm_system;

typedef struct ftlm_hamiltonian ftlm_hamiltonian; /* opaque */

/* Compiles the Hamiltonian (Sec. 2.1): one-site matrices h_i and the ladder
 * coefficients of every interacting pair, uploaded to device tables owned by the
 * handle.  Uses the current HIP device.  *out is set only on success. */
int ftlm_hamiltonian_create(const ftlm_system *sys, ftlm_hamiltonian **out);
void ftlm_hamiltonian_destroy(ftlm_hamiltonian *h);
/* dim = prod_i (2 s_i + 1) (Sec. 2.1). */
int ftlm_hamiltonian_dim(const ftlm_hamiltonian *h, uint64_t *dim);
/* Average number of stored non-zero matrix elements per row of H, counting the
 * diagonal once (the algorithmic work of H*v is 8 flops per non-zero). */
int ftlm_hamiltonian_nnz_per_row(const ftlm_hamiltonian *h, double *nnz);
/* Replaces the field B (tesla) and recompiles the field-dependent tables.
 * Synchronises the device.  Not thread-safe with concurrent apply/run. */
int ftlm_hamiltonian_set_field(ftlm_hamiltonian *h, const double B[3]);

/* w = H v for n_cols column-interleaved vectors (the matrix-free product at
 * the heart of every Lanczos step, Sec. 2.3).  v, w: device, [dim][n_cols]
 * complex of the given precision, 16-byte aligned, v != w, not overlapping.
 * 1 <= n_cols <= 64.  Allocates nothing. */
int ftlm_apply(const ftlm_hamiltonian *h, int32_t precision, int32_t n_cols, const void *v,
               void *w, void *stream);

/* Autotuner: times every admissible H*v configuration for (precision, n_cols) on
 * the caller's device buffers v, w ([dim][n_cols], as ftlm_apply) -- variants
 * 1 = direct gather (columns per lane 1, 2, 4, 8), 2 = windowed LDS passes,
 * 3 = LDS tile (spin 1/2, N >= 11), 4 = L2-window passes (one column), 5 = LDS
 * tile walked over L2 windows (spin 1/2, N >= 12; 256, 512 or 1024 threads per
 * tile, given in the columns-per-lane field as 1, 2 or 4 row groups), 6 = single pass
 * over LDS tiles of the low digits with coalesced partner reads for the terms
 * on outer sites (one column; Hamiltonians without s+- s^z pair pieces, i.e.
 * whose single-flip coefficients do not depend on the other sites; the
 * columns-per-lane field carries the block size in bits 0..3 -- 1: 256
 * threads for tiles of up to 4096 rows, else 1024 --, the log2 of the
 * tiles per XCD chunk in bits 4..7, and in bit 8 whether the partner tiles of
 * the pairs with one tile site are staged in LDS, one per outer site and move,
 * instead of read directly; not for systems of spins 1/2 only, where a launch
 * with bit 8 set fails with FTLM_EINVAL), each at 512, 1024, 2048 and 4096 blocks (variants 4, 5, 6: at most
 * 2048) --
 * with HIP events on the stream (blocking): three launches each, then the four
 * fastest again with ten launches each.  Stores the fastest of that second
 * round in the handle for later ftlm_apply / ftlm_run launches of the same
 * shape.  Outputs (may be NULL): the chosen variant, grid size, columns per
 * lane and its mean time over the ten launches. */
int ftlm_hamiltonian_autotune(ftlm_hamiltonian *h, int32_t precision, int32_t n_cols, const void *v,
                              void *w, void *stream, int32_t *variant, int32_t *grid_cap,
                              int32_t *kc, float *best_ms);
/* Sets the H*v configuration for (precision, n_cols) directly (e.g. from a cache
 * of earlier autotune results); variant 0 restores the built-in heuristic: for
 * one column of at least 2^20 rows the single-pass tile kernel (variant 6) when
 * the Hamiltonian has no s+- s^z pair pieces, else the LDS tile (spin 1/2, N >=
 * 11) or the windowed passes; below that the direct gather. */
int ftlm_hamiltonian_set_tuning(ftlm_hamiltonian *h, int32_t precision, int32_t n_cols,
                                int32_t variant, int32_t grid_cap, int32_t kc);

/* Start vectors of Eqs. (E-1-1), (E-1-2): out[nu*n_cols + c] = x + i y with x, y
 * independent standard normals for random vector r = r0 + c.  The bits come from
 * Philox4x32-10 (Salmon et al., SC'11) with key (seed low 32, seed high 32) and
 * counter (nu, r, field, instance); two 53-bit uniforms u1 in (0,1], u2 in [0,1)
 * give x + i y = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2) (Box-Muller).
 * out: device complex128 [dim][n_cols].  Not normalised.  The first call on a
 * device (per host thread) allocates a private 1 MB buffer for the kernel's norm
 * partials, kept until the process ends. */
int ftlm_gaussian_vectors(uint64_t seed, uint32_t instance, uint32_t field, uint32_t r0,
                          int32_t n_cols, uint64_t dim, void *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, loops that must not call hipMalloc): the same start vectors as
 * ftlm_gaussian_vectors (same arguments, same kernels, bitwise the same out),
 * with the kernel's norm partials kept in a file-scope device array of the
 * library instead of a buffer it allocates.  The array holds the partials of
 * at most 2048 blocks x 64 columns (1 MiB per GPU, held until the process
 * ends); n_cols > 64 is FTLM_ERANGE.  Calls no hipMalloc, hipFree or
 * allocating library routine.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU race on the partials (not on out).  The first
 * call on a device looks up the array's address there (hipGetSymbolAddress). */
int ftlm_gaussian_vectors_noalloc(uint64_t seed, uint32_t instance, uint32_t field, uint32_t r0,
                                  int32_t n_cols, uint64_t dim, void *out, void *stream);

/* Run parameters for ftlm_run / ftlm_run_batched. */
typedef struct {
  int32_t R;            /* random vectors per field, >= 1 */
  int32_t n_lanczos;    /* Lanczos steps N_L, 1 <= N_L <= 1024 */
  uint64_t seed;        /* key of the counter-based generator */
  uint32_t instance;    /* instance index used in the generator counter */
  const double *T;      /* [n_T] temperatures (K), all > 0; host */
  int32_t n_T;          /* >= 1 */
  const double *fields; /* [n_fields*3] fields (T) overriding the system's B; NULL =
                           the handle's current field (n_fields must then be 1);
                           the handle's field is restored on return */
  int32_t n_fields;
  int32_t precision;    /* ftlm_precision */
  int32_t columns;      /* K: random vectors iterated together, 1..64; 0 = automatic
                           (1 for dim >= 2^20, min(R, 4) for dim >= 2^17,
                           min(R, 16) for dim >= 2^14, else min(R, 64)) */
  const void *r_init;   /* optional device complex128 start vectors (not
                           normalised) replacing the generator, element (f, nu, r)
                           at offset (f*dim + nu)*R + r; NULL */
} ftlm_run_params;

/* Results; caller-owned host arrays (NULL entries are skipped). */
typedef struct {
  double *lnZ, *E, *C, *M;   /* [n_fields*n_T] */
  int32_t *n_lanczos_used;   /* [n_fields*R]; < N_L after a Lanczos breakdown */
  double *E_min;             /* [n_fields] lowest Ritz value over the R vectors */
  double *alpha, *beta;      /* [n_fields*R*N_L] tridiagonals (diagnostics) */
  double *hv_ms;             /* if non-NULL: summed duration (ms) of the run's Lanczos
                                H*v kernels, from HIP events recorded around each launch
                                on the run's stream (the run then skips graph replay) */
  int32_t *hv_launches;      /* number of H*v launches timed into *hv_ms */
} ftlm_result;

/* Bytes of device workspace ftlm_run needs for these parameters. */
int ftlm_run_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, size_t *bytes);

/* FTLM thermodynamics, Sec. 2.2: for every field, R random vectors run N_L
 * Lanczos steps (Paige order: u = H v_j - beta_{j-1} v_{j-1}; alpha_j =
 * Re<v_j|u>; u -= alpha_j v_j; beta_j = |u|; v_{j+1} = u/beta_j; with
 * y_j = <O v_1|v_j>); the Krylov eigenpairs eps_n, Q_1n and sum_a Q_an Re y_a
 * follow from the tridiagonal (implicit QL); the Boltzmann sums of Eqs. (E-2-C)
 * and (E-2-D) with Gamma = 1 give ln Z, E, C = (<eps^2> - <eps>^2)/T^2 and M.
 * A step with beta_j <= 1e-12 max(|alpha_<=j|, beta_<j) ends that vector's
 * recursion (recorded in n_lanczos_used; not an error).
 * Blocks on the stream before returning (results are host arrays). */
int ftlm_run(const ftlm_hamiltonian *h, const ftlm_run_params *p, void *workspace,
             size_t bytes, void *stream, ftlm_result *out);

/* Symmetric FTLM (sFTLM), Sec. 2.2, Eqs. (E-2-G) and (E-2-H), with pairs of
 * mutually time-reversed random vectors.  R (even) counts vectors: R/2 Gaussian
 * vectors (Philox vector index = pair index, as ftlm_gaussian_vectors) and their
 * time reverses (Theta x)[dim-1-nu] = (-1)^{sum_i (2 s_i - d_i(nu))} conj(x[nu]).
 * Each vector runs N_L Lanczos steps keeping all Krylov vectors; M is the ratio
 * sum_r <r|exp(-H/2T) O exp(-H/2T)|r> / sum_r <r|exp(-H/T)|r> with the double
 * sum of Eq. (E-2-H) over the Krylov eigenpairs, O = -sum_i g_i s_i.B_hat; ln Z,
 * E and C as ftlm_run.  Uses p->R, n_lanczos (<= 140), seed, instance, T, n_T,
 * fields, n_fields, precision; columns is ignored and r_init must be NULL.
 * Workspace: (2 N_L + 1) vectors plus O(R N_L^2) doubles; no allocation.
 * Blocks on the stream before returning. */
int ftlm_run_sftlm_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, size_t *bytes);
int ftlm_run_sftlm(const ftlm_hamiltonian *h, const ftlm_run_params *p, void *workspace,
                   size_t bytes, void *stream, ftlm_result *out);

/* Chebyshev (kernel polynomial) expansion of the thermal traces without a
 * smoothing kernel, the alternative to Lanczos named in Sec. 4: the same random
 * vectors and H*v launch, with exp(-H/T) = exp(-lo/T) sum_{n<=N} c_n(a/T)
 * T_n((H-b)/a), c_n(x) = (2 - delta_n0) (-1)^n exp(-x) I_n(x).  Spectral bounds
 * [lo, hi]: the extreme Krylov eigenvalues of p->n_lanczos Lanczos steps on the
 * first random vector of each field, widened by 2 % of their spread.  Moments
 * mu_n = Re<r|T_n|r>, nu_n = Re<O r|T_n|r> for n <= N + 2 (N + 2 H*v per
 * vector); ln Z, E = <H>, C = (<H^2> - <H>^2)/T^2 and M = <O> as in ftlm_run.
 * n_moments = N (2 <= N <= 1e6).  Truncation is not smoothed: N must exceed about
 * a/T_min for the lowest temperature to converge.  E_min receives lo;
 * bounds (host, may be NULL) receives [n_fields][lo, hi].  columns and r_init
 * are ignored / must be NULL.  Blocks on the stream before returning. */
int ftlm_run_kpm_workspace_size(const ftlm_hamiltonian *h, const ftlm_run_params *p, int32_t n_moments,
                                size_t *bytes);
int ftlm_run_kpm(const ftlm_hamiltonian *h, const ftlm_run_params *p, int32_t n_moments, void *workspace,
                 size_t bytes, void *stream, ftlm_result *out, double *bounds);

/* Batched form (grouping random vectors, field directions and instances so
 * that one launch applies H to many vectors: the paper's proposal against the
 * random access of H*v, Secs. 3.1 and 4): many Hamiltonian instances (uneven
 * dimensions) and their field directions run together; every Lanczos step is
 * one persistent launch over a work queue of (curve, row tile) units for all
 * curves of a wave, replayed as a HIP graph.  per_inst[k] describes instance k (R, N_L, n_T, precision and
 * columns must agree across instances).  columns = random vectors per work item,
 * one of 16, 8, 4, 2, 1 dividing R; 0 = automatic (4 when the largest instance
 * has >= 2^17 rows, else the largest dividing R).  out[k] receives instance k's
 * results.  Blocks on the stream before returning. */
int ftlm_run_batched_workspace_size(const ftlm_hamiltonian *const *hs, int32_t n_inst,
                                    const ftlm_run_params *per_inst, size_t *bytes);
int ftlm_run_batched(const ftlm_hamiltonian *const *hs, int32_t n_inst,
                     const ftlm_run_params *per_inst, void *workspace, size_t bytes,
                     void *stream, ftlm_result *out);

/* Launch choices of ftlm_run_batched on the calling host thread (the batched
 * autotuner's knobs; applying H to groups of random vectors at once is the
 * paper's remedy for the random access of H*v, Secs. 3.1 and 4): grid_cap =
 * blocks of the per-step launch (64..65536; 0 = 1024), unit_bits = log2 of the
 * rows of a work unit (11 or 12; 0 = 11), order = the order in which a wave's
 * items take their work units (0 = curve order, 1 = largest instance first),
 * block = threads per block of the H*v step launch (256, 512 or 1024; 0 = 512).
 * Results are bitwise independent of grid_cap and order (every work unit's
 * partial sums are formed alike and summed per item in unit order); unit_bits
 * and block change the summation tree of the dot products (rounding only).
 * FTLM_EINVAL (settings unchanged) for a value outside these.  If out[0].hv_ms is
 * non-NULL, ftlm_run_batched stores there the summed duration of the Lanczos
 * step launches (HIP events around each wave's step graph) and in
 * out[0].hv_launches the number of steps timed. */
int ftlm_batched_set_tuning(int32_t grid_cap, int32_t unit_bits, int32_t order, int32_t block);

/* Krylov eigen-decomposition step on the device (the tridiagonal eigenproblem of
 * Sec. 2.2): for every column c, the symmetric tridiagonal with diagonal
 * alpha[j*n_cols+c] and off-diagonal beta[j*n_cols+c] (j < n_used[c], or
 * n_lanczos when n_used is NULL) is diagonalised by implicit QL; eps[j*n_cols+c]
 * receives the eigenvalues, q1[...] the first components Q_1n and
 * qy[...] = sum_a Q_an y[a*n_cols+c] (y real, may be NULL).  Entries j >= n_used[c]
 * are set to 0.  All device pointers, [n_lanczos][n_cols] FP64; scratch holds
 * 4*n_lanczos*n_cols doubles. */
int ftlm_tridiag_eigen(int32_t n_cols, int32_t n_lanczos, const int32_t *n_used,
                       const double *alpha, const double *beta, const double *y, double *eps,
                       double *q1, double *qy, double *scratch, void *stream);

/* Boltzmann sums of Eqs. (E-2-C) and (E-2-D) on the device: columns
 * [f*R, (f+1)*R) form curve f.  Inputs from ftlm_tridiag_eigen (device); dims[f] is
 * the Hilbert dimension of curve f; T device [n_T].  Outputs device
 * [n_curves*n_T] lnZ, E, C, M and [n_curves] E_min. */
int ftlm_boltzmann(int32_t n_curves, int32_t R, int32_t n_lanczos, const int32_t *n_used,
                   const double *eps, const double *q1, const double *qy, const double *dims,
                   const double *T, int32_t n_T, double *lnZ, double *E, double *C, double *M,
                   double *E_min, void *stream);

/* ---- learned surrogate (an MLP 7 -> 256 -> 256 -> 256 -> 3, SiLU) ----
 * Weights W_k are [fan_in][fan_out] bf16 (layer k = 0..3), biases FP32; master
 * copies FP32 for the optimiser.  All pointers are device pointers. */
typedef struct {
  const uint16_t *W[4]; /* bf16 weights */
  const float *b[4];    /* biases */
} ftlm_mlp_weights;

/* y[B][3] = MLP(x[B][7]); acts (optional, may be NULL) receives the
 * pre-activations z_k [B][256] of the three hidden layers (FP32) and a_k
 * (bf16) for the backward pass: workspace of ftlm_mlp_workspace_size(B). */
int ftlm_mlp_workspace_size(int32_t batch, size_t *bytes);
int ftlm_mlp_forward(const ftlm_mlp_weights *w, int32_t batch, const float *x, float *y,
                     void *workspace, size_t bytes, void *stream);
/* Loss L = 1/(3B) sum (y - t)^2 and gradients dW (FP32 [fan_in][fan_out]) and db
 * for the batch, after ftlm_mlp_forward filled the same workspace.  loss: device
 * FP32 scalar (may be NULL). */
int ftlm_mlp_backward(const ftlm_mlp_weights *w, int32_t batch, const float *t, float *loss,
                      float *const dW[4], float *const db[4], void *workspace, size_t bytes,
                      void *stream);
/* Adam (Kingma & Ba) on n FP32 master parameters p with moments m, v; writes the
 * bf16 copy pb (may be NULL).  step counts from 1. */
int ftlm_adam_step(int64_t n, float *p, const float *grad, float *m, float *v, uint16_t *pb,
                   float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* Window sizes of the H*v planners, in KiB, for handles created (and plans
 * described) afterwards; 0 selects the default.  pass_kb: LDS windows of the
 * multi-pass kernel (variant 2; 4..128, default 64).  l2_kb: L2 windows of the
 * window kernels of variant 4 (4..65536, default 1024).  tile_kb: L2 windows of
 * the tile-window kernel (variant 5; 4..65536, default 2048, or a single window
 * when the vector is at most 160 MB).  Existing handles keep their plans.  The
 * setting is process-wide; calls concurrent with handle creation race.
 * FTLM_EINVAL (settings unchanged) for a value outside its range. */
int ftlm_set_plan_windows(int32_t pass_kb, int32_t l2_kb, int32_t tile_kb);

/* Host-only (no device work): compiles the Hamiltonian and reports the plan the
 * one-column H*v uses in the given precision.  Each pass stages windows of rows
 * that share every digit except those of its active sites and applies from LDS
 * the terms it owns.  Per pass p < max_pass: window_rows[p], n_active[p] (sites
 * spanning the window), n_pairs[p] (pair terms it applies), n_singles[p] (sites
 * whose single-site flips it applies); pair_sites (may be NULL) receives the
 * (i, j) sites of every pair term, pass by pass (2 * total pairs ints).
 * nnz_per_row (may be NULL) as ftlm_hamiltonian_nnz_per_row. */
int ftlm_describe_passes(const ftlm_system *sys, int32_t precision, int32_t max_pass,
                         int32_t *n_pass, uint32_t *window_rows, int32_t *n_active,
                         int32_t *n_pairs, int32_t *n_singles, int32_t *pair_sites,
                         double *nnz_per_row);

/* Host-only (no device work): the L2-window plan of the one-column H*v
 * (variant 4).  A window is the set of rows sharing the digits of every site
 * outside window_sites; its rows fit a share of one XCD's L2, and each pass walks
 * the windows so that all blocks of an XCD work on the same one, applying the
 * terms whose sites all lie in the window.  window_bytes <= 0 selects the library
 * setting (ftlm_set_plan_windows' l2_kb, default 1024).  Per pass p < max_pass:
 * window_rows[p], window_sites[p] (bit k = site k), n_pairs[p] and
 * single_sites[p] (bit k: the pass applies the single-site flips of site k);
 * pair_sites (may be NULL) receives the (i, j) sites of every pair term, pass by
 * pass.  Returns FTLM_ERANGE when no plan fits the window size. */
int ftlm_describe_windows(const ftlm_system *sys, int32_t precision, int64_t window_bytes,
                          int32_t max_pass, int32_t *n_pass, uint32_t *window_rows,
                          uint32_t *window_sites, int32_t *n_pairs, uint32_t *single_sites,
                          int32_t *pair_sites);

const char *ftlm_last_error(void);
int ftlm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FTLM_H */
