/*
 * clsel — selected inversion of the staggered Dirac matrix and the exact
 * complex-Langevin fermion drift, on AMD Instinct MI355X (gfx950).
 *
 * Problem (Bloch & Schenk, "Selected inversion as key to a stable Langevin
 * evolution across the QCD phase boundary", Lattice 2017):
 *   given SL(3,C) links U_{x,nu}, a quark mass m and a chemical potential mu,
 *   compute the entries of D(m,mu)^{-1} on the nonzero pattern of D (Sec. 3,
 *   selected-inversion paragraph) and the fermionic drift
 *   K^f_{a,x,nu} = tr[D^{-1} d_{a,x,nu} D] (Eq. 6) for every link, through the
 *   two-block reduction K = tr(P B) + tr(Q F) (Eq. 8).
 *
 * Operator (the paper names it only as the staggered operator of Eq. 1):
 *   D_{x,x} = m; D_{x,x+nu} = +1/2 eta_nu(x) s_nu(x) e^{+mu delta_{nu,3}} U_{x,nu};
 *   D_{x+nu,x} = -1/2 eta_nu(x) s_nu(x) e^{-mu delta_{nu,3}} U_{x,nu}^{-1};
 *   eta_nu(x) = (-1)^{x_0+...+x_{nu-1}}; s = -1 on the temporal hop that wraps
 *   (antiperiodic time), +1 otherwise; spatial directions periodic.
 * Derivative: left Lie derivative U -> e^{i alpha lambda_a} U (matches the
 * Langevin update U <- R U of Eqs. 3-4); lambda_a the Gell-Mann matrices.
 *
 * Layouts (all complex128 = two doubles, re then im, row-major colour indices):
 *   site index     x = x0 + L0*(x1 + L1*(x2 + L2*x3)), x3 = time
 *   links          [B][V][4][3][3]
 *   selected       [B][V][9][3][3]; slot 0 = Z_{x,x}, 1+nu = Z_{x,x+nu},
 *                  5+nu = Z_{x,x-nu}  (nu = 0..3)
 *   drift          [B][V][4][8]; component a-1 of K_{a,x,nu}
 *
 * Memory: device pointers are caller-owned and must stay valid until the work
 * enqueued on the batch's stream has passed them. Plans and batches own all
 * other memory. A batch references its plan: destroy batches first.
 *
 * Errors: functions return 0 (CL_OK) or a negative CL_E* code; cl_last_error()
 * gives a message. Numeric failures inside the enqueued work are recorded per
 * configuration and reported by cl_status; the outputs of a failed
 * configuration are NaN. There is one GPU code path and no CPU fallback: without
 * a usable gfx950 device every numeric call fails with CL_ENODEV or CL_EHIP.
 */
#ifndef CLSEL_H
#define CLSEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CL_OK 0
#define CL_EINVAL (-1)      /* bad argument: odd or < 4 extent, null pointer, batch < 1 */
#define CL_ENOMEM (-2)      /* device or host allocation failed */
#define CL_EORDER (-3)      /* call out of order, e.g. cl_selinv before cl_factor */
#define CL_ESINGULAR (-4)   /* non-finite pivot, zero pivot without perturbation, or a singular
                               low-rank correction matrix (per config) */
#define CL_ENONFINITE (-5)  /* non-finite or singular link (per config) */
#define CL_EHIP (-6)        /* a HIP runtime call failed */
#define CL_ENODEV (-7)      /* no usable GPU */
#define CL_ERANK (-8)       /* more perturbed pivots than the low-rank correction holds (per config) */

typedef struct cl_plan_s* cl_plan;
typedef struct cl_batch_s* cl_batch;

/* Options of the symbolic analysis. Zero fields take the defaults. */
typedef struct {
  int32_t leaf_sites;     /* nested dissection stops at boxes of <= this many sites (default 4) */
  int32_t max_pivot_rows; /* separators with more rows are split into a chain (<= 1536, default 1536) */
  int32_t nb;             /* block width of the frontal Gauss-Jordan sweep (1..64, default 64) */
  int32_t time_cuts;      /* 1: separators may cut the time direction; 0 (default): never */
  int32_t gemm_tile;      /* output tile of the plain products: 0 auto (64 x 64), 64, 12864, 128 */
  int32_t lowrank_cap;    /* perturbed pivots one configuration may have undone (0: default,
                             64 per 24576 rows of D, at least 128; at most 1024) */
  double pivot_floor;     /* pivot perturbation threshold in units of D's entries (0: default 0.3;
                             negative: no perturbation). See cl_factor. */
  int32_t smw_refine;     /* 1: one refinement step of the correction's solves against D~
                             formed from the links; 0 (default): none (0..1) */
} cl_plan_opts;

typedef struct {
  int32_t dims[4];
  int64_t volume;          /* V */
  int64_t n;               /* N = 3V */
  int32_t nfronts, nlevels, max_steps, max_front_rows, max_pivot_rows;
  int64_t pool_elems;      /* complex elements of one front pool, per configuration */
  double flops_factor;     /* executed by the factorisation kernels, per configuration */
  double flops_selinv;     /* executed by the selected-inversion kernels */
  double flops_factor_alg; /* standard block LU count: 8/3 p^3 + 8 s p^2 + 8 s^2 p per supernode */
  double flops_selinv_alg; /* standard selected inversion: 16/3 p^3 + 8 p^2 s + 16 s^2 p */
  double flops_dense_inverse; /* 8 N^3: what a full inverse would cost */
  int32_t lowrank_cap;     /* columns of the low-rank correction (0: perturbation off) */
  double pivot_floor;      /* pivot perturbation threshold (negative: off) */
  int32_t smw_refine;      /* refinement steps of the correction's solves */
} cl_plan_info_t;

/* Symbolic analysis of one lattice shape (host only, no device work). Every
 * extent must be even and between 4 and 254. The plan is immutable and may be shared by any
 * number of batches and threads. Sec. 3: sparse LU followed by selected
 * inversion; the ordering is geometric nested dissection. */
int cl_symbolic(const int32_t dims[4], cl_plan* out);
int cl_symbolic_ex(const int32_t dims[4], const cl_plan_opts* opts, cl_plan* out);
int cl_plan_info(cl_plan plan, cl_plan_info_t* out);
/* Device bytes a batch of `batch` configurations needs (for admission control). */
size_t cl_plan_bytes(cl_plan plan, int32_t batch);
/* Copies one plan table to host memory for inspection: what = 0 fronts (int64
 * rows of CL_FRONT_FIELDS), 1 front sites (int32), 2 parent->child row maps
 * (int32), 3 child->parent row maps (int32), 4 selected-block offsets (int64),
 * 5 elimination order (int64). With dst == NULL only *nbytes is set. */
#define CL_FRONT_FIELDS 28
int cl_plan_export(cl_plan plan, int32_t what, void* dst, size_t* nbytes);
void cl_plan_destroy(cl_plan plan);

/* Numeric workspace for up to `batch` configurations of one plan. Work is
 * ordered after, and before, work on `hip_stream` (NULL = the null stream); the
 * batch runs it on a private stream of default priority. */
int cl_batch_create(cl_plan plan, int32_t batch, void* hip_stream, cl_batch* out);
/* Configurations processed by the following calls: 1..batch (default batch). */
int cl_batch_set_active(cl_batch batch, int32_t n);
/* Enables (1) or disables (0) HIP-graph capture of cl_run. */
int cl_batch_use_graph(cl_batch batch, int32_t enable);
/* Lanes of cl_run: 1 runs the active configurations as one batch on the batch stream;
 * 2 runs the first half there and the second half on a second stream of the batch,
 * forked from it and joined back before cl_run's work ends (also under graph capture),
 * so that the latency-bound kernels of one half (pivot panels, assembly, gathers) run
 * beside the matrix-core products of the other. Every configuration is computed by the
 * same kernels either way, so the results are bitwise the same. 0 (the default) picks
 * 2 from 16 active configurations on, else 1; while GEMM launches are timed
 * (cl_batch_profile) cl_run uses one lane. CL_EINVAL outside 0..2. */
int cl_batch_set_lanes(cl_batch batch, int32_t lanes);
/* Assembles D for each configuration from `links_dev` (device, [B][V][4][3][3]
 * complex128, copied before the call returns control of it to the stream) and
 * m_host[b], mu_host[b], then runs the supernodal factorisation (partial
 * pivoting inside each supernode's own rows). Enqueues only.
 * Pivot perturbation: a pivot whose modulus, after partial pivoting, is below the plan's
 * pivot_floor is raised to that modulus (its phase kept). This factorises
 * D~ = D + sum_k delta_k e_{i_k} e_{j_k}^T, one rank-1 term per perturbed pivot, whose pivot
 * blocks are well conditioned. cl_selinv undoes the change exactly with the
 * Sherman-Morrison-Woodbury identity, so every result is that of D itself (Sec. 3: the
 * selected entries of D^{-1} are computed exactly, not approximated); cl_solve does the same.
 * A configuration with more perturbed pivots than the plan's lowrank_cap gets CL_ERANK. */
int cl_factor(cl_batch batch, const void* links_dev, const double* m_host, const double* mu_host);
/* Selected inversion (Takahashi / Erisman-Tinney recurrences in supernodal form):
 * the blocks of D~^{-1} on the filled pattern, root to leaves, gathered on the pattern of
 * D; then the low-rank correction of the perturbed pivots (see cl_factor):
 *   D^{-1} = D~^{-1} - X C Y,  X = D~^{-1} U,  Y = V^T D~^{-1},  C = (I + V^T X)^{-1},
 * with U = [-delta_k e_{i_k}] and V = [e_{j_k}]. X and Y come from r right and r left solves
 * through the same frontal factors (with the plan option smw_refine, each refined once
 * against D~ itself, the residual formed from the links); the r x r matrix C by
 * Gauss-Jordan elimination with partial pivoting. A singular C sets CL_ESINGULAR.
 * Enqueues only. */
int cl_selinv(cl_batch batch);
/* Drift K [B][V][4][8] complex128 into out_dev (device). Enqueues only. */
int cl_drift(cl_batch batch, void* out_dev);
/* Selected blocks [B][V][9][3][3] complex128 into out_dev (device). Enqueues only. */
int cl_selected(cl_batch batch, void* out_dev);
/* Fermionic observables from the selected blocks (Sec. 3: like the drift they need
 * only entries of D^{-1} where D is nonzero): out_dev (device) receives [B][2]
 * complex128 = { (1/V) tr D^{-1}  (chiral condensate, d/dm log det D / V),
 *                (1/V) tr(D^{-1} dD/dmu)  (quark number density, d/dmu log det D / V) }.
 * Deterministic reduction. Enqueues only; needs cl_selinv first. */
int cl_observables(cl_batch batch, void* out_dev);
/* Gauge drift K^g = -dS_g/dz for every link (Sec. 2, Eq. 5: the drift is K^g + K^f).
 * The paper names the Wilson gauge action without writing it; here it is the plaquette
 * action continued to SL(3,C) links, beta sum_P [1 - (tr P + tr P^{-1}) / 6], periodic in
 * every direction, differentiated with the same left Lie derivative as the fermion drift.
 * beta_host [B] (host, finite); out_dev (device) receives [B][V][4][8] complex128, K_a for
 * a = 1..8. Uses the links of the last cl_factor / cl_run. Enqueues only; CL_EORDER
 * before the first factorisation. */
int cl_gauge_drift(cl_batch batch, const double* beta_host, void* out_dev);
/* One Euler step of the complex Langevin evolution (Sec. 2, Eqs. 3-4) for every link:
 * U <- exp[i sum_a lambda_a (eps K_a + sqrt(eps) eta_a)] U, where U are the links of the
 * last cl_factor / cl_run and K = K^f + K^g.
 *   links_out_dev [B][V][4][3][3] complex128 (device): the new links; it may be the
 *                 buffer the links were read from.
 *   kf_dev        [B][V][4][8] complex128 (device): the fermion drift (cl_drift).
 *   kg_dev        same layout (cl_gauge_drift), or NULL for the fermion drift alone.
 *   eta_dev       [B][V][4][8] double (device): real Gaussian noise drawn by the caller
 *                 (<eta_a eta_b> = 2 delta_ab in the standard Euler scheme).
 *   eps_bar_host  [B] finite steps >= 0. kref_host [B] or NULL: where kref > 0 the step
 *                 is adaptive, eps = eps_bar * kref / max over links of
 *                 sqrt(sum_a |K_a|^2) (Sec. 4.1 uses an adaptive step without giving
 *                 the rule; this is the rule of Aarts, James, Seiler and Stamatescu,
 *                 2010), else eps = eps_bar.
 *   eps_out_dev   [B] double (device) or NULL: the step used.
 * The exponential is a scaled Taylor polynomial with squaring (relative error ~1e-15).
 * Enqueues only; CL_EORDER before the first factorisation, CL_EINVAL for a negative or
 * non-finite eps_bar or a non-finite kref. */
int cl_langevin_update(cl_batch batch, void* links_out_dev, const void* kf_dev, const void* kg_dev,
                       const void* eta_dev, const double* eps_bar_host, const double* kref_host,
                       void* eps_out_dev);
/* Solves D X = R for ns right-hand sides through the factors of the last cl_factor /
 * cl_run (forward sweep with -L^, backward sweep with A_JJ^{-1} and U^, front by front;
 * valid before and after cl_selinv, which leaves the factors in place). rhs_dev and
 * x_dev (device) are [B][N][ns] complex128 with row index 3*site + colour and the
 * right-hand sides contiguous. 1 <= ns <= 4096. The first call for a given ns builds
 * and checks its launch tables and allocates a workspace of 2 * (sum of front rows) * ns
 * complex128 per configuration; calls with the same ns reuse them. With perturbed pivots
 * (cl_factor) the solution of D~ is corrected to that of D: x = x~ - X C (V^T x~), with X and
 * C of the last cl_selinv, so cl_solve needs cl_selinv first where the plan perturbs
 * (CL_EORDER otherwise). Enqueues only; CL_EORDER before the first factorisation. */
int cl_solve(cl_batch batch, const void* rhs_dev, int32_t ns, void* x_dev);
/* Stochastic estimate of the selected blocks (Sec. 3, Eq. 7: the estimator that
 * selected inversion replaces): from noise columns xi and X = D^{-1} xi (cl_solve), both
 * [B][N][ns] complex128 (device), out_dev [B][V][9][3][3] complex128 receives
 * Z~_{x,y} = (1/ns) sum_s X_{x,s} xi_{y,s}^* in the slot order of cl_selected. With
 * E[xi xi^dagger] = 1 its expectation is the selected blocks of D^{-1}. Enqueues only. */
int cl_stochastic_blocks(cl_batch batch, const void* xi_dev, const void* x_dev, int32_t ns,
                         void* out_dev);
/* The drift contraction of cl_drift (Eq. 8) applied to caller-supplied blocks in the
 * layout of cl_selected (for example the stochastic estimate above), with the links and
 * mu of the last cl_factor / cl_run. out_dev [B][V][4][8] complex128. Enqueues only. */
int cl_drift_from_blocks(cl_batch batch, const void* blocks_dev, void* out_dev);
/* cl_factor + cl_selinv + cl_selected + cl_drift in one call; replayed from a
 * HIP graph when enabled. Either output pointer may be NULL. */
int cl_run(cl_batch batch, const void* links_dev, const double* m_host, const double* mu_host,
           void* selected_out_dev, void* drift_out_dev);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the work of cl_run (factorisation,
 * selected inversion with the low-rank correction, selected blocks, drift) for `batch`
 * configurations of `plan`, with every workspace and table in one static device array of
 * CL_NOALLOC_BYTES bytes per GPU instead of a batch. No device memory is allocated or
 * freed. links_dev, m_host, mu_host, selected_out_dev and drift_out_dev are as for
 * cl_factor and cl_run (either output may be NULL); status_host receives `batch` statuses
 * as cl_status gives them. The work runs on hip_stream (NULL: the null stream) and the
 * call returns after it has finished. A plan and batch whose workspace exceeds the array
 * is refused with CL_EINVAL (cl_last_error gives the bytes needed; 4^4 needs about 37 MiB
 * per configuration). The array is shared by every call on one GPU and keeps the last
 * call's contents: calls that overlap on one GPU (other threads, other streams) race and
 * must be serialised by the caller. */
#define CL_NOALLOC_BYTES (128u << 20)
int cl_run_noalloc(cl_plan plan, int32_t batch, const void* links_dev, const double* m_host,
                   const double* mu_host, void* selected_out_dev, void* drift_out_dev,
                   int32_t* status_host, void* hip_stream);
/* Waits for the batch's work and copies one status per active configuration:
 * 0, CL_ESINGULAR, CL_ENONFINITE or CL_ERANK. Returns 0 or an API error. */
int cl_status(cl_batch batch, int32_t* per_config_host);
/* Measurement support: with profiling on (eager path only), every launch of the
 * complex GEMM kernel in a selected mode is bracketed by HIP events on the batch
 * stream. gemm_modes is a bit mask: bit 0 = mode 0 (C = alpha*A*B [+ C0]: Schur
 * complements and the selected-inversion products), bit 1 = mode 1 (pivot-block
 * inverse times pivot rows), bit 2 = mode 2 (Gauss-Jordan elimination update);
 * 0 turns it off, 7 times every GEMM. _read waits for the stream, returns the
 * summed kernel time (ms), the summed algorithmic flops (8*M*N*K per product), the
 * summed algorithmic bytes (16 bytes per complex element: each operand read once,
 * the result written once, plus the C0 or base read where the mode has one) and the
 * number of timed launches since the last read, and resets the counters. */
int cl_batch_profile(cl_batch batch, int32_t gemm_modes);
int cl_batch_profile_read(cl_batch batch, double* gemm_ms, double* gemm_flops, double* gemm_bytes,
                          int64_t* launches);
/* The same launches one by one, in launch order, before _read resets them: fills up
 * to cap entries of ms, flops, bytes (host arrays of doubles) and mode (int32) and
 * sets *n to the number of timed launches (which may exceed cap). Waits for the
 * stream. NULL arrays are allowed only with cap == 0. */
int cl_batch_profile_launches(cl_batch batch, int64_t cap, double* ms, double* flops,
                              double* bytes, int32_t* mode, int64_t* n);
/* Test support (failure injection): in every following factorisation the assembled pivot
 * block of front `front` (an index of cl_plan_export table 0) of configuration `config` is
 * zero, as if D were singular there. front < 0 turns it off. The configuration then reports
 * CL_ESINGULAR (no perturbation: zero pivots) or CL_ERANK (more perturbed pivots than the
 * cap) with NaN outputs, and the other configurations are unaffected. */
int cl_batch_inject_fault(cl_batch batch, int32_t config, int32_t front);
/* Number of perturbed pivots of each active configuration in the last factorisation
 * (host array of batch entries; waits for the stream). */
int cl_batch_perturbations(cl_batch batch, int32_t* per_config_host);
/* Non-blocking: 1 if all work enqueued by the batch's last call has finished, 0 if
 * it is still running, negative on error. */
int cl_batch_query(cl_batch batch);
/* Waits for all work of the batch. */
int cl_batch_sync(cl_batch batch);
void cl_batch_destroy(cl_batch batch);

const char* cl_strerror(int code);
const char* cl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CLSEL_H */
