/*
 * kdqmc.h -- C ABI of the MI355X (gfx950) DQMC hot path for the attractive
 * Hubbard model on the L x L kagome lattice (N = 3 L^2 sites, 3-site cell).
 *
 * Method (Zhang, Li, Wang, "Accelerated quantum Monte Carlo simulations of
 * the attractive Hubbard model on the kagome lattice"):
 *   - the kinetic propagator exp(-dtau K) is applied to dense N x N matrices
 *     through the momentum-space block form of Eqs. (2)-(4): per vector, one
 *     2D FFT per sublattice, a 3x3 Bloch-block multiply per momentum, and
 *     the inverse FFT (Eq. (6), the product of Eq. (5));
 *   - the Ising auxiliary field is updated with the delay-update algorithm
 *     cited in Sec. II: accepted rank-one Green's-function updates are
 *     accumulated and added to G as one rank-k product.
 *
 * Conventions (all entry points):
 *   - Site order i = (x1*L + x2)*3 + s, s = 0,1,2 for sublattices A,B,C (the
 *     Kronecker order of Eq. (3)).  Matrices are row-major N x N.
 *   - Every pointer argument named *_dev is DEVICE memory owned by the
 *     caller; the library never allocates device memory.  All device work
 *     is enqueued on the stream given to kdqmc_init_lattice and is
 *     asynchronous: the caller synchronizes (kdqmc_sync) before reading
 *     results on the host.
 *   - Slices are 1-based: G(l) = [I + B_l ... B_1 B_{L_tau} ... B_{l+1}]^-1,
 *     B_l = exp(-dtau (K - mu)) exp(V_l), V_l = diag(alpha s_l),
 *     cosh(alpha) = exp(dtau |U| / 2) (discrete charge-channel decoupling).
 *   - Return value: KDQMC_OK (0) or a negative error code; the message of
 *     the last error on the calling thread is kdqmc_last_error().  A failed
 *     call leaves the context usable unless it returns KDQMC_EHIP.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Batched chains: a context made by kdqmc_init_batch holds n_chains
 *     independent Markov chains of one shape (same parameters except U);
 *     every call then acts on all of them at once (one launch per kernel,
 *     chains along the grid's z dimension).  Each device array argument then
 *     holds one record per chain, back to back, each laid out as documented
 *     for a single chain (record sizes: fields L_tau*N bytes, G N*N doubles,
 *     per-slice u/forced/accepted/ratio N elements, per-sweep ones L_tau*N,
 *     wrap_err 1 (kdqmc_stabilize) or L_tau/n_stab (kdqmc_sweep)).
 */
#ifndef KDQMC_H
#define KDQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KDQMC_OK = 0,
  KDQMC_EINVAL = -1,       /* bad argument (NULL, out of range, fields not +-1, ...) */
  KDQMC_EUNSUPPORTED = -2, /* lattice size or precision not compiled in */
  KDQMC_ESTATE = -3,       /* call out of order (slice index, stabilize point) */
  KDQMC_EHIP = -4,         /* a HIP runtime call failed */
  KDQMC_ENUMERIC = -5,     /* a stabilization found G drifted beyond the wrap-error
                              tolerance, or a non-finite value (see kdqmc_health) */
  KDQMC_ENOSPACE = -6      /* workspace smaller than kdqmc_workspace_bytes() */
};

typedef enum {
  KDQMC_FP64 = 0,       /* G, wrap, flush and stabilization in FP64 */
  KDQMC_MIXED_F16 = 1,  /* FP32 G and wrap; flush as split FP16 MFMA products
                           with FP32 accumulation; ratios and stabilization FP64 */
  KDQMC_MIXED_BF16 = 2  /* as MIXED_F16 with split BF16 products */
} kdqmc_prec;

typedef enum {
  KDQMC_KAGOME = 0,      /* 3 sites per cell, K of Eq. (3) */
  KDQMC_TRIANGULAR = 1,  /* 1 site per cell, K of App. A1 */
  KDQMC_HONEYCOMB = 2    /* 2 sites per cell, K of App. A2 */
} kdqmc_lattice;

typedef struct {
  int L;          /* cells per side; supported: 3, 6, 9, 12, 15, 18, 24 */
  double t;       /* hopping, K_ij = -t on nearest neighbours (Eq. (1)) */
  double U;       /* Hubbard interaction, U <= 0 (attractive) */
  double mu;      /* chemical potential (kdqmc_dirac_mu gives the Dirac energy) */
  double beta;    /* inverse temperature, beta = L_tau * dtau */
  double dtau;    /* imaginary-time step */
  int n_stab;     /* slices between stabilizations; must divide L_tau */
  int delay_k;    /* largest rank of one delayed flush, 1..512 */
  int window;     /* sites per decision window (at most 64), 0 = min(delay_k, 32) */
  int fft_tile;   /* complex vectors per wrap workgroup, 0 = automatic */
  int prec;       /* kdqmc_prec */
  int n_occ;      /* 0: finite temperature (grand canonical, beta = 1/T);
                     > 0: projector form of Sec. II with n_occ occupied trial
                     orbitals per spin (filling rho = 2 n_occ / N) projected
                     over beta (the projection length of Sec. III) */
  int lattice;    /* a kdqmc_lattice value, 0 = kagome: N = S L^2 sites with S = 3, 1, 2
                     sites per cell, ordered i = (x1 L + x2) S + s; the
                     measurements and kdqmc_trial_orbitals are kagome only */
} kdqmc_params;

typedef struct kdqmc_ctx kdqmc_ctx;

/* Bytes of device workspace the context needs for these parameters
 * (G, Bloch tables, fields, delay buffers, the two stabilization stacks of
 * L_tau/n_stab + 1 UDT entries each, and linear-algebra scratch).
 * Returns 0 for invalid parameters (kdqmc_last_error says why). */
size_t kdqmc_workspace_bytes(const kdqmc_params* p);

/* Bytes of device workspace for n_chains chains of one shape (1..65535):
 * n_chains per-chain blocks.  0 for invalid parameters. */
size_t kdqmc_workspace_bytes_batch(const kdqmc_params* p, int n_chains);

/* Projector form (Sec. II: the filling is set by a trial wave function that
 * occupies the lowest N_occ eigenstates of K, rho = 2 N_occ / N).
 * With params.n_occ > 0 the context computes
 *   G(l) = I - R(l) (L(l) R(l))^{-1} L(l),  R(l) = B_l ... B_1 P,
 *   L(l) = P^T B_{L_tau} ... B_{l+1},
 * (P: N x n_occ trial orbitals); the update, the flip ratio and the wrap are
 * those of the finite-temperature form, and the stabilization stacks hold
 * orthonormal N x n_occ panels (no scale factors).  G(L_tau) differs from
 * G(0): an upward pass runs from slice 0 to L_tau and ends there, a
 * downward pass from L_tau to 0, so passes alternate (upward first). */

/* Trial orbitals into P_host[N * n_occ] (host, row-major, site order above):
 * the lowest n_occ eigenvectors of K + eps (n_A - n_C) (a sublattice
 * potential on every cell; eps = 0.01 t splits the Dirac points of the
 * kagome bands, where the lowest N/3 levels of K end inside a degenerate
 * shell when 3 | L), as real orthonormal combinations of the Bloch states of
 * Eq. (4).  KDQMC_EINVAL if level n_occ is degenerate with level n_occ + 1. */
int kdqmc_trial_orbitals(int L, double t, int n_occ, double eps, double* P_host);

/* Loads the trial orbitals P_dev[N * n_occ] (device, row-major; one record
 * per chain for a batch) of a projector context.  Required before
 * kdqmc_set_fields; KDQMC_EINVAL for a finite-temperature context. */
int kdqmc_set_trial(kdqmc_ctx* c, const double* P_dev);

/* Chemical potential at the Dirac energy of the kagome bands: the energy at
 * which the two dispersive bands of the 3x3 Bloch block (Eq. (4)) touch,
 * -t (exact; the Dirac filling rho = 2/3 of Sec. IV). */
double kdqmc_dirac_mu(int L, double t);

/* Builds the Bloch tables (Eq. (4): H(k) per momentum; exp(-+dtau H(k)) and
 * exp(-dtau (H(k) - mu)) with the 1/L^2 of the FFT pair folded in), carves
 * the caller's workspace and binds the HIP stream (NULL = default stream).
 * The workspace must stay allocated until kdqmc_destroy.  No fields are set:
 * call kdqmc_set_fields (or kdqmc_set_G) next. */
int kdqmc_init_lattice(kdqmc_ctx** out, const kdqmc_params* p, void* workspace_dev,
                       size_t workspace_bytes, void* hip_stream);

/* As kdqmc_init_lattice for n_chains independent chains of the same shape
 * (the batched Monte Carlo of many Markov chains): U_host[n_chains] (host
 * memory, may be NULL = p->U for all) gives each chain's interaction, all
 * other parameters are shared.  The workspace must hold
 * kdqmc_workspace_bytes_batch(p, n_chains) bytes.  Array layouts of the
 * other calls: see "Batched chains" above. */
int kdqmc_init_batch(kdqmc_ctx** out, const kdqmc_params* p, int n_chains, const double* U_host,
                     void* workspace_dev, size_t workspace_bytes, void* hip_stream);

/* Chains held by the context (1 unless made by kdqmc_init_batch). */
int kdqmc_num_chains(const kdqmc_ctx* c);

/* Copies the Ising fields s_dev[L_tau][N] (int8, each +1 or -1), builds the
 * left stabilization stack from the top slice down, computes G(0) in FP64
 * from it, and sets the current slice to 0.  Invalid values -> KDQMC_EINVAL
 * (checked on the device; the call synchronizes for that check). */
int kdqmc_set_fields(kdqmc_ctx* c, const int8_t* s_dev);

/* Copies the current fields to s_dev[L_tau][N] (a checkpoint). */
int kdqmc_get_fields(kdqmc_ctx* c, int8_t* s_dev);

/* Loads an externally computed G(l) (FP64, N x N row-major) and sets the
 * current slice to l (0 <= l <= L_tau); for l > 0 an upward pass is then in
 * progress at slice l.  The stabilization stacks are not touched (they come
 * from kdqmc_set_fields and the passes); the next stabilization due becomes
 * the first one after slice l when the right stack holds the entries before
 * it, else the first of the pass. */
int kdqmc_set_G(kdqmc_ctx* c, const double* G_dev, int l);

/* The propagator wrap of Sec. II, Eqs. (5)-(6) applied on both sides of G:
 * G(l) = B_l G(l-1) B_l^{-1} with unchanged fields: the column pass applies
 * exp(V_l) then exp(-dtau K) to every column (batched 2D FFTs, 3x3 block
 * multiply, inverse FFTs), the row pass applies exp(+dtau K) to every row
 * (exp(dtau K) is symmetric).  Requires l == current slice + 1, and
 * KDQMC_ESTATE if slice l - 1 is a multiple of n_stab whose kdqmc_stabilize
 * call has not been made (the same holds for kdqmc_sweep_slice). */
int kdqmc_wrap_slice(kdqmc_ctx* c, int l);

/* One slice of the Monte Carlo sweep: the auxiliary-field update of the
 * delay-update algorithm cited in Sec. II, then the wrap of Eqs. (5)-(6)
 * (requires l == current slice + 1):
 * G~ = exp(V_l) G(l-1) exp(-V_l); sites i = 0..N-1 in order, in windows of
 * `window` sites; a flip of s_{l,i} is accepted iff u_dev[i] < ratio
 * (Metropolis) or, when forced_dev is not NULL, iff forced_dev[i] != 0;
 * ratio = exp(2 alpha s) R^2, R = 1 + Delta (1 - G~_ii),
 * Delta = exp(-2 alpha s) - 1, always in FP64.  Accepted rank-one updates
 * are accumulated and added to G~ as rank-<=delay_k products; then
 * G(l) = exp(-dtau K) G~ exp(dtau K).
 * u_dev[N] (float64) is required unless forced_dev[N] (uint8) is given;
 * accepted_dev[N] (uint8) and ratio_dev[N] (float64) are optional outputs. */
int kdqmc_sweep_slice(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                      uint8_t* accepted_dev, double* ratio_dev);

/* One slice of a downward pass (the same update read backwards, Eq. (5)'s
 * product traversed from slice L_tau to 1).  From G(l):
 * G~ = exp(dtau K) G(l) exp(-dtau K) = exp(V_l) G(l-1) exp(-V_l), the sites of
 * slice l are visited as in kdqmc_sweep_slice, then
 * G(l-1) = exp(-V_l') G~ exp(V_l') with the new fields V_l'.  A downward pass
 * starts from slice 0 (G(L_tau) = G(0)) with l = L_tau and continues with
 * l == current slice; afterwards the current slice is l - 1.  Arguments as in
 * kdqmc_sweep_slice.  KDQMC_ESTATE during an upward pass or when a
 * stabilization is due. */
int kdqmc_sweep_slice_down(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                           uint8_t* accepted_dev, double* ratio_dev);

/* Recomputes G(l) in FP64 for the current slice l of a pass from the
 * QR-stabilized stacks (UDT form, pre-pivoted Householder QR, Loh-Gubernatis
 * scale separation; the paper applies its propagator product, Eq. (5), inside
 * such chains but does not describe the stabilization itself), writes
 * max |G_current - G_fresh| to wrap_err_dev[0] (float64, optional) and
 * replaces G.  Synchronizes, then returns KDQMC_ENUMERIC when that wrap error
 * (of any chain) is not finite or above the tolerance (kdqmc_set_wrap_tolerance)
 * or a stabilization product had a non-finite column norm; G has been replaced
 * by the fresh FP64 value either way.  l must be a multiple of n_stab
 * reached by the pass (upward: n_stab..L_tau, downward: L_tau - n_stab..0),
 * with every earlier one of the pass stabilized, else KDQMC_ESTATE.  An
 * upward pass extends the right stack (B_l ... B_1) by one entry, a downward
 * pass the left stack ((B_{L_tau} ... B_{l+1})^T); the last stabilization of
 * a pass (l == L_tau upward, l == 0 downward) ends it at slice 0.  A stack
 * left stale by a pass in the other direction's absence (two upward passes
 * in a row) is rebuilt here from the current fields. */
int kdqmc_stabilize(kdqmc_ctx* c, double* wrap_err_dev);

/* A full upward sweep: kdqmc_sweep_slice for l = 1..L_tau with the uniforms
 * u_dev[L_tau][N] (float64) or forced_dev[L_tau][N], and kdqmc_stabilize
 * after every n_stab slices.  Optional outputs accepted_dev[L_tau][N],
 * ratio_dev[L_tau][N] and wrap_err_dev[L_tau / n_stab] (entry j - 1 for the
 * stabilization at slice j n_stab).  Requires the current slice to be 0
 * with no pass in progress. */
int kdqmc_sweep(kdqmc_ctx* c, const double* u_dev, const uint8_t* forced_dev,
                uint8_t* accepted_dev, double* ratio_dev, double* wrap_err_dev);

/* A full downward sweep: kdqmc_sweep_slice_down for l = L_tau..1 (the
 * uniforms and decisions of slice l at row l - 1 as above), kdqmc_stabilize
 * at every l - 1 that is a multiple of n_stab; wrap_err_dev[L_tau / n_stab]
 * has entry j for the stabilization at slice j n_stab.  Alternating upward
 * and downward sweeps keeps both stabilization stacks current without
 * rebuilding either. */
int kdqmc_sweep_down(kdqmc_ctx* c, const double* u_dev, const uint8_t* forced_dev,
                     uint8_t* accepted_dev, double* ratio_dev, double* wrap_err_dev);

/* Graph mode (default on): kdqmc_sweep captures its whole launch sequence
 * once per distinct set of pointer arguments into a HIP graph (on a
 * non-blocking stream the context creates) and replays it on the context's
 * stream; results are identical to the eager launches.  on = 0 launches
 * every kernel directly; while profiling is enabled sweeps also launch
 * directly (events inside a graph are not timed). */
int kdqmc_use_graphs(kdqmc_ctx* c, int on);

/* The equal-time Green's function from which the measurements of Secs. IV-V
 * are formed ("measurement" in the runtime breakdown of Sec. III): copies
 * G(current slice) to G_dev (FP64, N x N row-major, site order above). */
int kdqmc_measure_G(kdqmc_ctx* c, double* G_dev);

/* ---- equal-time measurements (Secs. IV-V) ----
 * Per-configuration estimators from the current G by Wick's theorem with
 * G_ab = <c_a c_b^+> for either spin (the charge decoupling keeps both spins
 * equal).  Real parts; the Monte-Carlo averages, the correlation ratio
 * R_Pair = 1 - S(Gamma + dk) / S(Gamma) and the order parameter
 * P = sqrt(S(Gamma) / N) of Sec. IV are formed from averages by the caller.
 *   SPAIR_*: S_Pair(Q) = (1/N) sum_ij e^{iQ.(r_i - r_j)}
 *            <c+_{i up} c+_{i dn} c_{j dn} c_{j up} + c_{j dn} c_{j up} c+_{i up} c+_{i dn}>
 *            (the symmetric form of Sec. IV) at Gamma and at the two
 *            smallest momenta Gamma + dk, dk = 2 pi b_1 / L and 2 pi b_2 / L;
 *   CDW2_*:  D(Q)^2 = <phi^+(Q) phi(Q)>, phi(Q) = (1/N) sum_cells e^{iQ.R}
 *            (n_A + e^{2 pi i/3} n_B + e^{4 pi i/3} n_C) (Sec. V), at Gamma and
 *            at the Dirac point K;
 *   DENSITY: particles per site, both spins.
 * Sites sit at x1 a1 + x2 a2 plus (0, 0), -a2/2, -a1/2 for A, B, C, with a1,
 * a2 at 60 degrees (every bond of Eq. (3) then has the same length). */
enum {
  KDQMC_OBS_SPAIR_GAMMA = 0,
  KDQMC_OBS_SPAIR_DK1 = 1,
  KDQMC_OBS_SPAIR_DK2 = 2,
  KDQMC_OBS_CDW2_GAMMA = 3,
  KDQMC_OBS_CDW2_K = 4,
  KDQMC_OBS_DENSITY = 5,
  KDQMC_NOBS = 6
};

/* Writes the KDQMC_NOBS estimators of G(current slice) to obs_dev[KDQMC_NOBS]
 * (device, float64; one record per chain for a batch).  Asynchronous; one
 * pass over G. */
int kdqmc_measure(kdqmc_ctx* c, double* obs_dev);

/* Numeric health.  Every stabilization (direct or inside kdqmc_sweep /
 * kdqmc_sweep_down) records its wrap error max |G_current - G_fresh| on the
 * device; one that is not finite or exceeds the context's tolerance, or a
 * non-finite column norm of a stabilization product, marks the chain.
 * Default tolerance: 1e-5 (FP64; the largest FP64 wrap error of the
 * workloads, U = -5 at 10-slice intervals, is about 1.4e-6), 1e-4 (mixed).  Sweeps do not
 * synchronize, so their marks are read here. */

/* Sets the largest accepted wrap error (tol > 0; INFINITY disables the check
 * of the size but keeps that of finiteness).  Captured sweep graphs are
 * dropped (they carry the old value). */
int kdqmc_set_wrap_tolerance(kdqmc_ctx* c, double tol);

/* Slice schedule of a single FP64 chain that uses the fused window launch
 * (the delayed update of the delay-update algorithm cited in Sec. II, one
 * flush per window): persistent != 0 runs each slice's window steps as one
 * resident launch (workgroups holding one to three 64 x 64 tiles of G in
 * registers for the slice, and one deciding workgroup, handing over through
 * counters in the workspace; possible when 1 + ceil(ceil(N/64)^2 / 3)
 * workgroups fit on the device at once, i.e. N <= 1728 on 256 compute
 * units, and the default then), 0 one launch per window.  Both
 * compute the same G, decisions and ratios bit for bit.  A wait that cannot
 * complete (the device shared with other resident work) is abandoned after a
 * bounded spin and leaves NaN in G, which the next stabilization reports as
 * KDQMC_ENUMERIC.  Returns 1 if the persistent launch is in use afterwards,
 * 0 if not, or a negative error code.  Captured sweep graphs are dropped. */
int kdqmc_set_slice_launch(kdqmc_ctx* c, int persistent);

/* Synchronizes; writes the largest wrap error of any chain since the last
 * call (or kdqmc_set_fields / kdqmc_set_G) to *worst_wrap_err (host, may be
 * NULL; NaN if one was not finite) and returns KDQMC_ENUMERIC if any chain was
 * marked in that time, else KDQMC_OK.  Clears the records. */
int kdqmc_health(kdqmc_ctx* c, double* worst_wrap_err);

/* Current slice index (0..L_tau), or a negative error code. */
int kdqmc_current_slice(const kdqmc_ctx* c);

/* Blocks until all work enqueued by this context has finished. */
int kdqmc_sync(kdqmc_ctx* c);

/* Frees the host-side context (not the caller's workspace). */
void kdqmc_destroy(kdqmc_ctx* c);

/* Message of the last failed call on this thread ("" if none). */
const char* kdqmc_last_error(void);

/* ---- profiling: HIP events around every kernel launch of the context ---- */

#define KDQMC_NPHASE 12
/* Phases: 0 wrap_cols, 1 wrap_rows (the two FFT passes of the wrap),
 * 2 decide, 3 extend, 4 prep (window decisions and delayed factors),
 * 5 flush (rank-k MFMA update), 6 bmul (B-chain products of the stacks),
 * 7 qr_panel, 8 gemm (stabilization linear algebra), 9 stabilize (whole
 * kdqmc_stabilize calls, which contain phases 6-8), 10 flush_decide (FP64
 * with a flush after every window: one launch per window that forms the
 * window's factors, flushes them and runs the next window's decisions),
 * 11 measure (kdqmc_measure). */

/* on != 0 starts recording (clearing earlier records); 0 stops. */
int kdqmc_profile_enable(kdqmc_ctx* c, int on);

/* Synchronizes, then writes the summed milliseconds ms[KDQMC_NPHASE] and the
 * launch counts launches[KDQMC_NPHASE] (host arrays) recorded since the last
 * enable/read, and clears the records. */
int kdqmc_profile_read(kdqmc_ctx* c, double* ms, int* launches);

/* Name of a phase index ("" if out of range). */
const char* kdqmc_phase_name(int phase);

/* ---- kernel-level entry points (the building blocks, for tests/tuning) ----
 * These act on caller matrices, not on chains: they need a single-chain
 * context (KDQMC_EINVAL otherwise). */

/* C(M x N) = alpha * op(A) op(B) + beta * C, FP64, row-major, on the
 * context's stream; op(X) = X or X^T (trans_* != 0).  lda/ldb/ldc are row
 * strides in elements.  FP64 MFMA kernel. */
int kdqmc_gemm_f64(kdqmc_ctx* c, int trans_a, int trans_b, int M, int N, int K, double alpha,
                   const double* A_dev, int lda, const double* B_dev, int ldb, double beta,
                   double* C_dev, int ldc);

/* The propagator product of Eq. (5) alone, by the three steps of Eq. (6):
 * A <- exp(sign dtau K) A for the first ncols columns of the N x N row-major
 * A_dev (row stride lda), sign = -1 or +1.  Needs a single-chain FP64
 * context (its tables).  The FFT side of the paper's Fig. 1 comparison. */
int kdqmc_expK_f64(kdqmc_ctx* c, double* A_dev, int lda, int ncols, int sign);

/* Householder QR of the n x n row-major A_dev (FP64) in place: on return
 * Q_dev holds Q (n x n), A_dev holds R in its upper triangle (zeros below).
 * No pivoting.  A_dev and Q_dev are N x N buffers (row stride N, N the
 * context's site count); the leading n x n block is factored (1 <= n <= N).
 * Uses the context's linear-algebra scratch. */
int kdqmc_qr_f64(kdqmc_ctx* c, int n, double* A_dev, double* Q_dev);

/* ---- for callers that cannot allocate device memory ----
 * Code under HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc cannot create a context (whose workspace the caller allocates).
 * This variant of kdqmc_qr_f64 needs no context: the same Householder QR
 * (same kernels, same result bit for bit) of the leading n x n block of A_dev
 * (row stride ld; R in its upper triangle, zeros below on return) with Q
 * (n x n, row stride ld) formed in Q_dev, enqueued on hip_stream (NULL = the
 * default stream).  Its scratch is a static device array of 4.6 MB held by
 * every GPU the library runs on until the process ends; nothing is allocated
 * and no allocating routine is called.  Limits: 1 <= n <= ld <= 512, else
 * KDQMC_EINVAL.  All calls on one GPU share that array: calls that overlap on
 * one GPU (concurrent streams, threads) race and must be serialized by the
 * caller. */
int kdqmc_qr_f64_noalloc(int n, int ld, double* A_dev, double* Q_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* KDQMC_H */
