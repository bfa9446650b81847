/*
 * pn.h -- C ABI of the MI355X (gfx950) library for batched, manifold-corrected
 * integration of spinning compact binaries in the conservative post-Newtonian
 * (PN) Hamiltonian formulation, with the two-nearby-trajectory fast Lyapunov
 * indicator (FLI) used in phase-space scans.
 *
 * Source: Ran, Liu & Zhong, "GPU accelerated manifold correction method for
 * spinning compact binaries", arXiv:1802.00147.
 *   Sec. 2, eq. (1)       Hamiltonian H = H_N + H_1PN + H_2PN + H_SO + H_SS
 *                         (3PN is not modelled; the 2.5PN reaction of eq. (6)
 *                         is optional, see pn_model)
 *   Sec. 2, eqs. (2)-(5)  spin-spin (S1S2) and quadrupole-monopole terms
 *   Sec. 2, eqs. (6)-(9)  Hamilton's equations and spin precession
 *   Sec. 2, eqs. (10)-(13) manifold correction (spin lengths; dual scaling)
 *   Sec. 3B               Newton iteration limit eps <= 1e-10
 *   Sec. 3C               FLI phase-space scans, chaos threshold 5.8 at t = 1e5
 *   Sec. 4, eq. (14)      gravitational-wave polarisations of recorded orbits
 * Beyond the paper: a persistent batch for orbits of uneven length, and a
 * neural surrogate of the scan's chaos label with integration as fallback.
 *
 * Units (Sec. 2): G = c = M = 1 with M = m1 + m2; r in M, p = P/mu, t in M,
 * H is the Hamiltonian per unit reduced mass mu.  beta = m1/m2 in (0, 1],
 * eta = mu/M.  Spin units: see pn_spin_units.
 *
 * State layout (all entry points): structure of arrays.  Component c of
 * orbit i is y[c * ld + i], c = 0..11 = (rx, ry, rz, px, py, pz, S1x, S1y,
 * S1z, S2x, S2y, S2z), ld >= n.  "[k][ld]" below means k rows of length ld.
 *
 * Memory: every array pointer is a DEVICE pointer (hipMalloc or a torch
 * CUDA tensor), 8-byte aligned; 256-byte alignment is recommended.  The
 * caller allocates and frees all device memory; the library allocates none
 * per call.  All work is enqueued on the given stream and is complete when
 * the stream is synchronised (calls that block are marked as such).  Inputs are not modified unless documented as
 * in/out.  Results depend only on each orbit's inputs and the settings, never
 * on the launch shape.
 *
 * Errors: every call returns a pn_status.  All argument validation happens on
 * the host before anything is launched; a call that returns PN_EINVAL has
 * touched no memory.  PN_EDEVICE reports a HIP launch error (the HIP error
 * text is available from pn_last_error()).  Physical failures of individual
 * orbits are not call errors: they are reported per orbit in the status
 * output (PN_ORBIT_*).
 */
#ifndef PN_H
#define PN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PN_OK = 0,
    PN_EINVAL = 1,   /* null pointer, n < 0 or n > 2^31 - 1, ld < n, parameter out of range, unknown enum */
    PN_ENOWS = 2,    /* workspace smaller than the documented size */
    PN_EDEVICE = 3   /* HIP error while launching */
} pn_status;

/* Per-orbit status codes (low byte) and flags. */
enum {
    PN_ORBIT_OK = 0,
    PN_ORBIT_MERGED = 1,        /* r fell below r_merge */
    PN_ORBIT_ESCAPED = 2,       /* r rose above r_esc */
    PN_ORBIT_NONFINITE = 3,     /* a state component became NaN or infinite */
    PN_ORBIT_UNBOUND_INIT = 4,  /* H(y0) >= 0: not a bound orbit (Sec. 3C removes these) */
    PN_ORBIT_BADPARAM = 5,      /* per-orbit beta / chi outside (0,1] / [0,1] */
    PN_ORBIT_NEWTON_NOCONV = 0x100 /* flag: some Newton solve hit max_iter */
};

/* Spin units.  The two choices describe the same Hamiltonian; they differ in
 * the unit of the spin variables and hence in the spin flow.
 *   PN_SPIN_PHYS:      spins in units of mu*M, |S_i| = chi_1 beta and chi_2 / beta;
 *                      dS_i/dt = (dH/dS_i) x S_i is the physical precession and
 *                      J = r x p + S1 + S2 is the conserved total angular momentum.
 *   PN_SPIN_PAPER_EQ8: spins in units of M^2, |S_i| = chi_i m_i^2; dH/dS_i is
 *                      exactly eqs. (8)-(9) and the flow is eq. (7) taken
 *                      literally (faster than the physical rate by 1/eta). */
typedef enum { PN_SPIN_PHYS = 0, PN_SPIN_PAPER_EQ8 = 1 } pn_spin_units;

typedef enum { PN_RK4 = 0, PN_RK5 = 1 } pn_method;

typedef enum {
    PN_CORR_NONE = 0,
    PN_CORR_SPIN = 1,  /* eq. (10) only */
    PN_CORR_SIX = 2,   /* eq. (10), then least-squares projection onto H = E0 and the
                          vector J = J0 followed by energy restoration by momentum scaling */
    PN_CORR_DUAL = 3   /* eq. (10), then the dual scaling of eqs. (11)-(13) */
} pn_corr_mode;

typedef enum { PN_THR_LITERAL = 0, PN_THR_LOG_T = 1 } pn_thr_scaling;

/* Terms of eq. (1).  pn_order: 0 Newtonian, 1 +1PN, 2 +1PN+2PN.
 * rad_reaction: 1 adds the 2.5PN radiation-reaction acceleration to dp/dt
 * (eq. 6; Sec. 3B, orbit 3).  The paper does not print it; this library uses
 * the leading-order reaction of a point-mass binary in the Iyer-Will gauge
 * family at (alpha, beta) = (4, 5), a = (8/5) eta / r^3 [(18 v^2 + 2/(3 r) -
 * 25 rdot^2) rdot n - (6 v^2 - 2/r - 15 rdot^2) v] with v = dH/dp (M = 1),
 * which radiates the quadrupole fluxes.  The system is then dissipative:
 * pn_rhs, pn_step and pn_trajectory accept it (with advancing references,
 * see pn_step); the FLI scans, batches and the surrogate integrate the
 * conservative system and return PN_EINVAL for it. */
typedef struct {
    int32_t pn_order;
    int32_t spin_orbit;  /* 1.5PN spin-orbit */
    int32_t spin_spin;   /* eq. (3) */
    int32_t quad_mono;   /* eqs. (4)-(5) */
    int32_t spin_units;  /* pn_spin_units */
    int32_t rad_reaction; /* 0 or 1 */
} pn_model;

/* Mass ratio and dimensionless spins.  Either per-orbit DEVICE arrays of
 * length n (all three non-NULL), or all three NULL and the host scalars
 * beta0, chi1_0, chi2_0 apply to every orbit.  Host scalars are validated
 * (beta in (0,1], chi in [0,1]); per-orbit values outside these ranges give
 * the orbit status PN_ORBIT_BADPARAM. */
typedef struct {
    const double* beta;
    const double* chi1;
    const double* chi2;
    double beta0, chi1_0, chi2_0;
} pn_params;

/* Fixed-step integrator.  PN_RK4: classical RK4.  PN_RK5: the paper's fifth-order
 * Runge-Kutta (Sec. 2, 3A), with the fifth-order weights of Dormand-Prince.
 * h > 0.  An integration to t_end takes ceil(t_end / h) steps. */
typedef struct {
    int32_t method;
    double h;
} pn_integrator;

/* Correction applied after every step (Sec. 2, eqs. 10-13).  tol is the
 * Newton iteration limit on the scale factors (the paper uses 1e-10, Sec. 3B);
 * max_iter caps each Newton solve (>= 1); sweeps (>= 1) is the number of
 * projection + momentum-scaling passes of PN_CORR_SIX; w1, w2 > 0 are the
 * weights of eq. (12) (the Newton root does not depend on them). */
typedef struct {
    int32_t mode;
    double tol;
    int32_t max_iter;
    int32_t sweeps;
    double w1, w2;
} pn_correction;

/* Fast Lyapunov indicator of two nearby trajectories (Sec. 3B-3C).  The shadow
 * starts at y0 + d0 e_{shadow_axis}; when the 12-component Euclidean separation
 * reaches d_renorm, log10(d/d0) is accumulated and the shadow is pulled back to
 * distance d0 along the same direction (its spin lengths and its own reference
 * integrals are then reset).  FLI(t_end) = sum + log10(d/d0).  An orbit is
 * labelled chaotic when FLI > threshold: thr_at_1e5 (5.8 in the paper) for
 * PN_THR_LITERAL, thr_at_1e5 + log10(t_end / 1e5) for PN_THR_LOG_T.  r_merge and
 * r_esc bound r (merged / escaped orbits are removed, Sec. 3C). */
typedef struct {
    double d0;
    double d_renorm;
    int32_t shadow_axis;
    double thr_at_1e5;
    int32_t thr_scaling;
    double r_merge;
    double r_esc;
} pn_fli_cfg;

/* Outputs of a scan.  fli, label, status are required; the rest may be NULL.
 *   fli[n]          FLI(t_end) (NaN for an orbit whose status is not OK)
 *   label[n]        1 chaotic, 0 regular, -1 invalid orbit
 *   status[n]       PN_ORBIT_* code, possibly with PN_ORBIT_NEWTON_NOCONV set
 *   y_final[12][ld] state of the orbit at t_end (or where it stopped)
 *   dH[n]           |H(y_final) - E0| / |E0|
 *   dJ[n]           |J(y_final) - J0| / |J0|
 *   newton_max[n]   largest Newton iteration count of any correction
 *   renorms[n]      number of shadow renormalisations
 *   trace[ntrace][ld] FLI after every trace_every steps (trace_every > 0;
 *                   entries past an orbit's last step are left untouched)
 *   steps[n]        steps the orbit completed (ceil(t_end / h) unless it was
 *                   removed; 0 for a state removed at t = 0) */
typedef struct {
    double* fli;
    int8_t* label;
    int32_t* status;
    double* y_final;
    double* dH;
    double* dJ;
    int32_t* newton_max;
    int64_t* renorms;
    double* trace;
    int64_t trace_every;
    int64_t ntrace;
    int64_t* steps;
} pn_scan_out;

/* Defaults used by the tests and benchmark (filled into caller structs). */
void pn_default_model(pn_model* m);
void pn_default_integrator(pn_integrator* in);
void pn_default_correction(pn_correction* c);
void pn_default_fli_cfg(pn_fli_cfg* f);

/* Initial conditions of a scan (Sec. 3B-3C, Sec. 4): r = (r0, 0, 0),
 * p = (0, p0, 0), S_i = |S_i| (sin th_i cos ph_i, sin th_i sin ph_i, cos th_i).
 * Inputs r0, p0, th1, ph1, th2, ph2 are [n] device arrays; output y0 [12][ld]. */
pn_status pn_init_state(const pn_model* model, pn_params params, int64_t n,
                        const double* r0, const double* p0, const double* th1,
                        const double* ph1, const double* th2, const double* ph2,
                        double* y0, int64_t ld, hipStream_t stream);

/* Right-hand side of Hamilton's equations and the spin precession (eqs. 6-9):
 * dydt = (dH/dp, -dH/dr, (dH/dS1) x S1, (dH/dS2) x S2).  y, dydt: [12][ld]. */
pn_status pn_rhs(const pn_model* model, pn_params params, int64_t n, const double* y,
                 int64_t ld, double* dydt, hipStream_t stream);

/* H and J = r x p + S1 + S2 per orbit.  H: [n]; J: [3][ld]. */
pn_status pn_invariants(const pn_model* model, pn_params params, int64_t n, const double* y,
                        int64_t ld, double* H, double* J, hipStream_t stream);

/* One manifold correction of each state against its reference integrals.
 * y: [12][ld] in/out.  ref: [4][ld] = (E0, J0x, J0y, J0z).  iters [n] (nullable):
 * total Newton iterations, negated when some solve hit max_iter. */
pn_status pn_manifold_correct(const pn_model* model, pn_params params,
                              const pn_correction* corr, int64_t n, double* y, int64_t ld,
                              const double* ref, int32_t* iters, hipStream_t stream);

/* nsteps integration steps of each state, each followed by the correction
 * (corr NULL or mode PN_CORR_NONE: no correction).  y: [12][ld] in/out.
 * ref: [4][ld] reference integrals, or NULL to capture them from y after its
 * spin lengths are set (only when a correction is requested).
 * With model->rad_reaction = 1 the references follow the dissipation
 * (integral-invariant relation, Sec. 3B): E and J advance with the state
 * through dE/dt = v.a and dJ/dt = r x a in the same Runge-Kutta step, the
 * correction targets the advanced values, and ref (when given) is in/out:
 * it holds the references at the end of the call.  Otherwise ref is only
 * read. */
pn_status pn_step(const pn_model* model, pn_params params, const pn_integrator* integ,
                  const pn_correction* corr, int64_t n, double* y, int64_t ld,
                  double* ref, int64_t nsteps, hipStream_t stream);

/* Fused FLI scan: for every orbit, integrate the orbit and its shadow from y0
 * to t_end with a correction after every step, and report the FLI, the
 * chaos label and the status (Sec. 3C).  y0: [12][ld] (not modified).
 * t_end: [n] device array, or NULL to use t_end_all for every orbit.
 * An orbit and its shadow run in two adjacent lanes of one wavefront. */
pn_status pn_fli_scan(const pn_model* model, pn_params params, const pn_integrator* integ,
                      const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                      const double* y0, int64_t ld, const double* t_end, double t_end_all,
                      const pn_scan_out* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Balanced scan of a grid whose orbits all integrate to the same end time
 * (the scans of Sec. 3C and Table 3).  Same computation and outputs as
 * pn_fli_scan, bit for bit; only the schedule differs.  With S steps per
 * orbit, the n orbits laid end to end form a tape of n S steps, and each of
 * P slots (an orbit pair of lanes) integrates a stretch of C >= n S / P steps
 * of it.  An orbit cut by the boundary between slots s and s + 1 is split as
 * in McNaughton's wrap-around rule: slot s + 1 integrates its first steps at
 * the start of its stretch and saves the pair state in the workspace, and
 * slot s integrates the rest, from that state, at the end of its stretch.
 * The stretches run in L launches of ceil(C / L) steps each; C - S >=
 * ceil(C / L) puts the two parts of every split orbit in different launches,
 * so no lane ever waits for another.  With P equal to the resident orbit
 * pairs of the device, every SIMD carries the same work, where the plain scan
 * of n > P equal orbits leaves a last round of resident wavefronts partly
 * filled.
 * ------------------------------------------------------------------------- */

/* Host-only plan: slot length C and launch count L for n orbits of `steps`
 * steps on `slots` slots.  C is the smallest length >= n steps / slots, raised
 * to steps + ceil(steps / 15) when smaller (the last slots then stay empty);
 * L is the smallest count in 2..16 with C - steps >= ceil(C / L).  PN_EINVAL
 * for n, steps or slots <= 0, slots > 2^24, n steps or slots C above 2^62. */
pn_status pn_balanced_plan(int64_t n, int64_t steps, int64_t slots, int64_t* slot_len, int32_t* launches);

/* Host-only: the piece that slot `slot` integrates at slot time tau of its
 * stretch (0 <= tau < its length, min(C, n steps - slot C)): steps
 * [*first_step, *end_step) of orbit *orbit, starting at slot time *start.
 * A piece with *first_step = 0 and *end_step < steps is the first part of a
 * split orbit (only ever at *start = 0), one with *first_step > 0 its second
 * part (the last piece of the stretch).  PN_EINVAL outside those ranges or
 * for slot_len <= steps. */
pn_status pn_balanced_piece(int64_t n, int64_t steps, int64_t slot_len, int64_t slot, int64_t tau,
                            int64_t* orbit, int64_t* first_step, int64_t* end_step, int64_t* start);

/* The schedule pn_fli_scan_balanced takes for n orbits to t_end_all:
 * *slots_used = P, *slot_len = C, *launches = L (outputs nullable).
 * slots = 0: P is the number of orbit pairs the balanced kernel keeps resident
 * on the current device, and the balanced schedule is taken only where its
 * predicted time (resident wavefronts per SIMD x C steps) is at least 2% below
 * the plain scan's (rounds of resident wavefronts x S steps); otherwise L = 0
 * and the call runs pn_fli_scan's kernel.  slots > 0: that many slots, always
 * balanced (for tests of the schedule; slots beyond residency simply run
 * later).  L = 0 also when n = 0 or S = 0.  PN_EINVAL for invalid arguments
 * or slots > 0 without a plan; PN_EDEVICE when slots = 0 and no device. */
pn_status pn_fli_scan_balanced_schedule(const pn_integrator* integ, const pn_correction* corr, int64_t n,
                                        double t_end_all, int64_t slots, int64_t* slots_used,
                                        int64_t* slot_len, int32_t* launches);

/* Bytes of workspace for a balanced scan on `slots` slots (the *slots_used of
 * pn_fli_scan_balanced_schedule): two tables of one pair record per slot,
 * about 320 bytes each.  0 for slots outside 1..2^24. */
size_t pn_fli_scan_balanced_workspace_size(int64_t slots);

/* pn_fli_scan of n orbits that all end at t_end_all, on the schedule
 * pn_fli_scan_balanced_schedule describes.  ws: device workspace of at least
 * pn_fli_scan_balanced_workspace_size(P) bytes, owned by the caller, contents
 * on entry irrelevant (the call first marks its records empty); may be NULL
 * when the schedule is the plain scan (L = 0).  Calls that share a workspace
 * must not overlap.  A saved part that is missing or names another orbit
 * (impossible with the planned launches) gives that orbit
 * PN_ORBIT_BADPARAM.  Errors as pn_fli_scan, plus PN_ENOWS for a short
 * workspace and the errors of pn_fli_scan_balanced_schedule. */
pn_status pn_fli_scan_balanced(const pn_model* model, pn_params params, const pn_integrator* integ,
                               const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                               const double* y0, int64_t ld, double t_end_all, const pn_scan_out* out,
                               int64_t slots, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Trajectories and gravitational waves (Sec. 4, eq. 14).
 * ------------------------------------------------------------------------- */

/* pn_step that also records the trajectory: after every `every` steps the
 * state is written to row k of traj ([rows][12][ld], row k = state after
 * (k + 1) * every steps, rows = nsteps / every).  traj: caller-owned device
 * array of rows * 12 * ld doubles (may be NULL when rows == 0); every >= 1.
 * y, ref, nsteps and errors as in pn_step. */
pn_status pn_trajectory(const pn_model* model, pn_params params, const pn_integrator* integ,
                        const pn_correction* corr, int64_t n, double* y, int64_t ld,
                        double* ref, int64_t nsteps, int64_t every, double* traj,
                        hipStream_t stream);

/* Gravitational-wave polarisations of eq. (14) from the leading
 * (mass-quadrupole) radiation field h_ij = (4 eta / D)(v_i v_j - n_i n_j / r)
 * (G = c = M = 1), with v = dr/dt = dH/dp of eq. (6) and eta = beta/(1+beta)^2:
 *   h_plus = 1/2 (p_i p_j - q_i q_j) h^TT_ij,  h_cross = 1/2 (p_i q_j + q_i p_j) h^TT_ij,
 * where N (nhat) points from the source to the observer, p (phat) lies along
 * the line of nodes and q = N x p.  nhat, phat: host 3-vectors, unit length
 * and orthogonal to 1e-12 (else PN_EINVAL).  dist: D in units of M (> 0).
 * y: [ns][12][ld] device array, ns sample rows of n states (e.g. the traj of
 * pn_trajectory); params per orbit (arrays of length >= n, indexed by the
 * column) or shared.  hp, hx: [ns][ld] device outputs, caller-owned; a column
 * whose per-orbit parameters are out of range gets NaN. */
pn_status pn_gw_polarizations(const pn_model* model, pn_params params, int64_t n, int64_t ns,
                              const double* y, int64_t ld, const double* nhat, const double* phat,
                              double dist, double* hp, double* hx, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batches of orbits of uneven length (persistent, work-stealing).
 * ------------------------------------------------------------------------- */

/* Launch shape of the persistent batch kernel.  block: threads per workgroup
 * (64, 128 or 256); waves_per_simd: wavefronts per SIMD in the grid (1 or 2;
 * with PN_RK4, 2 also selects the kernel build limited to 256 registers per
 * lane so that two stay resident); chunk_steps: steps a slot runs between
 * refills (>= 1). */
typedef struct {
    int32_t block;
    int32_t waves_per_simd;
    int32_t chunk_steps;
} pn_tuning;

void pn_default_tuning(pn_tuning* t);

/* Bytes of device workspace pn_batch_scan needs for n orbits. */
size_t pn_batch_workspace_size(int64_t n);

/* Resources of the fused scan kernel (pn_fli_scan) for one integrator and
 * correction mode on the current device, in the build that serves a shared
 * parameter set (every scan grid), as the runtime reports them:
 * vector registers per lane, scratch (spill) bytes per lane, and the
 * wavefronts per SIMD its 64-lane workgroups can keep resident.  Any output
 * pointer may be NULL (host memory).  PN_EINVAL for an unknown method or
 * mode, PN_EDEVICE without a device. */
pn_status pn_scan_kernel_resources(int32_t method, int32_t mode, int32_t* vgprs, int64_t* scratch_bytes,
                                   int32_t* waves_per_simd);

/* The same figures for the balanced scan's kernel (pn_fli_scan_balanced),
 * whose workgroups are 256 lanes (four wavefronts). */
pn_status pn_balanced_kernel_resources(int32_t method, int32_t mode, int32_t* vgprs, int64_t* scratch_bytes,
                                       int32_t* waves_per_simd);

/* Orbit pairs a pn_batch_scan launch keeps resident on the current device
 * with this tuning (NULL: the one pn_batch_scan would use): a batch of that
 * many equal orbits is one scheduling round.  0 when no device or an
 * invalid tuning. */
int64_t pn_batch_resident_pairs(const pn_tuning* tuning);

/* Same computation and outputs as pn_fli_scan (bitwise, for any tuning),
 * for orbits whose parameters and end times differ.  The orbits are ordered by
 * step count, longest first (binned, 8 bins per octave), into a queue in the
 * workspace; a persistent grid keeps every lane pair busy, claiming the next
 * orbit whenever its current one ends (one atomic per wavefront and refill).
 * t_end: [n] device array (required).  tuning: NULL uses the device's last
 * pn_autotune_batch result, else pn_default_tuning.  ws: device workspace of
 * at least pn_batch_workspace_size(n) bytes, owned by the caller; its contents
 * on entry are irrelevant; calls that share a workspace must not overlap.
 * Every orbit is claimed exactly once. */
pn_status pn_batch_scan(const pn_model* model, pn_params params, const pn_integrator* integ,
                        const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                        const double* y0, int64_t ld, const double* t_end, const pn_scan_out* out,
                        const pn_tuning* tuning, void* ws, size_t ws_bytes, hipStream_t stream);

/* Project-written autotuner: times the batch for block in {64, 128, 256} x
 * waves_per_simd in {1, 2} x chunk_steps in {32, 64, 256, 1024} with every
 * orbit's step count multiplied by step_scale (0 < step_scale <= 1), returns
 * the fastest in *best (and its time in *best_ms, nullable) and remembers it
 * for the current device.  Blocks the calling thread (synchronises the
 * stream).  The outputs in *out are overwritten with trial results. */
pn_status pn_autotune_batch(const pn_model* model, pn_params params, const pn_integrator* integ,
                            const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                            const double* y0, int64_t ld, const double* t_end, const pn_scan_out* out,
                            double step_scale, void* ws, size_t ws_bytes, pn_tuning* best,
                            float* best_ms, hipStream_t stream);

/* A batch captured once into a HIP graph (clear, bin, order, persistent scan)
 * and replayed with pn_graph_launch.  The pointers and sizes are frozen at
 * creation; the caller keeps every buffer alive until pn_graph_destroy.  The
 * graph holds only kernel nodes. */
typedef struct pn_graph pn_graph;
pn_status pn_batch_graph_create(const pn_model* model, pn_params params, const pn_integrator* integ,
                                const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                                const double* y0, int64_t ld, const double* t_end,
                                const pn_scan_out* out, const pn_tuning* tuning, void* ws,
                                size_t ws_bytes, pn_graph** graph);
pn_status pn_graph_launch(pn_graph* graph, hipStream_t stream);
void pn_graph_destroy(pn_graph* graph);

/* pn_batch_scan without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): the queue and the processing order live
 * in a static device array of the library, one per device, sized for at most
 * 2^20 orbits (4.2 MB); n above that returns PN_EINVAL (pn_last_error says
 * why) before anything is launched.  The call allocates nothing.  Every call
 * on a device shares that device's array: calls that overlap on one device
 * (on different streams, or from several threads) race and must be
 * serialised by the caller.  Arguments, outputs and results otherwise as
 * pn_batch_scan. */
pn_status pn_batch_scan_noalloc(const pn_model* model, pn_params params, const pn_integrator* integ,
                                const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                                int64_t ld, const double* t_end, const pn_scan_out* out, const pn_tuning* tuning,
                                hipStream_t stream);

/* Checkpoint and resume of a batch scan.  Long scans (t_end up to 1e6 steps
 * per orbit) can be interrupted after a bounded amount of work, saved, and
 * continued later, in the same process or after the workspace and outputs
 * were copied to host memory and back, with results identical bit for bit to
 * one uninterrupted pn_batch_scan (per-orbit arithmetic never depends on the
 * schedule, and the saved state is the exact state of every orbit in flight).
 *
 * Bytes of workspace for n orbits: the batch queue plus two tables of
 * min(n, 2^18) orbit records (324 bytes each). */
size_t pn_batch_ckpt_workspace_size(int64_t n);

/* pn_batch_scan with a checkpoint in ws (>= pn_batch_ckpt_workspace_size(n)
 * bytes, device memory owned by the caller).
 *   resume = 0: start the scan (the contents of ws on entry are irrelevant);
 *   resume = 1: continue the scan whose state a previous call left in ws; the
 *               model, parameters, settings, y0, t_end and out must be the
 *               same arrays (or copies) as in the call that started it; the
 *               tuning may differ.
 *   max_chunks > 0: every wavefront stops after max_chunks refills of
 *               tuning.chunk_steps steps; orbits still running are saved into
 *               ws, finished orbits have their results in *out.
 *   max_chunks = 0: run every remaining orbit to its end.
 * The scan is complete when pn_batch_scan_pending reports 0.  Traces are not
 * supported (out->trace_every must be 0).  Errors as pn_batch_scan, plus
 * PN_EINVAL for resume outside {0, 1} or max_chunks < 0. */
pn_status pn_batch_scan_resumable(const pn_model* model, pn_params params, const pn_integrator* integ,
                                  const pn_correction* corr, const pn_fli_cfg* fli, int64_t n,
                                  const double* y0, int64_t ld, const double* t_end,
                                  const pn_scan_out* out, const pn_tuning* tuning, int32_t resume,
                                  int32_t max_chunks, void* ws, size_t ws_bytes, hipStream_t stream);

/* Orbits of a resumable scan not finished yet (saved in flight plus never
 * started), read from ws after synchronising the stream (blocks). */
pn_status pn_batch_scan_pending(const void* ws, int64_t n, int64_t* pending, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate: a multilayer perceptron 7 -> 256 -> 256 -> 256 -> 2
 * (ReLU) that maps scan-point features to (chaos logit, FLI - log10 t_end),
 * trained on FLIs the scan itself produced, with integration as fallback.
 * Matrix products: bfloat16 operands, FP32 accumulation on MFMA.
 * ------------------------------------------------------------------------- */

/* Device buffers of the network, all owned by the caller.  Layer l (0..3) has
 * in_l = 7, 256, 256, 256 inputs and out_l = 256, 256, 256, 2 outputs.
 *   w[l]  FP32 master weights [out_l][in_l] row-major;  b[l]  FP32 biases [out_l]
 *   wb[l] bfloat16 copies of w[l] (bit patterns, uint16) read by the products
 *   mw, vw, mb, vb  Adam first/second moments of w and b (training only). */
typedef struct {
    float* w[4];
    float* b[4];
    uint16_t* wb[4];
    float* mw[4];
    float* vw[4];
    float* mb[4];
    float* vb[4];
} pn_mlp;

/* Elements of layer l's weights (which = 0) or biases (which = 1); 0 if l is
 * out of range. */
size_t pn_mlp_param_count(int32_t layer, int32_t which);

/* Refresh wb[] from w[] (round to nearest even bfloat16). */
pn_status pn_mlp_sync_bf16(pn_mlp* net, hipStream_t stream);

/* Standardised features of scan points into feat [n][8] (FP32, column 7 = 0):
 * (beta, chi1, chi2, r0, cos th1, cos th2, log10 t_end), each (x - mean[c]) /
 * stdv[c] with host arrays mean[7], stdv[7] (stdv > 0).  Point j takes row idx[j]
 * of the parameter arrays (idx NULL: row j).  t_end: [rows] array or NULL for
 * t_end_all > 0. */
pn_status pn_mlp_features(pn_params params, int64_t n, const double* r0, const double* th1,
                          const double* th2, const double* t_end, double t_end_all,
                          const int32_t* idx, const float* mean, const float* stdv, float* feat,
                          hipStream_t stream);

/* Training targets from a scan's outputs: lab[i] = 1 if label[i] == 1 else 0,
 * target[i] = fli[i] - log10 t_end (0 where the FLI is not finite).  t_end:
 * [n] array or NULL for t_end_all > 0. */
pn_status pn_mlp_targets(const double* fli, const int8_t* label, const double* t_end, double t_end_all,
                         int64_t n, float* lab, float* target, hipStream_t stream);

/* Bytes of workspace for one training step of `batch` samples. */
size_t pn_mlp_train_workspace_size(int32_t batch);

/* Byte offsets inside a pn_mlp_train_step workspace (of the same batch) of
 * the tensors a step leaves there, readable once the step has completed on
 * its stream (row-major, one row per batch sample):
 *   off[0]     X: the gathered features as bfloat16 [batch][8] (column 7 zero);
 *   off[1..3]  h1, h2, h3: the hidden activations after ReLU, bfloat16 [batch][256];
 *   off[4]     out: the outputs (logit, FLI - log10 t_end), FP32 [batch][2];
 *   off[5]     g4: d loss / d out, bfloat16 [batch][2];
 *   off[6..8]  g3, g2, g1: d loss / d (pre-activation of hidden layer 3, 2, 1),
 *              bfloat16 [batch][256].
 * The weight gradient of layer l is g_(l+1)^T a_l (a_0 = X, a_l = h_l) and
 * its bias gradient the column sums of g_(l+1); both are consumed by the
 * step's Adam update (the first step's moments are 0.1 g and 0.001 g^2).
 * off: 9 entries, caller-owned.  PN_EINVAL if batch <= 0 or off is NULL. */
pn_status pn_mlp_train_workspace_layout(int32_t batch, size_t* off);

/* One training step on rows idx[0..batch) of feat [rows][8] (16-byte aligned,
 * else PN_EINVAL), label [rows]
 * (1 chaotic, 0 regular) and target [rows] (FLI - log10 t_end): forward,
 * loss (binary cross-entropy of output 0 + Huber, delta 1, of output 1,
 * mean over the batch), backward, and an Adam update (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias correction for step >= 1) of w and b, with wb refreshed.
 * The batch's mean loss is ADDED to the device scalar *loss. */
pn_status pn_mlp_train_step(pn_mlp* net, const float* feat, const float* label, const float* target,
                            const int32_t* idx, int32_t batch, int32_t step, float lr, float* loss,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* nbatch training steps in one call, as pn_mlp_train_step each: batch b
 * (0 <= b < nbatch) trains on rows order[b * batch .. (b + 1) * batch) of
 * feat/label/target, with Adam step *adam_step + 1 + b; *adam_step (host,
 * in/out) is advanced by the steps done.  The batches' mean losses are ADDED
 * to the device scalar *loss.  order: device int32 array of nbatch * batch
 * row indices (the caller's data-loader order).  ws as for
 * pn_mlp_train_step(batch).  The first failing step's status is returned. */
pn_status pn_mlp_train(pn_mlp* net, int32_t* adam_step, const float* feat, const float* label,
                       const float* target, const int32_t* order, int64_t nbatch, int32_t batch,
                       float lr, float* loss, void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace for inference in chunks of `chunk` rows. */
size_t pn_mlp_infer_workspace_size(int64_t chunk);

/* Network outputs out [n][2] (FP32) for feat [n][8], `chunk` rows at a time. */
pn_status pn_mlp_infer(const pn_mlp* net, const float* feat, int64_t n, float* out, int64_t chunk,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/* The same outputs as pn_mlp_infer, bit for bit for finite features (a row
 * with a non-finite feature may differ between the two paths), from one
 * persistent kernel
 * that runs all four layers on 32-row tiles with the activations in LDS and
 * the hidden-layer weights in registers, layers 1-2 and layers 3-4 on two
 * halves of each workgroup as a two-stage pipeline.  No workspace;
 * feat [n][8] (16-byte aligned, else PN_EINVAL), out [n][2] device arrays
 * owned by the caller. */
pn_status pn_mlp_infer_fused(const pn_mlp* net, const float* feat, int64_t n, float* out,
                             hipStream_t stream);

/* Gate of the surrogate-assisted scan: label[i] = (out[i][0] > 0), fli_pred[i]
 * = out[i][1] (nullable), and every point with |logit| < margin or drawn for
 * the audit (SplitMix64(seed + i) / 2^64 < audit_frac) appended to list[]
 * (order unspecified); *count (device) receives the number appended. */
pn_status pn_surrogate_gate(const float* out, int64_t n, float margin, double audit_frac,
                            uint64_t seed, int8_t* label, float* fli_pred, int32_t* list,
                            unsigned long long* count, hipStream_t stream);

/* label[list[j]] = integrated[j] for j < m (the integrated labels win). */
pn_status pn_surrogate_merge(const int32_t* list, int64_t m, const int8_t* integrated, int8_t* label,
                             hipStream_t stream);

/* The matrix-core product used above, exposed for testing:
 * C = A B (+ bias[n]) (ReLU if relu) (times [mask(m,n) > 0] if mask), M x N,
 * A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (bfloat16 bit
 * patterns), FP32 accumulation; Cf (FP32, ld ldcf) and/or Cb (bfloat16). */
pn_status pn_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int64_t sam, int64_t sak,
                       const uint16_t* B, int64_t sbk, int64_t sbn, const float* bias, int32_t relu,
                       const uint16_t* mask, int64_t ldm, float* Cf, int64_t ldcf, uint16_t* Cb,
                       int64_t ldcb, hipStream_t stream);

/* Settings of pn_surrogate_scan (defaults from pn_default_surrogate_cfg). */
typedef struct {
    float margin;            /* points with |logit| < margin are integrated (0.5) */
    double audit_frac;       /* audit: SplitMix64(seed + i) / 2^64 < audit_frac (0.01) */
    uint64_t seed;           /* audit seed (5) */
    int32_t refine_epochs;   /* passes of training on the integrated audit (40; 0: none) */
    int32_t refine_batch;    /* samples per refinement step (2048) */
    float refine_lr;         /* Adam learning rate of the refinement (5e-4) */
    uint64_t refine_seed;    /* SplitMix64 seed of the sample order (51) */
    int32_t refine_cosine;   /* 1: learning rate refine_lr (1 + cos(pi e / epochs)) / 2 in
                                epoch e; 0: constant (0) */
    int64_t audit_split;     /* 0: the whole audit is integrated before the refinement (0);
                                1: only the largest whole number of rounds of the batch
                                kernel's resident orbit pairs (pn_batch_resident_pairs)
                                is, and the refinement sees only those; the rest of the
                                audit is integrated with the uncertain points, so that
                                only one of the two integrations ends in a partly idle
                                round; k > 1: as 1 with rounds of k points */
} pn_surrogate_cfg;

void pn_default_surrogate_cfg(pn_surrogate_cfg* cfg);

/* What one pn_surrogate_scan call did, from events on its stream and counts
 * read back by the call.  Index 0 is the audit integration (step 2), index 1
 * the fallback integration (step 5).
 *   phase_ms[4]     milliseconds of the audit (features, draw, integration),
 *                   the refinement, inference with the gate, and the
 *                   fallback integration (gathers and merge included)
 *   scan_ms[2]      milliseconds of the FP64 scan launches alone (the scan
 *                   call of each integration, nothing else)
 *   scan_kernel[2]  0 none, 1 the plain fused scan (k_fli_scan), 2 the
 *                   balanced schedule (k_wrap_scan), 3 the persistent batch
 *                   (k_batch_scan)
 *   scan_launches[2] launches of that scan kernel
 *   points[2]       points integrated
 *   orbit_steps[2]  orbit-steps integrated (the sum of the points' completed
 *                   steps; a removed orbit counts the steps it took) */
typedef struct {
    float phase_ms[4];
    float scan_ms[2];
    int32_t scan_kernel[2];
    int32_t scan_launches[2];
    int64_t points[2];
    int64_t orbit_steps[2];
} pn_surrogate_stats;

/* Bytes of workspace for pn_surrogate_scan over n points (0 if n is out of
 * range or refine_batch <= 0). */
size_t pn_surrogate_scan_workspace_size(int64_t n, int32_t refine_batch);

/* The surrogate-assisted scan of n points, end to end on the stream:
 *  1. features of every point (pn_mlp_features with mean/stdv);
 *  2. the audit sample (SplitMix64(seed + i) / 2^64 < audit_frac), sorted by
 *     point index, integrated: with t_end NULL (every point ends at
 *     t_end_all) by pn_fli_scan_balanced on the device's resident slots
 *     (the plain fused scan where that is predicted faster), else by the
 *     persistent batch scan (pn_batch_scan, cached tuning); the same for
 *     step 5 (all three give the same results bit for bit);
 *  3. refine_epochs passes of training (pn_mlp_train_step, Adam steps counted
 *     in *adam_step) on the valid audited orbits, in an order drawn from
 *     SplitMix64(refine_seed) (Fisher-Yates per epoch), when at least
 *     refine_batch of them were drawn;
 *  4. fused inference (pn_mlp_infer_fused); label[i] = (logit > 0);
 *  5. points with |logit| < margin not in the audit are integrated;
 *     integrated labels (-1 for removed orbits) replace the network's.
 * Point i has initial data r0[i], p0[i], th1[i], ph1[i], th2[i], ph2[i] (as
 * pn_init_state), parameters `params` (shared or per point), end time
 * t_end[i] or t_end_all.  label: [n] int8 device output; *integrated: host
 * output, the number of points integrated; points (nullable): [n] int32
 * device output whose first *integrated entries are the integrated points
 * (the sorted audit, then the uncertain ones); stats (nullable): host
 * output, timings and counts of the call (pn_surrogate_stats).  net is
 * updated by the refinement.  ws: caller-owned device workspace of at least
 * pn_surrogate_scan_workspace_size(n, cfg->refine_batch) bytes.  Blocks the
 * calling thread (it reads the audit and gate counts back); calls sharing a
 * workspace or a network must not overlap.  Errors: PN_EINVAL for invalid
 * arguments (checked before anything is launched), PN_ENOWS, PN_EDEVICE. */
pn_status pn_surrogate_scan(pn_mlp* net, int32_t* adam_step, const pn_model* model, pn_params params,
                            const pn_integrator* integ, const pn_correction* corr,
                            const pn_fli_cfg* fli, int64_t n, const double* r0, const double* p0,
                            const double* th1, const double* ph1, const double* th2,
                            const double* ph2, const double* t_end, double t_end_all,
                            const float* mean, const float* stdv, const pn_surrogate_cfg* cfg,
                            int8_t* label, int32_t* points, int64_t* integrated, pn_surrogate_stats* stats,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* Initial states of selected points: like pn_init_state, but point j takes
 * row idx[j] of r0, p0, th1, ph1, th2, ph2 (and of per-orbit parameters). */
pn_status pn_init_state_gather(const pn_model* model, pn_params params, int64_t m, const int32_t* idx,
                               const double* r0, const double* p0, const double* th1,
                               const double* ph1, const double* th2, const double* ph2, double* y0,
                               int64_t ld, hipStream_t stream);

/* Library version and last error text (thread-local; "" when none). */
/* Bytes of device workspace pn_fli_scan needs for n orbits: 0 (the fused scan
 * keeps everything in registers; the call exists so that callers can size
 * workspaces uniformly). */
size_t pn_fli_scan_workspace_size(int64_t n);

/* Forget the per-device autotune results kept by pn_autotune_batch (later
 * batches use pn_default_tuning until the next autotune).  The library holds
 * no other state. */
void pn_shutdown(void);

int32_t pn_version(void);
const char* pn_status_string(pn_status s);
const char* pn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PN_H */
