// pn_kernels.hip -- gfx950 kernels of the FP64 path and the C ABI of
// include/pn.h (except the network's entry points, in pn_mlp.hip).
//
// One lane integrates one trajectory: in the scans an orbit and its shadow
// occupy two adjacent lanes and trade state through DPP; the whole
// 12-component state, the Runge-Kutta stages and the correction live in
// registers; global memory is touched only to read initial states and to
// write results, in structure-of-arrays rows (coalesced across a wavefront).
// The physics path is scalar FP64 end to end.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "pn.h"
#include "pn_device.h"

// Text of the last device error of the calling thread, shared by every
// translation unit of the library and returned by pn_last_error().
namespace pn_detail {
thread_local char g_last_error[256] = "";
void set_last_error(const char* what, const char* msg) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, msg);
}
}  // namespace pn_detail

namespace {

constexpr int kBlock = 64;  // one wavefront per workgroup

void set_error(const char* what, hipError_t e) { pn_detail::set_last_error(what, hipGetErrorString(e)); }

// Parameters of a kernel: either per-orbit device arrays, or one shared
// coefficient table computed on the host (held in scalar registers).
struct ParamArgs {
    const double* beta;
    const double* chi1;
    const double* chi2;
    PnCoef coef;
    pn_model model;
};

__device__ __forceinline__ bool load_coef(const ParamArgs& pa, int64_t i, PnCoef& k) {
    if (pa.beta == nullptr) {
        k = pa.coef;
        return true;
    }
    return pn_make_coef(pa.model, pa.beta[i], pa.chi1[i], pa.chi2[i], k);
}

__device__ __forceinline__ void load_state(const double* y, int64_t ld, int64_t i, double* s) {
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = y[c * ld + i];
}

__device__ __forceinline__ void store_state(double* y, int64_t ld, int64_t i, const double* s) {
#pragma unroll
    for (int c = 0; c < 12; ++c) y[c * ld + i] = s[c];
}

__device__ __forceinline__ void capture_ref(const PnCoef& k, const double* y, double* ref) {
    ref[0] = pn_energy(k, y);
    pn_total_J(y, ref + 1);
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init_state(ParamArgs pa, int64_t n, const int32_t* idx,
                                                      const double* r0, const double* p0, const double* th1,
                                                      const double* ph1, const double* th2,
                                                      const double* ph2, double* y, int64_t ld) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t i = idx ? (int64_t)idx[j] : j;   // row of the inputs; output column j
    PnCoef k;
    load_coef(pa, i, k);
    double s[12];
    s[0] = r0[i]; s[1] = 0.0; s[2] = 0.0;
    s[3] = 0.0; s[4] = p0[i]; s[5] = 0.0;
    double sa, ca, sb, cb;
    sincos(th1[i], &sa, &ca);
    sincos(ph1[i], &sb, &cb);
    s[6] = k.s1 * sa * cb; s[7] = k.s1 * sa * sb; s[8] = k.s1 * ca;
    sincos(th2[i], &sa, &ca);
    sincos(ph2[i], &sb, &cb);
    s[9] = k.s2 * sa * cb; s[10] = k.s2 * sa * sb; s[11] = k.s2 * ca;
    store_state(y, ld, j, s);
}

// eta = m1 m2 (M = 1) of orbit i: from its mass ratio, or the shared value.
__device__ __forceinline__ double orbit_eta(const ParamArgs& pa, int64_t i, double eta0) {
    if (pa.beta == nullptr) return eta0;
    const double b = pa.beta[i];
    return b / ((1.0 + b) * (1.0 + b));
}

__global__ __launch_bounds__(kBlock) void k_rhs(ParamArgs pa, int64_t n, const double* y, int64_t ld,
                                               double* f, double eta0) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    PnCoef k;
    load_coef(pa, i, k);
    double s[12], d[12];
    load_state(y, ld, i, s);
    pn_rhs_eval(k, s, d);
    if (pa.model.rad_reaction) {
        double a[3];
        pn_rr_accel(orbit_eta(pa, i, eta0), s, d, a);
        d[3] += a[0]; d[4] += a[1]; d[5] += a[2];
    }
    store_state(f, ld, i, d);
}

__global__ __launch_bounds__(kBlock) void k_invariants(ParamArgs pa, int64_t n, const double* y,
                                                      int64_t ld, double* H, double* J) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    PnCoef k;
    load_coef(pa, i, k);
    double s[12], j[3];
    load_state(y, ld, i, s);
    H[i] = pn_energy(k, s);
    pn_total_J(s, j);
    J[i] = j[0];
    J[ld + i] = j[1];
    J[2 * ld + i] = j[2];
}

struct CorrArgs {
    double tol;
    int32_t max_iter;
    int32_t sweeps;
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_correct(ParamArgs pa, CorrArgs ca, int64_t n, double* y,
                                                   int64_t ld, const double* ref, int32_t* iters) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    PnCoef k;
    load_coef(pa, i, k);
    double s[12], r[4];
    load_state(y, ld, i, s);
#pragma unroll
    for (int c = 0; c < 4; ++c) r[c] = ref[c * ld + i];
    bool nc = false;
    const int it = pn_correct<MODE>(k, s, r, ca.tol, ca.max_iter, ca.sweeps, nc);
    store_state(y, ld, i, s);
    if (iters) iters[i] = nc ? -it : it;
}

// nsteps corrected steps per orbit; with traj set, the state after every
// `every` steps also goes to row (t / every - 1) of traj ([rows][12][ld]).
// RR: the dissipative system (2.5PN reaction); the references advance with
// the state (z = (y, E, J), one RK step for all 16 components) and are
// written back to ref when it is given.
template <int METHOD, int MODE, bool RR>
__global__ __launch_bounds__(kBlock) void k_step(ParamArgs pa, CorrArgs ca, double h, int64_t n,
                                                double* y, int64_t ld, double* ref,
                                                int64_t nsteps, double* traj, int64_t every, double eta0) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    PnCoef k;
    load_coef(pa, i, k);
    double z[RR ? 16 : 12];
    double* const s = z;
    double rloc[4];
    double* const r = RR ? z + 12 : rloc;
    load_state(y, ld, i, s);
    if (ref) {
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = ref[c * ld + i];
    } else {
        if (MODE != PN_CORR_NONE) pn_correct_spins(k, s);
        capture_ref(k, s, r);
    }
    const double eta = RR ? orbit_eta(pa, i, eta0) : 0.0;
    int64_t left = every;
    double* row = traj;
    for (int64_t t = 0; t < nsteps; ++t) {
        if constexpr (RR)
            pn_rk_step_rr<METHOD>(k, eta, z, h);
        else
            pn_rk_step<METHOD>(k, s, h);
        bool nc;
        pn_correct<MODE>(k, s, r, ca.tol, ca.max_iter, ca.sweeps, nc);
        if (row != nullptr && --left == 0) {
            store_state(row, ld, i, s);
            row += 12 * ld;
            left = every;
        }
    }
    store_state(y, ld, i, s);
    if (RR && ref) {
#pragma unroll
        for (int c = 0; c < 4; ++c) ref[c * ld + i] = r[c];
    }
}

// Gravitational-wave polarisations (Sec. 4, eq. 14) of the mass-quadrupole
// field h_ij = (4 eta / D)(v_i v_j - n_i n_j / r), v = dH/dp (eq. 6).  With p
// and q transverse to the line of sight the contractions of eq. (14) see only
// the transverse-traceless part, so they are taken on h_ij directly:
//   h_plus  = (2 eta / D) [(p.v)^2 - (q.v)^2 - ((p.n)^2 - (q.n)^2) / r]
//   h_cross = (4 eta / D) [(p.v)(q.v) - (p.n)(q.n) / r].
// One thread per (sample row, orbit) of y[ns][12][ld].
struct GwArgs {
    double px, py, pz, qx, qy, qz;   // line of nodes p and q = N x p
    double inv_dist;                 // 1 / D
    double eta0;                     // eta of a shared parameter set
};

// Orbit i = blockIdx.x * 256 + threadIdx.x, rows blockIdx.y, + gridDim.y, ...:
// consecutive lanes read consecutive orbits of one recorded row.
__global__ __launch_bounds__(256) void k_gw(ParamArgs pa, GwArgs ga, int64_t n, int64_t ns, const double* y,
                                            int64_t ld, double* hp, double* hx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    PnCoef k;
    const bool ok = load_coef(pa, i, k);
    double eta = ga.eta0;
    if (pa.beta != nullptr) {
        const double b = pa.beta[i];
        eta = b / ((1.0 + b) * (1.0 + b));
    }
    const double a = eta * ga.inv_dist;
    for (int64_t row = blockIdx.y; row < ns; row += gridDim.y) {
        double s[12], f[12];
        load_state(y + row * 12 * ld, ld, i, s);
        pn_rhs_eval(k, s, f);
        const double u = pn_rsqrt(dot3(s[0], s[1], s[2], s[0], s[1], s[2]));
        const double pv = dot3(ga.px, ga.py, ga.pz, f[0], f[1], f[2]);
        const double qv = dot3(ga.qx, ga.qy, ga.qz, f[0], f[1], f[2]);
        const double pr = dot3(ga.px, ga.py, ga.pz, s[0], s[1], s[2]) * u;
        const double qr = dot3(ga.qx, ga.qy, ga.qz, s[0], s[1], s[2]) * u;
        const double hplus = 2.0 * a * ((pv * pv - qv * qv) - (pr * pr - qr * qr) * u);
        const double hcross = 4.0 * a * (pv * qv - pr * qr * u);
        hp[row * ld + i] = ok ? hplus : __builtin_nan("");
        hx[row * ld + i] = ok ? hcross : __builtin_nan("");
    }
}

struct FliArgs {
    double h;
    CorrArgs corr;
    double d0, d_renorm2, rmerge2, resc2;
    double thr_at_1e5;
    int32_t thr_scaling;
    int32_t shadow_axis;
    const double* t_end;
    double t_end_all;
    pn_scan_out out;
    int64_t n, ld;
    const double* y0;
    double step_scale;      // 1 for real runs; < 1 shortens every orbit (autotune trials)
};

// Exchange a value with the partner lane (lanes 2j and 2j+1 of a wavefront)
// through DPP quad permutation [1,0,3,2]; no LDS traffic.  The two lanes of
// a pair always run the same control flow (their loop conditions are
// exchanged values), so the partner is active and every lane is written:
// the destination needs no prior value (no initialising move).
__device__ __forceinline__ int swap_pair_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
}

__device__ __forceinline__ double swap_pair(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)swap_pair_i32((int)(unsigned)b);
    const unsigned hi = (unsigned)swap_pair_i32((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Per-lane state of one trajectory of an orbit/shadow pair.  Each orbit
// occupies two adjacent lanes: the even lane integrates the orbit, the odd
// lane its shadow, so every lane holds a single trajectory.
struct PairState {
    double y[12], ref[4];
    double acc, d2, t_end;
    int64_t t, nsteps, renorms;
    int st, nmax;
    bool any_nc;
};

// End time and step count of orbit i, from the inputs.
__device__ __forceinline__ void pair_ends(PairState& ps, const FliArgs& fa, int64_t i) {
    ps.t_end = fa.t_end ? fa.t_end[i] : fa.t_end_all;
    ps.nsteps = ps.t_end > 0.0 ? (int64_t)ceil(ps.t_end / fa.h) : 0;
    if (fa.step_scale != 1.0) ps.nsteps = (int64_t)ceil((double)ps.nsteps * fa.step_scale);
}

// Separation of the pair, computed identically in both lanes: the lanes form
// e and -e exactly, so e * e and the sum carry the same bits.
__device__ __forceinline__ double pair_d2(const double* y) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double e = y[c] - swap_pair(y[c]);
        d2 = fma(e, e, d2);
    }
    return d2;
}

// Start orbit i in this pair: spin lengths (eq. 10), shadow offset,
// reference integrals, status at t = 0 (decided by the orbit lane).
__device__ __forceinline__ void pair_begin(PairState& ps, const PnCoef& k, bool param_ok, bool shadow,
                                           const FliArgs& fa, int64_t i) {
    load_state(fa.y0, fa.ld, i, ps.y);
    pn_correct_spins(k, ps.y);
    if (shadow) {
#pragma unroll
        for (int c = 0; c < 12; ++c) ps.y[c] += (c == fa.shadow_axis) ? fa.d0 : 0.0;
    }
    capture_ref(k, ps.y, ps.ref);
    pair_ends(ps, fa, i);
    int st = param_ok ? pn_validity(ps.y, fa.rmerge2, fa.resc2) : PN_ORBIT_BADPARAM;
    if (st == PN_ORBIT_OK && !(ps.ref[0] < 0.0)) st = PN_ORBIT_UNBOUND_INIT;
    const int other = swap_pair_i32(st);
    ps.st = shadow ? other : st;
    ps.acc = 0.0;
    ps.d2 = 0.0;
    ps.t = 0;
    ps.renorms = 0;
    ps.nmax = 0;
    ps.any_nc = false;
}

// One step of both trajectories (each lane its own), then the pair's
// validity, separation and, rarely, the shadow's renormalisation.
template <int METHOD, int MODE>
__device__ __forceinline__ void pair_step(PairState& ps, const PnCoef& k, bool shadow, const FliArgs& fa,
                                          int64_t i) {
    bool nc;
    pn_rk_step<METHOD>(k, ps.y, fa.h);
    const int it = pn_correct<MODE>(k, ps.y, ps.ref, fa.corr.tol, fa.corr.max_iter, fa.corr.sweeps, nc);
    ps.any_nc = ps.any_nc || nc;
    ps.nmax = max(ps.nmax, it);
    ps.t += 1;
    // Orbit verdict first, then the shadow's (same order in both lanes).
    const int mine = pn_validity(ps.y, fa.rmerge2, fa.resc2);
    const int other = swap_pair_i32(mine);
    const int vo = shadow ? other : mine, vs = shadow ? mine : other;
    ps.st = vo != PN_ORBIT_OK ? vo : vs;
    if (ps.st != PN_ORBIT_OK) return;
    ps.d2 = pair_d2(ps.y);
    if (ps.d2 >= fa.d_renorm2) {
        const double d = sqrt(ps.d2);
        ps.acc += log10(d / fa.d0);
        double yp[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) yp[c] = swap_pair(ps.y[c]);
        if (shadow) {
            const double f = fa.d0 / d;
#pragma unroll
            for (int c = 0; c < 12; ++c) ps.y[c] = fma(f, ps.y[c] - yp[c], yp[c]);
            pn_correct_spins(k, ps.y);
            capture_ref(k, ps.y, ps.ref);
        }
        ps.renorms += 1;
        ps.d2 = pair_d2(ps.y);
    }
    const int64_t tev = fa.out.trace_every;
    if (tev > 0 && (ps.t % tev) == 0 && !shadow) {
        const int64_t row = ps.t / tev - 1;
        if (row < fa.out.ntrace) fa.out.trace[row * fa.ld + i] = ps.acc + log10(sqrt(ps.d2) / fa.d0);
    }
}

__device__ __forceinline__ bool pair_running(const PairState& ps) {
    return ps.st == PN_ORBIT_OK && ps.t < ps.nsteps;
}

// Final separation and outputs of orbit i (written by the orbit lane).
__device__ __forceinline__ void pair_finish(PairState& ps, const PnCoef& k, bool shadow, const FliArgs& fa,
                                            int64_t i) {
    const double d2 = pair_d2(ps.y);
    const int nmax_other = swap_pair_i32(ps.nmax);
    const int nc_other = swap_pair_i32(ps.any_nc ? 1 : 0);
    if (shadow) return;
    const int64_t ld = fa.ld;
    const pn_scan_out& o = fa.out;
    if (o.y_final) store_state(o.y_final, ld, i, ps.y);
    if (o.dH || o.dJ) {
        double J[3];
        const double H = pn_energy(k, ps.y);
        pn_total_J(ps.y, J);
        const double* ref = ps.ref;
        if (o.dH) o.dH[i] = fabs(H - ref[0]) / fabs(ref[0]);
        if (o.dJ) {
            const double ex = J[0] - ref[1], ey = J[1] - ref[2], ez = J[2] - ref[3];
            o.dJ[i] = sqrt(dot3(ex, ey, ez, ex, ey, ez)) /
                      sqrt(dot3(ref[1], ref[2], ref[3], ref[1], ref[2], ref[3]));
        }
    }
    if (ps.st == PN_ORBIT_OK) {
        const double fli = ps.acc + log10(sqrt(d2) / fa.d0);
        const double thr = (fa.thr_scaling == PN_THR_LOG_T && ps.t_end > 0.0)
                               ? fa.thr_at_1e5 + log10(ps.t_end / 1e5) : fa.thr_at_1e5;
        o.fli[i] = fli;
        o.label[i] = fli > thr ? 1 : 0;
    } else {
        o.fli[i] = __builtin_nan("");
        o.label[i] = -1;
    }
    o.status[i] = ps.st | ((ps.any_nc || nc_other) ? PN_ORBIT_NEWTON_NOCONV : 0);
    if (o.newton_max) o.newton_max[i] = max(ps.nmax, nmax_other);
    if (o.renorms) o.renorms[i] = ps.renorms;
    if (o.steps) o.steps[i] = ps.t;
}

// Fused scan: orbit i on lanes (2i, 2i+1) from t = 0 to t_end.  SHARED:
// every orbit has the parameter set of pa.coef, whose table then stays in
// scalar registers.
template <int METHOD, int MODE, bool SHARED>
__global__ __launch_bounds__(kBlock) void k_fli_scan(ParamArgs pa, FliArgs fa) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = g >> 1;
    if (i >= fa.n) return;                 // pairs are whole: both lanes leave together
    const bool shadow = (g & 1) != 0;
    PnCoef k;
    bool param_ok = true;
    if (SHARED) {
        k = pa.coef;
        pn_coef_derive(k);
    } else {
        param_ok = load_coef(pa, i, k);
    }
    PairState ps;
    pair_begin(ps, k, param_ok, shadow, fa, i);
    while (pair_running(ps)) pair_step<METHOD, MODE>(ps, k, shadow, fa, i);
    pair_finish(ps, k, shadow, fa, i);
}

// ---------------------------------------------------------------------------
// Persistent work-stealing batch (orbits of uneven length and parameters).
// Workspace: queue head, bin counters, and the processing order.
// ---------------------------------------------------------------------------
constexpr int kBins = 256;           // 8 bins per octave of the step count

struct BatchWs {
    unsigned long long* head;        // next queue position to hand out
    unsigned int* bins;              // kBins counters, then kBins offsets
    int32_t* order;                  // queue position -> orbit index
};

__device__ __forceinline__ int step_bin(double t_end, double h) {
    const double ns = t_end > 0.0 ? ceil(t_end / h) : 0.0;
    int b = (int)floor(8.0 * log2(ns + 1.0));
    b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
    return kBins - 1 - b;            // longest first
}

__global__ __launch_bounds__(256) void k_batch_clear(BatchWs ws) {
    const int t = threadIdx.x;
    if (t == 0) *ws.head = 0ull;
    for (int b = t; b < 2 * kBins; b += 256) ws.bins[b] = 0u;
}

__global__ __launch_bounds__(256) void k_batch_bin_count(BatchWs ws, const double* t_end, double h, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    atomicAdd(&ws.bins[step_bin(t_end[i], h)], 1u);
}

// Exclusive prefix sum of the bin counters into the offsets (one workgroup).
__global__ __launch_bounds__(kBins) void k_batch_bin_scan(BatchWs ws) {
    __shared__ unsigned int sh[kBins];
    const int t = threadIdx.x;
    sh[t] = ws.bins[t];
    __syncthreads();
    for (int off = 1; off < kBins; off <<= 1) {
        const unsigned int v = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    ws.bins[kBins + t] = sh[t] - ws.bins[t];
}

__global__ __launch_bounds__(256) void k_batch_bin_scatter(BatchWs ws, const double* t_end, double h, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const unsigned int pos = atomicAdd(&ws.bins[kBins + step_bin(t_end[i], h)], 1u);
    ws.order[pos] = (int32_t)i;
}

// A table of saved orbit pairs: record r holds the orbit index and the exact
// state of lanes 2 r (orbit) and 2 r + 1 (shadow).
// Saved pair states: one record of kRecWords doubles per lane, contiguous
// (y[12], ref[4], acc, t, renorms, nmax | flags << 32), so that a lane
// addresses its record with one base address and constant offsets; records
// are written and read only where a piece or an orbit changes hands.
constexpr int kRecWords = 20;

struct RecTable {
    int32_t* id;                    // [cap] orbit index
    double* rec;                    // [2 cap][kRecWords]
    int64_t cap;                    // records
};

__device__ __forceinline__ void rec_save(const RecTable& T, int64_t r, const PairState& ps, bool shadow,
                                         int64_t cur) {
    double* R = T.rec + (2 * r + (shadow ? 1 : 0)) * kRecWords;
#pragma unroll
    for (int c = 0; c < 12; ++c) R[c] = ps.y[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) R[12 + c] = ps.ref[c];
    R[16] = ps.acc;
    R[17] = __builtin_bit_cast(double, ps.t);
    R[18] = __builtin_bit_cast(double, ps.renorms);
    const uint64_t fl = (uint64_t)(uint32_t)(ps.st | (ps.any_nc ? (1 << 16) : 0));
    R[19] = __builtin_bit_cast(double, (uint64_t)(uint32_t)ps.nmax | (fl << 32));
    if (!shadow) T.id[r] = (int32_t)cur;
}

// Restores what rec_save kept; returns the orbit index of the record (-1 if
// it names no orbit of this scan).
__device__ __forceinline__ int64_t rec_load(const RecTable& T, int64_t r, PairState& ps, bool shadow,
                                            const FliArgs& fa) {
    const int64_t i = T.id[r];
    if (i < 0 || i >= fa.n) return -1;
    const double* R = T.rec + (2 * r + (shadow ? 1 : 0)) * kRecWords;
#pragma unroll
    for (int c = 0; c < 12; ++c) ps.y[c] = R[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) ps.ref[c] = R[12 + c];
    ps.acc = R[16];
    ps.t = __builtin_bit_cast(int64_t, R[17]);
    ps.renorms = __builtin_bit_cast(int64_t, R[18]);
    const uint64_t w = __builtin_bit_cast(uint64_t, R[19]);
    ps.nmax = (int)(uint32_t)w;
    const int f = (int)(uint32_t)(w >> 32);
    ps.st = f & 0xFFFF;
    ps.any_nc = (f >> 16) != 0;
    ps.d2 = 0.0;
    pair_ends(ps, fa, i);
    return i;
}

// Checkpoint of an interrupted batch scan: the exact state of every orbit in
// flight, one record per orbit pair in each of two tables (the one a launch
// resumes from and the one it saves into, swapped after every launch).
// hdr: [0], [1] records in table 0 / 1; [2] read cursor of the input table;
// [3] index of the input table.
struct CkptArgs {
    unsigned long long* hdr;
    RecTable tab[2];
    int64_t cap;                    // records per table
    int32_t max_chunks;             // chunks per wavefront before it saves and leaves; 0: run to the end
};

// Persistent kernel: every wavefront keeps 32 orbit slots busy.  Between
// chunks of `chunk` steps, pairs whose orbit has ended write its results and
// claim the next queue position (one atomic per wavefront), so long orbits,
// started first, overlap with the short ones that fill the tail.  The
// wavefront leaves when the queue is drained and all its slots are empty.
// With CKPT, slots are first refilled from the orbits a previous launch
// saved, and after ck.max_chunks chunks (if > 0) every pair still running
// saves its state and the wavefront leaves.
template <int METHOD, int MODE, int OCC, bool CKPT>
__global__ __launch_bounds__(256, OCC) void k_batch_scan(ParamArgs pa, FliArgs fa, BatchWs ws, int32_t chunk,
                                                          CkptArgs ck) {
    const int lane = threadIdx.x & 63;
    const bool shadow = (lane & 1) != 0;
    const unsigned long long n = (unsigned long long)fa.n;
    int64_t cur = -1;                    // orbit in this pair's slot, -1 none
    bool drained = false;
    PnCoef k;
    PairState ps;
    int tin = 0;
    unsigned long long saved = 0ull;
    if (CKPT) {
        // Bounded reads of the header, so that a workspace that holds no
        // checkpoint cannot send a lane outside the tables.
        tin = (int)(ck.hdr[3] & 1ull);
        saved = ck.hdr[tin] < (unsigned long long)ck.cap ? ck.hdr[tin] : (unsigned long long)ck.cap;
    }
    int chunks = 0;
    for (;;) {
        if (CKPT) {
            // Saved orbits first: one atomic on the read cursor per wavefront.
            const bool need = (cur < 0) && !drained;
            const unsigned long long m = __ballot(need && !shadow);
            if (m != 0ull) {
                const int cnt = __popcll(m);
                const int leader = __ffsll((long long)m) - 1;
                unsigned long long base = 0ull;
                if (lane == leader) base = atomicAdd(&ck.hdr[2], (unsigned long long)cnt);
                base = __shfl(base, leader);
                if (need) {
                    const int even = lane & ~1;
                    const unsigned long long r = base + __popcll(m & ((1ull << even) - 1ull));
                    if (r < saved) {
                        const int64_t i = rec_load(ck.tab[tin], (int64_t)r, ps, shadow, fa);
                        if (i >= 0 && i < fa.n) {
                            cur = i;
                            load_coef(pa, cur, k);
                        }
                    }
                }
            }
        }
        // Refill empty slots: one atomic per wavefront for all claiming pairs.
        const bool need = (cur < 0) && !drained;
        const unsigned long long m = __ballot(need && !shadow);
        if (m != 0ull) {
            const int cnt = __popcll(m);
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0ull;
            if (lane == leader) base = atomicAdd(ws.head, (unsigned long long)cnt);
            base = __shfl(base, leader);
            if (need) {
                const int even = lane & ~1;
                const unsigned long long q = base + __popcll(m & ((1ull << even) - 1ull));
                if (q < n) {
                    cur = ws.order[q];
                    if (CKPT && (cur < 0 || cur >= fa.n)) {
                        cur = -1;       // not a queue this workspace set up: skip the position
                    } else {
                        const bool ok = load_coef(pa, cur, k);
                        pair_begin(ps, k, ok, shadow, fa, cur);
                    }
                } else {
                    drained = true;
                }
            }
        }
        if (__ballot(cur >= 0) == 0ull) break;
        if (cur >= 0) {
            for (int c = 0; c < chunk && pair_running(ps); ++c) pair_step<METHOD, MODE>(ps, k, shadow, fa, cur);
            if (!pair_running(ps)) {
                pair_finish(ps, k, shadow, fa, cur);
                cur = -1;
            }
        }
        if (CKPT && ck.max_chunks > 0 && ++chunks >= ck.max_chunks) {
            // Interrupted: save the pairs still running into the other table.
            const int tout = 1 - tin;
            const bool keep = cur >= 0;
            const unsigned long long m = __ballot(keep && !shadow);
            if (m != 0ull) {
                const int cnt = __popcll(m);
                const int leader = __ffsll((long long)m) - 1;
                unsigned long long base = 0ull;
                if (lane == leader) base = atomicAdd(&ck.hdr[tout], (unsigned long long)cnt);
                base = __shfl(base, leader);
                if (keep) {
                    const int even = lane & ~1;
                    const unsigned long long r = base + __popcll(m & ((1ull << even) - 1ull));
                    if (r < (unsigned long long)ck.cap) rec_save(ck.tab[tout], (int64_t)r, ps, shadow, cur);
                }
            }
            break;
        }
    }
}

// After an interrupted launch (one workgroup): saved orbits of the input table
// that no slot took are appended to the output table, which becomes the
// input of the next launch.
__global__ __launch_bounds__(256) void k_ckpt_carry(CkptArgs ck) {
    const unsigned long long cap = (unsigned long long)ck.cap;
    const int tin = (int)(ck.hdr[3] & 1ull), tout = 1 - tin;
    const unsigned long long saved = ck.hdr[tin] < cap ? ck.hdr[tin] : cap;
    const unsigned long long rd = ck.hdr[2] < saved ? ck.hdr[2] : saved;
    const unsigned long long base = ck.hdr[tout] < cap ? ck.hdr[tout] : cap;
    // The tables hold every orbit in flight (at most min(n, resident pairs));
    // the bound below only keeps a corrupted header inside them.
    const unsigned long long left = (saved - rd) < (cap - base) ? (saved - rd) : (cap - base);
    const RecTable& I = ck.tab[tin];
    const RecTable& O = ck.tab[tout];
    for (unsigned long long r = rd + threadIdx.x; r < rd + left; r += 256) {
        const unsigned long long d = base + (r - rd);
        O.id[d] = I.id[r];
        const double* src = I.rec + 2 * (int64_t)r * kRecWords;
        double* dst = O.rec + 2 * (int64_t)d * kRecWords;
        for (int w = 0; w < 2 * kRecWords; ++w) dst[w] = src[w];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ck.hdr[tout] = base + left;
        ck.hdr[tin] = 0ull;
        ck.hdr[2] = 0ull;
        ck.hdr[3] = (unsigned long long)tout;
    }
}

__global__ void k_ckpt_clear(CkptArgs ck) {
    if (threadIdx.x < 4) ck.hdr[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// Balanced scan of orbits that all take S steps.  Laid end to end, the n
// orbits form a tape of n S steps; slot s (one orbit pair of lanes) owns the
// stretch [s C, (s + 1) C) of it, so every slot carries the same work.  An
// orbit cut by the boundary between slots s and s + 1 is split the way
// McNaughton's wrap-around rule splits a preempted job: slot s + 1 integrates
// its first steps at the start of its stretch and saves the pair state
// (record s + 1 of the split table); slot s integrates the remaining steps at
// the end of its stretch, starting from that record.  The stretch runs in L
// launches of c slot-time steps; with C - S >= c the first part of a split
// orbit always ends in an earlier launch than the one in which its second part
// starts, so records are read one launch or more after they are written and
// no lane waits for another.  A piece cut by a launch boundary is saved in
// the slot's record of the carry table and resumed by the next launch.
// ---------------------------------------------------------------------------
struct WrapPiece {
    int64_t orbit;                  // orbit index
    int64_t a, b;                   // the piece integrates steps [a, b) of the orbit
    int64_t start;                  // slot time at which the piece starts
};

// The piece that slot s runs at slot time tau (0 <= tau < its stretch).
__host__ __device__ inline WrapPiece wrap_piece(int64_t n, int64_t S, int64_t C, int64_t s, int64_t tau) {
    const int64_t lo = s * C, total = n * S;
    const int64_t hi = total - lo < C ? total : lo + C;
    const int64_t j = (lo + tau) / S;
    const int64_t o_lo = j * S, o_hi = o_lo + S;
    const int64_t p_lo = o_lo > lo ? o_lo : lo, p_hi = o_hi < hi ? o_hi : hi;
    WrapPiece p;
    p.orbit = j;
    p.start = p_lo - lo;
    if (o_lo < lo) {                // begins in slot s - 1's stretch: run its first steps here
        p.a = 0;
        p.b = p_hi - p_lo;
    } else if (o_hi > hi) {         // ends in slot s + 1's stretch: run its last steps here
        p.a = S - (p_hi - p_lo);
        p.b = S;
    } else {
        p.a = 0;
        p.b = S;
    }
    return p;
}

struct WrapArgs {
    int64_t steps;                  // S
    int64_t slot_len;               // C
    int64_t slots;                  // orbit pairs of the schedule
    int64_t t0, t1;                 // slot-time window of this launch
    int32_t chunk;                  // steps between checks for the end of a piece
    RecTable carry, split;          // [slots] records each
};

// Where a piece's starting state comes from.
constexpr int kFromInputs = 0, kFromCarry = 1, kFromSplit = 2;

// Opens piece p in this pair: from the inputs when it starts at step 0, else
// from record r of the carry or split table.  A record that does not hold
// orbit p.orbit at step t_at (or stopped earlier with a final status) cannot
// occur under a valid plan; the orbit then reports PN_ORBIT_BADPARAM.
template <bool SHARED>
__device__ __forceinline__ void wrap_open(PairState& ps, PnCoef& k, const ParamArgs& pa, const FliArgs& fa,
                                          const WrapArgs& wa, int from, int64_t r, const WrapPiece& p,
                                          int64_t t_at, bool shadow) {
    const bool ok = SHARED ? true : load_coef(pa, p.orbit, k);
    if (from == kFromInputs) {
        pair_begin(ps, k, ok, shadow, fa, p.orbit);
        return;
    }
    const int64_t i = from == kFromCarry ? rec_load(wa.carry, r, ps, shadow, fa)
                                         : rec_load(wa.split, r, ps, shadow, fa);
    const bool match = i == p.orbit && (ps.st == PN_ORBIT_OK ? ps.t == t_at : ps.t <= t_at);
    if (!match) {
        pair_ends(ps, fa, p.orbit);
        ps.st = PN_ORBIT_BADPARAM;
    }
}

// SHARED: every orbit has the parameter set of pa.coef, whose table then stays
// in scalar registers for the whole launch instead of being rebuilt per piece
// in vector registers.
template <int METHOD, int MODE, int OCC, bool SHARED>
__global__ __launch_bounds__(256, OCC) void k_wrap_scan(ParamArgs pa, FliArgs fa, WrapArgs wa) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = g >> 1;
    const bool shadow = (g & 1) != 0;
    const int64_t S = wa.steps, C = wa.slot_len;
    const int64_t total = fa.n * S;
    int64_t len = 0;
    if (s < wa.slots && s * C < total) len = total - s * C < C ? total - s * C : C;
    const int64_t tend = wa.t1 < len ? wa.t1 : len;    // this launch ends the slot's work at tend
    int64_t tau = wa.t0;                               // slot time of the next piece to open
    bool active = tau < tend, open = active;
    int64_t orbit = 0, b = 0, pend = 0;                // open piece: orbit, last step + 1, end time
    PnCoef k;
    if (SHARED) {
        k = pa.coef;
        pn_coef_derive(k);
    }
    PairState ps;
    for (;;) {
        if (__ballot(active) == 0ull) break;
        if (open) {
            const WrapPiece p = wrap_piece(fa.n, S, C, s, tau);
            orbit = p.orbit;
            b = p.b;
            pend = p.start + (p.b - p.a);
            if (p.start < tau)          // cut by the previous launch's end
                wrap_open<SHARED>(ps, k, pa, fa, wa, kFromCarry, s, p, p.a + (tau - p.start), shadow);
            else
                wrap_open<SHARED>(ps, k, pa, fa, wa, p.a > 0 ? kFromSplit : kFromInputs, s + 1, p, p.a,
                                  shadow);
            open = false;
        }
        if (active) {
            // Steps left in this launch: up to b, less what lies past tend.
            const int64_t stop = pend <= tend ? b : b - (pend - tend);
            for (int c = 0; c < wa.chunk && ps.st == PN_ORBIT_OK && ps.t < stop; ++c)
                pair_step<METHOD, MODE>(ps, k, shadow, fa, orbit);
            if (!(ps.st == PN_ORBIT_OK && ps.t < stop)) {
                if (pend > tend) {
                    rec_save(wa.carry, s, ps, shadow, orbit);
                    active = false;
                } else {
                    if (b == S)
                        pair_finish(ps, k, shadow, fa, orbit);
                    else
                        rec_save(wa.split, s, ps, shadow, orbit);      // first part of a split orbit
                    tau = pend;
                    active = open = pend < tend;
                }
            }
        }
    }
}

// Marks every record of both tables empty before the first launch, so that a
// workspace's earlier contents can never be taken for this scan's records.
__global__ __launch_bounds__(256) void k_wrap_clear(WrapArgs wa) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < wa.slots) {
        wa.carry.id[r] = -1;
        wa.split.id[r] = -1;
    }
}

// ---------------------------------------------------------------------------
// Host-side validation and dispatch.
// ---------------------------------------------------------------------------
bool is_fin(double x) { return std::isfinite(x); }

pn_status check_model(const pn_model* m) {
    if (!m) return PN_EINVAL;
    if (m->pn_order < 0 || m->pn_order > 2) return PN_EINVAL;
    if ((m->spin_orbit | m->spin_spin | m->quad_mono) & ~1) return PN_EINVAL;
    if (m->spin_units != PN_SPIN_PHYS && m->spin_units != PN_SPIN_PAPER_EQ8) return PN_EINVAL;
    if (m->rad_reaction & ~1) return PN_EINVAL;
    return PN_OK;
}

pn_status make_params(const pn_model* m, const pn_params& p, ParamArgs& pa) {
    const int nnull = (p.beta == nullptr) + (p.chi1 == nullptr) + (p.chi2 == nullptr);
    if (nnull != 0 && nnull != 3) return PN_EINVAL;
    pa.beta = p.beta;
    pa.chi1 = p.chi1;
    pa.chi2 = p.chi2;
    pa.model = *m;
    std::memset(&pa.coef, 0, sizeof(pa.coef));
    if (nnull == 3) {
        if (!is_fin(p.beta0) || !is_fin(p.chi1_0) || !is_fin(p.chi2_0)) return PN_EINVAL;
        if (!pn_make_coef(*m, p.beta0, p.chi1_0, p.chi2_0, pa.coef)) return PN_EINVAL;
    }
    return PN_OK;
}

pn_status check_corr(const pn_correction* c) {
    if (!c) return PN_OK;
    if (c->mode < PN_CORR_NONE || c->mode > PN_CORR_DUAL) return PN_EINVAL;
    if (c->mode >= PN_CORR_SIX) {
        if (!(c->tol >= 0.0) || !is_fin(c->tol)) return PN_EINVAL;
        if (c->max_iter < 1 || c->max_iter > 1000) return PN_EINVAL;
        if (c->mode == PN_CORR_SIX && (c->sweeps < 1 || c->sweeps > 16)) return PN_EINVAL;
        if (!(c->w1 > 0.0) || !(c->w2 > 0.0)) return PN_EINVAL;
    }
    return PN_OK;
}

pn_status check_integ(const pn_integrator* in) {
    if (!in) return PN_EINVAL;
    if (in->method != PN_RK4 && in->method != PN_RK5) return PN_EINVAL;
    if (!(in->h > 0.0) || !is_fin(in->h)) return PN_EINVAL;
    return PN_OK;
}

CorrArgs corr_args(const pn_correction* c) {
    CorrArgs a;
    a.tol = c ? c->tol : 0.0;
    a.max_iter = c ? c->max_iter : 1;
    a.sweeps = c ? c->sweeps : 1;
    return a;
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Largest orbit count of a call: with two lanes per orbit a launch stays
// below HIP's limit of 2^32 work-items in x, and the balanced scan's pair
// records hold orbit indices in 32 bits.
constexpr int64_t kMaxN = ((int64_t)1 << 31) - 1;

pn_status launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(what, e);
        return PN_EDEVICE;
    }
    return PN_OK;
}

#define PN_REQUIRE(cond) do { if (!(cond)) return PN_EINVAL; } while (0)

template <int METHOD, int MODE>
void launch_step(const ParamArgs& pa, const CorrArgs& ca, double h, int64_t n, double* y, int64_t ld,
                 double* ref, int64_t nsteps, double* traj, int64_t every, double eta0, hipStream_t s) {
    if (pa.model.rad_reaction)
        hipLaunchKernelGGL((k_step<METHOD, MODE, true>), dim3(grid_for(n)), dim3(kBlock), 0, s, pa, ca, h, n, y,
                           ld, ref, nsteps, traj, every, eta0);
    else
        hipLaunchKernelGGL((k_step<METHOD, MODE, false>), dim3(grid_for(n)), dim3(kBlock), 0, s, pa, ca, h, n, y,
                           ld, ref, nsteps, traj, every, eta0);
}

template <int METHOD>
void launch_step_m(int mode, const ParamArgs& pa, const CorrArgs& ca, double h, int64_t n, double* y,
                   int64_t ld, double* ref, int64_t nsteps, double* traj, int64_t every, double eta0,
                   hipStream_t s) {
    switch (mode) {
        case PN_CORR_NONE:
            launch_step<METHOD, PN_CORR_NONE>(pa, ca, h, n, y, ld, ref, nsteps, traj, every, eta0, s); break;
        case PN_CORR_SPIN:
            launch_step<METHOD, PN_CORR_SPIN>(pa, ca, h, n, y, ld, ref, nsteps, traj, every, eta0, s); break;
        case PN_CORR_SIX:
            launch_step<METHOD, PN_CORR_SIX>(pa, ca, h, n, y, ld, ref, nsteps, traj, every, eta0, s); break;
        default:
            launch_step<METHOD, PN_CORR_DUAL>(pa, ca, h, n, y, ld, ref, nsteps, traj, every, eta0, s); break;
    }
}

// eta of a shared parameter set (unused with per-orbit arrays).
double shared_eta(const pn_params& p) { return p.beta ? 0.0 : p.beta0 / ((1.0 + p.beta0) * (1.0 + p.beta0)); }

template <int METHOD, int MODE>
void launch_scan(const ParamArgs& pa, const FliArgs& fa, hipStream_t s) {
    if (pa.beta == nullptr)
        hipLaunchKernelGGL((k_fli_scan<METHOD, MODE, true>), dim3(grid_for(2 * fa.n)), dim3(kBlock), 0, s, pa, fa);
    else
        hipLaunchKernelGGL((k_fli_scan<METHOD, MODE, false>), dim3(grid_for(2 * fa.n)), dim3(kBlock), 0, s, pa,
                           fa);
}

template <int METHOD>
void launch_scan_m(int mode, const ParamArgs& pa, const FliArgs& fa, hipStream_t s) {
    switch (mode) {
        case PN_CORR_NONE: launch_scan<METHOD, PN_CORR_NONE>(pa, fa, s); break;
        case PN_CORR_SPIN: launch_scan<METHOD, PN_CORR_SPIN>(pa, fa, s); break;
        case PN_CORR_SIX: launch_scan<METHOD, PN_CORR_SIX>(pa, fa, s); break;
        default: launch_scan<METHOD, PN_CORR_DUAL>(pa, fa, s); break;
    }
}

// Orbit pairs a persistent launch keeps resident.
int64_t batch_slots(const pn_tuning& tu, int ncu) { return (int64_t)ncu * 4 * tu.waves_per_simd * 32; }

template <int METHOD, int MODE, bool CKPT>
void launch_batch_c(const ParamArgs& pa, const FliArgs& fa, const BatchWs& ws, const pn_tuning& tu, int ncu,
                    const CkptArgs& ck, hipStream_t s) {
    const unsigned blocks = (unsigned)((int64_t)ncu * 4 * tu.waves_per_simd * 64 / tu.block);
    // Two resident waves per SIMD need <= 256 registers per lane: RK4 fits
    // (a few bytes of spill at most); the six-stage RK5 would spill hundreds
    // of bytes, so it keeps the one-wave build and only the grid grows.
    if constexpr (METHOD == PN_RK4) {
        if (tu.waves_per_simd == 2) {
            hipLaunchKernelGGL((k_batch_scan<METHOD, MODE, 2, CKPT>), dim3(blocks), dim3(tu.block), 0, s, pa, fa,
                               ws, tu.chunk_steps, ck);
            return;
        }
    }
    hipLaunchKernelGGL((k_batch_scan<METHOD, MODE, 1, CKPT>), dim3(blocks), dim3(tu.block), 0, s, pa, fa, ws,
                       tu.chunk_steps, ck);
}

template <int METHOD, int MODE>
void launch_batch(const ParamArgs& pa, const FliArgs& fa, const BatchWs& ws, const pn_tuning& tu, int ncu,
                  const CkptArgs* ck, hipStream_t s) {
    if (ck)
        launch_batch_c<METHOD, MODE, true>(pa, fa, ws, tu, ncu, *ck, s);
    else
        launch_batch_c<METHOD, MODE, false>(pa, fa, ws, tu, ncu, CkptArgs{}, s);
}

template <int METHOD>
void launch_batch_m(int mode, const ParamArgs& pa, const FliArgs& fa, const BatchWs& ws, const pn_tuning& tu,
                    int ncu, const CkptArgs* ck, hipStream_t s) {
    switch (mode) {
        case PN_CORR_NONE: launch_batch<METHOD, PN_CORR_NONE>(pa, fa, ws, tu, ncu, ck, s); break;
        case PN_CORR_SPIN: launch_batch<METHOD, PN_CORR_SPIN>(pa, fa, ws, tu, ncu, ck, s); break;
        case PN_CORR_SIX: launch_batch<METHOD, PN_CORR_SIX>(pa, fa, ws, tu, ncu, ck, s); break;
        default: launch_batch<METHOD, PN_CORR_DUAL>(pa, fa, ws, tu, ncu, ck, s); break;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t batch_ws_bytes(int64_t n) {
    return align256(sizeof(unsigned long long)) + align256(2 * kBins * sizeof(unsigned int)) +
           align256((size_t)n * sizeof(int32_t));
}

BatchWs carve(void* ws, int64_t n) {
    char* b = static_cast<char*>(ws);
    BatchWs w;
    w.head = reinterpret_cast<unsigned long long*>(b);
    b += align256(sizeof(unsigned long long));
    w.bins = reinterpret_cast<unsigned int*>(b);
    b += align256(2 * kBins * sizeof(unsigned int));
    w.order = reinterpret_cast<int32_t*>(b);
    (void)n;
    return w;
}

// The batch scan's workspace for callers that cannot allocate: a file-scope
// device array (every device the library runs on holds its own copy until
// the process ends) sized for kStaticBatchMaxOrbits orbits.  Host code uses
// only the device address that hipGetSymbolAddress reports for the current
// device, never the array's name.
constexpr int64_t kStaticBatchMaxOrbits = (int64_t)1 << 20;
constexpr size_t kStaticBatchBytes = 256 + ((2 * 256 * sizeof(unsigned int) + 255) / 256) * 256 +
                                     (((size_t)kStaticBatchMaxOrbits * sizeof(int32_t) + 255) / 256) * 256;
static __device__ __align__(256) unsigned char scratch[kStaticBatchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per
// device (nullptr and the HIP error text on failure).
void* static_scratch(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            set_error("pn_batch_scan_noalloc", e);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Checkpoint tables: records per table, bytes per table.
constexpr int64_t kCkptMaxPairs = (int64_t)1 << 18;

int64_t ckpt_cap(int64_t n) { return n < kCkptMaxPairs ? n : kCkptMaxPairs; }

size_t rec_table_bytes(int64_t cap) {
    return align256((size_t)cap * 4) + align256(2 * (size_t)cap * kRecWords * 8);
}

// Carves one record table of cap records at b and advances b past it.
RecTable carve_rec(char*& b, int64_t cap) {
    RecTable T;
    T.cap = cap;
    T.id = reinterpret_cast<int32_t*>(b);       b += align256((size_t)cap * 4);
    T.rec = reinterpret_cast<double*>(b);       b += align256(2 * (size_t)cap * kRecWords * 8);
    return T;
}

size_t ckpt_ws_bytes(int64_t n) { return batch_ws_bytes(n) + align256(4 * 8) + 2 * rec_table_bytes(ckpt_cap(n)); }

CkptArgs carve_ckpt(void* ws, int64_t n, int32_t max_chunks) {
    char* b = static_cast<char*>(ws) + batch_ws_bytes(n);
    CkptArgs ck;
    ck.cap = ckpt_cap(n);
    ck.max_chunks = max_chunks;
    ck.hdr = reinterpret_cast<unsigned long long*>(b);
    b += align256(4 * 8);
    for (int tab = 0; tab < 2; ++tab) ck.tab[tab] = carve_rec(b, ck.cap);
    return ck;
}

bool valid_tuning(const pn_tuning& t) {
    return (t.block == 64 || t.block == 128 || t.block == 256) && t.waves_per_simd >= 1 &&
           t.waves_per_simd <= 2 && t.chunk_steps >= 1 && t.chunk_steps <= (1 << 20);
}

// Last autotune result per device (guarded: calls on other threads may
// autotune or read it concurrently).
pn_tuning g_tuned[64];
bool g_has_tuned[64] = {false};
std::mutex g_tuned_mu;

// The tuning a batch uses: the caller's, else the device's last autotune
// result, else the defaults.
pn_tuning chosen_tuning(const pn_tuning* tuning, int dev) {
    pn_tuning tu;
    if (tuning) return *tuning;
    {
        std::lock_guard<std::mutex> lock(g_tuned_mu);
        if (dev >= 0 && dev < 64 && g_has_tuned[dev]) return g_tuned[dev];
    }
    pn_default_tuning(&tu);
    return tu;
}

void remember_tuning(int dev, const pn_tuning& tu) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    if (dev >= 0 && dev < 64) {
        g_tuned[dev] = tu;
        g_has_tuned[dev] = true;
    }
}

int device_cus(int& dev) {
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return ncu;
}

// Validation shared by the scan entry points; fills fa on success.
pn_status prepare_scan(const pn_model* model, const pn_params& params, const pn_integrator* integ,
                       const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0, int64_t ld,
                       const double* t_end, double t_end_all, const pn_scan_out* out, ParamArgs& pa,
                       FliArgs& fa) {
    if (check_model(model) != PN_OK || check_integ(integ) != PN_OK) return PN_EINVAL;
    if (model->rad_reaction) return PN_EINVAL;      // scans integrate the conservative system
    if (corr == nullptr || check_corr(corr) != PN_OK) return PN_EINVAL;
    if (fli == nullptr || out == nullptr) return PN_EINVAL;
    if (!(n >= 0 && n <= kMaxN && ld >= n)) return PN_EINVAL;
    if (!(fli->d0 > 0.0 && is_fin(fli->d0) && fli->d_renorm > fli->d0 && is_fin(fli->d_renorm))) return PN_EINVAL;
    if (fli->shadow_axis < 0 || fli->shadow_axis >= 12) return PN_EINVAL;
    if (!is_fin(fli->thr_at_1e5)) return PN_EINVAL;
    if (fli->thr_scaling != PN_THR_LITERAL && fli->thr_scaling != PN_THR_LOG_T) return PN_EINVAL;
    if (!(fli->r_merge >= 0.0 && fli->r_esc > fli->r_merge)) return PN_EINVAL;
    if (!(t_end != nullptr || (t_end_all >= 0.0 && is_fin(t_end_all)))) return PN_EINVAL;
    if (make_params(model, params, pa) != PN_OK) return PN_EINVAL;
    if (n > 0) {
        if (!(y0 && out->fli && out->label && out->status)) return PN_EINVAL;
        if (!(out->trace_every >= 0 && (out->trace_every == 0 || (out->trace && out->ntrace >= 0)))) return PN_EINVAL;
    }
    fa.h = integ->h;
    fa.corr = corr_args(corr);
    fa.d0 = fli->d0;
    fa.d_renorm2 = fli->d_renorm * fli->d_renorm;
    fa.rmerge2 = fli->r_merge * fli->r_merge;
    fa.resc2 = fli->r_esc * fli->r_esc;
    fa.thr_at_1e5 = fli->thr_at_1e5;
    fa.thr_scaling = fli->thr_scaling;
    fa.shadow_axis = fli->shadow_axis;
    fa.t_end = t_end;
    fa.t_end_all = t_end_all;
    fa.out = *out;
    fa.n = n;
    fa.ld = ld;
    fa.y0 = y0;
    fa.step_scale = 1.0;
    return PN_OK;
}

// Enqueue the whole batch: clear, bin by step count, order, persistent scan.
// With a checkpoint, `resume` skips the queue set-up and continues from the
// saved orbits, and the launch is followed by the carry-over of saved orbits.
void enqueue_batch(int method, int mode, const ParamArgs& pa, const FliArgs& fa, const BatchWs& w,
                   const pn_tuning& tu, int ncu, hipStream_t stream, const CkptArgs* ck = nullptr,
                   bool resume = false) {
    const unsigned g256 = (unsigned)((fa.n + 255) / 256);
    if (!resume) {
        hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(256), 0, stream, w);
        hipLaunchKernelGGL(k_batch_bin_count, dim3(g256), dim3(256), 0, stream, w, fa.t_end, fa.h, fa.n);
        hipLaunchKernelGGL(k_batch_bin_scan, dim3(1), dim3(kBins), 0, stream, w);
        hipLaunchKernelGGL(k_batch_bin_scatter, dim3(g256), dim3(256), 0, stream, w, fa.t_end, fa.h, fa.n);
        if (ck) hipLaunchKernelGGL(k_ckpt_clear, dim3(1), dim3(64), 0, stream, *ck);
    }
    if (method == PN_RK4)
        launch_batch_m<PN_RK4>(mode, pa, fa, w, tu, ncu, ck, stream);
    else
        launch_batch_m<PN_RK5>(mode, pa, fa, w, tu, ncu, ck, stream);
    if (ck) hipLaunchKernelGGL(k_ckpt_carry, dim3(1), dim3(256), 0, stream, *ck);
}

// Registers, private memory and resident wavefronts per SIMD of kernel f
// launched with workgroups of `block` threads.
pn_status func_resources(const char* what, const void* f, int block, int32_t* vgprs, int64_t* scratch_bytes,
                         int32_t* waves_per_simd) {
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, f);
    int blocks = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, block, 0);
    if (e != hipSuccess) {
        set_error(what, e);
        return PN_EDEVICE;
    }
    if (vgprs) *vgprs = at.numRegs;
    if (scratch_bytes) *scratch_bytes = (int64_t)at.localSizeBytes;
    if (waves_per_simd) *waves_per_simd = blocks * (block / 64) / 4;     // four SIMDs per CU
    return PN_OK;
}

// Balanced scan: kernel per method, correction and parameter mode.  RK4
// keeps two resident wavefronts per SIMD (at most 256 registers per lane):
// with a shared parameter set the RK4 build fits without spilling; the
// per-orbit build keeps a few values of the piece bookkeeping in scratch
// between piece events.  The six-stage RK5 keeps the registers of one.
constexpr int32_t kWrapMaxLaunches = 16;
constexpr int64_t kWrapMaxSlots = (int64_t)1 << 24;
constexpr int64_t kWrapMaxTape = (int64_t)1 << 62;
constexpr int32_t kWrapChunk = 256;

template <int METHOD, int MODE>
struct WrapK {
    static constexpr int OCC = METHOD == PN_RK4 ? 2 : 1;
    static const void* fn(bool shared) {
        return shared ? reinterpret_cast<const void*>(&k_wrap_scan<METHOD, MODE, OCC, true>)
                      : reinterpret_cast<const void*>(&k_wrap_scan<METHOD, MODE, OCC, false>);
    }
    static void launch(unsigned blocks, const ParamArgs& pa, const FliArgs& fa, const WrapArgs& wa,
                       hipStream_t s) {
        if (pa.beta == nullptr)
            hipLaunchKernelGGL((k_wrap_scan<METHOD, MODE, OCC, true>), dim3(blocks), dim3(256), 0, s, pa, fa, wa);
        else
            hipLaunchKernelGGL((k_wrap_scan<METHOD, MODE, OCC, false>), dim3(blocks), dim3(256), 0, s, pa, fa,
                               wa);
    }
};

// shared: the build for one parameter set shared by every orbit (its table in
// scalar registers), else the per-orbit build.
const void* wrap_fn(int method, int mode, bool shared = true) {
    switch (method * 4 + mode) {
        case 0: return WrapK<PN_RK4, PN_CORR_NONE>::fn(shared);
        case 1: return WrapK<PN_RK4, PN_CORR_SPIN>::fn(shared);
        case 2: return WrapK<PN_RK4, PN_CORR_SIX>::fn(shared);
        case 3: return WrapK<PN_RK4, PN_CORR_DUAL>::fn(shared);
        case 4: return WrapK<PN_RK5, PN_CORR_NONE>::fn(shared);
        case 5: return WrapK<PN_RK5, PN_CORR_SPIN>::fn(shared);
        case 6: return WrapK<PN_RK5, PN_CORR_SIX>::fn(shared);
        default: return WrapK<PN_RK5, PN_CORR_DUAL>::fn(shared);
    }
}

void wrap_launch(int method, int mode, unsigned blocks, const ParamArgs& pa, const FliArgs& fa,
                 const WrapArgs& wa, hipStream_t s) {
    switch (method * 4 + mode) {
        case 0: WrapK<PN_RK4, PN_CORR_NONE>::launch(blocks, pa, fa, wa, s); break;
        case 1: WrapK<PN_RK4, PN_CORR_SPIN>::launch(blocks, pa, fa, wa, s); break;
        case 2: WrapK<PN_RK4, PN_CORR_SIX>::launch(blocks, pa, fa, wa, s); break;
        case 3: WrapK<PN_RK4, PN_CORR_DUAL>::launch(blocks, pa, fa, wa, s); break;
        case 4: WrapK<PN_RK5, PN_CORR_NONE>::launch(blocks, pa, fa, wa, s); break;
        case 5: WrapK<PN_RK5, PN_CORR_SPIN>::launch(blocks, pa, fa, wa, s); break;
        case 6: WrapK<PN_RK5, PN_CORR_SIX>::launch(blocks, pa, fa, wa, s); break;
        default: WrapK<PN_RK5, PN_CORR_DUAL>::launch(blocks, pa, fa, wa, s); break;
    }
}

// Slot length C and launch count L of the balanced schedule of n orbits of S
// steps on P slots: C >= n S / P, and C - S >= ceil(C / L) so that the two
// parts of every split orbit fall in different launches.  C is raised to
// S + ceil(S / 15) when n S / P is smaller (the last slots then stay empty),
// which keeps L <= 16.
bool wrap_plan(int64_t n, int64_t S, int64_t P, int64_t& C, int32_t& L) {
    if (n <= 0 || S <= 0 || P <= 0 || P > kWrapMaxSlots) return false;
    if (n > kWrapMaxTape / S) return false;
    const int64_t total = n * S;
    C = total / P + (total % P != 0 ? 1 : 0);
    const int64_t cmin = S + (S + kWrapMaxLaunches - 2) / (kWrapMaxLaunches - 1);
    if (C < cmin) C = cmin;
    if (C > kWrapMaxTape / P) return false;
    for (L = 2; L <= kWrapMaxLaunches; ++L) {
        const int64_t c = C / L + (C % L != 0 ? 1 : 0);
        if (C - S >= c) return true;
    }
    return false;
}

// Orbit pairs the balanced kernel keeps resident on the current device (a
// full grid of them places the same number of wavefronts on every SIMD).
int64_t wrap_resident_pairs(int method, int mode, int64_t* waves_per_simd) {
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wrap_fn(method, mode), 256, 0) != hipSuccess ||
        blocks <= 0)
        return 0;
    if (waves_per_simd) *waves_per_simd = blocks;   // four wavefronts per workgroup, one per SIMD
    return (int64_t)ncu * blocks * 128;
}

int64_t steps_of(double t_end_all, double h) { return t_end_all > 0.0 ? (int64_t)ceil(t_end_all / h) : 0; }

// Schedule of pn_fli_scan_balanced: slots P, slot length C, launches L
// (L = 0: the plain fused scan).  With slots = 0 the device's resident pairs
// are used and the balanced schedule is taken only where its predicted time
// (wavefronts per SIMD x C) is at least 2% below the plain scan's (rounds of
// resident wavefronts x S); slots > 0 always takes it.
pn_status wrap_choose(int method, int mode, int64_t n, int64_t S, int64_t slots, int64_t& P, int64_t& C,
                      int32_t& L) {
    C = 0;
    L = 0;
    P = slots;
    if (slots < 0 || slots > kWrapMaxSlots) return PN_EINVAL;
    int64_t W = 0;
    if (slots == 0) {
        P = wrap_resident_pairs(method, mode, &W);
        if (P <= 0) {
            set_error("pn_fli_scan_balanced", hipErrorNoDevice);
            return PN_EDEVICE;
        }
    }
    if (n == 0 || S == 0) return PN_OK;
    if (!wrap_plan(n, S, P, C, L)) {
        C = 0;
        L = 0;
        return slots > 0 ? PN_EINVAL : PN_OK;
    }
    if (slots == 0) {
        const int64_t simds = P / (32 * W);
        const int64_t waves = (2 * n + 63) / 64;
        const double plain = (double)((waves + simds - 1) / simds) * (double)S;
        const double wrap = (double)W * (double)C;
        if (!(wrap * 1.02 < plain)) {
            C = 0;
            L = 0;
        }
    }
    return PN_OK;
}

size_t wrap_ws_bytes(int64_t P) { return 2 * rec_table_bytes(P); }

}  // namespace

// ===========================================================================
// C ABI.
// ===========================================================================
extern "C" {

void pn_default_model(pn_model* m) {
    if (!m) return;
    m->pn_order = 2;
    m->spin_orbit = 1;
    m->spin_spin = 1;
    m->quad_mono = 1;
    m->spin_units = PN_SPIN_PHYS;
    m->rad_reaction = 0;
}

void pn_default_integrator(pn_integrator* in) {
    if (!in) return;
    in->method = PN_RK4;
    in->h = 1.0;
}

void pn_default_correction(pn_correction* c) {
    if (!c) return;
    c->mode = PN_CORR_SIX;
    c->tol = 1e-10;
    c->max_iter = 20;
    c->sweeps = 2;
    c->w1 = 1.0;
    c->w2 = 1.0;
}

void pn_default_fli_cfg(pn_fli_cfg* f) {
    if (!f) return;
    f->d0 = 1e-8;
    f->d_renorm = 0.1;
    f->shadow_axis = 0;
    f->thr_at_1e5 = 5.8;
    f->thr_scaling = PN_THR_LOG_T;
    f->r_merge = 2.0;
    f->r_esc = 1e3;
}

int32_t pn_version(void) { return 1; }

const char* pn_status_string(pn_status s) {
    switch (s) {
        case PN_OK: return "ok";
        case PN_EINVAL: return "invalid argument";
        case PN_ENOWS: return "workspace too small";
        case PN_EDEVICE: return "device error";
    }
    return "unknown status";
}

const char* pn_last_error(void) { return pn_detail::g_last_error; }

void pn_shutdown(void) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    for (int d = 0; d < 64; ++d) g_has_tuned[d] = false;
}

size_t pn_fli_scan_workspace_size(int64_t n) {
    (void)n;
    return 0;
}

pn_status pn_init_state(const pn_model* model, pn_params params, int64_t n, const double* r0,
                        const double* p0, const double* th1, const double* ph1, const double* th2,
                        const double* ph2, double* y0, int64_t ld, hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && ld >= n);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0) return PN_OK;
    PN_REQUIRE(r0 && p0 && th1 && ph1 && th2 && ph2 && y0);
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(n)), dim3(kBlock), 0, stream, pa, n,
                       (const int32_t*)nullptr, r0, p0, th1, ph1, th2, ph2, y0, ld);
    return launched("pn_init_state");
}

pn_status pn_init_state_gather(const pn_model* model, pn_params params, int64_t m, const int32_t* idx,
                               const double* r0, const double* p0, const double* th1, const double* ph1,
                               const double* th2, const double* ph2, double* y0, int64_t ld,
                               hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(m >= 0 && m <= kMaxN && ld >= m);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (m == 0) return PN_OK;
    PN_REQUIRE(idx && r0 && p0 && th1 && ph1 && th2 && ph2 && y0);
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(m)), dim3(kBlock), 0, stream, pa, m, idx, r0, p0, th1, ph1,
                       th2, ph2, y0, ld);
    return launched("pn_init_state_gather");
}

pn_status pn_rhs(const pn_model* model, pn_params params, int64_t n, const double* y, int64_t ld,
                 double* dydt, hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && ld >= n);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0) return PN_OK;
    PN_REQUIRE(y && dydt);
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(n)), dim3(kBlock), 0, stream, pa, n, y, ld, dydt, shared_eta(params));
    return launched("pn_rhs");
}

pn_status pn_invariants(const pn_model* model, pn_params params, int64_t n, const double* y, int64_t ld,
                        double* H, double* J, hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && ld >= n);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0) return PN_OK;
    PN_REQUIRE(y && H && J);
    hipLaunchKernelGGL(k_invariants, dim3(grid_for(n)), dim3(kBlock), 0, stream, pa, n, y, ld, H, J);
    return launched("pn_invariants");
}

pn_status pn_manifold_correct(const pn_model* model, pn_params params, const pn_correction* corr,
                              int64_t n, double* y, int64_t ld, const double* ref, int32_t* iters,
                              hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(corr != nullptr && check_corr(corr) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && ld >= n);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0) return PN_OK;
    PN_REQUIRE(y && ref);
    const CorrArgs ca = corr_args(corr);
    const dim3 g(grid_for(n)), b(kBlock);
    switch (corr->mode) {
        case PN_CORR_NONE: hipLaunchKernelGGL(k_correct<PN_CORR_NONE>, g, b, 0, stream, pa, ca, n, y, ld, ref, iters); break;
        case PN_CORR_SPIN: hipLaunchKernelGGL(k_correct<PN_CORR_SPIN>, g, b, 0, stream, pa, ca, n, y, ld, ref, iters); break;
        case PN_CORR_SIX: hipLaunchKernelGGL(k_correct<PN_CORR_SIX>, g, b, 0, stream, pa, ca, n, y, ld, ref, iters); break;
        default: hipLaunchKernelGGL(k_correct<PN_CORR_DUAL>, g, b, 0, stream, pa, ca, n, y, ld, ref, iters); break;
    }
    return launched("pn_manifold_correct");
}

static pn_status step_impl(const char* what, const pn_model* model, pn_params params, const pn_integrator* integ,
                           const pn_correction* corr, int64_t n, double* y, int64_t ld, double* ref,
                           int64_t nsteps, double* traj, int64_t every, hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(check_integ(integ) == PN_OK);
    PN_REQUIRE(check_corr(corr) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && ld >= n && nsteps >= 0);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0 || nsteps == 0) return PN_OK;
    PN_REQUIRE(y);
    const int mode = corr ? corr->mode : PN_CORR_NONE;
    const CorrArgs ca = corr_args(corr);
    const double eta0 = shared_eta(params);
    if (integ->method == PN_RK4)
        launch_step_m<PN_RK4>(mode, pa, ca, integ->h, n, y, ld, ref, nsteps, traj, every, eta0, stream);
    else
        launch_step_m<PN_RK5>(mode, pa, ca, integ->h, n, y, ld, ref, nsteps, traj, every, eta0, stream);
    return launched(what);
}

pn_status pn_step(const pn_model* model, pn_params params, const pn_integrator* integ,
                  const pn_correction* corr, int64_t n, double* y, int64_t ld, double* ref,
                  int64_t nsteps, hipStream_t stream) {
    return step_impl("pn_step", model, params, integ, corr, n, y, ld, ref, nsteps, nullptr, 1, stream);
}

pn_status pn_trajectory(const pn_model* model, pn_params params, const pn_integrator* integ,
                        const pn_correction* corr, int64_t n, double* y, int64_t ld, double* ref,
                        int64_t nsteps, int64_t every, double* traj, hipStream_t stream) {
    PN_REQUIRE(every >= 1);
    PN_REQUIRE(traj != nullptr || nsteps / every == 0 || n == 0);
    return step_impl("pn_trajectory", model, params, integ, corr, n, y, ld, ref, nsteps,
                     nsteps / every > 0 ? traj : nullptr, every, stream);
}

pn_status pn_gw_polarizations(const pn_model* model, pn_params params, int64_t n, int64_t ns, const double* y,
                              int64_t ld, const double* nhat, const double* phat, double dist, double* hp,
                              double* hx, hipStream_t stream) {
    PN_REQUIRE(check_model(model) == PN_OK);
    PN_REQUIRE(n >= 0 && ns >= 0 && ld >= n);
    PN_REQUIRE(nhat != nullptr && phat != nullptr);
    PN_REQUIRE(dist > 0.0 && is_fin(dist));
    const double nn = nhat[0] * nhat[0] + nhat[1] * nhat[1] + nhat[2] * nhat[2];
    const double pp = phat[0] * phat[0] + phat[1] * phat[1] + phat[2] * phat[2];
    const double np = nhat[0] * phat[0] + nhat[1] * phat[1] + nhat[2] * phat[2];
    PN_REQUIRE(std::fabs(nn - 1.0) <= 1e-12 && std::fabs(pp - 1.0) <= 1e-12 && std::fabs(np) <= 1e-12);
    ParamArgs pa;
    PN_REQUIRE(make_params(model, params, pa) == PN_OK);
    if (n == 0 || ns == 0) return PN_OK;
    PN_REQUIRE(y && hp && hx);
    PN_REQUIRE(n <= (int64_t)1 << 40 && ns <= ((int64_t)1 << 62) / n);
    GwArgs ga;
    ga.px = phat[0]; ga.py = phat[1]; ga.pz = phat[2];
    ga.qx = nhat[1] * phat[2] - nhat[2] * phat[1];       // q = N x p
    ga.qy = nhat[2] * phat[0] - nhat[0] * phat[2];
    ga.qz = nhat[0] * phat[1] - nhat[1] * phat[0];
    ga.inv_dist = 1.0 / dist;
    ga.eta0 = params.beta0 / ((1.0 + params.beta0) * (1.0 + params.beta0));
    const int64_t blocks = (n + 255) / 256;
    PN_REQUIRE(blocks <= 0x7fffffffLL);
    const unsigned rows = (unsigned)(ns < 65535 ? ns : 65535);
    hipLaunchKernelGGL(k_gw, dim3((unsigned)blocks, rows), dim3(256), 0, stream, pa, ga, n, ns, y, ld, hp, hx);
    return launched("pn_gw_polarizations");
}

pn_status pn_fli_scan(const pn_model* model, pn_params params, const pn_integrator* integ,
                      const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                      int64_t ld, const double* t_end, double t_end_all, const pn_scan_out* out,
                      hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, t_end_all, out, pa, fa) == PN_OK);
    if (n == 0) return PN_OK;
    if (integ->method == PN_RK4)
        launch_scan_m<PN_RK4>(corr->mode, pa, fa, stream);
    else
        launch_scan_m<PN_RK5>(corr->mode, pa, fa, stream);
    return launched("pn_fli_scan");
}

pn_status pn_balanced_plan(int64_t n, int64_t steps, int64_t slots, int64_t* slot_len, int32_t* launches) {
    PN_REQUIRE(slot_len != nullptr && launches != nullptr);
    int64_t C = 0;
    int32_t L = 0;
    PN_REQUIRE(wrap_plan(n, steps, slots, C, L));
    *slot_len = C;
    *launches = L;
    return PN_OK;
}

pn_status pn_balanced_piece(int64_t n, int64_t steps, int64_t slot_len, int64_t slot, int64_t tau,
                            int64_t* orbit, int64_t* first_step, int64_t* end_step, int64_t* start) {
    PN_REQUIRE(orbit && first_step && end_step && start);
    PN_REQUIRE(n > 0 && steps > 0 && n <= kWrapMaxTape / steps && slot_len > steps && slot >= 0);
    const int64_t total = n * steps;
    PN_REQUIRE(slot <= total / slot_len && slot * slot_len < total);
    const int64_t len = total - slot * slot_len < slot_len ? total - slot * slot_len : slot_len;
    PN_REQUIRE(tau >= 0 && tau < len);
    const WrapPiece p = wrap_piece(n, steps, slot_len, slot, tau);
    *orbit = p.orbit;
    *first_step = p.a;
    *end_step = p.b;
    *start = p.start;
    return PN_OK;
}

pn_status pn_fli_scan_balanced_schedule(const pn_integrator* integ, const pn_correction* corr, int64_t n,
                                        double t_end_all, int64_t slots, int64_t* slots_used,
                                        int64_t* slot_len, int32_t* launches) {
    PN_REQUIRE(check_integ(integ) == PN_OK && corr != nullptr && check_corr(corr) == PN_OK);
    PN_REQUIRE(n >= 0 && n <= kMaxN && t_end_all >= 0.0 && is_fin(t_end_all) && t_end_all / integ->h < 4.0e18);
    int64_t P = 0, C = 0;
    int32_t L = 0;
    const pn_status st = wrap_choose(integ->method, corr->mode, n, steps_of(t_end_all, integ->h), slots, P, C, L);
    if (st != PN_OK) return st;
    if (slots_used) *slots_used = P;
    if (slot_len) *slot_len = C;
    if (launches) *launches = L;
    return PN_OK;
}

size_t pn_fli_scan_balanced_workspace_size(int64_t slots) {
    return slots > 0 && slots <= kWrapMaxSlots ? wrap_ws_bytes(slots) : 0;
}

pn_status pn_fli_scan_balanced(const pn_model* model, pn_params params, const pn_integrator* integ,
                               const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                               int64_t ld, double t_end_all, const pn_scan_out* out, int64_t slots, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, nullptr, t_end_all, out, pa, fa) ==
               PN_OK);
    PN_REQUIRE(t_end_all / integ->h < 4.0e18);
    PN_REQUIRE(slots >= 0 && slots <= kWrapMaxSlots);
    if (n == 0) return PN_OK;
    const int64_t S = steps_of(t_end_all, integ->h);
    int64_t P = 0, C = 0;
    int32_t L = 0;
    const pn_status st = wrap_choose(integ->method, corr->mode, n, S, slots, P, C, L);
    if (st != PN_OK) return st;
    if (L == 0) {
        if (integ->method == PN_RK4)
            launch_scan_m<PN_RK4>(corr->mode, pa, fa, stream);
        else
            launch_scan_m<PN_RK5>(corr->mode, pa, fa, stream);
        return launched("pn_fli_scan_balanced");
    }
    if (ws == nullptr || ws_bytes < wrap_ws_bytes(P)) return PN_ENOWS;
    WrapArgs wa;
    char* b = static_cast<char*>(ws);
    wa.carry = carve_rec(b, P);
    wa.split = carve_rec(b, P);
    wa.steps = S;
    wa.slot_len = C;
    wa.slots = P;
    wa.chunk = kWrapChunk;
    wa.t0 = wa.t1 = 0;
    hipLaunchKernelGGL(k_wrap_clear, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, wa);
    const int64_t c = C / L + (C % L != 0 ? 1 : 0);
    const unsigned blocks = (unsigned)((2 * P + 255) / 256);
    for (int32_t l = 0; l < L; ++l) {
        wa.t0 = l * c;
        wa.t1 = (l + 1) * c < C ? (l + 1) * c : C;
        wrap_launch(integ->method, corr->mode, blocks, pa, fa, wa, stream);
    }
    return launched("pn_fli_scan_balanced");
}

void pn_default_tuning(pn_tuning* t) {
    if (!t) return;
    t->block = 256;
    t->waves_per_simd = 2;
    t->chunk_steps = 256;
}

size_t pn_batch_workspace_size(int64_t n) { return n < 0 ? 0 : batch_ws_bytes(n); }

pn_status pn_scan_kernel_resources(int32_t method, int32_t mode, int32_t* vgprs, int64_t* scratch_bytes,
                                   int32_t* waves_per_simd) {
    PN_REQUIRE(method == PN_RK4 || method == PN_RK5);
    PN_REQUIRE(mode >= PN_CORR_NONE && mode <= PN_CORR_DUAL);
    const void* f = nullptr;
    switch (method * 4 + mode) {
        case 0: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK4, PN_CORR_NONE, true>); break;
        case 1: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK4, PN_CORR_SPIN, true>); break;
        case 2: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK4, PN_CORR_SIX, true>); break;
        case 3: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK4, PN_CORR_DUAL, true>); break;
        case 4: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK5, PN_CORR_NONE, true>); break;
        case 5: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK5, PN_CORR_SPIN, true>); break;
        case 6: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK5, PN_CORR_SIX, true>); break;
        default: f = reinterpret_cast<const void*>(&k_fli_scan<PN_RK5, PN_CORR_DUAL, true>); break;
    }
    return func_resources("pn_scan_kernel_resources", f, kBlock, vgprs, scratch_bytes, waves_per_simd);
}

pn_status pn_balanced_kernel_resources(int32_t method, int32_t mode, int32_t* vgprs, int64_t* scratch_bytes,
                                       int32_t* waves_per_simd) {
    PN_REQUIRE(method == PN_RK4 || method == PN_RK5);
    PN_REQUIRE(mode >= PN_CORR_NONE && mode <= PN_CORR_DUAL);
    return func_resources("pn_balanced_kernel_resources", wrap_fn(method, mode), 256, vgprs, scratch_bytes,
                          waves_per_simd);
}

int64_t pn_batch_resident_pairs(const pn_tuning* tuning) {
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) return 0;
    const pn_tuning tu = chosen_tuning(tuning, dev);
    if (!valid_tuning(tu)) return 0;
    return batch_slots(tu, ncu);
}

pn_status pn_batch_scan(const pn_model* model, pn_params params, const pn_integrator* integ,
                        const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                        int64_t ld, const double* t_end, const pn_scan_out* out, const pn_tuning* tuning,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(t_end != nullptr);
    PN_REQUIRE(n < 0x7fffffffLL);
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, 0.0, out, pa, fa) == PN_OK);
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) { set_error("pn_batch_scan", hipErrorInvalidDevice); return PN_EDEVICE; }
    const pn_tuning tu = chosen_tuning(tuning, dev);
    PN_REQUIRE(valid_tuning(tu));
    if (n == 0) return PN_OK;
    if (ws == nullptr || ws_bytes < batch_ws_bytes(n)) return PN_ENOWS;
    enqueue_batch(integ->method, corr->mode, pa, fa, carve(ws, n), tu, ncu, stream);
    return launched("pn_batch_scan");
}

pn_status pn_batch_scan_noalloc(const pn_model* model, pn_params params, const pn_integrator* integ,
                                const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                                int64_t ld, const double* t_end, const pn_scan_out* out, const pn_tuning* tuning,
                                hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(t_end != nullptr);
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, 0.0, out, pa, fa) == PN_OK);
    if (n > kStaticBatchMaxOrbits || batch_ws_bytes(n) > kStaticBatchBytes) {
        pn_detail::set_last_error("pn_batch_scan_noalloc", "more orbits than the static workspace holds (2^20)");
        return PN_EINVAL;
    }
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) { set_error("pn_batch_scan_noalloc", hipErrorInvalidDevice); return PN_EDEVICE; }
    const pn_tuning tu = chosen_tuning(tuning, dev);
    PN_REQUIRE(valid_tuning(tu));
    if (n == 0) return PN_OK;
    void* ws = static_scratch(dev);
    if (ws == nullptr) return PN_EDEVICE;
    // The queue head and bin counters start at zero: k_batch_clear (a kernel,
    // not a memset) clears them at the start of every call.
    enqueue_batch(integ->method, corr->mode, pa, fa, carve(ws, n), tu, ncu, stream);
    return launched("pn_batch_scan_noalloc");
}

size_t pn_batch_ckpt_workspace_size(int64_t n) { return n < 0 ? 0 : ckpt_ws_bytes(n); }

pn_status pn_batch_scan_resumable(const pn_model* model, pn_params params, const pn_integrator* integ,
                                  const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                                  int64_t ld, const double* t_end, const pn_scan_out* out,
                                  const pn_tuning* tuning, int32_t resume, int32_t max_chunks, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(t_end != nullptr);
    PN_REQUIRE(n < 0x7fffffffLL);
    PN_REQUIRE(resume == 0 || resume == 1);
    PN_REQUIRE(max_chunks >= 0);
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, 0.0, out, pa, fa) == PN_OK);
    PN_REQUIRE(out->trace_every == 0);
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) { set_error("pn_batch_scan_resumable", hipErrorInvalidDevice); return PN_EDEVICE; }
    const pn_tuning tu = chosen_tuning(tuning, dev);
    PN_REQUIRE(valid_tuning(tu));
    if (n == 0) return PN_OK;
    if (ws == nullptr || ws_bytes < ckpt_ws_bytes(n)) return PN_ENOWS;
    // Orbits in flight never exceed the orbits or the resident pairs of a
    // launch; the tables hold min(n, 2^18) records.
    PN_REQUIRE(n <= kCkptMaxPairs || batch_slots(tu, ncu) <= kCkptMaxPairs);
    const CkptArgs ck = carve_ckpt(ws, n, max_chunks);
    enqueue_batch(integ->method, corr->mode, pa, fa, carve(ws, n), tu, ncu, stream, &ck, resume != 0);
    return launched("pn_batch_scan_resumable");
}

pn_status pn_batch_scan_pending(const void* ws, int64_t n, int64_t* pending, hipStream_t stream) {
    PN_REQUIRE(pending != nullptr && n >= 0);
    *pending = 0;
    if (n == 0) return PN_OK;
    PN_REQUIRE(ws != nullptr);
    hipError_t e = hipStreamSynchronize(stream);
    unsigned long long head = 0ull, hdr[4] = {0ull, 0ull, 0ull, 0ull};
    if (e == hipSuccess) e = hipMemcpy(&head, ws, sizeof(head), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(hdr, static_cast<const char*>(ws) + batch_ws_bytes(n), sizeof(hdr), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_error("pn_batch_scan_pending", e);
        return PN_EDEVICE;
    }
    const unsigned long long tin = hdr[3] & 1ull;
    const unsigned long long queued = head < (unsigned long long)n ? (unsigned long long)n - head : 0ull;
    *pending = (int64_t)(hdr[tin] + queued);
    return PN_OK;
}

pn_status pn_autotune_batch(const pn_model* model, pn_params params, const pn_integrator* integ,
                            const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                            int64_t ld, const double* t_end, const pn_scan_out* out, double step_scale,
                            void* ws, size_t ws_bytes, pn_tuning* best, float* best_ms, hipStream_t stream) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(t_end != nullptr && best != nullptr);
    PN_REQUIRE(step_scale > 0.0 && step_scale <= 1.0);
    PN_REQUIRE(n < 0x7fffffffLL);
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, 0.0, out, pa, fa) == PN_OK);
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) { set_error("pn_autotune_batch", hipErrorInvalidDevice); return PN_EDEVICE; }
    pn_default_tuning(best);
    if (n == 0) return PN_OK;
    if (ws == nullptr || ws_bytes < batch_ws_bytes(n)) return PN_ENOWS;
    fa.step_scale = step_scale;
    const BatchWs w = carve(ws, n);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        set_error("pn_autotune_batch", hipErrorOutOfMemory);
        return PN_EDEVICE;
    }
    const int blocks[] = {64, 128, 256};
    const int waves[] = {1, 2};
    const int chunks[] = {32, 64, 256, 1024};
    float best_t = 1e30f;
    pn_status st = PN_OK;
    for (int b : blocks)
        for (int wv : waves)
            for (int c : chunks) {
                pn_tuning tu;
                tu.block = b;
                tu.waves_per_simd = wv;
                tu.chunk_steps = c;
                (void)hipEventRecord(e0, stream);
                enqueue_batch(integ->method, corr->mode, pa, fa, w, tu, ncu, stream);
                (void)hipEventRecord(e1, stream);
                if (launched("pn_autotune_batch") != PN_OK) { st = PN_EDEVICE; goto done; }
                if (hipEventSynchronize(e1) != hipSuccess) { set_error("pn_autotune_batch", hipGetLastError()); st = PN_EDEVICE; goto done; }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_t) { best_t = ms; *best = tu; }
            }
    remember_tuning(dev, *best);
    if (best_ms) *best_ms = best_t;
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

struct pn_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

pn_status pn_batch_graph_create(const pn_model* model, pn_params params, const pn_integrator* integ,
                                const pn_correction* corr, const pn_fli_cfg* fli, int64_t n, const double* y0,
                                int64_t ld, const double* t_end, const pn_scan_out* out,
                                const pn_tuning* tuning, void* ws, size_t ws_bytes, pn_graph** graph) {
    ParamArgs pa;
    FliArgs fa;
    PN_REQUIRE(graph != nullptr && t_end != nullptr && n > 0);
    PN_REQUIRE(n < 0x7fffffffLL);
    *graph = nullptr;
    PN_REQUIRE(prepare_scan(model, params, integ, corr, fli, n, y0, ld, t_end, 0.0, out, pa, fa) == PN_OK);
    int dev = 0;
    const int ncu = device_cus(dev);
    if (ncu <= 0) { set_error("pn_batch_graph_create", hipErrorInvalidDevice); return PN_EDEVICE; }
    const pn_tuning tu = chosen_tuning(tuning, dev);
    PN_REQUIRE(valid_tuning(tu));
    if (ws == nullptr || ws_bytes < batch_ws_bytes(n)) return PN_ENOWS;
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) { set_error("pn_batch_graph_create", e); return PN_EDEVICE; }
    pn_graph* g = new pn_graph;
    g->graph = nullptr;
    g->exec = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue_batch(integ->method, corr->mode, pa, fa, carve(ws, n), tu, ncu, cs);
        e = hipStreamEndCapture(cs, &g->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        set_error("pn_batch_graph_create", e);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return PN_EDEVICE;
    }
    *graph = g;
    return PN_OK;
}

pn_status pn_graph_launch(pn_graph* graph, hipStream_t stream) {
    PN_REQUIRE(graph != nullptr && graph->exec != nullptr);
    const hipError_t e = hipGraphLaunch(graph->exec, stream);
    if (e != hipSuccess) { set_error("pn_graph_launch", e); return PN_EDEVICE; }
    return PN_OK;
}

void pn_graph_destroy(pn_graph* graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
