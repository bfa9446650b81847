// pn_oracle.cpp -- plain, serial, FP64 CPU oracle for the manifold-corrected
// PN spinning-binary integrator and its fast Lyapunov indicator (FLI) scan.
//
// TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
// GPU library is compared against.  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it.  It shares no code, no
// header and no constant table with the GPU library.
//
// Style: one orbit at a time, every formula written out term by term in the
// paper's notation, no blocking, no fusion, no algebraic shortcuts.  All
// arithmetic is IEEE double with contraction disabled (-ffp-contract=off).
// Every routine is templated on the scalar type so that
//   * T = double                 : the reference itself,
//   * T = std::complex<double>   : complex-step derivatives of H (gradient pin),
//   * T = Counted                : algorithmic flop counts (+ - * / sqrt = 1).
//
// Sources (arXiv 1802.00147, "GPU accelerated manifold correction method for
// spinning compact binaries"):
//   Sec. 2, eq. (1)      H = H_N + H_PN + H_SO + H_SS (3PN dropped; the 2.5PN
//                        reaction of eq. (6) is an optional force on dp/dt)
//   Sec. 2, eqs. (2)-(5) spin-spin and quadrupole-monopole terms
//   Sec. 2, eq. (6)      dr/dt = dH/dp, dp/dt = -dH/dr (+ a_2.5PN, optional)
//   Sec. 3B (orbit 3)    dissipative orbit corrected against references that
//                        follow the integral-invariant relation
//   Sec. 2, eqs. (7)-(9) dS_i/dt = Omega_i x S_i
//   Sec. 2, eq. (10)     spin-length correction
//   Sec. 2, eqs. (11)-(13) dual (momentum-position) scaling, Newton solve
//   Sec. 3B              iteration limit eps <= 1e-10
//   Sec. 3C              two-nearby-trajectory FLI, threshold 5.8 at t = 1e5,
//                        removal of unbounded / merged orbits
//   Sec. 4, eq. (14)     gravitational-wave polarisations h_plus, h_cross
// The orbital N/1PN/2PN and spin-orbit terms are not printed in the paper
// (Sec. 2 cites them); the standard ADM-gauge expressions are used, and so
// is one reading of every other silent or garbled passage, stated where it
// is applied below.
//
// Parity pins that tie this file to the physics (not to itself) live in the
// tests: Kepler closed forms, the 2PN circular-orbit energy E(x), the 2PN
// periastron advance k(E, j), the eta -> 0 Schwarzschild limit, the spin-orbit
// circular-orbit coefficient, the paper's printed eqs. (8)-(9), complex-step
// gradients, Runge-Kutta stability polynomials and order slopes.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <atomic>

// ---------------------------------------------------------------------------
// Flop-counting scalar.  Counting rule: + - * / sqrt each count one flop;
// negation, comparisons, fabs and log10 count zero (log10 runs only on FLI
// renormalisation, off the per-step path).
// ---------------------------------------------------------------------------
static thread_local uint64_t g_flops = 0;

struct Counted {
    double v;
    Counted() : v(0.0) {}
    Counted(double x) : v(x) {}
};
static inline Counted operator+(Counted a, Counted b) { ++g_flops; return Counted(a.v + b.v); }
static inline Counted operator-(Counted a, Counted b) { ++g_flops; return Counted(a.v - b.v); }
static inline Counted operator*(Counted a, Counted b) { ++g_flops; return Counted(a.v * b.v); }
static inline Counted operator/(Counted a, Counted b) { ++g_flops; return Counted(a.v / b.v); }
static inline Counted operator-(Counted a) { return Counted(-a.v); }
static inline Counted operator+(Counted a, double b) { return a + Counted(b); }
static inline Counted operator+(double a, Counted b) { return Counted(a) + b; }
static inline Counted operator-(Counted a, double b) { return a - Counted(b); }
static inline Counted operator-(double a, Counted b) { return Counted(a) - b; }
static inline Counted operator*(Counted a, double b) { return a * Counted(b); }
static inline Counted operator*(double a, Counted b) { return Counted(a) * b; }
static inline Counted operator/(Counted a, double b) { return a / Counted(b); }
static inline Counted operator/(double a, Counted b) { return Counted(a) / b; }
static inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
static inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
static inline Counted& operator*=(Counted& a, Counted b) { a = a * b; return a; }
static inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
static inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
static inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
static inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
static inline Counted sqrt(Counted a) { ++g_flops; return Counted(std::sqrt(a.v)); }
static inline Counted fabs(Counted a) { return Counted(std::fabs(a.v)); }
static inline Counted log10(Counted a) { return Counted(std::log10(a.v)); }
static inline bool isfinite(Counted a) { return std::isfinite(a.v); }
static inline double val(Counted a) { return a.v; }
static inline double val(double a) { return a; }

using std::sqrt;
using std::fabs;
using std::log10;
using std::isfinite;

// ---------------------------------------------------------------------------
// Public plain-C structures of the oracle (its own; the GPU library has its
// own header and the test layer marshals into each separately).
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
    int32_t pn_order;    // 0: Newtonian only, 1: +1PN, 2: +1PN+2PN       (eq. 1)
    int32_t spin_orbit;  // 1.5PN spin-orbit on/off                          (eq. 1)
    int32_t spin_spin;   // S1-S2 coupling, eq. (3), on/off
    int32_t quad_mono;   // quadrupole-monopole S1S1, S2S2, eqs. (4)-(5), on/off
    int32_t spin_units;  // 0: physical spin flow (spins in mu*M), 1: eqs. (7)-(9) literal (spins in M^2)
    int32_t rad_reaction; // 2.5PN radiation-reaction acceleration on dp/dt (eq. 6), on/off
} or_model;

typedef struct {
    int32_t method;      // 0: classical RK4, 1: fifth-order Runge-Kutta (Dormand-Prince 5th-order weights)
    double h;            // fixed step
} or_integrator;

typedef struct {
    int32_t mode;        // 0 NONE, 1 SPIN (eq. 10), 2 SIX (spins + J vector + energy), 3 DUAL (eqs. 10-13)
    double tol;          // Newton iteration limit on the scale factors (Sec. 3B: 1e-10)
    int32_t max_iter;    // Newton iteration cap
    int32_t sweeps;      // SIX: number of (J projection, energy scaling) passes
    double w1, w2;       // eq. (12) weights (immaterial at an exact root)
} or_correction;

typedef struct {
    double d0;           // initial separation of the shadow trajectory
    double d_renorm;     // renormalise the shadow when the separation reaches this
    int32_t shadow_axis; // state component the shadow offset is applied to
    double thr_at_1e5;   // chaos threshold at t = 1e5 (Sec. 3C: 5.8)
    int32_t thr_scaling; // 0: literal threshold, 1: threshold + log10(t/1e5)
    double r_merge;      // r below this: merged
    double r_esc;        // r above this: escaped
} or_fli_cfg;

}  // extern "C"

enum { ST_OK = 0, ST_MERGED = 1, ST_ESCAPED = 2, ST_NONFINITE = 3, ST_UNBOUND_INIT = 4,
       ST_BADPARAM = 5, ST_NEWTON_NOCONV = 0x100 };

// Parameter ranges of Sec. 2: beta = m1/m2 in (0, 1]; Kerr spins chi in [0, 1].
#ifndef PN_SIX_MU
#define PN_SIX_MU 1e-5
#endif

static bool params_valid(double beta, double chi1, double chi2) {
    return beta > 0.0 && beta <= 1.0 && chi1 >= 0.0 && chi1 <= 1.0 && chi2 >= 0.0 && chi2 <= 1.0;
}

// ---------------------------------------------------------------------------
// Mass and spin coefficients (Sec. 2 mass definitions; eqs. (3)-(5), (8)-(9)).
// M = m1 + m2 = 1, beta = m1/m2 <= 1, eta = mu/M.  H is the Hamiltonian per
// unit reduced mass, r in M, p in mu.
// ---------------------------------------------------------------------------
struct Coef {
    double beta, eta;
    double cso1, cso2;   // spin-orbit:  H_SO = u^3 L.(cso1 S1 + cso2 S2)
    double c12;          // H_S1S2 = c12 u^3 [3(S1.n)(S2.n) - S1.S2]
    double c11, c22;     // H_SiSi = cii u^3 [3(Si.n)^2 - Si.Si]
    double s1, s2;       // spin lengths |S_i| in the chosen spin unit
};

static Coef make_coef(const or_model& m, double beta, double chi1, double chi2) {
    Coef c;
    c.beta = beta;
    const double m1 = beta / (1.0 + beta);   // M = 1
    const double m2 = 1.0 / (1.0 + beta);
    c.eta = m1 * m2;
    if (m.spin_units == 0) {
        // Spins in units of mu*M: S_phys = eta * S.  The physical SO energy
        // 2/r^3 (1 + 3 m2/(4 m1)) L.S1 + ... and eqs. (3)-(5), divided by mu,
        // pick up one factor of eta each.
        c.cso1 = c.eta * (2.0 + 3.0 / (2.0 * beta));
        c.cso2 = c.eta * (2.0 + 3.0 * beta / 2.0);
        c.c12 = c.eta;
        c.c11 = c.eta / (2.0 * beta);
        c.c22 = c.eta * beta / 2.0;
        c.s1 = chi1 * m1 * m1 / c.eta;  // = chi1 * beta
        c.s2 = chi2 * m2 * m2 / c.eta;  // = chi2 / beta
    } else {
        // Spins in units of M^2; dH/dS_i then equals eqs. (8)-(9) exactly.
        c.cso1 = 2.0 + 3.0 / (2.0 * beta);
        c.cso2 = 2.0 + 3.0 * beta / 2.0;
        c.c12 = 1.0 / c.eta;
        c.c11 = 1.0 / (2.0 * beta * c.eta);
        c.c22 = beta / (2.0 * c.eta);
        c.s1 = chi1 * m1 * m1;
        c.s2 = chi2 * m2 * m2;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Small vector helpers (plain, no conjugation: valid for complex-step).
// ---------------------------------------------------------------------------
template <class T> struct V3 { T x, y, z; };
template <class T> static inline V3<T> v3(T a, T b, T c) { V3<T> v; v.x = a; v.y = b; v.z = c; return v; }
template <class T> static inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> static inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return v3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T> static inline V3<T> add(const V3<T>& a, const V3<T>& b) { return v3<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> static inline V3<T> sub(const V3<T>& a, const V3<T>& b) { return v3<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T, class S> static inline V3<T> scl(S s, const V3<T>& a) { return v3<T>(s * a.x, s * a.y, s * a.z); }
template <class T> static inline V3<T> get3(const T* y, int off) { return v3<T>(y[off], y[off + 1], y[off + 2]); }
template <class T> static inline void put3(T* y, int off, const V3<T>& v) { y[off] = v.x; y[off + 1] = v.y; y[off + 2] = v.z; }

// State layout: y = (r[0..2], p[3..5], S1[6..8], S2[9..11]).

// ---------------------------------------------------------------------------
// Hamiltonian, eq. (1) without the 2.5PN and 3PN parts.
// ---------------------------------------------------------------------------
template <class T>
static T hamiltonian(const or_model& m, const Coef& c, const T* y) {
    const V3<T> r = get3(y, 0), p = get3(y, 3), S1 = get3(y, 6), S2 = get3(y, 9);
    const double eta = c.eta;
    const T rlen = sqrt(dot(r, r));
    const T u = 1.0 / rlen;
    const V3<T> n = scl(u, r);
    const T P2 = dot(p, p);
    const T NP = dot(n, p);

    // Newtonian part.
    T H = P2 / 2.0 - u;
    // 1PN (ADM).
    if (m.pn_order >= 1) {
        H += (3.0 * eta - 1.0) / 8.0 * (P2 * P2)
           - 0.5 * ((3.0 + eta) * P2 + eta * (NP * NP)) * u
           + 0.5 * (u * u);
    }
    // 2PN (ADM).
    if (m.pn_order >= 2) {
        H += (1.0 - 5.0 * eta + 5.0 * eta * eta) / 16.0 * (P2 * P2 * P2)
           + ((5.0 - 20.0 * eta - 3.0 * eta * eta) * (P2 * P2)
              - 2.0 * eta * eta * P2 * (NP * NP)
              - 3.0 * eta * eta * (NP * NP * NP * NP)) / 8.0 * u
           + ((5.0 + 8.0 * eta) * P2 + 3.0 * eta * (NP * NP)) / 2.0 * (u * u)
           - (1.0 + 3.0 * eta) / 4.0 * (u * u * u);
    }
    const T u3 = u * u * u;
    // 1.5PN spin-orbit: u^3 L . (cso1 S1 + cso2 S2), L = r x p.
    if (m.spin_orbit) {
        const V3<T> L = cross(r, p);
        H += u3 * (c.cso1 * dot(L, S1) + c.cso2 * dot(L, S2));
    }
    // eq. (3): S1-S2 coupling.
    if (m.spin_spin) {
        H += c.c12 * u3 * (3.0 * dot(S1, n) * dot(S2, n) - dot(S1, S2));
    }
    // eqs. (4)-(5): quadrupole-monopole terms.
    if (m.quad_mono) {
        H += c.c11 * u3 * (3.0 * dot(S1, n) * dot(S1, n) - dot(S1, S1));
        H += c.c22 * u3 * (3.0 * dot(S2, n) * dot(S2, n) - dot(S2, S2));
    }
    return H;
}

// ---------------------------------------------------------------------------
// Gradient of H: dH/dr, dH/dp, dH/dS1, dH/dS2, written term by term.
// Orbital part: H_orb(P2, NP, u) with P2 = p.p, NP = n.p, u = 1/r;
//   dP2/dp = 2p, dNP/dp = n, dNP/dr = u (p - NP n), du/dr = -u^2 n.
// ---------------------------------------------------------------------------
template <class T>
struct Grad { V3<T> dr, dp, dS1, dS2; };

// With only_p set, just dH/dp is formed (all that the momentum-scaling Newton
// derivative needs); the other fields are then left zero.
template <class T>
static Grad<T> gradient(const or_model& m, const Coef& c, const T* y, bool only_p = false) {
    const V3<T> r = get3(y, 0), p = get3(y, 3), S1 = get3(y, 6), S2 = get3(y, 9);
    const double eta = c.eta;
    const T rlen = sqrt(dot(r, r));
    const T u = 1.0 / rlen;
    const V3<T> n = scl(u, r);
    const T P2 = dot(p, p);
    const T NP = dot(n, p);

    // Partial derivatives of H_orb with respect to P2, NP and u.
    T H_P2 = T(0.5);
    T H_NP = T(0.0);
    T H_u = T(-1.0);
    if (m.pn_order >= 1) {
        H_P2 += (3.0 * eta - 1.0) / 8.0 * (2.0 * P2) - 0.5 * (3.0 + eta) * u;
        H_NP += -0.5 * eta * (2.0 * NP) * u;
    }
    if (m.pn_order >= 2) {
        H_P2 += (1.0 - 5.0 * eta + 5.0 * eta * eta) / 16.0 * (3.0 * P2 * P2)
              + ((5.0 - 20.0 * eta - 3.0 * eta * eta) * (2.0 * P2)
                 - 2.0 * eta * eta * (NP * NP)) / 8.0 * u
              + (5.0 + 8.0 * eta) / 2.0 * (u * u);
        H_NP += (-2.0 * eta * eta * P2 * (2.0 * NP)
                 - 3.0 * eta * eta * (4.0 * NP * NP * NP)) / 8.0 * u
              + 3.0 * eta * (2.0 * NP) / 2.0 * (u * u);
    }

    Grad<T> g;
    g.dr = v3<T>(T(0.0), T(0.0), T(0.0));
    g.dS1 = v3<T>(T(0.0), T(0.0), T(0.0));
    g.dS2 = v3<T>(T(0.0), T(0.0), T(0.0));
    // Orbital contributions.
    g.dp = add(scl(2.0 * H_P2, p), scl(H_NP, n));
    const T u3 = u * u * u;
    if (only_p) {
        if (m.spin_orbit) {
            const V3<T> Seff = add(scl(c.cso1, S1), scl(c.cso2, S2));
            g.dp = add(g.dp, scl(u3, cross(Seff, r)));
        }
        return g;
    }
    if (m.pn_order >= 1) {
        H_u += -0.5 * ((3.0 + eta) * P2 + eta * (NP * NP)) + u;
    }
    if (m.pn_order >= 2) {
        H_u += ((5.0 - 20.0 * eta - 3.0 * eta * eta) * (P2 * P2)
                - 2.0 * eta * eta * P2 * (NP * NP)
                - 3.0 * eta * eta * (NP * NP * NP * NP)) / 8.0
             + ((5.0 + 8.0 * eta) * P2 + 3.0 * eta * (NP * NP)) / 2.0 * (2.0 * u)
             - (1.0 + 3.0 * eta) / 4.0 * (3.0 * u * u);
    }
    g.dr = sub(scl(H_NP * u, sub(p, scl(NP, n))), scl(H_u * u * u, n));

    const T u4 = u3 * u;
    if (m.spin_orbit) {
        const V3<T> L = cross(r, p);
        const V3<T> Seff = add(scl(c.cso1, S1), scl(c.cso2, S2));
        // d/dp [ u^3 (r x p).Seff ] = u^3 (Seff x r)
        g.dp = add(g.dp, scl(u3, cross(Seff, r)));
        // d/dr [ u^3 (r x p).Seff ] = u^3 (p x Seff) - 3 u^4 (L.Seff) n
        g.dr = add(g.dr, sub(scl(u3, cross(p, Seff)), scl(3.0 * u4 * dot(L, Seff), n)));
        g.dS1 = add(g.dS1, scl(c.cso1 * u3, L));
        g.dS2 = add(g.dS2, scl(c.cso2 * u3, L));
    }
    const T a1 = dot(S1, n), a2 = dot(S2, n);
    if (m.spin_spin) {
        const T S12 = dot(S1, S2);
        // d/dr: -3 u^4 (3 a1 a2 - S1.S2) n + 3 u^4 [a2 (S1 - a1 n) + a1 (S2 - a2 n)]
        g.dr = add(g.dr, scl(c.c12, add(scl(-3.0 * u4 * (3.0 * a1 * a2 - S12), n),
                                        scl(3.0 * u4, add(scl(a2, sub(S1, scl(a1, n))),
                                                          scl(a1, sub(S2, scl(a2, n))))))));
        g.dS1 = add(g.dS1, scl(c.c12 * u3, sub(scl(3.0 * a2, n), S2)));
        g.dS2 = add(g.dS2, scl(c.c12 * u3, sub(scl(3.0 * a1, n), S1)));
    }
    if (m.quad_mono) {
        const T S11 = dot(S1, S1), S22 = dot(S2, S2);
        g.dr = add(g.dr, scl(c.c11, add(scl(-3.0 * u4 * (3.0 * a1 * a1 - S11), n),
                                        scl(6.0 * u4 * a1, sub(S1, scl(a1, n))))));
        g.dr = add(g.dr, scl(c.c22, add(scl(-3.0 * u4 * (3.0 * a2 * a2 - S22), n),
                                        scl(6.0 * u4 * a2, sub(S2, scl(a2, n))))));
        g.dS1 = add(g.dS1, scl(c.c11 * u3, sub(scl(6.0 * a1, n), scl(2.0, S1))));
        g.dS2 = add(g.dS2, scl(c.c22 * u3, sub(scl(6.0 * a2, n), scl(2.0, S2))));
    }
    return g;
}

// The 2.5PN radiation-reaction acceleration of eq. (6).  The paper takes it
// from Levin et al. (2011) without printing it; here it is the leading-order
// reaction acceleration of a point-mass binary in the two-parameter gauge
// family of Iyer and Will (1993),
//   a = (8/5) eta / r^3 [ A rdot n - B v ],
//   A = 3(1 + be) v^2 + (23 + 6 al - 9 be) / (3 r) - 5 be rdot^2,
//   B = (2 + al) v^2 + (2 - al) / r - 3 (1 + al) rdot^2,
// at al = 4, be = 5 (the harmonic-coordinate form of Damour and Deruelle),
// with v = dH/dp the velocity of the Hamiltonian flow and rdot = n.v (M = 1).
// Every member of the family radiates the quadrupole energy and angular
// momentum fluxes on average over an orbit (-(32/5) eta^2 / r^5 on a circle).
template <class T>
static V3<T> rr_accel(const Coef& c, const T* y, const V3<T>& v) {
    const V3<T> r = get3(y, 0);
    const T rr = sqrt(dot(r, r));
    const V3<T> n = scl(T(1.0) / rr, r);
    const T rdot = dot(n, v), v2 = dot(v, v);
    const double al = 4.0, be = 5.0;
    const T A = 3.0 * (1.0 + be) * v2 + ((23.0 + 6.0 * al - 9.0 * be) / 3.0) / rr - 5.0 * be * rdot * rdot;
    const T B = (2.0 + al) * v2 + (2.0 - al) / rr - 3.0 * (1.0 + al) * rdot * rdot;
    const T pre = (8.0 / 5.0) * c.eta / (rr * rr * rr);
    return sub(scl(pre * A * rdot, n), scl(pre * B, v));
}

// Hamilton's equations (eq. 6) and spin precession (eq. 7):
//   dr/dt = dH/dp,  dp/dt = -dH/dr (+ a_2.5PN),  dS_i/dt = (dH/dS_i) x S_i.
template <class T>
static void rhs(const or_model& m, const Coef& c, const T* y, T* dydt) {
    const Grad<T> g = gradient(m, c, y);
    const V3<T> S1 = get3(y, 6), S2 = get3(y, 9);
    put3(dydt, 0, g.dp);
    if (m.rad_reaction)
        put3(dydt, 3, add(scl(-1.0, g.dr), rr_accel(c, y, g.dp)));
    else
        put3(dydt, 3, scl(-1.0, g.dr));
    put3(dydt, 6, cross(g.dS1, S1));
    put3(dydt, 9, cross(g.dS2, S2));
}

// The dissipative system with its reference integrals (Sec. 3B, integral
// invariant relation): z = (y, E, J), dz/dt = (f(y), v.a, r x a).  The
// Hamiltonian and total angular momentum change only through the reaction
// acceleration (the spin flow conserves both), so E(t) and J(t) are the
// values the corrected state must carry.
static void rhs_with_refs(const or_model& m, const Coef& c, const double* z, double* dz) {
    rhs<double>(m, c, z, dz);
    const V3<double> v = get3(dz, 0);
    const V3<double> a = rr_accel(c, z, v);
    dz[12] = dot(v, a);
    const V3<double> dJ = cross(get3(z, 0), a);
    dz[13] = dJ.x; dz[14] = dJ.y; dz[15] = dJ.z;
}

// Total angular momentum J = r x p + S1 + S2.
template <class T>
static V3<T> total_J(const T* y) {
    return add(add(cross(get3(y, 0), get3(y, 3)), get3(y, 6)), get3(y, 9));
}

// ---------------------------------------------------------------------------
// Fixed-step Runge-Kutta on a D-dimensional system y' = f(y).
// RK4: classical Kutta tableau.  RK5: the fifth-order weights of the
// Dormand-Prince 5(4) pair used as a plain fixed-step six-stage method.
// ---------------------------------------------------------------------------
template <int D, class T, class F>
static void rk_step(int method, double h, F f, T* y) {
    if (method == 0) {
        T k1[D], k2[D], k3[D], k4[D], tmp[D];
        f(y, k1);
        for (int i = 0; i < D; ++i) tmp[i] = y[i] + (h / 2.0) * k1[i];
        f(tmp, k2);
        for (int i = 0; i < D; ++i) tmp[i] = y[i] + (h / 2.0) * k2[i];
        f(tmp, k3);
        for (int i = 0; i < D; ++i) tmp[i] = y[i] + h * k3[i];
        f(tmp, k4);
        for (int i = 0; i < D; ++i)
            y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        return;
    }
    // Dormand-Prince coefficients (Butcher tableau rows a_ij, weights b_i).
    static const double a21 = 1.0 / 5.0;
    static const double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    static const double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    static const double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0,
                        a53 = 64448.0 / 6561.0, a54 = -212.0 / 729.0;
    static const double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                        a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    static const double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                        b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    T k1[D], k2[D], k3[D], k4[D], k5[D], k6[D], tmp[D];
    f(y, k1);
    for (int i = 0; i < D; ++i) tmp[i] = y[i] + h * (a21 * k1[i]);
    f(tmp, k2);
    for (int i = 0; i < D; ++i) tmp[i] = y[i] + h * (a31 * k1[i] + a32 * k2[i]);
    f(tmp, k3);
    for (int i = 0; i < D; ++i) tmp[i] = y[i] + h * (a41 * k1[i] + a42 * k2[i] + a43 * k3[i]);
    f(tmp, k4);
    for (int i = 0; i < D; ++i)
        tmp[i] = y[i] + h * (a51 * k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i]);
    f(tmp, k5);
    for (int i = 0; i < D; ++i)
        tmp[i] = y[i] + h * (a61 * k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] + a65 * k5[i]);
    f(tmp, k6);
    for (int i = 0; i < D; ++i)
        y[i] = y[i] + h * (b1 * k1[i] + b3 * k3[i] + b4 * k4[i] + b5 * k5[i] + b6 * k6[i]);
}

// ---------------------------------------------------------------------------
// Manifold correction.
// ---------------------------------------------------------------------------

// eq. (10): restore the spin lengths, S_i <- s_i S_i* / |S_i*|.
template <class T>
static void correct_spins(const Coef& c, T* y) {
    V3<T> S1 = get3(y, 6), S2 = get3(y, 9);
    const T l1 = sqrt(dot(S1, S1));
    const T l2 = sqrt(dot(S2, S2));
    if (val(l1) > 0.0) S1 = scl(c.s1 / l1, S1);
    if (val(l2) > 0.0) S2 = scl(c.s2 / l2, S2);
    put3(y, 6, S1);
    put3(y, 9, S2);
}

// Energy by momentum scaling (velocity scaling, cited in Sec. 1): find a with
// H(r, a p, S) = E0 by Newton's method, g(a) = H - E0, g'(a) = dH/dp(r, a p, S) . p.
// Returns the iteration count; *conv = false when the cap was reached.
template <class T>
static int energy_scale(const or_model& m, const Coef& c, const or_correction& cc,
                        T* y, double E0, bool* conv) {
    const V3<T> p0 = get3(y, 3);
    T a = T(1.0);
    T ys[12];
    int it = 0;
    *conv = false;
    while (it < cc.max_iter) {
        for (int i = 0; i < 12; ++i) ys[i] = y[i];
        put3(ys, 3, scl(a, p0));
        const T g = hamiltonian(m, c, ys) - E0;
        const Grad<T> gr = gradient(m, c, ys, true);
        const T dg = dot(gr.dp, p0);
        const T da = -(g / dg);
        a = a + da;
        ++it;
        if (val(fabs(da)) <= cc.tol) { *conv = true; break; }
    }
    put3(y, 3, scl(a, p0));
    return it;
}

// Joint least-squares projection onto the four integrals H = E0 and
// J = J0 (Nacozy's shortest path, cited in Sec. 1), spins held fixed: the
// smallest (dr, dp) in the Euclidean norm that satisfies the linearised
// constraints G d = -c, with G the 4x6 Jacobian of (J, H) in (r, p) and c the
// residual: d = -G^T lam with (G G^T) lam = c.  The system is solved by block
// elimination of the J block M (3x3, Cholesky): with M u = c_J, M v = a (a the
// J-energy coupling column), the energy multiplier is t/s where s = A33 - a.v
// is the Schur complement and t = c_E - a.u the reduced residual.  Near
// circular orbits the energy row becomes dependent on the J rows (a circular
// orbit extremises H at fixed J) and s -> 0; the multiplier is then damped
// smoothly, lam_E = t s / (s^2 + (mu A33)^2), so that it never amplifies the
// rounding of the energy residual by more than 1/(2 mu A33).  Whatever energy
// error remains goes to the momentum scaling that follows.
template <class T>
static void project_EJ(const or_model& m, const Coef& c, T* y, const double* ref, double mu) {
    const V3<T> r = get3(y, 0), p = get3(y, 3);
    const Grad<T> g = gradient(m, c, y);
    const T H = hamiltonian(m, c, y);
    const V3<T> J = total_J(y);
    // Rows 0..2: grad of J_k = (p x e_k, e_k x r); row 3: grad H = (dH/dr, dH/dp).
    const T rv[3] = {r.x, r.y, r.z}, pv[3] = {p.x, p.y, p.z};
    const T rr = dot(r, r), pp = dot(p, p);
    T M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i][j] = (i == j ? rr + pp : T(0.0)) - rv[i] * rv[j] - pv[i] * pv[j];
    // (p x e_k).dH/dr + (e_k x r).dH/dp = e_k . (dH/dr x p + r x dH/dp)
    const V3<T> cx = add(cross(g.dr, p), cross(r, g.dp));
    const T a[3] = {cx.x, cx.y, cx.z};
    const T A33 = dot(g.dr, g.dr) + dot(g.dp, g.dp);
    const T cJ[3] = {J.x - ref[1], J.y - ref[2], J.z - ref[3]};
    const T cE = H - ref[0];
    // Cholesky of the J block, M = L L^T.
    T L[3][3] = {{T(0.0), T(0.0), T(0.0)}, {T(0.0), T(0.0), T(0.0)}, {T(0.0), T(0.0), T(0.0)}};
    for (int j = 0; j < 3; ++j) {
        T s = M[j][j];
        for (int k = 0; k < j; ++k) s = s - L[j][k] * L[j][k];
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < 3; ++i) {
            T t = M[i][j];
            for (int k = 0; k < j; ++k) t = t - L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    auto solve = [&](const T* b, T* x) {
        T z[3];
        for (int i = 0; i < 3; ++i) {
            T t = b[i];
            for (int k = 0; k < i; ++k) t = t - L[i][k] * z[k];
            z[i] = t / L[i][i];
        }
        for (int i = 2; i >= 0; --i) {
            T t = z[i];
            for (int k = i + 1; k < 3; ++k) t = t - L[k][i] * x[k];
            x[i] = t / L[i][i];
        }
    };
    T u[3], v[3];
    solve(cJ, u);
    solve(a, v);
    const T s = A33 - (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]);
    const T t = cE - (a[0] * u[0] + a[1] * u[1] + a[2] * u[2]);
    const T damp = mu * A33;
    const T lamE = t * s / (s * s + damp * damp);
    const V3<T> lJ = v3<T>(u[0] - v[0] * lamE, u[1] - v[1] * lamE, u[2] - v[2] * lamE);
    // d = -G^T lam: dr = -(p x lamJ) - lamE dH/dr, dp = -(lamJ x r) - lamE dH/dp.
    const V3<T> dr = sub(scl(-1.0, cross(p, lJ)), scl(lamE, g.dr));
    const V3<T> dp = sub(scl(-1.0, cross(lJ, r)), scl(lamE, g.dp));
    put3(y, 0, add(r, dr));
    put3(y, 3, add(p, dp));
}

// Dual scaling, eqs. (11)-(13): p = alpha p*, r = b r* (the paper calls the
// second factor beta; b avoids the clash with the mass ratio).  Newton on
//   f1 = H(b r*, alpha p*, S) - E0,  f2 = |alpha b L* + S1 + S2| - |J0|,
// which is Gauss-Newton on Phi of eq. (12) and shares its root for any
// positive weights.  When the 2x2 Jacobian is near singular (the two
// constraints are then locally dependent) the step falls back to energy-only
// momentum scaling.
template <class T>
static int dual_scale(const or_model& m, const Coef& c, const or_correction& cc,
                      T* y, double E0, double J0norm, bool* conv, bool* singular) {
    const V3<T> r0 = get3(y, 0), p0 = get3(y, 3), S1 = get3(y, 6), S2 = get3(y, 9);
    const V3<T> L0 = cross(r0, p0);
    const V3<T> Ssum = add(S1, S2);
    T al = T(1.0), b = T(1.0);
    T ys[12];
    int it = 0;
    *conv = false;
    *singular = false;
    while (it < cc.max_iter) {
        for (int i = 0; i < 12; ++i) ys[i] = y[i];
        put3(ys, 0, scl(b, r0));
        put3(ys, 3, scl(al, p0));
        const T f1 = hamiltonian(m, c, ys) - E0;
        const Grad<T> gr = gradient(m, c, ys);
        const V3<T> J = add(scl(al * b, L0), Ssum);
        const T Jn = sqrt(dot(J, J));
        const T f2 = Jn - J0norm;
        const T JhL = dot(J, L0) / Jn;           // Jhat . L*
        const T j11 = dot(gr.dp, p0);            // df1/dalpha
        const T j12 = dot(gr.dr, r0);            // df1/db
        const T j21 = b * JhL;                   // df2/dalpha
        const T j22 = al * JhL;                  // df2/db
        const T det = j11 * j22 - j12 * j21;
        if (val(fabs(det)) < 1e-3 * val(fabs(j22)) * val(fabs(j11))) {
            *singular = true;
            break;
        }
        const T dal = -(j22 * f1 - j12 * f2) / det;
        const T db = -(-j21 * f1 + j11 * f2) / det;
        al = al + dal;
        b = b + db;
        ++it;
        if (val(fabs(dal)) <= cc.tol && val(fabs(db)) <= cc.tol) { *conv = true; break; }
    }
    if (*singular) {
        // Fall back: keep r*, restore the energy by momentum scaling.
        return it + energy_scale(m, c, cc, y, E0, conv);
    }
    put3(y, 0, scl(b, r0));
    put3(y, 3, scl(al, p0));
    return it;
}

// One correction of a state against its reference ref = (E0, J0x, J0y, J0z).
// Returns the Newton iteration count; sets *noconv when any solve hit the cap.
template <class T>
static int correct(const or_model& m, const Coef& c, const or_correction& cc,
                   T* y, const double* ref, bool* noconv) {
    *noconv = false;
    if (cc.mode == 0) return 0;
    correct_spins(c, y);  // eq. (10) comes first in every mode
    if (cc.mode == 1) return 0;
    int iters = 0;
    bool conv = true;
    if (cc.mode == 2) {
        for (int s = 0; s < cc.sweeps; ++s) {
            project_EJ(m, c, y, ref, PN_SIX_MU);
            iters += energy_scale(m, c, cc, y, ref[0], &conv);
            if (!conv) *noconv = true;
        }
        return iters;
    }
    // mode 3: dual scaling.
    const double J0n = std::sqrt(ref[1] * ref[1] + ref[2] * ref[2] + ref[3] * ref[3]);
    bool sing = false;
    iters = dual_scale(m, c, cc, y, ref[0], J0n, &conv, &sing);
    if (!conv) *noconv = true;
    return iters;
}

// One integration step: RK then correction.
template <class T>
static int step_once(const or_model& m, const Coef& c, const or_integrator& in,
                     const or_correction& cc, T* y, const double* ref, bool* noconv) {
    auto f = [&](const T* yy, T* dd) { rhs(m, c, yy, dd); };
    rk_step<12>(in.method, in.h, f, y);
    return correct(m, c, cc, y, ref, noconv);
}

// One step of the dissipative system: the state and its references advance
// together with the same Runge-Kutta stages, then the state is corrected
// against the advanced references.
static int step_once_rr(const or_model& m, const Coef& c, const or_integrator& in,
                        const or_correction& cc, double* y, double* ref, bool* noconv) {
    double z[16];
    for (int i = 0; i < 12; ++i) z[i] = y[i];
    for (int i = 0; i < 4; ++i) z[12 + i] = ref[i];
    auto f = [&](const double* zz, double* dd) { rhs_with_refs(m, c, zz, dd); };
    rk_step<16>(in.method, in.h, f, z);
    for (int i = 0; i < 12; ++i) y[i] = z[i];
    for (int i = 0; i < 4; ++i) ref[i] = z[12 + i];
    return correct(m, c, cc, y, ref, noconv);
}

// Orbit validity (Sec. 3C removes unbounded or merged orbits).
template <class T>
static int validity(const or_fli_cfg& fc, const T* y) {
    for (int i = 0; i < 12; ++i)
        if (!isfinite(y[i])) return ST_NONFINITE;
    const double r = std::sqrt(val(y[0]) * val(y[0]) + val(y[1]) * val(y[1]) + val(y[2]) * val(y[2]));
    if (r < fc.r_merge) return ST_MERGED;
    if (r > fc.r_esc) return ST_ESCAPED;
    return ST_OK;
}

template <class T>
static void capture_ref(const or_model& m, const Coef& c, const T* y, double* ref) {
    ref[0] = val(hamiltonian(m, c, y));
    const V3<T> J = total_J(y);
    ref[1] = val(J.x); ref[2] = val(J.y); ref[3] = val(J.z);
}

static double threshold(const or_fli_cfg& fc, double t_end) {
    if (fc.thr_scaling == 1 && t_end > 0.0) return fc.thr_at_1e5 + std::log10(t_end / 1e5);
    return fc.thr_at_1e5;
}

// ---------------------------------------------------------------------------
// FLI run of one orbit and its shadow (Sec. 3B/3C, two nearby trajectories).
// Per step: both trajectories take an RK step and a correction against their
// own reference; the separation d over all 12 state components is measured;
// when d reaches d_renorm the accumulated sum gets log10(d/d0), the shadow is
// pulled back to distance d0 along the same direction, its spin lengths are
// restored and its reference integrals are re-captured.
// FLI(t_end) = sum + log10(d/d0).
// ---------------------------------------------------------------------------
struct FliResult {
    double fli;
    int8_t label;
    int32_t status;
    double y_final[12];
    double dH, dJ;
    int32_t newton_max;
    int64_t newton_total;
    int64_t renorms;
    int64_t steps_done;
};

template <class T>
static FliResult fli_run(const or_model& m, const Coef& c, const or_integrator& in,
                         const or_correction& cc, const or_fli_cfg& fc,
                         const double* y0, double t_end, double* trace, int64_t trace_every) {
    FliResult res;
    res.newton_max = 0;
    res.newton_total = 0;
    res.renorms = 0;
    res.steps_done = 0;
    res.status = ST_OK;
    T y[12], ys[12];
    for (int i = 0; i < 12; ++i) y[i] = T(y0[i]);
    // The reference integrals are taken after the spin lengths are set.
    correct_spins(c, y);
    for (int i = 0; i < 12; ++i) ys[i] = y[i];
    ys[fc.shadow_axis] = ys[fc.shadow_axis] + fc.d0;
    double ref[4], refs[4];
    capture_ref(m, c, y, ref);
    capture_ref(m, c, ys, refs);
    const int64_t nsteps = (t_end > 0.0) ? (int64_t)std::ceil(t_end / in.h) : 0;

    int st = validity(fc, y);
    if (st == ST_OK && !(ref[0] < 0.0)) st = ST_UNBOUND_INIT;

    T acc = T(0.0);
    bool any_noconv = false;
    for (int64_t k = 0; k < nsteps && st == ST_OK; ++k) {
        bool nc = false;
        int it = step_once(m, c, in, cc, y, ref, &nc);
        any_noconv = any_noconv || nc;
        res.newton_max = std::max(res.newton_max, it);
        res.newton_total += it;
        it = step_once(m, c, in, cc, ys, refs, &nc);
        any_noconv = any_noconv || nc;
        res.newton_max = std::max(res.newton_max, it);
        res.newton_total += it;
        res.steps_done = k + 1;
        st = validity(fc, y);
        if (st == ST_OK) st = validity(fc, ys);
        if (st != ST_OK) break;
        T d2 = T(0.0);
        for (int i = 0; i < 12; ++i) d2 = d2 + (ys[i] - y[i]) * (ys[i] - y[i]);
        const T d = sqrt(d2);
        if (val(d) >= fc.d_renorm) {
            acc = acc + log10(d / fc.d0);
            const T f = fc.d0 / d;
            for (int i = 0; i < 12; ++i) ys[i] = y[i] + f * (ys[i] - y[i]);
            correct_spins(c, ys);
            capture_ref(m, c, ys, refs);
            res.renorms += 1;
        }
        if (trace && trace_every > 0 && (k + 1) % trace_every == 0) {
            T e2 = T(0.0);
            for (int i = 0; i < 12; ++i) e2 = e2 + (ys[i] - y[i]) * (ys[i] - y[i]);
            trace[(k + 1) / trace_every - 1] = val(acc + log10(sqrt(e2) / fc.d0));
        }
    }
    for (int i = 0; i < 12; ++i) res.y_final[i] = val(y[i]);
    {
        const double H = val(hamiltonian(m, c, y));
        res.dH = std::fabs(H - ref[0]) / std::fabs(ref[0]);
        const V3<T> J = total_J(y);
        const double dx = val(J.x) - ref[1], dy = val(J.y) - ref[2], dz = val(J.z) - ref[3];
        const double j0 = std::sqrt(ref[1] * ref[1] + ref[2] * ref[2] + ref[3] * ref[3]);
        res.dJ = std::sqrt(dx * dx + dy * dy + dz * dz) / j0;
    }
    if (st == ST_OK) {
        T e2 = T(0.0);
        for (int i = 0; i < 12; ++i) e2 = e2 + (ys[i] - y[i]) * (ys[i] - y[i]);
        res.fli = val(acc + log10(sqrt(e2) / fc.d0));
        res.label = (res.fli > threshold(fc, t_end)) ? 1 : 0;
    } else {
        res.fli = NAN;
        res.label = -1;
    }
    res.status = st | (any_noconv ? ST_NEWTON_NOCONV : 0);
    return res;
}

// ---------------------------------------------------------------------------
// Initial conditions (Sec. 3B/3C, Sec. 4): r = (r0, 0, 0), p = (0, p0, 0),
// unit spins (sin th cos ph, sin th sin ph, cos th), S_i = s_i * unit spin.
// ---------------------------------------------------------------------------
static void init_state(const Coef& c, double r0, double p0, double th1, double ph1,
                       double th2, double ph2, double* y) {
    y[0] = r0; y[1] = 0.0; y[2] = 0.0;
    y[3] = 0.0; y[4] = p0; y[5] = 0.0;
    y[6] = c.s1 * std::sin(th1) * std::cos(ph1);
    y[7] = c.s1 * std::sin(th1) * std::sin(ph1);
    y[8] = c.s1 * std::cos(th1);
    y[9] = c.s2 * std::sin(th2) * std::cos(ph2);
    y[10] = c.s2 * std::sin(th2) * std::sin(ph2);
    y[11] = c.s2 * std::cos(th2);
}

static inline double pick(const double* a, int64_t stride, int64_t i) { return a[stride * i]; }

// ===========================================================================
// extern "C" entry points (AoS: each state is 12 consecutive doubles).
// Parameters beta, chi1, chi2 are arrays with a stride (0 = one value for all).
// ===========================================================================
extern "C" {

// Coefficient table, for inspection by tests:
// out = [eta, cso1, cso2, c12, c11, c22, s1, s2].
void or_coefficients(const or_model* m, double beta, double chi1, double chi2, double* out) {
    const Coef c = make_coef(*m, beta, chi1, chi2);
    out[0] = c.eta; out[1] = c.cso1; out[2] = c.cso2; out[3] = c.c12;
    out[4] = c.c11; out[5] = c.c22; out[6] = c.s1; out[7] = c.s2;
}

void or_hamiltonian(const or_model* m, double beta, double chi1, double chi2,
                    int64_t n, const double* y, double* H) {
    const Coef c = make_coef(*m, beta, chi1, chi2);
    for (int64_t i = 0; i < n; ++i) H[i] = hamiltonian<double>(*m, c, y + 12 * i);
}

// Analytic gradient: g = (dH/dr, dH/dp, dH/dS1, dH/dS2) per state.
void or_gradient(const or_model* m, double beta, double chi1, double chi2,
                 int64_t n, const double* y, double* g) {
    const Coef c = make_coef(*m, beta, chi1, chi2);
    for (int64_t i = 0; i < n; ++i) {
        const Grad<double> gr = gradient<double>(*m, c, y + 12 * i);
        double* o = g + 12 * i;
        put3(o, 0, gr.dr); put3(o, 3, gr.dp); put3(o, 6, gr.dS1); put3(o, 9, gr.dS2);
    }
}

// Complex-step gradient of H: Im H(y + i delta e_k) / delta for each k.
void or_gradient_complex_step(const or_model* m, double beta, double chi1, double chi2,
                              int64_t n, const double* y, double delta, double* g) {
    const Coef c = make_coef(*m, beta, chi1, chi2);
    typedef std::complex<double> C;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 12; ++k) {
            C yc[12];
            for (int j = 0; j < 12; ++j) yc[j] = C(y[12 * i + j], 0.0);
            yc[k] = C(y[12 * i + k], delta);
            g[12 * i + k] = std::imag(hamiltonian<C>(*m, c, yc)) / delta;
        }
    }
}

void or_rhs(const or_model* m, const double* beta, const double* chi1, const double* chi2,
            int64_t pstride, int64_t n, const double* y, double* dydt) {
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        rhs<double>(*m, c, y + 12 * i, dydt + 12 * i);
    }
}

// H and J = r x p + S1 + S2 per state: out[4*i] = H, out[4*i+1..3] = J.
void or_invariants(const or_model* m, const double* beta, const double* chi1, const double* chi2,
                   int64_t pstride, int64_t n, const double* y, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        capture_ref<double>(*m, c, y + 12 * i, out + 4 * i);
    }
}

void or_init_state(const or_model* m, const double* beta, const double* chi1, const double* chi2,
                   int64_t pstride, int64_t n, const double* r0, const double* p0,
                   const double* th1, const double* ph1, const double* th2, const double* ph2,
                   double* y) {
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        init_state(c, r0[i], p0[i], th1[i], ph1[i], th2[i], ph2[i], y + 12 * i);
    }
}

// One correction of each state against ref (4 doubles per state: E0, J0).
// iters[i] receives the Newton iteration count (negative when not converged).
void or_manifold_correct(const or_model* m, const double* beta, const double* chi1,
                         const double* chi2, int64_t pstride, const or_correction* cc,
                         int64_t n, double* y, const double* ref, int32_t* iters) {
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        bool nc = false;
        const int it = correct<double>(*m, c, *cc, y + 12 * i, ref + 4 * i, &nc);
        if (iters) iters[i] = nc ? -it : it;
    }
}

// nsteps steps (RK + optional correction) of each state.  When ref is NULL
// the references are captured from each state after its spin lengths are set
// (only when a correction is requested).  With radiation reaction the
// references advance with the state and are written back to ref (when given).
void or_step(const or_model* m, const double* beta, const double* chi1, const double* chi2,
             int64_t pstride, const or_integrator* in, const or_correction* cc,
             int64_t n, double* y, double* ref, int64_t nsteps) {
    or_correction none;
    std::memset(&none, 0, sizeof(none));
    const or_correction& use = cc ? *cc : none;
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        double* yi = y + 12 * i;
        double r[4];
        if (ref) {
            for (int k = 0; k < 4; ++k) r[k] = ref[4 * i + k];
        } else {
            if (use.mode != 0) correct_spins(c, yi);
            capture_ref<double>(*m, c, yi, r);
        }
        for (int64_t k = 0; k < nsteps; ++k) {
            bool nc = false;
            if (m->rad_reaction)
                step_once_rr(*m, c, *in, use, yi, r, &nc);
            else
                step_once<double>(*m, c, *in, use, yi, r, &nc);
        }
        if (ref && m->rad_reaction)
            for (int k = 0; k < 4; ++k) ref[4 * i + k] = r[k];
    }
}

// One Runge-Kutta step of the scalar linear equation y' = z y from y = 1 with
// h = 1: returns the stability function R(z) of the chosen tableau.
double or_rk_linear_step(int32_t method, double z) {
    double y[1] = {1.0};
    auto f = [&](const double* yy, double* dd) { dd[0] = z * yy[0]; };
    rk_step<1>(method, 1.0, f, y);
    return y[0];
}

// Full FLI run for n orbits, parallel over orbits with nthreads std::threads.
// Outputs (each nullable except fli/label/status): y_final[12*n], dH[n], dJ[n],
// newton_max[n], renorms[n], steps[n] (steps the orbit completed before its
// run ended), trace[n * ntrace] with ntrace = nsteps/trace_every.
void or_fli_scan(const or_model* m, const double* beta, const double* chi1, const double* chi2,
                 int64_t pstride, const or_integrator* in, const or_correction* cc,
                 const or_fli_cfg* fc, int64_t n, const double* y0, const double* t_end,
                 int64_t tstride, double* fli, int8_t* label, int32_t* status,
                 double* y_final, double* dH, double* dJ, int32_t* newton_max,
                 int64_t* renorms, int64_t* steps, double* trace, int64_t trace_every,
                 int64_t ntrace, int32_t nthreads) {
    std::atomic<int64_t> next(0);
    auto worker = [&]() {
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= n) break;
            // Scans follow the conservative system (the paper's scans of
            // Sec. 3C); a model with radiation reaction is refused per orbit.
            if (m->rad_reaction ||
                !params_valid(pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i))) {
                fli[i] = NAN;
                label[i] = -1;
                status[i] = ST_BADPARAM;
                if (y_final) for (int k = 0; k < 12; ++k) y_final[12 * i + k] = y0[12 * i + k];
                if (dH) dH[i] = NAN;
                if (dJ) dJ[i] = NAN;
                if (newton_max) newton_max[i] = 0;
                if (renorms) renorms[i] = 0;
                if (steps) steps[i] = 0;
                continue;
            }
            const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
            const FliResult r = fli_run<double>(*m, c, *in, *cc, *fc, y0 + 12 * i, t_end[tstride * i],
                                                trace ? trace + ntrace * i : nullptr, trace_every);
            fli[i] = r.fli;
            label[i] = r.label;
            status[i] = r.status;
            if (y_final) for (int k = 0; k < 12; ++k) y_final[12 * i + k] = r.y_final[k];
            if (dH) dH[i] = r.dH;
            if (dJ) dJ[i] = r.dJ;
            if (newton_max) newton_max[i] = r.newton_max;
            if (renorms) renorms[i] = r.renorms;
            if (steps) steps[i] = r.steps_done;
        }
    };
    if (nthreads <= 1) {
        worker();
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < nthreads; ++t) th.emplace_back(worker);
        for (auto& t : th) t.join();
    }
}

// Algorithmic flop counts with the counting scalar.
// out = [rhs, rk_step (incl. its RHS calls), correction (mean per call over the
//        run), fli run total, orbit-steps done, newton total, renorms].
void or_count_flops(const or_model* m, double beta, double chi1, double chi2,
                    const or_integrator* in, const or_correction* cc, const or_fli_cfg* fc,
                    const double* y0, double t_end, double* out) {
    const Coef c = make_coef(*m, beta, chi1, chi2);
    Counted y[12], d[12];
    for (int i = 0; i < 12; ++i) y[i] = Counted(y0[i]);
    g_flops = 0;
    rhs<Counted>(*m, c, y, d);
    out[0] = (double)g_flops;
    g_flops = 0;
    {
        Counted yy[12];
        for (int i = 0; i < 12; ++i) yy[i] = y[i];
        auto f = [&](const Counted* a, Counted* b) { rhs<Counted>(*m, c, a, b); };
        rk_step<12>(in->method, in->h, f, yy);
        out[1] = (double)g_flops;
        double ref[4];
        capture_ref<double>(*m, c, y0, ref);
        g_flops = 0;
        bool nc = false;
        correct<Counted>(*m, c, *cc, yy, ref, &nc);
        out[2] = (double)g_flops;
    }
    g_flops = 0;
    const FliResult r = fli_run<Counted>(*m, c, *in, *cc, *fc, y0, t_end, nullptr, 0);
    out[3] = (double)g_flops;
    out[4] = (double)r.steps_done;
    out[5] = (double)r.newton_total;
    out[6] = (double)r.renorms;
}

// Gravitational-wave polarisations, Sec. 4, eq. (14), from the leading
// (mass-quadrupole) radiation field written out as its definition:
//   h_ij    = (4 eta / D) (v_i v_j - n_i n_j / r)      (G = c = M = 1, D in M)
//   h^TT    = P h P - (1/2) P tr(P h),   P = I - N N^T   (transverse-traceless part)
//   h_plus  = (1/2) (p_i p_j - q_i q_j) h^TT_ij
//   h_cross = (1/2) (p_i q_j + q_i p_j) h^TT_ij,        q = N x p
// with v = dr/dt = dH/dp (eq. 6) and eta = mu / M.  N points from the source to
// the observer and p lies along the line of nodes (Sec. 4).  States y are n
// rows of 12; out[2*i] = h_plus, out[2*i+1] = h_cross.
void or_gw_polarizations(const or_model* m, const double* beta, const double* chi1, const double* chi2,
                         int64_t pstride, int64_t n, const double* y, const double* N, const double* pn,
                         double dist, double* out) {
    double q[3] = {N[1] * pn[2] - N[2] * pn[1], N[2] * pn[0] - N[0] * pn[2], N[0] * pn[1] - N[1] * pn[0]};
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - N[a] * N[b];
    for (int64_t i = 0; i < n; ++i) {
        const Coef c = make_coef(*m, pick(beta, pstride, i), pick(chi1, pstride, i), pick(chi2, pstride, i));
        const double* yi = y + 12 * i;
        const Grad<double> g = gradient<double>(*m, c, yi);
        const double v[3] = {g.dp.x, g.dp.y, g.dp.z};
        const double r = std::sqrt(yi[0] * yi[0] + yi[1] * yi[1] + yi[2] * yi[2]);
        const double nn[3] = {yi[0] / r, yi[1] / r, yi[2] / r};
        double h[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) h[a][b] = 4.0 * c.eta / dist * (v[a] * v[b] - nn[a] * nn[b] / r);
        double Ph[3][3], PhP[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                Ph[a][b] = 0.0;
                for (int k = 0; k < 3; ++k) Ph[a][b] += P[a][k] * h[k][b];
            }
        double tr = Ph[0][0] + Ph[1][1] + Ph[2][2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                PhP[a][b] = 0.0;
                for (int k = 0; k < 3; ++k) PhP[a][b] += Ph[a][k] * P[k][b];
            }
        double hp = 0.0, hx = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double tt = PhP[a][b] - 0.5 * P[a][b] * tr;
                hp += 0.5 * (pn[a] * pn[b] - q[a] * q[b]) * tt;
                hx += 0.5 * (pn[a] * q[b] + q[a] * pn[b]) * tt;
            }
        out[2 * i] = hp;
        out[2 * i + 1] = hx;
    }
}

int32_t or_abi_version(void) { return 1; }

}  // extern "C"
