// pn_device.h -- register-resident FP64 physics of one trajectory per lane.
//
// Hamiltonian (arXiv:1802.00147, Sec. 2, eq. 1) per unit reduced mass in ADM
// variables, as a table-driven polynomial in P2 = p.p, NP = n.p and u = 1/r:
//   H_orb = P2/2 - u + a1 P2^2 + (a2 P2 + a3 NP^2) u + a4 u^2
//         + b1 P2^3 + (b2 P2^2 + b3 P2 NP^2 + b4 NP^4) u + (b5 P2 + b6 NP^2) u^2 + b7 u^3
//   H_SO  = u^3 L.(cso1 S1 + cso2 S2)                              (1.5PN spin-orbit)
//   H_SS  = u^3 { c12 [3 (S1.n)(S2.n) - S1.S2]                      (eq. 3)
//               + c11 [3 (S1.n)^2 - S1.S1] + c22 [3 (S2.n)^2 - S2.S2] }  (eqs. 4-5)
// Terms that a model switches off have zero coefficients, so every kernel
// evaluates one branch-free expression.  The gradient is written out by hand
// (combined terms, one reciprocal square root per evaluation); equations of
// motion follow eqs. (6)-(7).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pn.h"

#define PN_HD __host__ __device__ __forceinline__

#ifndef PN_SIX_MU
#define PN_SIX_MU 1e-5
#endif

struct PnCoef {
    double a1, a2, a3, a4;                 // 1PN
    double b1, b2, b3, b4, b5, b6, b7;     // 2PN
    double cso1, cso2, c12, c11, c22;      // spin couplings
    double s1, s2;                         // spin lengths
    // Multiples of the above that the equations of motion use, formed once
    // per table (pn_orbit_partials, pn_rhs_eval).
    double m4a1, m6b1, m2a2, m4b2, m2b3, m2b5;   // 2 dH/dP2
    double m2a3, m4b4, m2b6;                     // dH/dNP / (u NP), with m2b3
    double m2a4, m3b7;                           // dH/du, with m2b5 and m2b6
    double m3c12, m6c11, m6c22;                  // spin-spin weights w_i
};

// The multiples of a table's coefficients (the same IEEE products wherever
// they are formed).  A kernel whose orbits share one table receives it in
// scalar registers and re-forms these on the device, so that they sit in
// vector registers: the scalar registers then hold only the base table.
PN_HD void pn_coef_derive(PnCoef& k) {
    k.m4a1 = 4.0 * k.a1; k.m6b1 = 6.0 * k.b1; k.m2a2 = 2.0 * k.a2; k.m4b2 = 4.0 * k.b2;
    k.m2b3 = 2.0 * k.b3; k.m2b5 = 2.0 * k.b5;
    k.m2a3 = 2.0 * k.a3; k.m4b4 = 4.0 * k.b4; k.m2b6 = 2.0 * k.b6;
    k.m2a4 = 2.0 * k.a4; k.m3b7 = 3.0 * k.b7;
    k.m3c12 = 3.0 * k.c12; k.m6c11 = 6.0 * k.c11; k.m6c22 = 6.0 * k.c22;
}

// Coefficient table of one parameter set (Sec. 2: M = 1, eta = m1 m2).
// Returns false when beta or chi is out of range (or not finite).
PN_HD bool pn_make_coef(const pn_model& m, double beta, double chi1, double chi2, PnCoef& k) {
    const bool ok = (beta > 0.0) && (beta <= 1.0) && (chi1 >= 0.0) && (chi1 <= 1.0) &&
                    (chi2 >= 0.0) && (chi2 <= 1.0);
    if (!ok) beta = 1.0;  // keep the table finite; the caller flags the orbit
    const double m1 = beta / (1.0 + beta), m2 = 1.0 / (1.0 + beta);
    const double eta = m1 * m2;
    const double o1 = m.pn_order >= 1 ? 1.0 : 0.0;
    const double o2 = m.pn_order >= 2 ? 1.0 : 0.0;
    k.a1 = o1 * (3.0 * eta - 1.0) / 8.0;
    k.a2 = o1 * -(3.0 + eta) / 2.0;
    k.a3 = o1 * -eta / 2.0;
    k.a4 = o1 * 0.5;
    k.b1 = o2 * (1.0 - 5.0 * eta + 5.0 * eta * eta) / 16.0;
    k.b2 = o2 * (5.0 - 20.0 * eta - 3.0 * eta * eta) / 8.0;
    k.b3 = o2 * -(eta * eta) / 4.0;
    k.b4 = o2 * -3.0 * eta * eta / 8.0;
    k.b5 = o2 * (5.0 + 8.0 * eta) / 2.0;
    k.b6 = o2 * 3.0 * eta / 2.0;
    k.b7 = o2 * -(1.0 + 3.0 * eta) / 4.0;
    // Spin units: a spin in M^2 is eta times the same spin in mu M, so the
    // couplings linear in the spins (spin-orbit) carry one factor of eta and
    // the quadratic ones (eqs. 3-5) two factors relative to M^2 units, where
    // dH/dS_i reproduces eqs. (8)-(9) exactly.
    const double f = (m.spin_units == PN_SPIN_PHYS) ? eta : 1.0;
    const double so = m.spin_orbit ? 1.0 : 0.0;
    const double ss = m.spin_spin ? 1.0 : 0.0;
    const double qm = m.quad_mono ? 1.0 : 0.0;
    k.cso1 = so * f * (2.0 + 1.5 / beta);
    k.cso2 = so * f * (2.0 + 1.5 * beta);
    k.c12 = ss * f * f / eta;
    k.c11 = qm * f * f / (2.0 * beta * eta);
    k.c22 = qm * f * f * beta / (2.0 * eta);
    if (m.spin_units == PN_SPIN_PHYS) {
        k.s1 = chi1 * beta;         // chi1 m1^2 / (mu M)
        k.s2 = chi2 / beta;         // chi2 m2^2 / (mu M)
    } else {
        k.s1 = chi1 * m1 * m1;
        k.s2 = chi2 * m2 * m2;
    }
    pn_coef_derive(k);
    return ok;
}

// 1/sqrt(x) to ~1 ulp: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double pn_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// 1/x to ~1 ulp: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double pn_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    return y;
}

__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz) {
    return fma(ax, bx, fma(ay, by, az * bz));
}

// Partial derivatives of H_orb(P2, NP, u) in nested (Horner) form:
//   cp = 2 dH/dP2 = 1 + P2 (4 a1 + 6 b1 P2) + u (2 a2 + 4 b2 P2 + 2 b3 NP2 + 2 b5 u)
//   dH/dNP = NP u hw,  hw = 2 a3 + 2 b3 P2 + 4 b4 NP2 + 2 b6 u
//   dH/du = -1 + P2 (a2 + b2 P2 + b3 NP2) + NP2 (a3 + b4 NP2) + u (2 a4 + 2 b5 P2 + 2 b6 NP2 + 3 b7 u)
struct PnOrbPartials { double cp, hw, Hu, Hu0; };

__device__ __forceinline__ PnOrbPartials pn_orbit_partials(const PnCoef& k, double P2, double NP2, double u) {
    PnOrbPartials o;
    const double ca = fma(fma(k.m6b1, P2, k.m4a1), P2, 1.0);
    const double cb = fma(k.m2b5, u, fma(k.m2b3, NP2, fma(k.m4b2, P2, k.m2a2)));
    o.cp = fma(cb, u, ca);
    o.hw = fma(k.m2b6, u, fma(k.m4b4, NP2, fma(k.m2b3, P2, k.m2a3)));
    const double t1 = fma(k.b3, NP2, fma(k.b2, P2, k.a2));
    const double t2 = fma(k.b4, NP2, k.a3);
    const double t3 = fma(k.m3b7, u, fma(k.m2b6, NP2, fma(k.m2b5, P2, k.m2a4)));
    o.Hu0 = fma(t2, NP2, fma(t1, P2, -1.0));
    o.Hu = fma(t3, u, o.Hu0);
    return o;
}

// Right-hand side: f = (dH/dp, -dH/dr, Omega1 x S1, Omega2 x S2).
__device__ __forceinline__ void pn_rhs_eval(const PnCoef& k, const double* y, double* f) {
    const double rx = y[0], ry = y[1], rz = y[2];
    const double px = y[3], py = y[4], pz = y[5];
    const double s1x = y[6], s1y = y[7], s1z = y[8];
    const double s2x = y[9], s2y = y[10], s2z = y[11];
    const double r2 = dot3(rx, ry, rz, rx, ry, rz);
    const double u = pn_rsqrt(r2);
    const double u2 = u * u, u3 = u2 * u, u4 = u2 * u2;
    const double nx = rx * u, ny = ry * u, nz = rz * u;
    const double P2 = dot3(px, py, pz, px, py, pz);
    const double NP = dot3(nx, ny, nz, px, py, pz);
    const double NP2 = NP * NP;
    const PnOrbPartials o = pn_orbit_partials(k, P2, NP2, u);
    const double HNP = (u * o.hw) * NP;   // dH/dNP
    const double Ap = HNP * u;

    // Spin geometry; eu = u^3 S_eff, S_eff = cso1 S1 + cso2 S2.
    const double Lx = ry * pz - rz * py, Ly = rz * px - rx * pz, Lz = rx * py - ry * px;
    const double A1 = u3 * k.cso1, A2 = u3 * k.cso2, C12 = u3 * k.c12;
    const double eux = fma(A1, s1x, A2 * s2x);
    const double euy = fma(A1, s1y, A2 * s2y);
    const double euz = fma(A1, s1z, A2 * s2z);
    const double LSu = dot3(Lx, Ly, Lz, eux, euy, euz);   // u^3 L.S_eff
    const double sn1 = dot3(s1x, s1y, s1z, nx, ny, nz);
    const double sn2 = dot3(s2x, s2y, s2z, nx, ny, nz);
    const double S12 = dot3(s1x, s1y, s1z, s2x, s2y, s2z);
    const double S11 = dot3(s1x, s1y, s1z, s1x, s1y, s1z);
    const double S22 = dot3(s2x, s2y, s2z, s2x, s2y, s2z);
    // Spin-spin weights: dH/dS_i holds u^3 w_i n (eqs. 3-5).
    const double w1 = fma(k.m3c12, sn2, k.m6c11 * sn1);
    const double w2 = fma(k.m3c12, sn1, k.m6c22 * sn2);
    // Bracket of dH/dr along n (eqs. 3-5): sum c (5 a a - S.S), with
    // w1 a1 + w2 a2 = 6 sum c a a.
    const double Hss5 = fma(5.0 / 6.0, fma(w1, sn1, w2 * sn2), -fma(k.c12, S12, fma(k.c11, S11, k.c22 * S22)));

    // dH/dp = cp p + HNP n + u^3 (S_eff x r).
    f[0] = fma(euy, rz, fma(-euz, ry, fma(HNP, nx, o.cp * px)));
    f[1] = fma(euz, rx, fma(-eux, rz, fma(HNP, ny, o.cp * py)));
    f[2] = fma(eux, ry, fma(-euy, rx, fma(HNP, nz, o.cp * pz)));

    // dH/dr = An n + Ap p + u^4 (w1 S1 + w2 S2) + u^3 (p x S_eff),
    // An = -Ap NP - Hu u^2 - 3 u^4 (L.S_eff + Hss5).
    const double An = fma(-3.0 * u, fma(u3, Hss5, LSu), fma(-o.Hu, u2, -Ap * NP));
    const double B1 = u4 * w1, B2 = u4 * w2;
    f[3] = -fma(euz, py, fma(-euy, pz, fma(B2, s2x, fma(B1, s1x, fma(Ap, px, An * nx)))));
    f[4] = -fma(eux, pz, fma(-euz, px, fma(B2, s2y, fma(B1, s1y, fma(Ap, py, An * ny)))));
    f[5] = -fma(euy, px, fma(-eux, py, fma(B2, s2z, fma(B1, s1z, fma(Ap, pz, An * nz)))));

    // Spin precession, eq. (7): Omega1 = u^3 (cso1 L + w1 n - c12 S2), and
    // u^3 w1 n = u^4 w1 r = B1 r.
    const double o1x = fma(A1, Lx, fma(B1, rx, -C12 * s2x));
    const double o1y = fma(A1, Ly, fma(B1, ry, -C12 * s2y));
    const double o1z = fma(A1, Lz, fma(B1, rz, -C12 * s2z));
    const double o2x = fma(A2, Lx, fma(B2, rx, -C12 * s1x));
    const double o2y = fma(A2, Ly, fma(B2, ry, -C12 * s1y));
    const double o2z = fma(A2, Lz, fma(B2, rz, -C12 * s1z));
    f[6] = o1y * s1z - o1z * s1y;
    f[7] = o1z * s1x - o1x * s1z;
    f[8] = o1x * s1y - o1y * s1x;
    f[9] = o2y * s2z - o2z * s2y;
    f[10] = o2z * s2x - o2x * s2z;
    f[11] = o2x * s2y - o2y * s2x;
}

// Quantities of the spins alone, fixed while a correction moves r and p:
// the effective spin-orbit vector S_eff = cso1 S1 + cso2 S2 and the spin
// products.
struct PnSpinInv { double ex, ey, ez, S11, S22, S12, Sq; };

__device__ __forceinline__ PnSpinInv pn_spin_inv(const PnCoef& k, const double* y) {
    const double s1x = y[6], s1y = y[7], s1z = y[8];
    const double s2x = y[9], s2y = y[10], s2z = y[11];
    PnSpinInv v;
    v.ex = k.cso1 * s1x + k.cso2 * s2x;
    v.ey = k.cso1 * s1y + k.cso2 * s2y;
    v.ez = k.cso1 * s1z + k.cso2 * s2z;
    v.S11 = dot3(s1x, s1y, s1z, s1x, s1y, s1z);
    v.S22 = dot3(s2x, s2y, s2z, s2x, s2y, s2z);
    v.S12 = dot3(s1x, s1y, s1z, s2x, s2y, s2z);
    v.Sq = fma(k.c12, v.S12, fma(k.c11, v.S11, k.c22 * v.S22));   // sum c S.S of eqs. 3-5
    return v;
}

// Geometry of the position with fixed spins: u = 1/r and its powers, n, the
// spin projections a_i = S_i.n and the spin-spin brackets of H (3 a a - S.S,
// eqs. 3-5), of dH/dr along n (5 a a - S.S) and of dH/dr along S_i (w_i).
// It does not depend on p, so a momentum scaling leaves it valid.
struct PnRGeom { double u, u2, u3, u4, nx, ny, nz, Hss3, Hss5, w1, w2; };

__device__ __forceinline__ PnRGeom pn_rgeom(const PnCoef& k, const PnSpinInv& si, const double* y) {
    const double rx = y[0], ry = y[1], rz = y[2];
    PnRGeom g;
    g.u = pn_rsqrt(dot3(rx, ry, rz, rx, ry, rz));
    g.u2 = g.u * g.u;
    g.u3 = g.u2 * g.u;
    g.u4 = g.u2 * g.u2;
    g.nx = rx * g.u;
    g.ny = ry * g.u;
    g.nz = rz * g.u;
    const double sn1 = dot3(y[6], y[7], y[8], g.nx, g.ny, g.nz);
    const double sn2 = dot3(y[9], y[10], y[11], g.nx, g.ny, g.nz);
    g.w1 = fma(k.m3c12, sn2, k.m6c11 * sn1);
    g.w2 = fma(k.m3c12, sn1, k.m6c22 * sn2);
    // w1 a1 + w2 a2 = 6 sum c a a, so the brackets are multiples of it less sum c S.S.
    const double q6 = fma(g.w1, sn1, g.w2 * sn2);
    g.Hss3 = fma(0.5, q6, -si.Sq);
    g.Hss5 = fma(5.0 / 6.0, q6, -si.Sq);
    return g;
}

// Energy as a polynomial in a momentum scale factor a (r and spins fixed):
// H(r, a p, S) = K0 + K1 a + K2 a^2 + K4 a^4 + K6 a^6.
struct PnEnergyPoly { double K0, K1, K2, K4, K6; };

__device__ __forceinline__ PnEnergyPoly pn_energy_poly_g(const PnCoef& k, const PnSpinInv& si, const PnRGeom& g,
                                                         const double* y) {
    const double rx = y[0], ry = y[1], rz = y[2];
    const double px = y[3], py = y[4], pz = y[5];
    const double P2 = dot3(px, py, pz, px, py, pz);
    const double NP = dot3(g.nx, g.ny, g.nz, px, py, pz);
    const double NP2 = NP * NP;
    const double Lx = ry * pz - rz * py, Ly = rz * px - rx * pz, Lz = rx * py - ry * px;
    const double LS = dot3(Lx, Ly, Lz, si.ex, si.ey, si.ez);
    PnEnergyPoly e;
    e.K0 = -g.u + k.a4 * g.u2 + k.b7 * g.u3 + g.u3 * g.Hss3;
    e.K1 = g.u3 * LS;
    e.K2 = 0.5 * P2 + fma(k.a2, P2, k.a3 * NP2) * g.u + fma(k.b5, P2, k.b6 * NP2) * g.u2;
    e.K4 = k.a1 * P2 * P2 + (k.b2 * P2 * P2 + k.b3 * P2 * NP2 + k.b4 * NP2 * NP2) * g.u;
    e.K6 = k.b1 * P2 * P2 * P2;
    return e;
}

__device__ __forceinline__ PnEnergyPoly pn_energy_poly(const PnCoef& k, const double* y) {
    const PnSpinInv si = pn_spin_inv(k, y);
    return pn_energy_poly_g(k, si, pn_rgeom(k, si, y), y);
}

__device__ __forceinline__ double pn_energy(const PnCoef& k, const double* y) {
    const PnEnergyPoly e = pn_energy_poly(k, y);
    return e.K0 + e.K1 + e.K2 + e.K4 + e.K6;
}

// H and its gradient with respect to r and p (spins held fixed), given the
// geometry of r.
__device__ __forceinline__ void pn_energy_grad_g(const PnCoef& k, const PnSpinInv& si, const PnRGeom& g,
                                                 const double* y, double& H, double* gr, double* gp) {
    const double rx = y[0], ry = y[1], rz = y[2];
    const double px = y[3], py = y[4], pz = y[5];
    const double u = g.u, u2 = g.u2, u3 = g.u3, u4 = g.u4;
    const double nx = g.nx, ny = g.ny, nz = g.nz;
    const double ex = si.ex, ey = si.ey, ez = si.ez;
    const double P2 = dot3(px, py, pz, px, py, pz);
    const double NP = dot3(nx, ny, nz, px, py, pz);
    const double NP2 = NP * NP;
    const PnOrbPartials o = pn_orbit_partials(k, P2, NP2, u);
    const double HNP = (u * o.hw) * NP;
    const double Ap = HNP * u;
    const double Lx = ry * pz - rz * py, Ly = rz * px - rx * pz, Lz = rx * py - ry * px;
    const double LS = dot3(Lx, Ly, Lz, ex, ey, ez);
    // H = P2 (1/2 + P2 (a1 + b1 P2)) + u (dH/du at u = 0 + u (a4 + b5 P2 + b6 NP2 + u (b7 + LS + Hss3))).
    const double hA = fma(fma(k.b1, P2, k.a1), P2, 0.5) * P2;
    const double hB = fma(k.b7 + (LS + g.Hss3), u, fma(k.b6, NP2, fma(k.b5, P2, k.a4)));
    H = fma(fma(hB, u, o.Hu0), u, hA);
    const double eux = u3 * ex, euy = u3 * ey, euz = u3 * ez;
    gp[0] = fma(euy, rz, fma(-euz, ry, fma(HNP, nx, o.cp * px)));
    gp[1] = fma(euz, rx, fma(-eux, rz, fma(HNP, ny, o.cp * py)));
    gp[2] = fma(eux, ry, fma(-euy, rx, fma(HNP, nz, o.cp * pz)));
    const double An = fma(-3.0 * u4, LS + g.Hss5, fma(-o.Hu, u2, -Ap * NP));
    const double B1 = u4 * g.w1, B2 = u4 * g.w2;
    gr[0] = fma(euz, py, fma(-euy, pz, fma(B2, y[9], fma(B1, y[6], fma(Ap, px, An * nx)))));
    gr[1] = fma(eux, pz, fma(-euz, px, fma(B2, y[10], fma(B1, y[7], fma(Ap, py, An * ny)))));
    gr[2] = fma(euy, px, fma(-eux, py, fma(B2, y[11], fma(B1, y[8], fma(Ap, pz, An * nz)))));
}

__device__ __forceinline__ void pn_energy_grad_rp(const PnCoef& k, const double* y, double& H,
                                                  double* gr, double* gp) {
    const PnSpinInv si = pn_spin_inv(k, y);
    pn_energy_grad_g(k, si, pn_rgeom(k, si, y), y, H, gr, gp);
}

// Total angular momentum J = r x p + S1 + S2.
__device__ __forceinline__ void pn_total_J(const double* y, double* J) {
    J[0] = y[1] * y[5] - y[2] * y[4] + y[6] + y[9];
    J[1] = y[2] * y[3] - y[0] * y[5] + y[7] + y[10];
    J[2] = y[0] * y[4] - y[1] * y[3] + y[8] + y[11];
}

// eq. (10): S_i <- s_i S_i / |S_i| (a zero spin stays zero).
__device__ __forceinline__ void pn_correct_spins(const PnCoef& k, double* y) {
    const double l1 = dot3(y[6], y[7], y[8], y[6], y[7], y[8]);
    const double l2 = dot3(y[9], y[10], y[11], y[9], y[10], y[11]);
    const double f1 = l1 > 0.0 ? k.s1 * pn_rsqrt(l1) : 0.0;
    const double f2 = l2 > 0.0 ? k.s2 * pn_rsqrt(l2) : 0.0;
    y[6] *= f1; y[7] *= f1; y[8] *= f1;
    y[9] *= f2; y[10] *= f2; y[11] *= f2;
}

// 1/x to a relative error near the square of the hardware estimate's (one
// Newton step): for the Newton updates and the multipliers of the
// projection, whose results are corrections of order 1e-10 of the state and
// need far fewer correct bits than the state itself.
__device__ __forceinline__ double pn_rcp1(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// Energy restoration by momentum scaling: Newton on a for
// g(a) = H(r, a p, S) - E0 using the polynomial form of H in a.
// Returns the iteration count; *conv is false if max_iter was reached.
__device__ __forceinline__ int pn_energy_scale_poly(const PnEnergyPoly& e, double* y, double E0, double tol,
                                                    int max_iter, bool& conv) {
    double a = 1.0;
    int it = 0;
    conv = false;
    while (it < max_iter) {
        const double a2 = a * a, a3 = a2 * a;
        const double g = fma(fma(fma(e.K6, a2, e.K4), a2, e.K2), a2, fma(e.K1, a, e.K0)) - E0;
        const double dg = fma(fma(6.0 * e.K6, a2, 4.0 * e.K4), a3, fma(2.0 * e.K2, a, e.K1));
        const double da = -g * pn_rcp1(dg);
        a += da;
        ++it;
        if (fabs(da) <= tol) { conv = true; break; }
    }
    y[3] *= a; y[4] *= a; y[5] *= a;
    return it;
}

__device__ __forceinline__ int pn_energy_scale(const PnCoef& k, double* y, double E0, double tol,
                                               int max_iter, bool& conv) {
    return pn_energy_scale_poly(pn_energy_poly(k, y), y, E0, tol, max_iter, conv);
}

// Least-squares projection of (r, p) onto H = E0, J = J0 (spins fixed): the
// smallest displacement d with G d = -c, d = -G^T lam, (G G^T) lam = c, where
// the rows of G are grad J_x, grad J_y, grad J_z, grad H.  Solved by LDL^T.
// Near circular orbits the energy row is nearly a combination of the J rows
// and its pivot d3 vanishes; its multiplier is damped (Tikhonov),
// lam3 = z3 d3 / (d3^2 + (mu A33)^2) with mu = PN_SIX_MU, which bounds how far
// rounding in z3 can move the state.  g is the geometry of the current r.
__device__ __forceinline__ void pn_project_EJ_g(const PnCoef& k, const PnSpinInv& si, const PnRGeom& geo,
                                                double* y, const double* ref) {
    double H, gr[3], gp[3], J[3];
    pn_energy_grad_g(k, si, geo, y, H, gr, gp);
    pn_total_J(y, J);
    const double rx = y[0], ry = y[1], rz = y[2];
    const double px = y[3], py = y[4], pz = y[5];
    const double s = dot3(rx, ry, rz, rx, ry, rz) + dot3(px, py, pz, px, py, pz);
    const double A00 = s - rx * rx - px * px, A11 = s - ry * ry - py * py, A22 = s - rz * rz - pz * pz;
    const double A10 = -(ry * rx + py * px), A20 = -(rz * rx + pz * px), A21 = -(rz * ry + pz * py);
    // Cross terms e_k . (dH/dr x p + r x dH/dp).
    const double A30 = (gr[1] * pz - gr[2] * py) + (ry * gp[2] - rz * gp[1]);
    const double A31 = (gr[2] * px - gr[0] * pz) + (rz * gp[0] - rx * gp[2]);
    const double A32 = (gr[0] * py - gr[1] * px) + (rx * gp[1] - ry * gp[0]);
    const double A33 = dot3(gr[0], gr[1], gr[2], gr[0], gr[1], gr[2]) + dot3(gp[0], gp[1], gp[2], gp[0], gp[1], gp[2]);
    const double c0 = J[0] - ref[1], c1 = J[1] - ref[2], c2 = J[2] - ref[3], c3 = H - ref[0];
    // LDL^T.
    const double d0 = A00, i0 = pn_rcp1(d0);
    const double l10 = A10 * i0, l20 = A20 * i0, l30 = A30 * i0;
    const double d1 = A11 - l10 * l10 * d0, i1 = pn_rcp1(d1);
    const double l21 = (A21 - l20 * l10 * d0) * i1;
    const double l31 = (A31 - l30 * l10 * d0) * i1;
    const double d2 = A22 - l20 * l20 * d0 - l21 * l21 * d1, i2 = pn_rcp1(d2);
    const double l32 = (A32 - l30 * l20 * d0 - l31 * l21 * d1) * i2;
    const double d3 = A33 - l30 * l30 * d0 - l31 * l31 * d1 - l32 * l32 * d2;
    const double z0 = c0, z1 = c1 - l10 * z0, z2 = c2 - l20 * z0 - l21 * z1;
    const double z3 = c3 - l30 * z0 - l31 * z1 - l32 * z2;
    const double damp = PN_SIX_MU * A33;
    const double lam3 = z3 * d3 * pn_rcp1(fma(d3, d3, damp * damp));
    const double lam2 = z2 * i2 - l32 * lam3;
    const double lam1 = z1 * i1 - l21 * lam2 - l31 * lam3;
    const double lam0 = z0 * i0 - l10 * lam1 - l20 * lam2 - l30 * lam3;
    // d = -G^T lam: dr = -(p x lamJ) - lam3 dH/dr, dp = -(lamJ x r) - lam3 dH/dp.
    y[0] = rx - (py * lam2 - pz * lam1) - lam3 * gr[0];
    y[1] = ry - (pz * lam0 - px * lam2) - lam3 * gr[1];
    y[2] = rz - (px * lam1 - py * lam0) - lam3 * gr[2];
    y[3] = px - (lam1 * rz - lam2 * ry) - lam3 * gp[0];
    y[4] = py - (lam2 * rx - lam0 * rz) - lam3 * gp[1];
    y[5] = pz - (lam0 * ry - lam1 * rx) - lam3 * gp[2];
}

// The six-integral correction after the spin lengths: `sweeps` passes of the
// joint projection followed by the energy's momentum scaling.  The spins do
// not move, and the momentum scaling leaves r (so its geometry) unchanged:
// the geometry computed for the scaling serves the next pass's projection.
__device__ __forceinline__ int pn_correct_six(const PnCoef& k, double* y, const double* ref, double tol,
                                              int max_iter, int sweeps, bool& noconv) {
    const PnSpinInv si = pn_spin_inv(k, y);
    PnRGeom geo = pn_rgeom(k, si, y);
    int iters = 0;
    for (int s = 0; s < sweeps; ++s) {
        pn_project_EJ_g(k, si, geo, y, ref);
        geo = pn_rgeom(k, si, y);
        bool conv;
        iters += pn_energy_scale_poly(pn_energy_poly_g(k, si, geo, y), y, ref[0], tol, max_iter, conv);
        noconv = noconv || !conv;
    }
    return iters;
}

// Dual scaling of eqs. (11)-(13): p = alpha p*, r = b r*, Newton on
// f1 = H(b r*, alpha p*, S) - E0 and f2 = |alpha b L* + S1 + S2| - |J0|
// (Gauss-Newton on eq. 12, same root for any weights).  A Jacobian whose
// determinant is below 1e-3 of |j11 j22| falls back to energy-only momentum
// scaling for this step.
__device__ __forceinline__ int pn_dual_scale(const PnCoef& k, double* y, const double* ref, double tol,
                                             int max_iter, bool& conv) {
    const double r0x = y[0], r0y = y[1], r0z = y[2];
    const double p0x = y[3], p0y = y[4], p0z = y[5];
    const double Lx = r0y * p0z - r0z * p0y, Ly = r0z * p0x - r0x * p0z, Lz = r0x * p0y - r0y * p0x;
    const double Sx = y[6] + y[9], Sy = y[7] + y[10], Sz = y[8] + y[11];
    const double J0n = sqrt(ref[1] * ref[1] + ref[2] * ref[2] + ref[3] * ref[3]);
    double al = 1.0, b = 1.0;
    int it = 0;
    conv = false;
    bool singular = false;
    double ys[12];
#pragma unroll
    for (int c = 6; c < 12; ++c) ys[c] = y[c];
    while (it < max_iter) {
        ys[0] = b * r0x; ys[1] = b * r0y; ys[2] = b * r0z;
        ys[3] = al * p0x; ys[4] = al * p0y; ys[5] = al * p0z;
        double H, gr[3], gp[3];
        pn_energy_grad_rp(k, ys, H, gr, gp);
        const double f1 = H - ref[0];
        const double ab = al * b;
        const double Jx = ab * Lx + Sx, Jy = ab * Ly + Sy, Jz = ab * Lz + Sz;
        const double Jn = sqrt(dot3(Jx, Jy, Jz, Jx, Jy, Jz));
        const double f2 = Jn - J0n;
        const double JhL = dot3(Jx, Jy, Jz, Lx, Ly, Lz) / Jn;
        const double j11 = dot3(gp[0], gp[1], gp[2], p0x, p0y, p0z);
        const double j12 = dot3(gr[0], gr[1], gr[2], r0x, r0y, r0z);
        const double j21 = b * JhL;
        const double j22 = al * JhL;
        const double det = j11 * j22 - j12 * j21;
        if (fabs(det) < 1e-3 * fabs(j22) * fabs(j11)) { singular = true; break; }
        const double dal = -(j22 * f1 - j12 * f2) / det;
        const double db = -(-j21 * f1 + j11 * f2) / det;
        al += dal;
        b += db;
        ++it;
        if (fabs(dal) <= tol && fabs(db) <= tol) { conv = true; break; }
    }
    if (singular) return it + pn_energy_scale(k, y, ref[0], tol, max_iter, conv);
    y[0] = b * r0x; y[1] = b * r0y; y[2] = b * r0z;
    y[3] = al * p0x; y[4] = al * p0y; y[5] = al * p0z;
    return it;
}

// One correction against ref = (E0, J0x, J0y, J0z); returns Newton iterations.
template <int MODE>
__device__ __forceinline__ int pn_correct(const PnCoef& k, double* y, const double* ref, double tol,
                                          int max_iter, int sweeps, bool& noconv) {
    noconv = false;
    if (MODE == PN_CORR_NONE) return 0;
    pn_correct_spins(k, y);
    if (MODE == PN_CORR_SPIN) return 0;
    if (MODE == PN_CORR_SIX) return pn_correct_six(k, y, ref, tol, max_iter, sweeps, noconv);
    bool conv = true;
    const int iters = pn_dual_scale(k, y, ref, tol, max_iter, conv);
    noconv = !conv;
    return iters;
}

// One fixed step of RK4 or of the Dormand-Prince fifth-order weights.
template <int METHOD>
__device__ __forceinline__ void pn_rk_step(const PnCoef& k, double* y, double h) {
    double kk[12], acc[12], t[12];
    if (METHOD == PN_RK4) {
        pn_rhs_eval(k, y, kk);
#pragma unroll
        for (int c = 0; c < 12; ++c) { acc[c] = kk[c]; t[c] = fma(0.5 * h, kk[c], y[c]); }
        pn_rhs_eval(k, t, kk);
#pragma unroll
        for (int c = 0; c < 12; ++c) { acc[c] = fma(2.0, kk[c], acc[c]); t[c] = fma(0.5 * h, kk[c], y[c]); }
        pn_rhs_eval(k, t, kk);
#pragma unroll
        for (int c = 0; c < 12; ++c) { acc[c] = fma(2.0, kk[c], acc[c]); t[c] = fma(h, kk[c], y[c]); }
        pn_rhs_eval(k, t, kk);
        const double h6 = h / 6.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = fma(h6, acc[c] + kk[c], y[c]);
        return;
    }
    // Dormand-Prince: the stage derivatives are folded into running stage
    // inputs so that only the current derivative is live.
    constexpr double a21 = 1.0 / 5.0;
    constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                     a54 = -212.0 / 729.0;
    constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                     a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                     b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    double s3[12], s4[12], s5[12], s6[12];
    pn_rhs_eval(k, y, kk);  // k1
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        t[c] = fma(h * a21, kk[c], y[c]);
        s3[c] = fma(h * a31, kk[c], y[c]);
        s4[c] = fma(h * a41, kk[c], y[c]);
        s5[c] = fma(h * a51, kk[c], y[c]);
        s6[c] = fma(h * a61, kk[c], y[c]);
        acc[c] = fma(h * b1, kk[c], y[c]);
    }
    pn_rhs_eval(k, t, kk);  // k2
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        s3[c] = fma(h * a32, kk[c], s3[c]);
        s4[c] = fma(h * a42, kk[c], s4[c]);
        s5[c] = fma(h * a52, kk[c], s5[c]);
        s6[c] = fma(h * a62, kk[c], s6[c]);
    }
    pn_rhs_eval(k, s3, kk);  // k3
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        s4[c] = fma(h * a43, kk[c], s4[c]);
        s5[c] = fma(h * a53, kk[c], s5[c]);
        s6[c] = fma(h * a63, kk[c], s6[c]);
        acc[c] = fma(h * b3, kk[c], acc[c]);
    }
    pn_rhs_eval(k, s4, kk);  // k4
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        s5[c] = fma(h * a54, kk[c], s5[c]);
        s6[c] = fma(h * a64, kk[c], s6[c]);
        acc[c] = fma(h * b4, kk[c], acc[c]);
    }
    pn_rhs_eval(k, s5, kk);  // k5
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        s6[c] = fma(h * a65, kk[c], s6[c]);
        acc[c] = fma(h * b5, kk[c], acc[c]);
    }
    pn_rhs_eval(k, s6, kk);  // k6
#pragma unroll
    for (int c = 0; c < 12; ++c) y[c] = fma(h * b6, kk[c], acc[c]);
}

// 2.5PN radiation-reaction acceleration of eq. (6) (M = 1): the
// leading-order reaction of a point-mass binary in the Iyer-Will gauge family
// at (alpha, beta) = (4, 5), the harmonic-coordinate form,
//   a = (8/5) eta / r^3 [(18 v^2 + 2 / (3 r) - 25 rdot^2) rdot n
//                        - (6 v^2 - 2 / r - 15 rdot^2) v],
// with v = dH/dp and rdot = n.v.
__device__ __forceinline__ void pn_rr_accel(double eta, const double* y, const double* v, double* a) {
    const double r2 = dot3(y[0], y[1], y[2], y[0], y[1], y[2]);
    const double u = pn_rsqrt(r2);
    const double nx = y[0] * u, ny = y[1] * u, nz = y[2] * u;
    const double rdot = dot3(nx, ny, nz, v[0], v[1], v[2]);
    const double v2 = dot3(v[0], v[1], v[2], v[0], v[1], v[2]);
    const double rd2 = rdot * rdot;
    const double A = 18.0 * v2 + (2.0 / 3.0) * u - 25.0 * rd2;
    const double B = 6.0 * v2 - 2.0 * u - 15.0 * rd2;
    const double pre = 1.6 * eta * u * u * u;
    const double cn = pre * A * rdot, cv = -pre * B;
    a[0] = cn * nx + cv * v[0];
    a[1] = cn * ny + cv * v[1];
    a[2] = cn * nz + cv * v[2];
}

// The dissipative system with its reference integrals: z = (y, E, J) and
// dz/dt = (f(y) with a_2.5PN on dp/dt, v.a, r x a).  The spin flow conserves
// H and J, so the references change only through the reaction.
__device__ __forceinline__ void pn_rhs_rr(const PnCoef& k, double eta, const double* z, double* f) {
    pn_rhs_eval(k, z, f);
    double a[3];
    pn_rr_accel(eta, z, f, a);
    f[3] += a[0]; f[4] += a[1]; f[5] += a[2];
    f[12] = dot3(f[0], f[1], f[2], a[0], a[1], a[2]);
    f[13] = z[1] * a[2] - z[2] * a[1];
    f[14] = z[2] * a[0] - z[0] * a[2];
    f[15] = z[0] * a[1] - z[1] * a[0];
}

// One fixed RK4 or Dormand-Prince fifth-order step of the 16-component
// dissipative system (state and references together).
template <int METHOD>
__device__ void pn_rk_step_rr(const PnCoef& k, double eta, double* z, double h) {
    constexpr int D = 16;
    double k1[D], k2[D], k3[D], k4[D], t[D];
    if (METHOD == PN_RK4) {
        pn_rhs_rr(k, eta, z, k1);
        for (int c = 0; c < D; ++c) t[c] = fma(0.5 * h, k1[c], z[c]);
        pn_rhs_rr(k, eta, t, k2);
        for (int c = 0; c < D; ++c) t[c] = fma(0.5 * h, k2[c], z[c]);
        pn_rhs_rr(k, eta, t, k3);
        for (int c = 0; c < D; ++c) t[c] = fma(h, k3[c], z[c]);
        pn_rhs_rr(k, eta, t, k4);
        for (int c = 0; c < D; ++c) z[c] = fma(h / 6.0, k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c], z[c]);
        return;
    }
    double k5[D], k6[D];
    pn_rhs_rr(k, eta, z, k1);
    for (int c = 0; c < D; ++c) t[c] = z[c] + h * (1.0 / 5.0) * k1[c];
    pn_rhs_rr(k, eta, t, k2);
    for (int c = 0; c < D; ++c) t[c] = z[c] + h * ((3.0 / 40.0) * k1[c] + (9.0 / 40.0) * k2[c]);
    pn_rhs_rr(k, eta, t, k3);
    for (int c = 0; c < D; ++c)
        t[c] = z[c] + h * ((44.0 / 45.0) * k1[c] + (-56.0 / 15.0) * k2[c] + (32.0 / 9.0) * k3[c]);
    pn_rhs_rr(k, eta, t, k4);
    for (int c = 0; c < D; ++c)
        t[c] = z[c] + h * ((19372.0 / 6561.0) * k1[c] + (-25360.0 / 2187.0) * k2[c] + (64448.0 / 6561.0) * k3[c] +
                           (-212.0 / 729.0) * k4[c]);
    pn_rhs_rr(k, eta, t, k5);
    for (int c = 0; c < D; ++c)
        t[c] = z[c] + h * ((9017.0 / 3168.0) * k1[c] + (-355.0 / 33.0) * k2[c] + (46732.0 / 5247.0) * k3[c] +
                           (49.0 / 176.0) * k4[c] + (-5103.0 / 18656.0) * k5[c]);
    pn_rhs_rr(k, eta, t, k6);
    for (int c = 0; c < D; ++c)
        z[c] = z[c] + h * ((35.0 / 384.0) * k1[c] + (500.0 / 1113.0) * k3[c] + (125.0 / 192.0) * k4[c] +
                           (-2187.0 / 6784.0) * k5[c] + (11.0 / 84.0) * k6[c]);
}

// Orbit validity in the order: non-finite, merged, escaped.  The sum of
// y[c] * 0 is NaN exactly when some component is NaN or infinite.
__device__ __forceinline__ int pn_validity(const double* y, double rmerge2, double resc2) {
    double z = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) z = fma(y[c], 0.0, z);
    if (!isfinite(z)) return PN_ORBIT_NONFINITE;
    const double r2 = dot3(y[0], y[1], y[2], y[0], y[1], y[2]);
    if (r2 < rmerge2) return PN_ORBIT_MERGED;
    if (r2 > resc2) return PN_ORBIT_ESCAPED;
    return PN_ORBIT_OK;
}
