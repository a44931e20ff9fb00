// Device arithmetic of the three-dimensional moment equations: the
// ten-moment system (rho, rho u_i, E_ij = P_ij + rho u_i u_j) with zero heat
// flux (Sec. 2, eqs. (2)-(4) in three dimensions; ten eigenvalues, Sec. 3.3),
// characteristic MUSCL-Hancock with HLL fluxes as in two dimensions.
//
// States are 10-vectors in registers: primitive (rho, u, v, w, Pxx, Pxy, Pxz,
// Pyy, Pyz, Pzz), conserved (rho, rho u, rho v, rho w, Exx, ..., Ezz).  Each
// direction N (0, 1, 2) is a template argument, so every index below is a
// compile-time constant and the vectors stay in registers.  Along axis n with
// transverse axes t1 < t2 the eigen-system is (eigenvalues ascending)
//   u - a, u - c (t1), u - c (t2), u (rho, P_t1t1, P_t1t2, P_t2t2),
//   u + c (t1), u + c (t2), u + a,    a = sqrt(3 P_nn / rho), c = sqrt(P_nn / rho),
// projected and back-projected in closed form (q_t = P_nt / P_nn); the
// tracing uses the collapsed form of eqs. (27)-(32) with the HLL terms, which
// needs only the extreme speeds u -+ a.
#pragma once

#include "csh_device.h"

namespace csh {
namespace d3 {

constexpr int NV = 10;

struct V10 {
    double v[NV];
};

// index of P_ij / E_ij
CSH_HD constexpr int P(int i, int j)
{
    return (i == 0) ? 4 + j : (i == 1) ? (j == 0 ? 5 : 6 + j) : (j == 0 ? 6 : j == 1 ? 8 : 9);
}

template <int N>
struct Axes {
    static constexpr int t1 = (N == 0) ? 1 : 0;
    static constexpr int t2 = (N == 2) ? 1 : 2;
};

CSH_HD V10 to_prim(const V10& U, double ir)
{
    V10 w;
    w.v[0] = U.v[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) w.v[1 + i] = U.v[1 + i] * ir;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) w.v[P(i, j)] = U.v[P(i, j)] - U.v[1 + i] * w.v[1 + j];
    return w;
}

CSH_HD V10 to_cons(const V10& w)
{
    V10 U;
    U.v[0] = w.v[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) U.v[1 + i] = w.v[0] * w.v[1 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) U.v[P(i, j)] = w.v[P(i, j)] + U.v[1 + i] * w.v[1 + j];
    return U;
}

// flux along N: rho u_n, rho u_i u_n + P_in, E_ij u_n + P_ni u_j + P_nj u_i
template <int N>
CSH_HD V10 flux(const V10& w, const V10& U)
{
    V10 F;
    const double un = w.v[1 + N];
    F.v[0] = U.v[1 + N];
#pragma unroll
    for (int i = 0; i < 3; ++i) F.v[1 + i] = U.v[1 + i] * un + w.v[P(i, N)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            F.v[P(i, j)] = U.v[P(i, j)] * un + w.v[P(N, i)] * w.v[1 + j] + w.v[P(N, j)] * w.v[1 + i];
    return F;
}

// A d with A the primitive Jacobian along N
template <int N>
CSH_HD V10 jac(const V10& w, double ir, const V10& d)
{
    V10 o;
    const double un = w.v[1 + N];
    o.v[0] = un * d.v[0] + w.v[0] * d.v[1 + N];
#pragma unroll
    for (int i = 0; i < 3; ++i) o.v[1 + i] = un * d.v[1 + i] + ir * d.v[P(i, N)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            o.v[P(i, j)] = un * d.v[P(i, j)] + w.v[P(i, j)] * d.v[1 + N] + w.v[P(i, N)] * d.v[1 + j] +
                           w.v[P(j, N)] * d.v[1 + i];
    return o;
}

template <int N>
struct Eig {
    double a, c, h2a, h2c, ip, q1, q2;
};

template <int N>
CSH_HD Eig<N> eig(const V10& w, double ir)
{
    constexpr int t1 = Axes<N>::t1, t2 = Axes<N>::t2;
    Eig<N> e;
    const double pnn = w.v[P(N, N)];
    const double t = pnn * ir;
    const double y = rsqrt(t);  // 1 / c
    e.c = t * y;
    e.a = 1.7320508075688772935 * e.c;
    e.h2c = 0.5 * y;
    e.h2a = 0.28867513459481288225 * y;
    e.ip = rcp(pnn);
    e.q1 = w.v[P(N, t1)] * e.ip;
    e.q2 = w.v[P(N, t2)] * e.ip;
    return e;
}

// amplitudes on the ten waves, in the order of the header comment
template <int N>
CSH_HD V10 project(const V10& w, const Eig<N>& e, const V10& d)
{
    constexpr int t1 = Axes<N>::t1, t2 = Axes<N>::t2;
    const double dnn = d.v[P(N, N)];
    const double f1 = dnn * e.ip * (1.0 / 6.0), f2 = d.v[1 + N] * e.h2a;
    const double hip = 0.5 * e.ip;
    const double s1 = (d.v[P(N, t1)] - e.q1 * dnn) * hip, h1 = (e.q1 * d.v[1 + N] - d.v[1 + t1]) * e.h2c;
    const double s2 = (d.v[P(N, t2)] - e.q2 * dnn) * hip, h2 = (e.q2 * d.v[1 + N] - d.v[1 + t2]) * e.h2c;
    const double third = dnn * (1.0 / 3.0);
    V10 al;
    al.v[0] = f1 - f2;
    al.v[9] = f1 + f2;
    al.v[1] = h1 + s1;
    al.v[7] = s1 - h1;
    al.v[2] = h2 + s2;
    al.v[8] = s2 - h2;
    al.v[3] = d.v[0] - w.v[0] * e.ip * third;
    al.v[4] = d.v[P(t1, t1)] - 2.0 * e.q1 * d.v[P(N, t1)] + (4.0 * e.q1 * e.q1 - w.v[P(t1, t1)] * e.ip) * third;
    al.v[5] = d.v[P(t1, t2)] - e.q2 * d.v[P(N, t1)] - e.q1 * d.v[P(N, t2)] +
              (4.0 * e.q1 * e.q2 - w.v[P(t1, t2)] * e.ip) * third;
    al.v[6] = d.v[P(t2, t2)] - 2.0 * e.q2 * d.v[P(N, t2)] + (4.0 * e.q2 * e.q2 - w.v[P(t2, t2)] * e.ip) * third;
    return al;
}

template <int N>
CSH_HD V10 backproject(const V10& w, const Eig<N>& e, const V10& al)
{
    constexpr int t1 = Axes<N>::t1, t2 = Axes<N>::t2;
    const double S = al.v[0] + al.v[9], D = al.v[9] - al.v[0];
    const double S1 = al.v[1] + al.v[7], D1 = al.v[7] - al.v[1];
    const double S2 = al.v[2] + al.v[8], D2 = al.v[8] - al.v[2];
    const double pnn = w.v[P(N, N)], pn1 = w.v[P(N, t1)], pn2 = w.v[P(N, t2)];
    V10 d;
    d.v[0] = w.v[0] * S + al.v[3];
    d.v[1 + N] = e.a * D;
    d.v[1 + t1] = e.a * e.q1 * D + e.c * D1;
    d.v[1 + t2] = e.a * e.q2 * D + e.c * D2;
    d.v[P(N, N)] = 3.0 * pnn * S;
    d.v[P(N, t1)] = 3.0 * pn1 * S + pnn * S1;
    d.v[P(N, t2)] = 3.0 * pn2 * S + pnn * S2;
    d.v[P(t1, t1)] = (w.v[P(t1, t1)] + 2.0 * pn1 * e.q1) * S + 2.0 * pn1 * S1 + al.v[4];
    d.v[P(t1, t2)] = (w.v[P(t1, t2)] + pn1 * e.q2 + pn2 * e.q1) * S + pn2 * S1 + pn1 * S2 + al.v[5];
    d.v[P(t2, t2)] = (w.v[P(t2, t2)] + 2.0 * pn2 * e.q2) * S + 2.0 * pn2 * S2 + al.v[6];
    return d;
}

// characteristic MC-limited slope along N (eqs. (19)-(26))
template <int N>
CSH_HD V10 limited_slope(const V10& w, const Eig<N>& e, const V10& wm, const V10& wp)
{
    V10 dl, dr;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        dl.v[m] = w.v[m] - wm.v[m];
        dr.v[m] = wp.v[m] - w.v[m];
    }
    const V10 l = project<N>(w, e, dl), r = project<N>(w, e, dr);
    V10 am;
#pragma unroll
    for (int m = 0; m < NV; ++m) am.v[m] = mc(l.v[m], r.v[m]);
    return backproject<N>(w, e, am);
}

// HLL flux along N between face states (Davis speeds)
template <int N>
CSH_HD V10 hll(const V10& wl, const V10& wr)
{
    const V10 Ul = to_cons(wl), Ur = to_cons(wr);
    const V10 Fl = flux<N>(wl, Ul), Fr = flux<N>(wr, Ur);
    const double tl = 3.0 * wl.v[P(N, N)], tr = 3.0 * wr.v[P(N, N)];
    const double al = tl * rsqrt(tl * wl.v[0]), ar = tr * rsqrt(tr * wr.v[0]);
    const double sl = fmin(fmin(wl.v[1 + N] - al, wr.v[1 + N] - ar), 0.0);
    const double sr = fmax(fmax(wl.v[1 + N] + al, wr.v[1 + N] + ar), 0.0);
    const double inv = rcp(sr - sl);
    const double a = sr * inv, b = sl * inv, c = sl * a;
    V10 F;
#pragma unroll
    for (int m = 0; m < NV; ++m) F.v[m] = a * Fl.v[m] - b * Fr.v[m] + c * (Ur.v[m] - Ul.v[m]);
    return F;
}

// CFL rate: sum over the axes of (|u_k| + sqrt(3 P_kk / rho)) / h_k
CSH_HD double signal_rate(const V10& w, const double ih[3])
{
    const double ir = rcp(w.v[0]);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double t = 3.0 * w.v[P(k, k)] * ir;
        s += (fabs(w.v[1 + k]) + t * rsqrt(t)) * ih[k];
    }
    return s;
}

CSH_HD bool physical(const V10& w)
{
    const double pxx = w.v[4], pxy = w.v[5], pxz = w.v[6], pyy = w.v[7], pyz = w.v[8], pzz = w.v[9];
    const double m2 = pxx * pyy - pxy * pxy;
    const double det = pxx * (pyy * pzz - pyz * pyz) - pxy * (pxy * pzz - pyz * pxz) + pxz * (pxy * pyz - pyy * pxz);
    double sum = 0.0;
#pragma unroll
    for (int m = 0; m < NV; ++m) sum += w.v[m];
    return w.v[0] > 0.0 && pxx > 0.0 && m2 > 0.0 && det > 0.0 && isfinite(sum);
}

}  // namespace d3
}  // namespace csh
