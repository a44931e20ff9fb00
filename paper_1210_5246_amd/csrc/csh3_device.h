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
// needs only the extreme speeds u -+ a.  As in two dimensions the kernels carry
// half slopes (the face-state coefficients take the factor 2) and form each
// wave's amplitude up to a positive per-cell scale.
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
    double a, c, h2c, ip, q1, q2;  // a = sqrt(3 Pnn / rho), c = sqrt(Pnn / rho), h2c = 1/(2c), ip = 1/Pnn
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
    e.ip = y * y * ir;          // (rho / Pnn) / rho
    e.q1 = w.v[P(N, t1)] * e.ip;
    e.q2 = w.v[P(N, t2)] * e.ip;
    return e;
}

// Half the MC limiter, mc(dl, dr) / 2, from order statistics: with
// q = (dl + dr) / 4 the result is the median of (min(dl, dr, q), 0,
// max(dl, dr, q)).
CSH_HD double mc_half(double dl, double dr)
{
    const double q = 0.25 * (dl + dr);
    const double A = fmin(fmin(dl, dr), q), B = fmax(fmax(dl, dr), q);
    return fmax(A, fmin(B, 0.0));
}

// Half the characteristic MC-limited slope along N (eqs. (19)-(26)).  The
// limiter commutes with a positive factor common to its two arguments, so the
// amplitudes are formed up to per-cell positive scales:
//   u -+ a:          dPnn -+ rho a du_n                          (6 Pnn times l . d)
//   u -+ c (t):      (dPnt - q_t dPnn) -+ rho c (q_t du_n - du_t)  (2 Pnn times)
//   u (4 waves):     drho - rho dPnn / (3 Pnn) and the three transverse-stress
//                    combinations, unscaled;
// the back-projection divides the scales out.
template <int N>
CSH_HD V10 half_slope(const V10& w, double ir, const Eig<N>& e, const V10& wm, const V10& wp)
{
    constexpr int t1 = Axes<N>::t1, t2 = Axes<N>::t2;
    constexpr int nn = P(N, N), n1 = P(N, t1), n2 = P(N, t2), s11 = P(t1, t1), s12 = P(t1, t2), s22 = P(t2, t2);
    const double rho = w.v[0];
    const double ra = rho * e.a, rc = rho * e.c, rip = rho * e.ip;
    const double kr = rip * (1.0 / 3.0);
    const double k11 = (4.0 * e.q1 * e.q1 - w.v[s11] * e.ip) * (1.0 / 3.0);
    const double k12 = (4.0 * e.q1 * e.q2 - w.v[s12] * e.ip) * (1.0 / 3.0);
    const double k22 = (4.0 * e.q2 * e.q2 - w.v[s22] * e.ip) * (1.0 / 3.0);
    const double q1x2 = e.q1 + e.q1, q2x2 = e.q2 + e.q2;
    auto project = [&](const V10& d, double (&al)[NV]) {
        const double dnn = d.v[nn], dun = d.v[1 + N];
        al[0] = dnn - ra * dun;
        al[9] = dnn + ra * dun;
        const double s1 = d.v[n1] - e.q1 * dnn, h1 = e.q1 * dun - d.v[1 + t1];
        const double s2 = d.v[n2] - e.q2 * dnn, h2 = e.q2 * dun - d.v[1 + t2];
        al[1] = s1 + rc * h1;
        al[7] = s1 - rc * h1;
        al[2] = s2 + rc * h2;
        al[8] = s2 - rc * h2;
        al[3] = d.v[0] - kr * dnn;
        al[4] = d.v[s11] - q1x2 * d.v[n1] + k11 * dnn;
        al[5] = d.v[s12] - e.q2 * d.v[n1] - e.q1 * d.v[n2] + k12 * dnn;
        al[6] = d.v[s22] - q2x2 * d.v[n2] + k22 * dnn;
    };
    double l[NV], r[NV], m[NV];
    {
        V10 dl, dr;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            dl.v[k] = w.v[k] - wm.v[k];
            dr.v[k] = wp.v[k] - w.v[k];
        }
        project(dl, l);
        project(dr, r);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = mc_half(l[k], r[k]);
    const double S = m[0] + m[9], D = m[9] - m[0];
    const double S1 = m[1] + m[7], D1 = m[7] - m[1];
    const double S2 = m[2] + m[8], D2 = m[8] - m[2];
    const double i6 = e.ip * (1.0 / 6.0), bu = e.a * i6, bc = e.h2c * ir;  // a / (6 Pnn), c / (2 Pnn)
    const double pn1 = w.v[n1], pn2 = w.v[n2];
    V10 d;
    d.v[0] = (rip * (1.0 / 6.0)) * S + m[3];
    d.v[1 + N] = bu * D;
    d.v[1 + t1] = (bu * e.q1) * D + bc * D1;
    d.v[1 + t2] = (bu * e.q2) * D + bc * D2;
    d.v[nn] = 0.5 * S;
    d.v[n1] = 0.5 * (e.q1 * S + S1);
    d.v[n2] = 0.5 * (e.q2 * S + S2);
    d.v[s11] = ((w.v[s11] + q1x2 * pn1) * i6) * S + e.q1 * S1 + m[4];
    d.v[s12] = ((w.v[s12] + pn1 * e.q2 + pn2 * e.q1) * i6) * S + 0.5 * (e.q2 * S1 + e.q1 * S2) + m[5];
    d.v[s22] = ((w.v[s22] + q2x2 * pn2) * i6) * S + e.q2 * S2 + m[6];
    return d;
}

// F - s U along N, formed from the primitive state: with s' = u_n - s and
// m = rho s', X_rho = m, X_i = m u_i + P_in, X_ij = u_j X_i + s' P_ij + P_nj u_i,
// which for i = n is u_j X_n + P_nj (s' + u_n).
template <int N>
CSH_HD V10 moving_flux(const V10& w, double s)
{
    const double un = w.v[1 + N], sp = un - s, m = w.v[0] * sp, g = sp + un;
    V10 X;
    X.v[0] = m;
#pragma unroll
    for (int i = 0; i < 3; ++i) X.v[1 + i] = m * w.v[1 + i] + w.v[P(i, N)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            if (i == N) X.v[P(i, j)] = w.v[1 + j] * X.v[1 + N] + w.v[P(N, j)] * g;
            else if (j == N) X.v[P(i, j)] = w.v[1 + i] * X.v[1 + N] + w.v[P(N, i)] * g;
            else X.v[P(i, j)] = w.v[1 + j] * X.v[1 + i] + sp * w.v[P(i, j)] + w.v[P(N, j)] * w.v[1 + i];
        }
    return X;
}

// HLL flux along N between face states (Davis speeds); with the clamped
// outer speeds S_L' = min(S_L, 0), S_R' = max(S_R, 0) it is
// (S_R' X_L - S_L' X_R) / (S_R' - S_L'), X_K = F_K - S_K' U_K.
template <int N>
CSH_HD V10 hll(const V10& wl, const V10& wr)
{
    const double tl = 3.0 * wl.v[P(N, N)], tr = 3.0 * wr.v[P(N, N)];
    const double al = tl * rsqrt(tl * wl.v[0]), ar = tr * rsqrt(tr * wr.v[0]);
    const double sl = fmin(fmin(wl.v[1 + N] - al, wr.v[1 + N] - ar), 0.0);
    const double sr = fmax(fmax(wl.v[1 + N] + al, wr.v[1 + N] + ar), 0.0);
    const double inv = rcp(sr - sl);
    const double a = sr * inv, b = sl * inv;
    const V10 XL = moving_flux<N>(wl, sl), XR = moving_flux<N>(wr, sr);
    V10 F;
#pragma unroll
    for (int m = 0; m < NV; ++m) F.v[m] = a * XL.v[m] - b * XR.v[m];
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
    return (w.v[0] > 0.0) & (pxx > 0.0) & (m2 > 0.0) & (det > 0.0) & isfinite(sum);
}

}  // namespace d3
}  // namespace csh
