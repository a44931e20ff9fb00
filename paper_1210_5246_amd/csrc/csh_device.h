// Device arithmetic of the collisionless-stellar-hydrodynamics sweep
// (Mitchell, Vorobyov & Hensler, arXiv:1210.5246), gfx950.
//
// Formulation used on the GPU (the scheme is the paper's; the arithmetic is
// arranged for registers):
//  * the eigenvectors of Sec. 3.3, eqs. (14)-(18), extended to the full
//    symmetric 2-D stress tensor, are never stored: the projections on the
//    left eigenvectors and the back-projection on the right ones are written
//    out in closed form from their sparsity (about 14 FMAs each);
//  * the characteristic tracing of eqs. (27)-(32) with the HLL terms added
//    counts every wave once, and its per-wave sums collapse through
//    sum_a lam_a (l_a.dw) r_a = A dw to
//        w_hi = w + [1/2 + k min(lamM, 0)] dw - k A dw
//        w_lo = w - [1/2 - k max(lam0, 0)] dw - k A dw ,
//    with A the sparse primitive Jacobian;
//  * with the transverse predictor of the unsplit scheme, all four face
//    states of a cell share one centre value
//        base = w - (dt/2dx) A dw_x - (dt/2dy) B dw_y ;
//  * HLL (Davis speeds) in the branch-free form with S_L' = min(S_L, 0) and
//    S_R' = max(S_R, 0), which equals the three-case formula.
// Variables: primitive W = (rho, u, v, Pxx, Pxy, Pyy), conserved
// U = (rho, rho u, rho v, Exx, Exy, Eyy), E_ij = P_ij + rho u_i u_j (Sec. 2).
// The y direction is the x direction applied to the state with the axes
// exchanged (swap()).
#pragma once

#include <hip/hip_runtime.h>

// host-and-device arithmetic (also exercised on the CPU by the tests)
#define CSH_HD __host__ __device__ __forceinline__

namespace csh {

// Reciprocal and reciprocal square root from the hardware approximations plus
// one Newton step.  gfx950's FP64 v_rcp/v_rsq are accurate to ~5e-8 relative;
// one step brings them to ~4e-15, well inside the scheme's parity tolerance,
// at about half the instructions of the IEEE-exact sequences.  FP32 uses the
// single-precision instructions (~1 ulp).  On the host (tests) they are exact;
// the refinement steps themselves are host-callable, so the tests run them
// from approximations with the hardware's error.
//   r' = r + r (1 - x r)            (relative error e -> e^2)
CSH_HD double rcp_refine(double x, double r) { return fma(fma(-x, r, 1.0), r, r); }
//   y' = y + (y / 2)(1 - x y^2)     (e -> 3/2 e^2)
CSH_HD double rsqrt_refine(double x, double y) { return fma(0.5 * y, fma(-x * y, y, 1.0), y); }
//   s = x y, s' = s + (s / 2)(1 - s y)   (the square root from y ~ 1/sqrt(x))
CSH_HD double sqrt_refine(double x, double y)
{
    const double s = x * y;
    return fma(0.5 * s, fma(-s, y, 1.0), s);
}

CSH_HD double rcp(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return rcp_refine(x, __builtin_amdgcn_rcp(x));
#else
    return 1.0 / x;
#endif
}
CSH_HD float rcp(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
CSH_HD double rsqrt(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return rsqrt_refine(x, __builtin_amdgcn_rsq(x));
#else
    return 1.0 / sqrt(x);
#endif
}
CSH_HD float rsqrt(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

// Square root of a positive number: on the device s0 = x rsq(x) from the
// hardware approximation, then one Newton step of the square root written
// with the same reciprocal root (sqrt_refine; ~4e-15, one instruction fewer
// than refining the reciprocal root and multiplying by x).  NaN for x <= 0
// (as x rsqrt(x)).
CSH_HD double sqrt_pos(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return sqrt_refine(x, __builtin_amdgcn_rsq(x));
#else
    return x * (1.0 / sqrt(x));
#endif
}
CSH_HD float sqrt_pos(float x) { return x * rsqrt(x); }

template <typename T>
struct Prim {
    T r, u, v, pxx, pxy, pyy;
};

template <typename T>
struct Cons {
    T r, mx, my, exx, exy, eyy;
};

// characteristic amplitudes of the waves (u-a, u-c, u[rho], u[Pyy], u+c, u+a)
template <typename T>
struct Char {
    T a1, a2, a3, a4, a5, a6;
};

template <typename T>
CSH_HD Prim<T> swap(const Prim<T>& w)
{
    return {w.r, w.v, w.u, w.pyy, w.pxy, w.pxx};
}

template <typename T>
CSH_HD Cons<T> swap(const Cons<T>& U)
{
    return {U.r, U.my, U.mx, U.eyy, U.exy, U.exx};
}

template <typename T>
CSH_HD Prim<T> sub(const Prim<T>& a, const Prim<T>& b)
{
    return {a.r - b.r, a.u - b.u, a.v - b.v, a.pxx - b.pxx, a.pxy - b.pxy, a.pyy - b.pyy};
}

// Sec. 2: E_ij = P_ij + rho u_i u_j
template <typename T>
CSH_HD Prim<T> to_prim(const Cons<T>& U, T ir)
{
    const T u = U.mx * ir, v = U.my * ir;
    return {U.r, u, v, U.exx - U.mx * u, U.exy - U.mx * v, U.eyy - U.my * v};
}

template <typename T>
CSH_HD Prim<T> to_prim(const Cons<T>& U)
{
    return to_prim(U, rcp(U.r));
}

template <typename T>
CSH_HD Cons<T> to_cons(const Prim<T>& w)
{
    const T mx = w.r * w.u, my = w.r * w.v;
    return {w.r, mx, my, w.pxx + mx * w.u, w.pxy + mx * w.v, w.pyy + my * w.v};
}

// x flux of eqs. (2)-(4) (k = x terms), from the primitive state and its
// conserved form: (rho u, rho u u + Pxx, rho v u + Pxy, (Exx + 2 Pxx) u,
// (Exy + Pxy) u + Pxx v, Eyy u + 2 Pxy v)
template <typename T>
CSH_HD Cons<T> flux_x(const Prim<T>& w, const Cons<T>& U)
{
    return {U.mx,
            U.mx * w.u + w.pxx,
            U.my * w.u + w.pxy,
            (U.exx + T(2) * w.pxx) * w.u,
            (U.exy + w.pxy) * w.u + w.pxx * w.v,
            U.eyy * w.u + T(2) * w.pxy * w.v};
}

// Per-cell coefficients of the x-direction eigen-system (eqs. (14)-(18),
// full tensor): fast speed a = sqrt(3 Pxx / rho) (eq. (15), gamma = 3),
// shear speed c = sqrt(Pxx / rho), q = Pxy / Pxx.
template <typename T>
struct Eig {
    T a, c, h2a, h2c, ip, q;  // h2a = 1/(2a), h2c = 1/(2c), ip = 1/Pxx
};

template <typename T>
CSH_HD Eig<T> eig_x(const Prim<T>& w, T ir)
{
    Eig<T> e;
    const T t = w.pxx * ir;
    const T y = rsqrt(t);                 // 1 / c
    e.c = t * y;
    e.a = T(1.7320508075688772935) * e.c;  // sqrt(3) c
    e.h2c = T(0.5) * y;
    e.h2a = T(0.28867513459481288225) * y;  // 1 / (2 sqrt(3) c)
    e.ip = y * y * ir;                      // 1 / Pxx = (rho / Pxx) / rho
    e.q = w.pxy * e.ip;
    return e;
}

// alpha = L d: amplitudes of a primitive difference on the six waves.
template <typename T>
CSH_HD Char<T> project(const Prim<T>& w, const Eig<T>& e, const Prim<T>& d)
{
    const T t1 = d.pxx * e.ip * T(1.0 / 6.0);
    const T t2 = d.u * e.h2a;
    const T s = (d.pxy - e.q * d.pxx) * (T(0.5) * e.ip);
    const T h = (e.q * d.u - d.v) * e.h2c;
    Char<T> al;
    al.a1 = t1 - t2;
    al.a6 = t1 + t2;
    al.a2 = h + s;
    al.a5 = s - h;
    al.a3 = d.r - w.r * d.pxx * e.ip * T(1.0 / 3.0);
    al.a4 = d.pyy - T(2) * e.q * d.pxy + (T(4) * e.q * e.q - w.pyy * e.ip) * d.pxx * T(1.0 / 3.0);
    return al;
}

// d = R alpha: back-projection on the right eigenvectors.
template <typename T>
CSH_HD Prim<T> backproject(const Prim<T>& w, const Eig<T>& e, const Char<T>& al)
{
    const T S = al.a1 + al.a6, D = al.a6 - al.a1;
    const T S25 = al.a2 + al.a5, D25 = al.a5 - al.a2;
    Prim<T> d;
    d.r = w.r * S + al.a3;
    d.u = e.a * D;
    d.v = e.a * e.q * D + e.c * D25;
    d.pxx = T(3) * w.pxx * S;
    d.pxy = T(3) * w.pxy * S + w.pxx * S25;
    d.pyy = (w.pyy + T(2) * w.pxy * e.q) * S + T(2) * w.pxy * S25 + al.a4;
    return d;
}

// Monotonised-central limiter, eq. (25), zero at extrema (the TVD clause).
// With dl * dr > 0 the centred difference has the sign of both.
template <typename T>
CSH_HD T mc(T dl, T dr)
{
    // dr with dl's sign taken off is positive iff the two agree in sign; the
    // clamp at zero then covers the extremum case
    const T a = fmin(fabs(dl), copysign(T(1), dl) * dr);
    const T m = fmax(fmin(a + a, T(0.5) * fabs(dl + dr)), T(0));
    return copysign(m, dl);
}

// Limited primitive slope along x: eqs. (19)-(26) with dl = w_i - w_{i-1},
// dr = w_{i+1} - w_i; the centred amplitudes are the mean of the one-sided ones.
template <typename T>
CSH_HD Prim<T> limited_slope(const Prim<T>& w, const Eig<T>& e, const Prim<T>& dl,
                                                 const Prim<T>& dr)
{
    const Char<T> l = project(w, e, dl), r = project(w, e, dr);
    Char<T> m;
    m.a1 = mc(l.a1, r.a1);
    m.a2 = mc(l.a2, r.a2);
    m.a3 = mc(l.a3, r.a3);
    m.a4 = mc(l.a4, r.a4);
    m.a5 = mc(l.a5, r.a5);
    m.a6 = mc(l.a6, r.a6);
    return backproject(w, e, m);
}

// Half the MC limiter, mc(dl, dr) / 2, from order statistics: with
// q = (dl + dr) / 4, lo = min(dl, dr), hi = max(dl, dr), A = min(lo, q) <= q <=
// B = max(hi, q), and the result is the median of (A, 0, B): A when both
// differences are positive, B when both are negative, 0 otherwise.  Equal to
// the sign-tested form value for value (up to the sign of a zero); the factor
// 2 it omits goes into the face-state coefficients.
template <typename T>
CSH_HD T mc_half(T dl, T dr)
{
    const T q = T(0.25) * (dl + dr);
    const T A = fmin(fmin(dl, dr), q), B = fmax(fmax(dl, dr), q);
    return fmax(A, fmin(B, T(0)));
}

// Half the characteristic MC-limited slope (eqs. (19)-(26)) in scaled form.
// The limiter commutes with a positive factor common to its two arguments, so
// each wave's amplitude is formed up to a per-cell positive scale and the
// back-projection divides it out.  Amplitudes, x direction (q = Pxy / Pxx):
//   u -+ a:  dPxx -+ rho a du                          (6 Pxx times l . d)
//   u -+ c:  (dPxy - q dPxx) -+ rho c (q du - dv)      (2 Pxx times)
//   u:       drho - rho / (3 Pxx) dPxx,  dPyy - 2 q dPxy + (4 q^2 - Pyy / Pxx) / 3 dPxx
// and with S, D the sum and difference of the u -+ a pair, S', D' of the
// u -+ c pair, the slope is
//   (rho S / (6 Pxx) + m_rho, a D / (6 Pxx), a q D / (6 Pxx) + c D' / (2 Pxx),
//    S / 2, (q S + S') / 2, (Pyy + 2 Pxy q) S / (6 Pxx) + q S' + m_Pyy).
template <typename T>
CSH_HD Prim<T> half_slope(const Prim<T>& w, T ir, const Eig<T>& e, const Prim<T>& dl, const Prim<T>& dr)
{
    const T ra = w.r * e.a, rc = w.r * e.c, q2 = e.q + e.q;
    const T rip = w.r * e.ip;  // rho / Pxx
    const T kr = rip * T(1.0 / 3.0);
    const T k4 = (T(4) * e.q * e.q - w.pyy * e.ip) * T(1.0 / 3.0);
    auto project = [&](const Prim<T>& d, T (&al)[6]) {
        al[0] = d.pxx - ra * d.u;
        al[5] = d.pxx + ra * d.u;
        const T s = d.pxy - e.q * d.pxx, h = e.q * d.u - d.v;
        al[1] = s + rc * h;
        al[4] = s - rc * h;
        al[2] = d.r - kr * d.pxx;
        al[3] = d.pyy - q2 * d.pxy + k4 * d.pxx;
    };
    T l[6], r[6], m[6];
    project(dl, l);
    project(dr, r);
#pragma unroll
    for (int k = 0; k < 6; ++k) m[k] = mc_half(l[k], r[k]);
    const T i6 = e.ip * T(1.0 / 6.0);
    const T S = m[0] + m[5], D = m[5] - m[0], S2 = m[1] + m[4], D2 = m[4] - m[1];
    const T bu = e.a * i6;
    Prim<T> d;
    d.r = (rip * T(1.0 / 6.0)) * S + m[2];
    d.u = bu * D;
    d.v = (bu * e.q) * D + (e.h2c * ir) * D2;  // c / (2 Pxx) = 1 / (2 c rho)
    d.pxx = T(0.5) * S;
    d.pxy = T(0.5) * (e.q * S + S2);
    d.pyy = ((w.pyy + q2 * w.pxy) * i6) * S + e.q * S2 + m[3];
    return d;
}

// A d with A the primitive x Jacobian (rows: u d_rho + rho d_u, u d_u + d_Pxx/rho,
// u d_v + d_Pxy/rho, u d_Pxx + 3 Pxx d_u, u d_Pxy + 2 Pxy d_u + Pxx d_v,
// u d_Pyy + Pyy d_u + 2 Pxy d_v).
template <typename T>
CSH_HD Prim<T> jac_x(const Prim<T>& w, T ir, const Prim<T>& d)
{
    Prim<T> o;
    o.r = w.u * d.r + w.r * d.u;
    o.u = w.u * d.u + ir * d.pxx;
    o.v = w.u * d.v + ir * d.pxy;
    o.pxx = w.u * d.pxx + T(3) * w.pxx * d.u;
    o.pxy = w.u * d.pxy + T(2) * w.pxy * d.u + w.pxx * d.v;
    o.pyy = w.u * d.pyy + w.pyy * d.u + T(2) * w.pxy * d.v;
    return o;
}

template <typename T>
CSH_HD Prim<T> axpy(T a, const Prim<T>& x, const Prim<T>& y)
{
    return {y.r + a * x.r, y.u + a * x.u, y.v + a * x.v, y.pxx + a * x.pxx, y.pxy + a * x.pxy,
            y.pyy + a * x.pyy};
}

// A face state with the quantities its Riemann problem needs.
template <typename T>
struct Face {
    Prim<T> w;
    Cons<T> U;
    T a;  // normal fast speed sqrt(3 Pnn / rho)
};

// x-face state from a primitive state (normal direction x)
template <typename T>
CSH_HD Face<T> make_face_x(const Prim<T>& w)
{
    Face<T> f;
    f.w = w;
    f.U = to_cons(w);
    const T t = T(3) * w.pxx;
    f.a = t * rsqrt(t * w.r);  // sqrt(3 Pxx / rho)
    return f;
}

// F - s U for an x-face state, formed from the primitive state alone: with
// s' = u - s and m = rho s', F - s U = s' U + N (N = (0, Pxx, Pxy, 2 Pxx u,
// Pxy u + Pxx v, 2 Pxy v), the stress part of the flux) regroups to
// (m, m u + Pxx, m v + Pxy, u X_mx + Pxx (s' + u), v X_mx + Pxy (s' + u),
//  v (X_my + Pxy) + Pyy s').
template <typename T>
CSH_HD Cons<T> moving_flux_x(const Prim<T>& w, T s)
{
    const T sp = w.u - s;
    const T m = w.r * sp;
    const T xmx = m * w.u + w.pxx;
    const T xmy = m * w.v + w.pxy;
    const T g = sp + w.u;
    return {m, xmx, xmy, w.u * xmx + w.pxx * g, w.v * xmx + w.pxy * g, w.v * (xmy + w.pxy) + w.pyy * sp};
}

// HLL flux in x (Davis speed estimates), branch-free form: with the outer
// speeds clamped, S_L' = min(S_L, 0) and S_R' = max(S_R, 0), the three-case
// flux is (S_R' F_L - S_L' F_R + S_L' S_R' (U_R - U_L)) / (S_R' - S_L'), which
// is (S_R' X_L - S_L' X_R) / (S_R' - S_L') with X_K = F_K - S_K' U_K.
template <typename T>
CSH_HD Cons<T> hll_x(const Face<T>& L, const Face<T>& R)
{
    const T sl = fmin(fmin(L.w.u - L.a, R.w.u - R.a), T(0));
    const T sr = fmax(fmax(L.w.u + L.a, R.w.u + R.a), T(0));
    const T inv = rcp(sr - sl);
    const T a = sr * inv, b = sl * inv;
    const Cons<T> XL = moving_flux_x(L.w, sl), XR = moving_flux_x(R.w, sr);
    return {a * XL.r - b * XR.r,     a * XL.mx - b * XR.mx,   a * XL.my - b * XR.my,
            a * XL.exx - b * XR.exx, a * XL.exy - b * XR.exy, a * XL.eyy - b * XR.eyy};
}

// HLLC flux in x for the moment equations: outer speeds as for HLL, one
// contact S*, and a star region with one velocity (S*, v*) and one pair of
// x-stresses (Pxx*, Pxy*); with D_K = rho_K (S_K - u_K),
//   S* = (Pxx_R - Pxx_L + D_L u_L - D_R u_R) / (D_L - D_R),
//   v* = (Pxy_R - Pxy_L + D_L v_L - D_R v_R) / (D_L - D_R),
// and each star density from the jump condition across S_K with the star
// flux q* S* + N*:  q*_K (S_K - S*) = q_K (S_K - u_K) + N* - N_K,
// N = (0, Pxx, Pxy, 2 Pxx u, Pxy u + Pxx v, 2 Pxy v).  The side K of the
// contact that holds x = 0 is selected first (S* >= 0: left), so one star
// state is formed; with S_K' the outer speed clamped at 0 the flux is
// F_K + S_K' (U*_K - U_K), which is F_L / F_R in the supersonic cases.
template <typename T>
CSH_HD Cons<T> hllc_x(const Face<T>& L, const Face<T>& R)
{
    const T sl = fmin(L.w.u - L.a, R.w.u - R.a);
    const T sr = fmax(L.w.u + L.a, R.w.u + R.a);
    const T dl = L.w.r * (sl - L.w.u), dr = R.w.r * (sr - R.w.u);
    const T idd = rcp(dl - dr);
    const T ss = (R.w.pxx - L.w.pxx + dl * L.w.u - dr * R.w.u) * idd;
    const T vs = (R.w.pxy - L.w.pxy + dl * L.w.v - dr * R.w.v) * idd;
    const bool left = ss >= T(0);
    const Face<T>& K = left ? L : R;
    const T sk = left ? sl : sr, dk = left ? dl : dr;
    const T skc = left ? fmin(sl, T(0)) : fmax(sr, T(0));
    const Prim<T>& w = K.w;
    const T pnn = w.pxx + dk * (ss - w.u), pnt = w.pxy + dk * (vs - w.v);
    const T g = skc * rcp(sk - ss);  // S_K' / (S_K - S*)
    // S_K' (U*_K - U_K) = S_K' [U_K (S* - u_K) + N* - N_K] / (S_K - S*)
    const T c = ss - w.u;
    const Cons<T> F = flux_x(w, K.U);
    return {F.r + g * (K.U.r * c),
            F.mx + g * (K.U.mx * c + pnn - w.pxx),
            F.my + g * (K.U.my * c + pnt - w.pxy),
            F.exx + g * (K.U.exx * c + T(2) * (pnn * ss - w.pxx * w.u)),
            F.exy + g * (K.U.exy * c + pnt * ss + pnn * vs - w.pxy * w.u - w.pxx * w.v),
            F.eyy + g * (K.U.eyy * c + T(2) * (pnt * vs - w.pxy * w.v))};
}

// The face flux of the characteristic scheme: RS = 0 HLL, RS = 1 HLLC.
template <int RS, typename T>
CSH_HD Cons<T> riemann_x(const Face<T>& L, const Face<T>& R)
{
    if constexpr (RS == 1) return hllc_x(L, R);
    else return hll_x(L, R);
}

template <typename T>
CSH_HD Face<T> swap(const Face<T>& f)
{
    return {swap(f.w), swap(f.U), f.a};
}

// The four time-centred face states of a cell (primitive, axes not exchanged)
// from the cell and its four neighbours: limited slopes in x and y, and the
// Hancock predictor with the tracing coefficients of eqs. (27)-(32) and the
// transverse terms.  1-D: only xhi / xlo, no y terms.
template <typename T>
struct Faces {
    Prim<T> xhi, xlo, yhi, ylo;
};

// The same from the one-sided differences along x (dlx = w_i - w_{i-1}, drx =
// w_{i+1} - w_i) and y: a march that holds them already (the left difference of
// a cell is the right difference of its left neighbour, and of the row below)
// passes them in and forms each once.
template <typename T, bool TWOD>
CSH_HD Faces<T> face_states_d(const Prim<T>& W0, T ir, const Prim<T>& dlx, const Prim<T>& drx, const Prim<T>& dly,
                              const Prim<T>& dry, T kx, T ky)
{
    // with the half slopes h = dm / 2 every coefficient doubles:
    // base = w - 2k A h, w_hi = base + (1 + 2k min(lamM, 0)) h, w_lo = base - (1 - 2k max(lam0, 0)) h
    const T kx2 = kx + kx;
    const Eig<T> ex = eig_x(W0, ir);
    const Prim<T> hx = half_slope(W0, ir, ex, dlx, drx);
    Prim<T> base = axpy(-kx2, jac_x(W0, ir, hx), W0);
    Faces<T> f;
    const T chix = T(1) + kx2 * fmin(W0.u + ex.a, T(0));
    const T clox = T(1) - kx2 * fmax(W0.u - ex.a, T(0));
    if constexpr (TWOD) {
        const T ky2 = ky + ky;
        const Prim<T> W0s = swap(W0);
        const Eig<T> ey = eig_x(W0s, ir);
        const Prim<T> hys = half_slope(W0s, ir, ey, swap(dly), swap(dry));
        base = axpy(-ky2, swap(jac_x(W0s, ir, hys)), base);
        const Prim<T> hy = swap(hys);
        const T chiy = T(1) + ky2 * fmin(W0.v + ey.a, T(0));
        const T cloy = T(1) - ky2 * fmax(W0.v - ey.a, T(0));
        f.yhi = axpy(chiy, hy, base);
        f.ylo = axpy(-cloy, hy, base);
    }
    f.xhi = axpy(chix, hx, base);
    f.xlo = axpy(-clox, hx, base);
    return f;
}

template <typename T, bool TWOD>
CSH_HD Faces<T> face_states(const Prim<T>& W0, T ir, const Prim<T>& Wl, const Prim<T>& Wr, const Prim<T>& Wm,
                            const Prim<T>& Wp, T kx, T ky)
{
    return face_states_d<T, TWOD>(W0, ir, sub(W0, Wl), sub(Wr, W0), sub(W0, Wm), sub(Wp, W0), kx, ky);
}

// ---- Kurganov-Tadmor central scheme (Sec. 3.2) ------------------------------------------------

// half the component-wise MC-limited slope of the primitive variables
template <typename T>
CSH_HD Prim<T> mc_half_slope(const Prim<T>& wm, const Prim<T>& w0, const Prim<T>& wp)
{
    return {mc_half(w0.r - wm.r, wp.r - w0.r),       mc_half(w0.u - wm.u, wp.u - w0.u),
            mc_half(w0.v - wm.v, wp.v - w0.v),       mc_half(w0.pxx - wm.pxx, wp.pxx - w0.pxx),
            mc_half(w0.pxy - wm.pxy, wp.pxy - w0.pxy), mc_half(w0.pyy - wm.pyy, wp.pyy - w0.pyy)};
}

// Twice the x flux of eq. (6), 2H = F(u-) + F(u+) - a (u+ - u-), from the face
// states u- = wl, u+ = wr, a = max over the two of |u| + sqrt(3 Pxx / rho)
// (eqs. (7)-(8)); as (F - s U) at s = -a on the left plus s = a on the right,
// formed from the primitive states (moving_flux_x).
template <typename T>
CSH_HD Cons<T> kt_flux2_x(const Prim<T>& wl, const Prim<T>& wr)
{
    const T tl = T(3) * wl.pxx, tr = T(3) * wr.pxx;
    const T a = fmax(fabs(wl.u) + tl * rsqrt(tl * wl.r), fabs(wr.u) + tr * rsqrt(tr * wr.r));
    const Cons<T> XL = moving_flux_x(wl, -a), XR = moving_flux_x(wr, a);
    return {XL.r + XR.r, XL.mx + XR.mx, XL.my + XR.my, XL.exx + XR.exx, XL.exy + XR.exy, XL.eyy + XR.eyy};
}

// External flat-rotation-curve potential (Sec. 3.3, last paragraph): exact
// kick of the velocity by dt * a for a fixed field a (rho and the stress
// unchanged): rho u_i += dt rho a_i, E_ij += dt (a_i m_j + m_i a_j) + dt^2 rho a_i a_j.
// P carries vc2 (0: no field), rc2, x0, y0, dx, dy of the grid.  Evaluated
// in the state's precision (an FP32 state's kick in FP32: its rounding is that
// of the state it updates).
template <typename T, typename P>
__device__ __forceinline__ void kick(Cons<T>& U, const P& p, double dt, int i, int j, bool twod)
{
    if (p.vc2 == 0.0) return;
    const T x = T(p.x0) + (T(i) + T(0.5)) * T(p.dx);
    const T y = twod ? T(p.y0) + (T(j) + T(0.5)) * T(p.dy) : T(0);
    // velocity increment g = dt a, a = -vc2 (x, y) / (x^2 + y^2 + rc^2)
    const T f = T(-p.vc2 * dt) * rcp(x * x + y * y + T(p.rc2));
    const T gx = f * x, gy = f * y;
    // m' = m + rho g; E' = E + g_i m_j + m_i g_j + rho g_i g_j, i.e.
    // E'_xx = E_xx + g_x (m_x + m'_x), E'_xy = E_xy + g_x m_y + g_y m'_x
    const T mx = U.mx + U.r * gx, my = U.my + U.r * gy;
    U.exx = U.exx + gx * (U.mx + mx);
    U.exy = U.exy + gx * U.my + gy * mx;
    U.eyy = U.eyy + gy * (U.my + my);
    U.mx = mx;
    U.my = my;
}

// CFL rate of a cell (the timestep is C / max over cells of this):
// (|u| + a_x)/dx + (|v| + a_y)/dy, 1-D: (|u| + a_x)/dx.  Evaluated in the
// state's precision (FP32 for an FP32 state: a relative rounding of ~1e-7 in
// a quantity that only sets the timestep) and returned as a double.
template <typename T, bool TWOD>
CSH_HD double signal_rate(const Prim<T>& w, double idx, double idy)
{
    const T ir = rcp(w.r);
    const T tx = T(3) * w.pxx * ir;
    T s = (fabs(w.u) + sqrt_pos(tx)) * T(idx);
    if (TWOD) {
        const T ty = T(3) * w.pyy * ir;
        s += (fabs(w.v) + sqrt_pos(ty)) * T(idy);
    }
    return double(s);
}

// CFL rate of a new 2-D state together with the test of physical() (rho > 0,
// positive-definite stress, everything finite), sharing the work: a NaN or an
// infinity in u, v, Pxx or Pyy makes the rate NaN or infinite, one in Pxy
// fails det > 0, one in rho fails rho > 0 or makes rate + rho infinite.
template <typename T>
CSH_HD double checked_rate(const Cons<T>& U, double idx, double idy, bool& bad)
{
    const Prim<T> w = to_prim(U);
    const double s = signal_rate<T, true>(w, idx, idy);
    const bool ok = (w.r > T(0)) & (w.pxx > T(0)) & (w.pyy > T(0)) & (w.pxx * w.pyy - w.pxy * w.pxy > T(0)) &
                    isfinite(s + double(w.r));
    bad |= !ok;
    return s;
}

// rho > 0, positive-definite stress, everything finite
template <typename T>
CSH_HD bool physical(const Prim<T>& w)
{
    // every test evaluated (no short-circuit: no lane-divergent branches)
    const bool pd = (w.r > T(0)) & (w.pxx > T(0)) & (w.pyy > T(0)) & (w.pxx * w.pyy - w.pxy * w.pxy > T(0));
    // a NaN or infinity in any component makes the sum NaN or infinite
    return pd & isfinite(w.r + w.u + w.v + w.pxx + w.pxy + w.pyy);
}

// ---- wavefront primitives --------------------------------------------------------------------

// Value held by lane (lane + D), D = +1 or -1, by a DPP whole-wavefront shift
// (wave_shl:1 / wave_shr:1; lane layout checked on gfx950).  The lane at the
// end the shift comes from receives 0; callers never use it (it is halo).
template <int D>
__device__ __forceinline__ double lane_shift(double x)
{
    constexpr int ctrl = D > 0 ? 0x130 : 0x138;
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), ctrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), ctrl, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int D>
__device__ __forceinline__ float lane_shift(float x)
{
    constexpr int ctrl = D > 0 ? 0x130 : 0x138;
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, true));
}

template <int D, typename T>
__device__ __forceinline__ Prim<T> lane_shift(const Prim<T>& w)
{
    return {lane_shift<D>(w.r), lane_shift<D>(w.u), lane_shift<D>(w.v),
            lane_shift<D>(w.pxx), lane_shift<D>(w.pxy), lane_shift<D>(w.pyy)};
}

template <int D, typename T>
__device__ __forceinline__ Cons<T> lane_shift(const Cons<T>& U)
{
    return {lane_shift<D>(U.r), lane_shift<D>(U.mx), lane_shift<D>(U.my),
            lane_shift<D>(U.exx), lane_shift<D>(U.exy), lane_shift<D>(U.eyy)};
}

// Index of the calling wavefront in its workgroup, as a wave-uniform value
// (threadIdx.x / 64 is the same on every lane of a wavefront, but the compiler
// cannot see that; without the readfirstlane every branch on it is compiled
// as lane-divergent control flow).
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// max over the wavefront
__device__ __forceinline__ double wave_max(double x)
{
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// positive doubles order like their bit patterns
__device__ __forceinline__ void atomic_max_pos(unsigned long long* slot, double x)
{
    atomicMax(slot, (unsigned long long)__double_as_longlong(x));
}

// ---- one-dimensional sweep of a wavefront's 64 cells ------------------------------------------

// HLL flux through the high face (c + 1/2) of the lane's cell c, from the
// conserved states of the 64 consecutive cells the wavefront holds: slopes,
// characteristic limiting, tracing (eqs. (19)-(32)), HLL.  Valid on lanes
// 1..61 (the two edge lanes on each side lack a neighbour's slope).
template <typename T, int RS = 0>
__device__ __forceinline__ Cons<T> flux_1d(const Cons<T>& U0, T kx)
{
    const T ir = rcp(U0.r);
    const Prim<T> W0 = to_prim(U0, ir);
    const Prim<T> dr = sub(lane_shift<+1>(W0), W0);
    const Faces<T> f = face_states_d<T, false>(W0, ir, lane_shift<-1>(dr), dr, dr, dr, kx, T(0));
    return riemann_x<RS>(make_face_x(f.xhi), make_face_x(lane_shift<+1>(f.xlo)));
}

template <typename T>
CSH_HD Cons<T> update(const Cons<T>& U, T c, const Cons<T>& Fp, const Cons<T>& Fm)
{
    return {U.r - c * (Fp.r - Fm.r),       U.mx - c * (Fp.mx - Fm.mx),
            U.my - c * (Fp.my - Fm.my),    U.exx - c * (Fp.exx - Fm.exx),
            U.exy - c * (Fp.exy - Fm.exy), U.eyy - c * (Fp.eyy - Fm.eyy)};
}

// ---- state access ------------------------------------------------------------------------------

template <typename T>
CSH_HD Cons<T> load_cons(const T* __restrict__ U, size_t plane, size_t c)
{
    return {U[c], U[plane + c], U[2 * plane + c], U[3 * plane + c], U[4 * plane + c], U[5 * plane + c]};
}

template <typename T>
CSH_HD void store_cons(T* __restrict__ U, size_t plane, size_t c, const Cons<T>& v)
{
    U[c] = v.r;
    U[plane + c] = v.mx;
    U[2 * plane + c] = v.my;
    U[3 * plane + c] = v.exx;
    U[4 * plane + c] = v.exy;
    U[5 * plane + c] = v.eyy;
}

// The six planes of a state as wave-uniform base pointers, addressed with a
// 32-bit byte offset (planes are limited to 4 GiB at init), so each access is
// a scalar base plus one vector offset.
template <typename T>
struct Planes {
    const char* b[6];
    CSH_HD Planes(const T* U, size_t plane)
    {
        for (int k = 0; k < 6; ++k) b[k] = reinterpret_cast<const char*>(U + k * plane);
    }
    CSH_HD Cons<T> load(unsigned cell) const
    {
        const unsigned o = cell * (unsigned)sizeof(T);
        return {*reinterpret_cast<const T*>(b[0] + o), *reinterpret_cast<const T*>(b[1] + o),
                *reinterpret_cast<const T*>(b[2] + o), *reinterpret_cast<const T*>(b[3] + o),
                *reinterpret_cast<const T*>(b[4] + o), *reinterpret_cast<const T*>(b[5] + o)};
    }
};

template <typename T>
struct OutPlanes {
    char* b[6];
    CSH_HD OutPlanes(T* U, size_t plane)
    {
        for (int k = 0; k < 6; ++k) b[k] = reinterpret_cast<char*>(U + k * plane);
    }
    CSH_HD void store(unsigned cell, const Cons<T>& v) const
    {
        const unsigned o = cell * (unsigned)sizeof(T);
        *reinterpret_cast<T*>(b[0] + o) = v.r;
        *reinterpret_cast<T*>(b[1] + o) = v.mx;
        *reinterpret_cast<T*>(b[2] + o) = v.my;
        *reinterpret_cast<T*>(b[3] + o) = v.exx;
        *reinterpret_cast<T*>(b[4] + o) = v.exy;
        *reinterpret_cast<T*>(b[5] + o) = v.eyy;
    }
};

CSH_HD int map_index(int i, int n, int bc)
{
    if (bc == 0) {  // periodic
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);  // zero-gradient outflow
}

// map_index for -n <= i < 2n (the stencil rows of a grid with n >= 2): no division
CSH_HD int map_near(int i, int n, int bc)
{
    if (bc == 0) return i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace csh
