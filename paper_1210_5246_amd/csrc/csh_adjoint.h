// Reverse-mode pieces of the sweep (FP64): vector-Jacobian products of every
// stage of csh_device.h, written out by hand statement by statement in reverse
// order, and the per-cell bodies of the adjoint kernels.
//
// Conventions: a function foo_vjp(inputs..., ybar, xbar...) ADDS the
// contribution of ybar to the adjoints xbar of foo's inputs.  At the kinks of
// min/max/|.| the subgradient of one branch is taken: MC takes the centred
// difference first, then 2|dl|, then 2|dr| (first minimal argument); the
// tracing coefficients have zero slope where their eigenvalue is exactly 0;
// HLL speed estimates take the first argument on ties and zero slope where
// they are clipped at 0.  All __host__ __device__, so the tests can run them
// on the CPU.
#pragma once

#include "csh_device.h"
#include "csh_xcd.h"

namespace csh {

using P = Prim<double>;
using C = Cons<double>;
using A6 = Char<double>;
using E = Eig<double>;

CSH_HD void acc(P& a, const P& b)
{
    a.r += b.r; a.u += b.u; a.v += b.v; a.pxx += b.pxx; a.pxy += b.pxy; a.pyy += b.pyy;
}
CSH_HD P scale(double s, const P& a) { return {s * a.r, s * a.u, s * a.v, s * a.pxx, s * a.pxy, s * a.pyy}; }
CSH_HD double dot(const P& a, const P& b)
{
    return a.r * b.r + a.u * b.u + a.v * b.v + a.pxx * b.pxx + a.pxy * b.pxy + a.pyy * b.pyy;
}
CSH_HD P zero_p() { return {0, 0, 0, 0, 0, 0}; }
CSH_HD C zero_c() { return {0, 0, 0, 0, 0, 0}; }

// eig_x(w, ir): c = sqrt(pxx ir), a = sqrt3 c, h2c = 0.5/c, h2a = k/c, ip = 1/pxx, q = pxy ip
CSH_HD void eig_vjp(const P& w, double ir, const E& e, const E& eb, P& wb, double& irb)
{
    double cb = eb.c;
    double ipb = eb.ip;
    // q = pxy * ip
    wb.pxy += e.ip * eb.q;
    ipb += w.pxy * eb.q;
    // ip = 1 / pxx
    wb.pxx += -e.ip * e.ip * ipb;
    // h2a = k / c ; h2c = 0.5 / c ; a = sqrt3 c  (1 / c = 2 h2c)
    const double ic = 2.0 * e.h2c;
    cb += -e.h2a * ic * eb.h2a;
    cb += -e.h2c * ic * eb.h2c;
    cb += 1.7320508075688772935 * eb.a;
    // c = sqrt(pxx ir)
    const double tb = cb * e.h2c;
    wb.pxx += ir * tb;
    irb += w.pxx * tb;
}

// project(w, e, d) -> alpha
CSH_HD void project_vjp(const P& w, const E& e, const P& d, const A6& ab, P& wb, E& eb, P& db)
{
    const double t1b = ab.a1 + ab.a6, t2b = ab.a6 - ab.a1;
    const double hb = ab.a2 - ab.a5, sb = ab.a2 + ab.a5;
    // a3 = d.r - w.r d.pxx ip / 3
    db.r += ab.a3;
    constexpr double third = 1.0 / 3.0, sixth = 1.0 / 6.0;
    wb.r += -d.pxx * e.ip * third * ab.a3;
    db.pxx += -w.r * e.ip * third * ab.a3;
    eb.ip += -w.r * d.pxx * third * ab.a3;
    // a4 = d.pyy - 2 q d.pxy + (4 q^2 - pyy ip) d.pxx / 3
    db.pyy += ab.a4;
    eb.q += (-2.0 * d.pxy + 8.0 * e.q * d.pxx * third) * ab.a4;
    db.pxy += -2.0 * e.q * ab.a4;
    wb.pyy += -e.ip * d.pxx * third * ab.a4;
    eb.ip += -w.pyy * d.pxx * third * ab.a4;
    db.pxx += (4.0 * e.q * e.q - w.pyy * e.ip) * third * ab.a4;
    // h = (q d.u - d.v) h2c
    const double X = e.q * d.u - d.v;
    const double Xb = e.h2c * hb;
    eb.h2c += X * hb;
    eb.q += d.u * Xb;
    db.u += e.q * Xb;
    db.v -= Xb;
    // s = (d.pxy - q d.pxx) (ip / 2)
    const double Y = d.pxy - e.q * d.pxx;
    const double Yb = 0.5 * e.ip * sb;
    eb.ip += 0.5 * Y * sb;
    db.pxy += Yb;
    eb.q -= d.pxx * Yb;
    db.pxx -= e.q * Yb;
    // t2 = d.u h2a
    db.u += e.h2a * t2b;
    eb.h2a += d.u * t2b;
    // t1 = d.pxx ip / 6
    db.pxx += e.ip * sixth * t1b;
    eb.ip += d.pxx * sixth * t1b;
}

// backproject(w, e, alpha) -> d
CSH_HD void backproject_vjp(const P& w, const E& e, const A6& al, const P& db, P& wb, E& eb, A6& ab)
{
    const double S = al.a1 + al.a6, D = al.a6 - al.a1;
    const double S25 = al.a2 + al.a5, D25 = al.a5 - al.a2;
    const double Sb = w.r * db.r + 3.0 * w.pxx * db.pxx + 3.0 * w.pxy * db.pxy + (w.pyy + 2.0 * w.pxy * e.q) * db.pyy;
    const double Db = e.a * db.u + e.a * e.q * db.v;
    const double S25b = w.pxx * db.pxy + 2.0 * w.pxy * db.pyy;
    const double D25b = e.c * db.v;
    ab.a3 += db.r;
    ab.a4 += db.pyy;
    wb.r += S * db.r;
    eb.a += D * db.u + e.q * D * db.v;
    eb.q += e.a * D * db.v + 2.0 * w.pxy * S * db.pyy;
    eb.c += D25 * db.v;
    wb.pxx += 3.0 * S * db.pxx + S25 * db.pxy;
    wb.pxy += 3.0 * S * db.pxy + 2.0 * e.q * S * db.pyy + 2.0 * S25 * db.pyy;
    wb.pyy += S * db.pyy;
    ab.a1 += Sb - Db;
    ab.a6 += Sb + Db;
    ab.a2 += S25b - D25b;
    ab.a5 += S25b + D25b;
}

// MC: m = sgn(dc) min(2|dl|, |dc|, 2|dr|) if dl and dr are nonzero with one
// sign, else 0 (the forward form tests the signs, not the product).  The
// branch taken sets the weights of the two inputs (0.5 / 0.5 centred, 2 / 0
// or 0 / 2 one-sided, 0 / 0 off); written without branches so the two
// adjoints stay in registers.
CSH_HD void mc_vjp(double dl, double dr, double mb, double& dlb, double& drb)
{
    const bool on = dl != 0.0 && dr != 0.0 && (dl < 0.0) == (dr < 0.0);
    const double adc = fabs(0.5 * (dl + dr)), al2 = 2.0 * fabs(dl), ar2 = 2.0 * fabs(dr);
    const bool cen = adc <= al2 && adc <= ar2;  // centred difference
    const bool left = al2 <= ar2;               // else 2 dl (same sign as dc), else 2 dr
    const double wl = on ? (cen ? 0.5 : (left ? 2.0 : 0.0)) : 0.0;
    const double wr = on ? (cen ? 0.5 : (left ? 0.0 : 2.0)) : 0.0;
    dlb += wl * mb;
    drb += wr * mb;
}

// limited_slope(w, e, dl, dr) -> dm
CSH_HD void limited_slope_vjp(const P& w, const E& e, const P& dl, const P& dr, const P& dmb, P& wb, E& eb,
                              P& dlb, P& drb)
{
    const A6 l = project(w, e, dl), r = project(w, e, dr);
    A6 m;
    m.a1 = mc(l.a1, r.a1);
    m.a2 = mc(l.a2, r.a2);
    m.a3 = mc(l.a3, r.a3);
    m.a4 = mc(l.a4, r.a4);
    m.a5 = mc(l.a5, r.a5);
    m.a6 = mc(l.a6, r.a6);
    A6 mb{0, 0, 0, 0, 0, 0};
    backproject_vjp(w, e, m, dmb, wb, eb, mb);
    A6 lb{0, 0, 0, 0, 0, 0}, rb{0, 0, 0, 0, 0, 0};
    mc_vjp(l.a1, r.a1, mb.a1, lb.a1, rb.a1);
    mc_vjp(l.a2, r.a2, mb.a2, lb.a2, rb.a2);
    mc_vjp(l.a3, r.a3, mb.a3, lb.a3, rb.a3);
    mc_vjp(l.a4, r.a4, mb.a4, lb.a4, rb.a4);
    mc_vjp(l.a5, r.a5, mb.a5, lb.a5, rb.a5);
    mc_vjp(l.a6, r.a6, mb.a6, lb.a6, rb.a6);
    project_vjp(w, e, dl, lb, wb, eb, dlb);
    project_vjp(w, e, dr, rb, wb, eb, drb);
}

// jac_x(w, ir, d) -> o
CSH_HD void jac_vjp(const P& w, double ir, const P& d, const P& ob, P& wb, double& irb, P& db)
{
    wb.u += d.r * ob.r + d.u * ob.u + d.v * ob.v + d.pxx * ob.pxx + d.pxy * ob.pxy + d.pyy * ob.pyy;
    wb.r += d.u * ob.r;
    irb += d.pxx * ob.u + d.pxy * ob.v;
    wb.pxx += 3.0 * d.u * ob.pxx + d.v * ob.pxy;
    wb.pxy += 2.0 * d.u * ob.pxy + 2.0 * d.v * ob.pyy;
    wb.pyy += d.u * ob.pyy;
    db.r += w.u * ob.r;
    db.u += w.r * ob.r + w.u * ob.u + 3.0 * w.pxx * ob.pxx + 2.0 * w.pxy * ob.pxy + w.pyy * ob.pyy;
    db.v += w.u * ob.v + w.pxx * ob.pxy + 2.0 * w.pxy * ob.pyy;
    db.pxx += ir * ob.u + w.u * ob.pxx;
    db.pxy += ir * ob.v + w.u * ob.pxy;
    db.pyy += w.u * ob.pyy;
}

CSH_HD P swapb(const P& a) { return swap(a); }  // the adjoint of a permutation that is its own inverse

// face_states<TWOD>(W0, Wl, Wr, Wm, Wp, kx, ky): adjoints of the five input states
// The reverse pass of face_states in two parts that add up to it: the y part
// (the y slope, its tracing coefficients and transverse term; adjoints of Wm,
// Wp and its share of W0) and the x part (the rest: the x slope, its
// coefficients and term, and the identity part of base; Wl, Wr and the rest of
// W0).  Both need the summed face adjoints of base; each adds its own 1/rho
// term.  W0b accumulates y first, then x.
CSH_HD P base_adjoint(const Faces<double>& fb, bool twod)
{
    P baseb = zero_p();
    // xhi = base + chix dxm ; xlo = base - clox dxm ; the same for y
    acc(baseb, fb.xhi);
    acc(baseb, fb.xlo);
    if (twod) {
        acc(baseb, fb.yhi);
        acc(baseb, fb.ylo);
    }
    return baseb;
}

CSH_HD void face_states_vjp_y(const P& W0, const P& Wm, const P& Wp, double ky, const Faces<double>& fb, P& W0b,
                              P& Wmb, P& Wpb)
{
    // ---- forward recompute ----
    const double ir = rcp(W0.r);
    const P W0s = swap(W0);
    const E ey = eig_x(W0s, ir);
    const P dlys = swap(sub(W0, Wm)), drys = swap(sub(Wp, W0));
    const P dyms = limited_slope(W0s, ey, dlys, drys);
    const P dym = swap(dyms);
    const double chiy = 0.5 + ky * fmin(W0.v + ey.a, 0.0);
    const double cloy = 0.5 - ky * fmax(W0.v - ey.a, 0.0);
    // ---- reverse ----
    const P baseb = base_adjoint(fb, true);
    double irb = 0.0;
    E eyb{0, 0, 0, 0, 0, 0};
    P dymb = zero_p();
    acc(dymb, scale(chiy, fb.yhi));
    acc(dymb, scale(-cloy, fb.ylo));
    const double chiyb = dot(dym, fb.yhi), cloyb = -dot(dym, fb.ylo);
    // chiy = 1/2 + ky min(v + ay, 0) ; cloy = 1/2 - ky max(v - ay, 0)
    if (W0.v + ey.a < 0.0) {
        W0b.v += ky * chiyb;
        eyb.a += ky * chiyb;
    }
    if (W0.v - ey.a > 0.0) {
        W0b.v -= ky * cloyb;
        eyb.a += ky * cloyb;
    }
    // base -= ky swap(jac_x(W0s, ir, dyms))
    P W0sb = zero_p(), dymsb = swapb(dymb);
    jac_vjp(W0s, ir, dyms, scale(-ky, swapb(baseb)), W0sb, irb, dymsb);
    // dyms = limited_slope(W0s, ey, dlys, drys)
    P dlysb = zero_p(), drysb = zero_p();
    limited_slope_vjp(W0s, ey, dlys, drys, dymsb, W0sb, eyb, dlysb, drysb);
    eig_vjp(W0s, ir, ey, eyb, W0sb, irb);
    acc(W0b, swapb(W0sb));
    // dlys = swap(W0 - Wm), drys = swap(Wp - W0)
    const P dlyb = swapb(dlysb), dryb = swapb(drysb);
    acc(W0b, dlyb);
    acc(Wmb, scale(-1.0, dlyb));
    acc(Wpb, dryb);
    acc(W0b, scale(-1.0, dryb));
    // ir = 1 / W0.r
    W0b.r += -ir * ir * irb;
}

template <bool TWOD>
CSH_HD void face_states_vjp_x(const P& W0, const P& Wl, const P& Wr, double kx, const Faces<double>& fb, P& W0b,
                              P& Wlb, P& Wrb)
{
    // ---- forward recompute ----
    const double ir = rcp(W0.r);
    const E ex = eig_x(W0, ir);
    const P dlx = sub(W0, Wl), drx = sub(Wr, W0);
    const P dxm = limited_slope(W0, ex, dlx, drx);
    const double chix = 0.5 + kx * fmin(W0.u + ex.a, 0.0);
    const double clox = 0.5 - kx * fmax(W0.u - ex.a, 0.0);
    // ---- reverse ----
    const P baseb = base_adjoint(fb, TWOD);
    double irb = 0.0;
    E exb{0, 0, 0, 0, 0, 0};
    P dxmb = zero_p();
    acc(dxmb, scale(chix, fb.xhi));
    acc(dxmb, scale(-clox, fb.xlo));
    const double chixb = dot(dxm, fb.xhi), cloxb = -dot(dxm, fb.xlo);
    // chix = 1/2 + kx min(u + ax, 0) ; clox = 1/2 - kx max(u - ax, 0)
    if (W0.u + ex.a < 0.0) {
        W0b.u += kx * chixb;
        exb.a += kx * chixb;
    }
    if (W0.u - ex.a > 0.0) {
        W0b.u -= kx * cloxb;
        exb.a += kx * cloxb;
    }
    // base = W0 - kx jac_x(W0, ir, dxm) (- the transverse term, in the y part)
    acc(W0b, baseb);
    jac_vjp(W0, ir, dxm, scale(-kx, baseb), W0b, irb, dxmb);
    P dlxb = zero_p(), drxb = zero_p();
    limited_slope_vjp(W0, ex, dlx, drx, dxmb, W0b, exb, dlxb, drxb);
    eig_vjp(W0, ir, ex, exb, W0b, irb);
    // dlx = W0 - Wl, drx = Wr - W0
    acc(W0b, dlxb);
    acc(Wlb, scale(-1.0, dlxb));
    acc(Wrb, drxb);
    acc(W0b, scale(-1.0, drxb));
    // ir = 1 / W0.r
    W0b.r += -ir * ir * irb;
}

// reverse of face_states<double, TWOD>(W0, ir, Wl, Wr, Wm, Wp, kx, ky)
template <bool TWOD>
CSH_HD void face_states_vjp(const P& W0, const P& Wl, const P& Wr, const P& Wm, const P& Wp, double kx, double ky,
                            const Faces<double>& fb, P& W0b, P& Wlb, P& Wrb, P& Wmb, P& Wpb)
{
    if constexpr (TWOD) face_states_vjp_y(W0, Wm, Wp, ky, fb, W0b, Wmb, Wpb);
    face_states_vjp_x<TWOD>(W0, Wl, Wr, kx, fb, W0b, Wlb, Wrb);
}

// to_cons(w): mx = r u, my = r v, exx = pxx + mx u, exy = pxy + mx v, eyy = pyy + my v
CSH_HD void to_cons_vjp(const P& w, const C& Ub, P& wb)
{
    const double mx = w.r * w.u, my = w.r * w.v;
    wb.pxx += Ub.exx;
    wb.pxy += Ub.exy;
    wb.pyy += Ub.eyy;
    const double mxb = Ub.mx + w.u * Ub.exx + w.v * Ub.exy;
    const double myb = Ub.my + w.v * Ub.eyy;
    wb.u += mx * Ub.exx + w.r * mxb;
    wb.v += mx * Ub.exy + my * Ub.eyy + w.r * myb;
    wb.r += Ub.r + w.u * mxb + w.v * myb;
}

// to_prim(U): u = mx ir, v = my ir, pxx = exx - mx u, pxy = exy - mx v, pyy = eyy - my v
CSH_HD void to_prim_vjp(const C& U, const P& wb, C& Ub)
{
    const double ir = rcp(U.r);
    const double u = U.mx * ir, v = U.my * ir;
    Ub.exx += wb.pxx;
    Ub.exy += wb.pxy;
    Ub.eyy += wb.pyy;
    const double ub = wb.u - U.mx * wb.pxx;
    const double vb = wb.v - U.mx * wb.pxy - U.my * wb.pyy;
    Ub.mx += -u * wb.pxx - v * wb.pxy + ir * ub;
    Ub.my += -v * wb.pyy + ir * vb;
    const double irb = U.mx * ub + U.my * vb;
    Ub.r += wb.r - ir * ir * irb;
}

// flux_x(w, U)
CSH_HD void flux_vjp(const P& w, const C& U, const C& Fb, P& wb, C& Ub)
{
    Ub.mx += Fb.r + w.u * Fb.mx;
    Ub.my += w.u * Fb.my;
    Ub.exx += w.u * Fb.exx;
    Ub.exy += w.u * Fb.exy;
    Ub.eyy += w.u * Fb.eyy;
    wb.u += U.mx * Fb.mx + U.my * Fb.my + (U.exx + 2.0 * w.pxx) * Fb.exx + (U.exy + w.pxy) * Fb.exy + U.eyy * Fb.eyy;
    wb.v += w.pxx * Fb.exy + 2.0 * w.pxy * Fb.eyy;
    wb.pxx += Fb.mx + 2.0 * w.u * Fb.exx + w.v * Fb.exy;
    wb.pxy += Fb.my + w.u * Fb.exy + 2.0 * w.v * Fb.eyy;
}

// hll_x(make_face_x(wl), make_face_x(wr)): adjoints of the two primitive face states
CSH_HD void hll_vjp(const P& wl, const P& wr, const C& Fb, P& wlb, P& wrb)
{
    const Face<double> L = make_face_x(wl), R = make_face_x(wr);
    const double A1 = L.w.u - L.a, B1 = R.w.u - R.a;
    const double C1 = L.w.u + L.a, D1 = R.w.u + R.a;
    const double sl = fmin(fmin(A1, B1), 0.0);
    const double sr = fmax(fmax(C1, D1), 0.0);
    const double inv = rcp(sr - sl);
    const double slr = sl * sr;
    const C FL = flux_x(L.w, L.U), FR = flux_x(R.w, R.U);
    const double fl[6] = {FL.r, FL.mx, FL.my, FL.exx, FL.exy, FL.eyy};
    const double fr[6] = {FR.r, FR.mx, FR.my, FR.exx, FR.exy, FR.eyy};
    const double ul[6] = {L.U.r, L.U.mx, L.U.my, L.U.exx, L.U.exy, L.U.eyy};
    const double ur[6] = {R.U.r, R.U.mx, R.U.my, R.U.exx, R.U.exy, R.U.eyy};
    const double fb[6] = {Fb.r, Fb.mx, Fb.my, Fb.exx, Fb.exy, Fb.eyy};
    double flb[6], frb[6], ulb[6], urb[6];
    double srb = 0, slb = 0, invb = 0, slrb = 0;
    for (int k = 0; k < 6; ++k) {
        const double du = ur[k] - ul[k];
        const double N = sr * fl[k] - sl * fr[k] + slr * du;
        const double Nb = inv * fb[k];
        invb += N * fb[k];
        flb[k] = sr * Nb;
        frb[k] = -sl * Nb;
        srb += fl[k] * Nb;
        slb -= fr[k] * Nb;
        slrb += du * Nb;
        urb[k] = slr * Nb;
        ulb[k] = -slr * Nb;
    }
    srb += sl * slrb;
    slb += sr * slrb;
    // inv = 1 / (sr - sl)
    srb += -inv * inv * invb;
    slb += inv * inv * invb;
    double ulwb = 0, urwb = 0, alb = 0, arb = 0;  // adjoints of u_L, u_R, a_L, a_R
    if (fmin(A1, B1) < 0.0) {
        if (A1 <= B1) { ulwb += slb; alb -= slb; }
        else { urwb += slb; arb -= slb; }
    }
    if (fmax(C1, D1) > 0.0) {
        if (C1 >= D1) { ulwb += srb; alb += srb; }
        else { urwb += srb; arb += srb; }
    }
    C ULb = {ulb[0], ulb[1], ulb[2], ulb[3], ulb[4], ulb[5]};
    C URb = {urb[0], urb[1], urb[2], urb[3], urb[4], urb[5]};
    flux_vjp(L.w, L.U, C{flb[0], flb[1], flb[2], flb[3], flb[4], flb[5]}, wlb, ULb);
    flux_vjp(R.w, R.U, C{frb[0], frb[1], frb[2], frb[3], frb[4], frb[5]}, wrb, URb);
    to_cons_vjp(L.w, ULb, wlb);
    to_cons_vjp(R.w, URb, wrb);
    wlb.u += ulwb;
    wrb.u += urwb;
    // a = sqrt(3 pxx / r): da/dpxx = a / (2 pxx), da/dr = -a / (2 r)
    const double hl = 0.5 * L.a * alb, hr = 0.5 * R.a * arb;
    wlb.pxx += hl * rcp(L.w.pxx);
    wlb.r -= hl * rcp(L.w.r);
    wrb.pxx += hr * rcp(R.w.pxx);
    wrb.r -= hr * rcp(R.w.r);
}

// the fixed-field kick is affine in U with a constant Jacobian K; lam' = K^T lam
CSH_HD C kick_vjp(const C& lb, double h, double ax, double ay)
{
    C o = lb;
    o.r += h * ax * lb.mx + h * ay * lb.my + h * h * (ax * ax * lb.exx + ax * ay * lb.exy + ay * ay * lb.eyy);
    o.mx += 2.0 * h * ax * lb.exx + h * ay * lb.exy;
    o.my += h * ax * lb.exy + 2.0 * h * ay * lb.eyy;
    return o;
}

// ---- per-cell bodies of the adjoint kernels ----------------------------------------------

struct AdjArgs {
    int nx, ny, bcx, bcy;
    int ex, ey;          // extended grid: ex = nx + 2, ey = ny + 2 (1-D: 1)
    double dx, dy, dt;
    double kx, ky;       // dt / (2 dx), dt / (2 dy) (1-D: ky = 0)
    double cx, cy;       // dt / dx, dt / dy
    double vc2, rc2, x0, y0;
    const double* U;     // [6][ny][nx]
    const double* lam1;  // lam^{n+1}
    double* lam0;        // lam^n
    double* FS;          // [4 faces][6][ext]
    double* FSb;         // [4][6][ext]
    double* Cs;          // [3 roles][6][ext]: the y part's shares (SELF, DOWN, UP)
    double* XS;          // [6][ey][nx + 4]: per padded position (column -2 .. nx + 1 of an extended
                         // row), SELF and the x part's shares summed
};

// the step factors of AdjArgs from dt, dx, dy (IEEE divisions, once per call)
CSH_HD void set_step_factors(AdjArgs& a)
{
    a.kx = a.dt / (2.0 * a.dx);
    a.ky = a.ey > 1 ? a.dt / (2.0 * a.dy) : 0.0;
    a.cx = a.dt / a.dx;
    a.cy = a.ey > 1 ? a.dt / a.dy : 0.0;
}

enum { XHI = 0, XLO = 1, YHI = 2, YLO = 3 };
enum { SELF = 0, DOWN = 1, UP = 2 };

CSH_HD P load_p(const double* B, size_t plane, size_t slot, size_t idx)
{
    const double* b = B + slot * 6 * plane;
    return {b[idx], b[plane + idx], b[2 * plane + idx], b[3 * plane + idx], b[4 * plane + idx], b[5 * plane + idx]};
}
CSH_HD void store_p(double* B, size_t plane, size_t slot, size_t idx, const P& v)
{
    double* b = B + slot * 6 * plane;
    b[idx] = v.r;
    b[plane + idx] = v.u;
    b[2 * plane + idx] = v.v;
    b[3 * plane + idx] = v.pxx;
    b[4 * plane + idx] = v.pxy;
    b[5 * plane + idx] = v.pyy;
}

// map_index for -2n <= i < 3n (the reverse pass reads at most two cells past
// the extended ring, so any n >= 1 is covered): no division
CSH_HD int map_wide(int i, int n, int bc)
{
    if (bc == 0) {
        if (i < 0) i += n;
        if (i < 0) i += n;
        if (i >= n) i -= n;
        if (i >= n) i -= n;
        return i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// primitive state of the (possibly ghost) cell (i, j)
CSH_HD P prim_at(const AdjArgs& a, int i, int j, bool twod)
{
    const int gi = map_wide(i, a.nx, a.bcx);
    const int gj = twod ? map_wide(j, a.ny, a.bcy) : 0;
    return to_prim(load_cons<double>(a.U, (size_t)a.nx * a.ny, (size_t)gj * a.nx + gi));
}

CSH_HD size_t ext_index(const AdjArgs& a, int i, int j) { return (size_t)(j + (a.ey > 1 ? 1 : 0)) * a.ex + (i + 1); }

// lam' of interior cell (i, j): the kick's transpose applied to lam^{n+1}
CSH_HD C lam_prime(const AdjArgs& a, int i, int j, bool twod)
{
    const C l = load_cons<double>(a.lam1, (size_t)a.nx * a.ny, (size_t)j * a.nx + i);
    if (a.vc2 == 0.0) return l;
    const double x = a.x0 + (i + 0.5) * a.dx;
    const double y = twod ? a.y0 + (j + 0.5) * a.dy : 0.0;
    const double f = -a.vc2 * rcp(x * x + y * y + a.rc2);
    return kick_vjp(l, a.dt, f * x, f * y);
}

template <bool TWOD>
CSH_HD void faces_cell(const AdjArgs& a, int i, int j)
{
    const double kx = a.kx, ky = TWOD ? a.ky : 0.0;
    const P W0 = prim_at(a, i, j, TWOD);
    const P Wl = prim_at(a, i - 1, j, TWOD), Wr = prim_at(a, i + 1, j, TWOD);
    const P Wm = TWOD ? prim_at(a, i, j - 1, TWOD) : W0, Wp = TWOD ? prim_at(a, i, j + 1, TWOD) : W0;
    const Faces<double> f = face_states<double, TWOD>(W0, rcp(W0.r), Wl, Wr, Wm, Wp, kx, ky);
    const size_t ne = (size_t)a.ex * a.ey, e = ext_index(a, i, j);
    store_p(a.FS, ne, XHI, e, f.xhi);
    store_p(a.FS, ne, XLO, e, f.xlo);
    if (TWOD) {
        store_p(a.FS, ne, YHI, e, f.yhi);
        store_p(a.FS, ne, YLO, e, f.ylo);
    }
}

CSH_HD C csub(const C& p, const C& q, double s)
{
    return {s * (p.r - q.r), s * (p.mx - q.mx), s * (p.my - q.my), s * (p.exx - q.exx), s * (p.exy - q.exy),
            s * (p.eyy - q.eyy)};
}

template <bool TWOD>
CSH_HD void hll_cell(const AdjArgs& a, int i, int j)
{
    const size_t ne = (size_t)a.ex * a.ey;
    const size_t e = ext_index(a, i, j);
    const C z = zero_c();
    // face-state adjoint slots of this cell that no face writes (the outer
    // faces of the ring) are cleared here; every other slot is written by the
    // one face that uses that state
    const bool jin = !TWOD || (j >= 0 && j < a.ny), iin = i >= 0 && i < a.nx;
    if (!(i <= a.nx - 1 && jin)) store_p(a.FSb, ne, XHI, e, zero_p());
    if (!(i >= 0 && jin)) store_p(a.FSb, ne, XLO, e, zero_p());
    if (TWOD) {
        if (!(j <= a.ny - 1 && iin)) store_p(a.FSb, ne, YHI, e, zero_p());
        if (!(j >= 0 && iin)) store_p(a.FSb, ne, YLO, e, zero_p());
    }
    // x face i + 1/2 in an interior row: between extended cells (i, j) and (i + 1, j)
    if (i <= a.nx - 1 && (!TWOD || (j >= 0 && j < a.ny))) {
        const int jj = TWOD ? j : 0;
        const C lp = (i + 1 <= a.nx - 1) ? lam_prime(a, i + 1, jj, TWOD) : z;
        const C lm = (i >= 0) ? lam_prime(a, i, jj, TWOD) : z;
        const C Fb = csub(lp, lm, a.cx);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(load_p(a.FS, ne, XHI, e), load_p(a.FS, ne, XLO, e + 1), Fb, wlb, wrb);
        store_p(a.FSb, ne, XHI, e, wlb);
        store_p(a.FSb, ne, XLO, e + 1, wrb);
    }
    if (TWOD && j <= a.ny - 1 && i >= 0 && i < a.nx) {
        const C lp = (j + 1 <= a.ny - 1) ? lam_prime(a, i, j + 1, true) : z;
        const C lm = (j >= 0) ? lam_prime(a, i, j, true) : z;
        const C Gb = csub(lp, lm, a.cy);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(swap(load_p(a.FS, ne, YHI, e)), swap(load_p(a.FS, ne, YLO, e + a.ex)), swap(Gb), wlb, wrb);
        store_p(a.FSb, ne, YHI, e, swapb(wlb));
        store_p(a.FSb, ne, YLO, e + a.ex, swapb(wrb));
    }
}

CSH_HD Faces<double> load_face_adjoints(const AdjArgs& a, size_t ne, size_t e, bool twod)
{
    Faces<double> fb;
    fb.xhi = load_p(a.FSb, ne, XHI, e);
    fb.xlo = load_p(a.FSb, ne, XLO, e);
    if (twod) {
        fb.yhi = load_p(a.FSb, ne, YHI, e);
        fb.ylo = load_p(a.FSb, ne, YLO, e);
    } else {
        fb.yhi = fb.ylo = zero_p();
    }
    return fb;
}

// y part of the face-state adjoint of extended cell (i, j) (2-D): slots SELF
// (its share), DOWN, UP
CSH_HD void cells_cell_y(const AdjArgs& a, int i, int j)
{
    const double ky = a.ky;
    const size_t ne = (size_t)a.ex * a.ey, e = ext_index(a, i, j);
    const P W0 = prim_at(a, i, j, true);
    const P Wm = prim_at(a, i, j - 1, true), Wp = prim_at(a, i, j + 1, true);
    const Faces<double> fb = load_face_adjoints(a, ne, e, true);
    P b0 = zero_p(), bm = zero_p(), bp = zero_p();
    face_states_vjp_y(W0, Wm, Wp, ky, fb, b0, bm, bp);
    store_p(a.Cs, ne, SELF, e, b0);
    store_p(a.Cs, ne, DOWN, e, bm);
    store_p(a.Cs, ne, UP, e, bp);
}

// x part of extended cell (i, j): b0 = its SELF share (2-D: the y part's plus
// this part's), bl, br its LEFT and RIGHT shares (to positions i - 1, i + 1)
template <bool TWOD>
CSH_HD void cells_x_vjp(const AdjArgs& a, int i, int j, P& b0, P& bl, P& br)
{
    const double kx = a.kx;
    const size_t ne = (size_t)a.ex * a.ey, e = ext_index(a, i, j);
    const P W0 = prim_at(a, i, j, TWOD);
    const P Wl = prim_at(a, i - 1, j, TWOD), Wr = prim_at(a, i + 1, j, TWOD);
    const Faces<double> fb = load_face_adjoints(a, ne, e, TWOD);
    b0 = TWOD ? load_p(a.Cs, ne, SELF, e) : zero_p();
    bl = zero_p();
    br = zero_p();
    face_states_vjp_x<TWOD>(W0, Wl, Wr, kx, fb, b0, bl, br);
}

// index of padded position (px, j), px in [-2, nx + 1], j an extended row, in XS
CSH_HD size_t xs_index(const AdjArgs& a, int px, int j) { return (size_t)(j + (a.ey > 1 ? 1 : 0)) * (a.nx + 4) + (px + 2); }

// positions p in [-2, n+1] (the ghost-padded range the stencil reads) with
// map(p) == i; returns their count (at most 5)
CSH_HD int preimages(int i, int n, int bc, int* p)
{
    int k = 0;
    if (bc == 0) {  // periodic: p = i + m n
        for (int m = -3; m <= 3; ++m) {
            const int q = i + m * n;
            if (q >= -2 && q <= n + 1) p[k++] = q;
        }
    } else {        // outflow: clamp(p) == i
        const int lo = (i == 0) ? -2 : i, hi = (i == n - 1) ? n + 1 : i;
        for (int q = lo; q <= hi; ++q) p[k++] = q;
    }
    return k;
}

// sum of the shares that land on padded position (pi, pj): the x-part sum of
// its row (extended rows only) and the y part's DOWN and UP shares of the
// extended cells above and below
template <bool TWOD>
CSH_HD P pad_sum(const AdjArgs& a, int pi, int pj)
{
    const size_t ne = (size_t)a.ex * a.ey, nxs = (size_t)(a.nx + 4) * a.ey;
    auto in_ext = [&](int i, int j) { return i >= -1 && i <= a.nx && (!TWOD || (j >= -1 && j <= a.ny)); };
    P s = zero_p();
    if (!TWOD || (pj >= -1 && pj <= a.ny)) acc(s, load_p(a.XS, nxs, 0, xs_index(a, pi, pj)));
    if (TWOD) {
        if (in_ext(pi, pj + 1)) acc(s, load_p(a.Cs, ne, DOWN, ext_index(a, pi, pj + 1)));
        if (in_ext(pi, pj - 1)) acc(s, load_p(a.Cs, ne, UP, ext_index(a, pi, pj - 1)));
    }
    return s;
}

template <bool TWOD>
CSH_HD void gather_cell(const AdjArgs& a, int i, int j)
{
    int px[5], py[5];
    const int nx_ = preimages(i, a.nx, a.bcx, px);
    const int ny_ = TWOD ? preimages(j, a.ny, a.bcy, py) : 1;
    if (!TWOD) py[0] = 0;
    P wb = zero_p();
    for (int u = 0; u < nx_; ++u)
        for (int v = 0; v < ny_; ++v) acc(wb, pad_sum<TWOD>(a, px[u], py[v]));
    const size_t plane = (size_t)a.nx * a.ny, c = (size_t)j * a.nx + i;
    C out = lam_prime(a, i, j, TWOD);
    to_prim_vjp(load_cons<double>(a.U, plane, c), wb, out);
    store_cons(a.lam0, plane, c, out);
}

// ---- the tiled two-kernel reverse pass (2-D) ----------------------------------------------
//
// Kernel A (faces and fluxes) and kernel B (face states and gather) replace the
// five one-thread-per-cell stages on 2-D grids.  Each works on a tile held in
// LDS, so the face states, the shares of the face-state reverse pass and
// their sums never travel through device memory; only the face-state
// adjoints (FSb) pass from A to B.
//
// Periodic axes are treated as a pure wrap: a virtual cell outside [0, n) is
// the wrapped cell (its state, its lam' and its face-state adjoints), every
// face is a real face, and an output cell gathers only the shares that land on
// itself.  Outflow axes keep the extended ring (cells -1 and n, lam' = 0
// outside [0, n)), and the shares landing on ghost positions (-2, -1, n,
// n + 1) are folded into the boundary cell.  Both are the transpose of the
// same forward step; they differ from the five-stage pass only in the order
// of the sums.
//
// The bodies below are the per-thread work of each phase between the
// workgroup barriers, written so a CPU loop over tiles, phases and threads
// runs them unchanged (tests/host).

// kernel A: a tile of kA_TX x kA_TY extended cells, one thread per cell
constexpr int kA_TX = 32, kA_TY = 8, kA_THREADS = kA_TX * kA_TY;
constexpr int kA_WX = kA_TX + 3, kA_WY = kA_TY + 3;  // states: cells [X0 - 1, X0 + TX + 2)
constexpr int kA_FX = kA_TX + 1, kA_FY = kA_TY + 1;  // face states: cells [X0, X0 + TX + 1)
constexpr int kA_NW = kA_WX * kA_WY, kA_NF = kA_FX * kA_FY;
constexpr int kA_LDS = 6 * kA_NW + 12 * kA_NF;       // doubles of LDS: states, low x and y face states

// kernel B: a tile of kB_W x kB_H virtual cells (four rows per wavefront),
// the outputs its inner (kB_W - 2) x (kB_H - 2) cells.  16 x 16 rather than
// 64 x 8: 77 KB of LDS, so two workgroups share a CU and one's barriers
// overlap the other's work, and at 512^2 1369 tiles fill three rounds of 512
// (64 x 8: 774 tiles, four rounds of one workgroup per CU)
constexpr int kB_W = 16, kB_H = 16, kB_THREADS = kB_W * kB_H;
constexpr int kB_OX = kB_W - 2, kB_OY = kB_H - 2;
enum { SH_LEFT = 0, SH_RIGHT = 1, SH_DOWN = 2, SH_UP = 3, SH_TOT = 4 };
constexpr int kB_SX = kB_W + 2, kB_SY = kB_H + 2, kB_NS = kB_SX * kB_SY;  // states: the tile and a ring
constexpr int kB_LDS = 5 * 6 * kB_THREADS + 6 * kB_NS;  // doubles of LDS (the states after the shares)

CSH_HD void lds_put(double* L, int stride, int base, int k, const P& v)
{
    L[base + 0 * stride + k] = v.r;
    L[base + 1 * stride + k] = v.u;
    L[base + 2 * stride + k] = v.v;
    L[base + 3 * stride + k] = v.pxx;
    L[base + 4 * stride + k] = v.pxy;
    L[base + 5 * stride + k] = v.pyy;
}
CSH_HD P lds_get(const double* L, int stride, int base, int k)
{
    return {L[base + k], L[base + stride + k], L[base + 2 * stride + k], L[base + 3 * stride + k],
            L[base + 4 * stride + k], L[base + 5 * stride + k]};
}

// lam' of a virtual cell: wrapped on periodic axes; zero outside the grid on outflow ones
CSH_HD C lam_prime_virtual(const AdjArgs& a, int i, int j)
{
    if (a.bcx != 0 && (i < 0 || i >= a.nx)) return zero_c();
    if (a.bcy != 0 && (j < 0 || j >= a.ny)) return zero_c();
    return lam_prime(a, map_wide(i, a.nx, a.bcx), map_wide(j, a.ny, a.bcy), true);
}

// A1: primitive states of the cells [X0 - 1, X0 + TX + 2) x [Y0 - 1, Y0 + TY + 2)
// (coordinates past [-2, n + 1] are clamped into it: those cells only feed
// face states of cells beyond the extended ring, which no face uses)
CSH_HD void tileA_states(const AdjArgs& a, int X0, int Y0, int t, double* L)
{
    for (int k = t; k < kA_NW; k += kA_THREADS) {
        const int i0 = X0 - 1 + k % kA_WX, j0 = Y0 - 1 + k / kA_WX;
        const int i = i0 < -2 ? -2 : (i0 > a.nx + 1 ? a.nx + 1 : i0);
        const int j = j0 < -2 ? -2 : (j0 > a.ny + 1 ? a.ny + 1 : j0);
        lds_put(L, kA_NW, 0, k, prim_at(a, i, j, true));
    }
}

// face states of cell k of the face-state block [X0, X0 + TX + 1) x [Y0, Y0 + TY + 1)
CSH_HD Faces<double> tileA_face_states(const AdjArgs& a, int k, const double* L)
{
    const int lx = k % kA_FX + 1, ly = k / kA_FX + 1;  // position in the state block
    const int c = ly * kA_WX + lx;
    const P W0 = lds_get(L, kA_NW, 0, c);
    return face_states<double, true>(W0, rcp(W0.r), lds_get(L, kA_NW, 0, c - 1), lds_get(L, kA_NW, 0, c + 1),
                                     lds_get(L, kA_NW, 0, c - kA_WX), lds_get(L, kA_NW, 0, c + kA_WX), a.kx, a.ky);
}

// A2: the face states of the thread's own cell e = (X0 + t % TX, Y0 + t / TX):
// the high ones kept (returned), the low ones written to LDS for the faces of
// the cells to the left and below; then the low x face states of the column
// to the right of the tile and the low y face states of the row above it
CSH_HD void tileA_faces(const AdjArgs& a, int t, double* L, P& xhi, P& yhi)
{
    double* X = L + 6 * kA_NW;
    double* Y = X + 6 * kA_NF;
    const int k = (t / kA_TX) * kA_FX + t % kA_TX;
    const Faces<double> f = tileA_face_states(a, k, L);
    xhi = f.xhi;
    yhi = f.yhi;
    lds_put(X, kA_NF, 0, k, f.xlo);
    lds_put(Y, kA_NF, 0, k, f.ylo);
    if (t < kA_TY + kA_TX) {
        const bool col = t < kA_TY;  // the column x = X0 + TX, else the row y = Y0 + TY
        const int k2 = col ? t * kA_FX + kA_TX : kA_TY * kA_FX + (t - kA_TY);
        const Faces<double> g = tileA_face_states(a, k2, L);
        if (col) lds_put(X, kA_NF, 0, k2, g.xlo);
        else lds_put(Y, kA_NF, 0, k2, g.ylo);
    }
}

// A3: the extended cell e of the thread: the flux adjoints of its high x and
// y faces, through HLL into the adjoints of the two face states of each
// (written to FSb); the slots of the ring that no face writes are cleared
CSH_HD void tileA_fluxes(const AdjArgs& a, int X0, int Y0, int t, const double* L, const P& xhi, const P& yhi)
{
    const double* X = L + 6 * kA_NW;
    const double* Y = X + 6 * kA_NF;
    const int i = X0 + t % kA_TX, j = Y0 + t / kA_TX;
    if (i > a.nx || j > a.ny) return;  // outside the extended grid
    const size_t ne = (size_t)a.ex * a.ey, e = ext_index(a, i, j);
    const int k = (t / kA_TX) * kA_FX + t % kA_TX;  // e in the face-state block
    if (i == a.nx) store_p(a.FSb, ne, XHI, e, zero_p());
    if (i == -1) store_p(a.FSb, ne, XLO, e, zero_p());
    if (j == a.ny) store_p(a.FSb, ne, YHI, e, zero_p());
    if (j == -1) store_p(a.FSb, ne, YLO, e, zero_p());
    if (i == a.nx && j == a.ny) return;
    const C l0 = lam_prime_virtual(a, i, j);
    if (i <= a.nx - 1) {  // x face i + 1/2
        const C Fb = csub(lam_prime_virtual(a, i + 1, j), l0, a.cx);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(xhi, lds_get(X, kA_NF, 0, k + 1), Fb, wlb, wrb);
        store_p(a.FSb, ne, XHI, e, wlb);
        store_p(a.FSb, ne, XLO, e + 1, wrb);
    }
    if (j <= a.ny - 1) {  // y face j + 1/2
        const C Gb = csub(lam_prime_virtual(a, i, j + 1), l0, a.cy);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(swap(yhi), swap(lds_get(Y, kA_NF, 0, k + kA_FX)), swap(Gb), wlb, wrb);
        store_p(a.FSb, ne, YHI, e, swapb(wlb));
        store_p(a.FSb, ne, YLO, e + a.ex, swapb(wrb));
    }
}

// index of a virtual cell in the extended face-state arrays, -1 for a cell
// beyond the ring [-1, n] (its shares reach no output: on an outflow axis its
// face states feed no face, on a periodic one it is not next to an output);
// a ring cell of a periodic axis is the wrapped cell
CSH_HD long ext_of_virtual(const AdjArgs& a, int i, int j)
{
    if (i < -1 || i > a.nx || j < -1 || j > a.ny) return -1;
    if (a.bcx == 0) i = map_wide(i, a.nx, 0);
    if (a.bcy == 0) j = map_wide(j, a.ny, 0);
    return (long)ext_index(a, i, j);
}

// B0: primitive states of the tile and its ring, cells [X0 - 2, X0 + kB_W) x
// [Y0 - 2, Y0 + kB_H) (coordinates clamped into [-2, n + 1], as in A1)
CSH_HD void tileB_states(const AdjArgs& a, int X0, int Y0, int t, double* L)
{
    double* S = L + 5 * 6 * kB_THREADS;
    for (int k = t; k < kB_NS; k += kB_THREADS) {
        const int i0 = X0 - 2 + k % kB_SX, j0 = Y0 - 2 + k / kB_SX;
        const int i = i0 < -2 ? -2 : (i0 > a.nx + 1 ? a.nx + 1 : i0);
        const int j = j0 < -2 ? -2 : (j0 > a.ny + 1 ? a.ny + 1 : j0);
        lds_put(S, kB_NS, 0, k, prim_at(a, i, j, true));
    }
}

// the face-state adjoints of the thread's cell; zero beyond the ring
CSH_HD Faces<double> tileB_face_adjoints(const AdjArgs& a, int X0, int Y0, int t)
{
    const long e = ext_of_virtual(a, X0 - 1 + t % kB_W, Y0 - 1 + t / kB_W);
    if (e < 0) return {zero_p(), zero_p(), zero_p(), zero_p()};
    return load_face_adjoints(a, (size_t)a.ex * a.ey, (size_t)e, true);
}

// B1: the face-state reverse pass of the virtual cell at column l, row w of the
// tile (X0 - 1 + l, Y0 - 1 + w) from its face-state adjoints fb: its own share
// returned, the four it gives its neighbours written to LDS
CSH_HD P tileB_shares(const AdjArgs& a, int X0, int Y0, int t, double* L, const Faces<double>& fb)
{
    const double* S = L + 5 * 6 * kB_THREADS;
    const int l = t % kB_W, w = t / kB_W;
    const int i = X0 - 1 + l, j = Y0 - 1 + w;
    const int c = (w + 1) * kB_SX + (l + 1);  // the cell in the state block
    P b0 = zero_p();
    const long e = ext_of_virtual(a, i, j);
    // the y part first, its two neighbour shares stored before the x part
    // starts (fewer values live at once)
    const P W0 = e >= 0 ? lds_get(S, kB_NS, 0, c) : zero_p();
    {
        P bm = zero_p(), bp = zero_p();
        if (e >= 0)
            face_states_vjp_y(W0, lds_get(S, kB_NS, 0, c - kB_SX), lds_get(S, kB_NS, 0, c + kB_SX), a.ky, fb, b0, bm,
                              bp);
        lds_put(L, kB_THREADS, SH_DOWN * 6 * kB_THREADS, t, bm);
        lds_put(L, kB_THREADS, SH_UP * 6 * kB_THREADS, t, bp);
    }
    P bl = zero_p(), br = zero_p();
    if (e >= 0)
        face_states_vjp_x<true>(W0, lds_get(S, kB_NS, 0, c - 1), lds_get(S, kB_NS, 0, c + 1), a.kx, fb, b0, bl, br);
    lds_put(L, kB_THREADS, SH_LEFT * 6 * kB_THREADS, t, bl);
    lds_put(L, kB_THREADS, SH_RIGHT * 6 * kB_THREADS, t, br);
    return b0;
}

// B2: everything that lands on the position of column l, row w from inside the tile
CSH_HD P tileB_total(int t, const P& self, const double* L)
{
    const int l = t % kB_W, w = t / kB_W;
    P s = self;
    if (l + 1 < kB_W) acc(s, lds_get(L, kB_THREADS, SH_LEFT * 6 * kB_THREADS, t + 1));
    if (l >= 1) acc(s, lds_get(L, kB_THREADS, SH_RIGHT * 6 * kB_THREADS, t - 1));
    if (w >= 1) acc(s, lds_get(L, kB_THREADS, SH_UP * 6 * kB_THREADS, t - kB_W));
    if (w + 1 < kB_H) acc(s, lds_get(L, kB_THREADS, SH_DOWN * 6 * kB_THREADS, t + kB_W));
    return s;
}

CSH_HD void tileB_put_total(int t, const P& s, double* L) { lds_put(L, kB_THREADS, SH_TOT * 6 * kB_THREADS, t, s); }

// what lands on tile position (lp, wp), lp in [-1, kB_W], wp in [-1, kB_H]:
// the total inside the tile, or the one share a tile cell gives a position just
// outside it (the cells beyond it feed only ghost positions of outflow axes
// through shares that are zero: they lie past the extended ring)
CSH_HD P tileB_landing(int lp, int wp, const double* L)
{
    const bool xin = lp >= 0 && lp < kB_W, yin = wp >= 0 && wp < kB_H;
    if (xin && yin) return lds_get(L, kB_THREADS, SH_TOT * 6 * kB_THREADS, wp * kB_W + lp);
    if (yin && lp == -1) return lds_get(L, kB_THREADS, SH_LEFT * 6 * kB_THREADS, wp * kB_W);
    if (yin && lp == kB_W) return lds_get(L, kB_THREADS, SH_RIGHT * 6 * kB_THREADS, wp * kB_W + kB_W - 1);
    if (xin && wp == -1) return lds_get(L, kB_THREADS, SH_DOWN * 6 * kB_THREADS, lp);
    if (xin && wp == kB_H) return lds_get(L, kB_THREADS, SH_UP * 6 * kB_THREADS, (kB_H - 1) * kB_W + lp);
    return zero_p();
}

// positions whose shares belong to output coordinate i on one axis: itself, and
// on an outflow axis the ghost positions the boundary cell stands for
CSH_HD int fold_positions(int i, int n, int bc, int* p)
{
    int k = 0;
    p[k++] = i;
    if (bc != 0) {
        if (i == 0) { p[k++] = -1; p[k++] = -2; }
        if (i == n - 1) { p[k++] = n; p[k++] = n + 1; }
    }
    return k;
}

// B3: the output cell at column l, row w (inner cells only): the folded total of
// the shares on its positions, through W(U), plus lam' itself
CSH_HD void tileB_gather(const AdjArgs& a, int X0, int Y0, int t, const double* L)
{
    const int l = t % kB_W, w = t / kB_W;
    if (l < 1 || l > kB_OX || w < 1 || w > kB_OY) return;
    const int i = X0 - 1 + l, j = Y0 - 1 + w;
    if (i >= a.nx || j >= a.ny) return;
    int px[5], py[5];
    const int nx_ = fold_positions(i, a.nx, a.bcx, px), ny_ = fold_positions(j, a.ny, a.bcy, py);
    P wb = zero_p();
    for (int u = 0; u < nx_; ++u)
        for (int v = 0; v < ny_; ++v) acc(wb, tileB_landing(px[u] - (X0 - 1), py[v] - (Y0 - 1), L));
    const size_t plane = (size_t)a.nx * a.ny, c = (size_t)j * a.nx + i;
    C out = lam_prime(a, i, j, true);
    to_prim_vjp(load_cons<double>(a.U, plane, c), wb, out);
    store_cons(a.lam0, plane, c, out);
}

}  // namespace csh
