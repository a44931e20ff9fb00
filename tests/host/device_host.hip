// CPU harness for the forward sweep's per-state arithmetic (csh_device.h and
// csh3_device.h are host-callable): one state or one face at a time, so the
// tests can compare the kernels' closed forms with the oracle's per-state
// functions on random states without a GPU.  Test infrastructure only.
#include "csh_device.h"
#include "csh3_device.h"

using namespace csh;
using P = Prim<double>;

static P ld(const double* a) { return {a[0], a[1], a[2], a[3], a[4], a[5]}; }
static void st(double* o, const P& w)
{
    o[0] = w.r;
    o[1] = w.u;
    o[2] = w.v;
    o[3] = w.pxx;
    o[4] = w.pxy;
    o[5] = w.pyy;
}
static void stc(double* o, const Cons<double>& U)
{
    o[0] = U.r;
    o[1] = U.mx;
    o[2] = U.my;
    o[3] = U.exx;
    o[4] = U.exy;
    o[5] = U.eyy;
}
static P dir_in(int dir, const P& w) { return dir ? swap(w) : w; }

extern "C" double dev_mc_half(double dl, double dr) { return mc_half(dl, dr); }

// the characteristic MC slope (twice the kernels' half slope) along x or y
extern "C" void dev_slope(int dir, const double* wm, const double* w0, const double* wp, double* out)
{
    const P m = dir_in(dir, ld(wm)), c = dir_in(dir, ld(w0)), p = dir_in(dir, ld(wp));
    const double ir = rcp(c.r);
    const P h = half_slope(c, ir, eig_x(c, ir), sub(c, m), sub(p, c));
    st(out, dir_in(dir, {2 * h.r, 2 * h.u, 2 * h.v, 2 * h.pxx, 2 * h.pxy, 2 * h.pyy}));
}

// the two x-face states of a cell in one dimension, k = dt / (2 dx)
extern "C" void dev_faces_1d(const double* wl, const double* w0, const double* wr, double k, double* lo, double* hi)
{
    const P c = ld(w0);
    const Faces<double> f = face_states<double, false>(c, rcp(c.r), ld(wl), ld(wr), c, c, k, 0.0);
    st(lo, f.xlo);
    st(hi, f.xhi);
}

template <int RS>
static void face_flux(int dir, const double* wl, const double* wr, double* out)
{
    const Cons<double> F = riemann_x<RS>(make_face_x(dir_in(dir, ld(wl))), make_face_x(dir_in(dir, ld(wr))));
    stc(out, dir ? swap(F) : F);
}
extern "C" void dev_hll(int dir, const double* wl, const double* wr, double* out) { face_flux<0>(dir, wl, wr, out); }
extern "C" void dev_hllc(int dir, const double* wl, const double* wr, double* out) { face_flux<1>(dir, wl, wr, out); }

// the Kurganov-Tadmor flux of eq. (6) (the kernels form twice it)
extern "C" void dev_kt_flux(int dir, const double* wl, const double* wr, double* out)
{
    const Cons<double> F2 = kt_flux2_x(dir_in(dir, ld(wl)), dir_in(dir, ld(wr)));
    const Cons<double> F = {0.5 * F2.r, 0.5 * F2.mx, 0.5 * F2.my, 0.5 * F2.exx, 0.5 * F2.exy, 0.5 * F2.eyy};
    stc(out, dir ? swap(F) : F);
}

// three dimensions: the characteristic MC slope and the HLL flux along an axis
static d3::V10 ld10(const double* a)
{
    d3::V10 x;
    for (int m = 0; m < d3::NV; ++m) x.v[m] = a[m];
    return x;
}
template <int N>
static void slope3(const double* wm, const double* w0, const double* wp, double* out)
{
    const d3::V10 c = ld10(w0);
    const double ir = rcp(c.v[0]);
    const d3::V10 h = d3::half_slope<N>(c, ir, d3::eig<N>(c, ir), ld10(wm), ld10(wp));
    for (int m = 0; m < d3::NV; ++m) out[m] = 2 * h.v[m];
}
template <int N>
static void hll3(const double* wl, const double* wr, double* out)
{
    const d3::V10 F = d3::hll<N>(ld10(wl), ld10(wr));
    for (int m = 0; m < d3::NV; ++m) out[m] = F.v[m];
}
extern "C" void dev_slope3(int axis, const double* wm, const double* w0, const double* wp, double* out)
{
    if (axis == 0) slope3<0>(wm, w0, wp, out);
    else if (axis == 1) slope3<1>(wm, w0, wp, out);
    else slope3<2>(wm, w0, wp, out);
}
extern "C" void dev_hll3(int axis, const double* wl, const double* wr, double* out)
{
    if (axis == 0) hll3<0>(wl, wr, out);
    else if (axis == 1) hll3<1>(wl, wr, out);
    else hll3<2>(wl, wr, out);
}

// the Newton refinements of the device's reciprocal, reciprocal square root and
// square root, fed an approximation from the caller
extern "C" double dev_rcp_refine(double x, double r) { return rcp_refine(x, r); }
extern "C" double dev_rsqrt_refine(double x, double y) { return rsqrt_refine(x, y); }
extern "C" double dev_sqrt_refine(double x, double y) { return sqrt_refine(x, y); }
