// CPU harness for the adjoint: runs the per-cell bodies of the adjoint kernels
// and the forward face/flux arithmetic in host loops, so the tests can check
// the hand-written reverse pass against finite differences and the oracle's
// dense Jacobian without a GPU.  Test infrastructure only.
#include <algorithm>
#include <cstring>
#include <limits>
#include <vector>

#include "csh_adjoint.h"

using namespace csh;

static AdjArgs make_args(int nx, int ny, int bcx, int bcy, double dx, double dy, double dt, double vc, double rc,
                         double x0, double y0, const double* U)
{
    AdjArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.bcx = bcx;
    a.bcy = bcy;
    a.ex = nx + 2;
    a.ey = ny > 1 ? ny + 2 : 1;
    a.dx = dx;
    a.dy = ny > 1 ? dy : 1.0;
    a.dt = dt;
    set_step_factors(a);
    a.vc2 = vc * vc;
    a.rc2 = rc * rc;
    a.x0 = x0;
    a.y0 = y0;
    a.U = U;
    return a;
}

template <bool TWOD>
static void adjoint_loops(AdjArgs& a)
{
    const int j0 = TWOD ? -1 : 0, j1 = TWOD ? a.ny : 0;
    for (int j = j0; j <= j1; ++j)
        for (int i = -1; i <= a.nx; ++i) faces_cell<TWOD>(a, i, j);
    for (int j = j0; j <= j1; ++j)
        for (int i = -1; i <= a.nx; ++i) hll_cell<TWOD>(a, i, j);
    if constexpr (TWOD)
        for (int j = j0; j <= j1; ++j)
            for (int i = -1; i <= a.nx; ++i) cells_cell_y(a, i, j);
    // x part: self, left and right shares per extended cell, then one sum per
    // padded position in the kernel's order (self, left share of the cell to
    // the right, right share of the cell to the left; zero outside the range)
    const size_t ne = (size_t)a.ex * a.ey, nxs = (size_t)(a.nx + 4) * a.ey;
    std::vector<P> b0(ne, zero_p()), bl(ne, zero_p()), br(ne, zero_p());
    for (int j = j0; j <= j1; ++j)
        for (int i = -1; i <= a.nx; ++i) {
            const size_t e = ext_index(a, i, j);
            cells_x_vjp<TWOD>(a, i, j, b0[e], bl[e], br[e]);
        }
    auto share = [&](const std::vector<P>& v, int i, int j) { return i >= -1 && i <= a.nx ? v[ext_index(a, i, j)] : zero_p(); };
    for (int j = j0; j <= j1; ++j)
        for (int px = -2; px <= a.nx + 1; ++px) {
            const P s0 = share(b0, px, j), l = share(bl, px + 1, j), r = share(br, px - 1, j);
            const P sum = {s0.r + l.r + r.r,       s0.u + l.u + r.u,       s0.v + l.v + r.v,
                           s0.pxx + l.pxx + r.pxx, s0.pxy + l.pxy + r.pxy, s0.pyy + l.pyy + r.pyy};
            store_p(a.XS, nxs, 0, xs_index(a, px, j), sum);
        }
    for (int j = 0; j < (TWOD ? a.ny : 1); ++j)
        for (int i = 0; i < a.nx; ++i) gather_cell<TWOD>(a, i, j);
}

extern "C" int host_adjoint_step(int nx, int ny, int bcx, int bcy, double dx, double dy, double dt, double vc,
                                 double rc, double x0, double y0, const double* U, const double* lam1, double* lam0)
{
    AdjArgs a = make_args(nx, ny, bcx, bcy, dx, dy, dt, vc, rc, x0, y0, U);
    const size_t ne = (size_t)a.ex * a.ey;
    // NaN-filled: every slot the reverse pass reads must have been written by it
    std::vector<double> ws(66 * ne + 6 * (size_t)(nx + 4) * a.ey, std::numeric_limits<double>::quiet_NaN());
    a.FS = ws.data();
    a.FSb = ws.data() + 24 * ne;
    a.Cs = ws.data() + 48 * ne;
    a.XS = ws.data() + 66 * ne;
    a.lam1 = lam1;
    a.lam0 = lam0;
    if (ny > 1) adjoint_loops<true>(a);
    else adjoint_loops<false>(a);
    return 0;
}

// The tiled two-kernel reverse pass of 2-D grids (kernels A and B) run on the
// CPU: per tile, each phase for every thread, a host array standing for LDS;
// the tiles in the GPU's numbering order.  NaN-filled buffers: a slot read
// before it is written shows in the result.
extern "C" int host_adjoint_step_tiled(int nx, int ny, int bcx, int bcy, double dx, double dy, double dt, double vc,
                                       double rc, double x0, double y0, const double* U, const double* lam1,
                                       double* lam0)
{
    if (ny < 2) return -1;
    AdjArgs a = make_args(nx, ny, bcx, bcy, dx, dy, dt, vc, rc, x0, y0, U);
    const size_t ne = (size_t)a.ex * a.ey;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> fsb(24 * ne, nan);
    a.FSb = fsb.data();
    a.lam1 = lam1;
    a.lam0 = lam0;
    std::vector<double> L((size_t)(kA_LDS > kB_LDS ? kA_LDS : kB_LDS));
    const int tax = (a.ex + kA_TX - 1) / kA_TX, tay = (a.ey + kA_TY - 1) / kA_TY;
    std::vector<P> xhi(kA_THREADS), yhi(kA_THREADS);
    for (int ty = 0; ty < tay; ++ty)
        for (int tx = 0; tx < tax; ++tx) {
            const int X0 = -1 + tx * kA_TX, Y0 = -1 + ty * kA_TY;
            std::fill(L.begin(), L.end(), nan);
            for (int t = 0; t < kA_THREADS; ++t) tileA_states(a, X0, Y0, t, L.data());
            for (int t = 0; t < kA_THREADS; ++t) tileA_faces(a, t, L.data(), xhi[t], yhi[t]);
            for (int t = 0; t < kA_THREADS; ++t) tileA_fluxes(a, X0, Y0, t, L.data(), xhi[t], yhi[t]);
        }
    const int tbx = (nx + kB_OX - 1) / kB_OX, tby = (ny + kB_OY - 1) / kB_OY;
    std::vector<P> self(kB_THREADS), tot(kB_THREADS);
    std::vector<Faces<double>> fbs(kB_THREADS);
    for (int ty = 0; ty < tby; ++ty)
        for (int tx = 0; tx < tbx; ++tx) {
            const int X0 = tx * kB_OX, Y0 = ty * kB_OY;
            std::fill(L.begin(), L.end(), nan);
            for (int t = 0; t < kB_THREADS; ++t) {
                fbs[t] = tileB_face_adjoints(a, X0, Y0, t);
                tileB_states(a, X0, Y0, t, L.data());
            }
            for (int t = 0; t < kB_THREADS; ++t) self[t] = tileB_shares(a, X0, Y0, t, L.data(), fbs[t]);
            for (int t = 0; t < kB_THREADS; ++t) tot[t] = tileB_total(t, self[t], L.data());
            for (int t = 0; t < kB_THREADS; ++t) tileB_put_total(t, tot[t], L.data());
            for (int t = 0; t < kB_THREADS; ++t) tileB_gather(a, X0, Y0, t, L.data());
        }
    return 0;
}

// the forward step with the same face-state, HLL, update and kick arithmetic
template <bool TWOD>
static void step_loops(AdjArgs& a, double* Un)
{
    const int j0 = TWOD ? -1 : 0, j1 = TWOD ? a.ny : 0;
    for (int j = j0; j <= j1; ++j)
        for (int i = -1; i <= a.nx; ++i) faces_cell<TWOD>(a, i, j);
    const size_t ne = (size_t)a.ex * a.ey, plane = (size_t)a.nx * a.ny;
    const double cx = a.dt / a.dx, cy = a.dt / a.dy;
    for (int j = 0; j < (TWOD ? a.ny : 1); ++j)
        for (int i = 0; i < a.nx; ++i) {
            const size_t e = ext_index(a, i, j);
            const C Fp = hll_x(make_face_x(load_p(a.FS, ne, XHI, e)), make_face_x(load_p(a.FS, ne, XLO, e + 1)));
            const C Fm = hll_x(make_face_x(load_p(a.FS, ne, XHI, e - 1)), make_face_x(load_p(a.FS, ne, XLO, e)));
            C u = update(load_cons<double>(a.U, plane, (size_t)j * a.nx + i), cx, Fp, Fm);
            if (TWOD) {
                const C Gp = swap(hll_x(make_face_x(swap(load_p(a.FS, ne, YHI, e))),
                                        make_face_x(swap(load_p(a.FS, ne, YLO, e + a.ex)))));
                const C Gm = swap(hll_x(make_face_x(swap(load_p(a.FS, ne, YHI, e - a.ex))),
                                        make_face_x(swap(load_p(a.FS, ne, YLO, e)))));
                u = update(u, cy, Gp, Gm);
            }
            if (a.vc2 != 0.0) {
                const double x = a.x0 + (i + 0.5) * a.dx, y = TWOD ? a.y0 + (j + 0.5) * a.dy : 0.0;
                const double f = -a.vc2 / (x * x + y * y + a.rc2), ax = f * x, ay = f * y, h = a.dt;
                const double mx = u.mx, my = u.my;
                u.mx = mx + h * u.r * ax;
                u.my = my + h * u.r * ay;
                u.exx = u.exx + h * ax * (2.0 * mx + h * u.r * ax);
                u.exy = u.exy + h * (ax * my + mx * ay + h * u.r * ax * ay);
                u.eyy = u.eyy + h * ay * (2.0 * my + h * u.r * ay);
            }
            store_cons(Un, plane, (size_t)j * a.nx + i, u);
        }
}

extern "C" int host_step(int nx, int ny, int bcx, int bcy, double dx, double dy, double dt, double vc, double rc,
                         double x0, double y0, const double* U, double* Un)
{
    AdjArgs a = make_args(nx, ny, bcx, bcy, dx, dy, dt, vc, rc, x0, y0, U);
    const size_t ne = (size_t)a.ex * a.ey;
    std::vector<double> fs(24 * ne, 0.0);
    a.FS = fs.data();
    if (ny > 1) step_loops<true>(a, Un);
    else step_loops<false>(a, Un);
    return 0;
}

// W -> U and its transpose, per cell
extern "C" void host_init_adjoint(int64_t n, const double* W, const double* lamU, double* lamW)
{
    for (int64_t c = 0; c < n; ++c) {
        const P w = {W[c], W[n + c], W[2 * n + c], W[3 * n + c], W[4 * n + c], W[5 * n + c]};
        P wb = zero_p();
        to_cons_vjp(w, load_cons<double>(lamU, (size_t)n, (size_t)c), wb);
        const double v[6] = {wb.r, wb.u, wb.v, wb.pxx, wb.pxy, wb.pyy};
        for (int m = 0; m < 6; ++m) lamW[m * n + c] = v[m];
    }
}

// the adjoint kernels' workgroup renumbering, for the bijection test
extern "C" unsigned host_xcd_block(unsigned b, unsigned nb)
{
    return csh::xcd_block(b, nb);
}
