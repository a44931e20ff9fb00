// Adjoint of one sweep at frozen timestep (FP64): lam^n = (d S_dt / d U^n)^T lam^{n+1}.
//
// The forward step reads primitive states at "extended" cells e = (i, j),
// i in [-1, nx], j in [-1, ny] (2-D), whose values come from the mapped cells
// map(e) of the boundary conditions; each extended cell builds its four face
// states from itself and its four neighbours; every face flux uses the high
// state of one extended cell and the low state of the next; the update of an
// interior cell uses its four faces.  The reverse pass follows the same
// structure in four kernels, with fixed slots instead of atomics so the
// result is deterministic:
//   1. faces:  recompute the face states of every extended cell -> FS
//   2. hll:    per face, lam' = K^T lam^{n+1} (kick), flux adjoint
//              dt/dx (lam'_{i+1} - lam'_i), HLL vjp -> adjoints of the two face
//              states, each written to its one slot in FSb
//   3. cells:  per extended cell, the vjp of its face-state computation gives
//              the adjoints of its five input primitive states -> slots
//              C[self, left, right, down, up]
//   4. gather: per interior cell, sum the slots that land on each padded
//              position, fold the padded positions that the boundary mapping
//              sends to this cell, chain through W(U) and add lam' itself.
#include <string>

#include "csh_adjoint.h"
#include "csh_api_util.h"

namespace csh {

struct AdjArgs {
    int nx, ny, bcx, bcy;
    int ex, ey;          // extended grid: ex = nx + 2, ey = ny + 2 (1-D: 1)
    double dx, dy, dt;
    double vc2, rc2, x0, y0;
    const double* U;     // [6][ny][nx]
    const double* lam1;  // lam^{n+1}
    double* lam0;        // lam^n
    double* FS;          // [4 faces][6][ext]
    double* FSb;         // [4][6][ext]
    double* Cs;          // [5 roles][6][ext]
};

enum { XHI = 0, XLO = 1, YHI = 2, YLO = 3 };
enum { SELF = 0, LEFT = 1, RIGHT = 2, DOWN = 3, UP = 4 };

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

// primitive state of the (possibly ghost) cell (i, j)
CSH_HD P prim_at(const AdjArgs& a, int i, int j, bool twod)
{
    const int gi = map_index(i, a.nx, a.bcx);
    const int gj = twod ? map_index(j, a.ny, a.bcy) : 0;
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
    const double f = -a.vc2 / (x * x + y * y + a.rc2);
    return kick_vjp(l, a.dt, f * x, f * y);
}

template <bool TWOD>
CSH_HD void faces_cell(const AdjArgs& a, int i, int j)
{
    const double kx = a.dt / (2.0 * a.dx), ky = TWOD ? a.dt / (2.0 * a.dy) : 0.0;
    const P W0 = prim_at(a, i, j, TWOD);
    const P Wl = prim_at(a, i - 1, j, TWOD), Wr = prim_at(a, i + 1, j, TWOD);
    const P Wm = TWOD ? prim_at(a, i, j - 1, TWOD) : W0, Wp = TWOD ? prim_at(a, i, j + 1, TWOD) : W0;
    const Faces<double> f = face_states<double, TWOD>(W0, Wl, Wr, Wm, Wp, kx, ky);
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
    // x face i + 1/2 in an interior row: between extended cells (i, j) and (i + 1, j)
    if (i <= a.nx - 1 && (!TWOD || (j >= 0 && j < a.ny))) {
        const int jj = TWOD ? j : 0;
        const C lp = (i + 1 <= a.nx - 1) ? lam_prime(a, i + 1, jj, TWOD) : z;
        const C lm = (i >= 0) ? lam_prime(a, i, jj, TWOD) : z;
        const C Fb = csub(lp, lm, a.dt / a.dx);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(load_p(a.FS, ne, XHI, e), load_p(a.FS, ne, XLO, e + 1), Fb, wlb, wrb);
        store_p(a.FSb, ne, XHI, e, wlb);
        store_p(a.FSb, ne, XLO, e + 1, wrb);
    }
    if (TWOD && j <= a.ny - 1 && i >= 0 && i < a.nx) {
        const C lp = (j + 1 <= a.ny - 1) ? lam_prime(a, i, j + 1, true) : z;
        const C lm = (j >= 0) ? lam_prime(a, i, j, true) : z;
        const C Gb = csub(lp, lm, a.dt / a.dy);
        P wlb = zero_p(), wrb = zero_p();
        hll_vjp(swap(load_p(a.FS, ne, YHI, e)), swap(load_p(a.FS, ne, YLO, e + a.ex)), swap(Gb), wlb, wrb);
        store_p(a.FSb, ne, YHI, e, swapb(wlb));
        store_p(a.FSb, ne, YLO, e + a.ex, swapb(wrb));
    }
}

template <bool TWOD>
CSH_HD void cells_cell(const AdjArgs& a, int i, int j)
{
    const double kx = a.dt / (2.0 * a.dx), ky = TWOD ? a.dt / (2.0 * a.dy) : 0.0;
    const size_t ne = (size_t)a.ex * a.ey, e = ext_index(a, i, j);
    const P W0 = prim_at(a, i, j, TWOD);
    const P Wl = prim_at(a, i - 1, j, TWOD), Wr = prim_at(a, i + 1, j, TWOD);
    const P Wm = TWOD ? prim_at(a, i, j - 1, TWOD) : W0, Wp = TWOD ? prim_at(a, i, j + 1, TWOD) : W0;
    Faces<double> fb;
    fb.xhi = load_p(a.FSb, ne, XHI, e);
    fb.xlo = load_p(a.FSb, ne, XLO, e);
    if (TWOD) {
        fb.yhi = load_p(a.FSb, ne, YHI, e);
        fb.ylo = load_p(a.FSb, ne, YLO, e);
    } else {
        fb.yhi = fb.ylo = zero_p();
    }
    P b0 = zero_p(), bl = zero_p(), br = zero_p(), bm = zero_p(), bp = zero_p();
    face_states_vjp<TWOD>(W0, Wl, Wr, Wm, Wp, kx, ky, fb, b0, bl, br, bm, bp);
    store_p(a.Cs, ne, SELF, e, b0);
    store_p(a.Cs, ne, LEFT, e, bl);
    store_p(a.Cs, ne, RIGHT, e, br);
    if (TWOD) {
        store_p(a.Cs, ne, DOWN, e, bm);
        store_p(a.Cs, ne, UP, e, bp);
    }
}

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

// sum of the slots that land on padded position (pi, pj)
template <bool TWOD>
CSH_HD P pad_sum(const AdjArgs& a, int pi, int pj)
{
    const size_t ne = (size_t)a.ex * a.ey;
    auto in_ext = [&](int i, int j) { return i >= -1 && i <= a.nx && (!TWOD || (j >= -1 && j <= a.ny)); };
    P s = zero_p();
    if (in_ext(pi, pj)) acc(s, load_p(a.Cs, ne, SELF, ext_index(a, pi, pj)));
    if (in_ext(pi + 1, pj)) acc(s, load_p(a.Cs, ne, LEFT, ext_index(a, pi + 1, pj)));
    if (in_ext(pi - 1, pj)) acc(s, load_p(a.Cs, ne, RIGHT, ext_index(a, pi - 1, pj)));
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

// ---- kernels ----------------------------------------------------------------------------------------

template <bool TWOD, int STAGE>
__global__ __launch_bounds__(256) void adjoint_kernel(AdjArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (STAGE == 4) {  // interior cells
        if (t >= (int64_t)a.nx * a.ny) return;
        gather_cell<TWOD>(a, (int)(t % a.nx), (int)(t / a.nx));
        return;
    }
    if (t >= (int64_t)a.ex * a.ey) return;  // extended cells
    const int i = (int)(t % a.ex) - 1;
    const int j = TWOD ? (int)(t / a.ex) - 1 : 0;
    if (STAGE == 1) faces_cell<TWOD>(a, i, j);
    if (STAGE == 2) hll_cell<TWOD>(a, i, j);
    if (STAGE == 3) cells_cell<TWOD>(a, i, j);
}

__global__ __launch_bounds__(256) void zero_kernel(double* p, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0.0;
}

// W -> U (primitive to conserved) transposed: lam_W = (dU/dW)^T lam_U
__global__ __launch_bounds__(256) void init_adjoint_kernel(const double* W, const double* lamU, double* lamW, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const P w = {W[c], W[n + c], W[2 * n + c], W[3 * n + c], W[4 * n + c], W[5 * n + c]};
    P wb = zero_p();
    to_cons_vjp(w, load_cons<double>(lamU, (size_t)n, (size_t)c), wb);
    lamW[c] = wb.r;
    lamW[n + c] = wb.u;
    lamW[2 * n + c] = wb.v;
    lamW[3 * n + c] = wb.pxx;
    lamW[4 * n + c] = wb.pxy;
    lamW[5 * n + c] = wb.pyy;
}

}  // namespace csh

size_t csh_adjoint_workspace_doubles(int nx, int ny)
{
    const size_t ne = (size_t)(nx + 2) * (ny > 1 ? ny + 2 : 1);
    return ne * 6 * (4 + 4 + 5);
}

int csh_adjoint_impl(csh_grid_view v, double dt, const void* U, const void* lam_next, void* lam, double* ws,
                     hipStream_t s)
{
    using namespace csh;
    const bool twod = v.ny > 1;
    AdjArgs a{};
    a.nx = v.nx;
    a.ny = v.ny;
    a.bcx = v.bcx;
    a.bcy = v.bcy;
    a.ex = v.nx + 2;
    a.ey = twod ? v.ny + 2 : 1;
    a.dx = v.dx;
    a.dy = v.dy;
    a.dt = dt;
    a.vc2 = v.vc * v.vc;
    a.rc2 = v.rc * v.rc;
    a.x0 = v.x0;
    a.y0 = v.y0;
    a.U = static_cast<const double*>(U);
    a.lam1 = static_cast<const double*>(lam_next);
    a.lam0 = static_cast<double*>(lam);
    const size_t ne = (size_t)a.ex * a.ey;
    a.FS = ws;
    a.FSb = ws + 24 * ne;
    a.Cs = ws + 48 * ne;
    const unsigned be = (unsigned)((ne + 255) / 256), bi = (unsigned)(((size_t)v.nx * v.ny + 255) / 256);
    unsigned bz = (unsigned)((24 * ne + 255) / 256);
    if (bz > 8192) bz = 8192;
    zero_kernel<<<bz, 256, 0, s>>>(a.FSb, (int64_t)(24 * ne));
    if (twod) {
        adjoint_kernel<true, 1><<<be, 256, 0, s>>>(a);
        adjoint_kernel<true, 2><<<be, 256, 0, s>>>(a);
        adjoint_kernel<true, 3><<<be, 256, 0, s>>>(a);
        adjoint_kernel<true, 4><<<bi, 256, 0, s>>>(a);
    } else {
        adjoint_kernel<false, 1><<<be, 256, 0, s>>>(a);
        adjoint_kernel<false, 2><<<be, 256, 0, s>>>(a);
        adjoint_kernel<false, 3><<<be, 256, 0, s>>>(a);
        adjoint_kernel<false, 4><<<bi, 256, 0, s>>>(a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return csh_fail(CSH_ERR_HIP, std::string("adjoint_step: ") + hipGetErrorString(e));
    return CSH_OK;
}

int csh_init_adjoint_impl(int64_t n, const void* W, const void* lamU, void* lamW, hipStream_t s)
{
    csh::init_adjoint_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        static_cast<const double*>(W), static_cast<const double*>(lamU), static_cast<double*>(lamW), n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return csh_fail(CSH_ERR_HIP, std::string("init_state_adjoint: ") + hipGetErrorString(e));
    return CSH_OK;
}
