// Adjoint of one sweep at frozen timestep (FP64): lam^n = (d S_dt / d U^n)^T lam^{n+1}.
//
// 2-D grids: two LDS-tiled kernels (adjoint_tileA_kernel, adjoint_tileB_kernel,
// the phase bodies in csh_adjoint.h): A recomputes the face states of a tile
// and takes the flux adjoints of its faces through HLL into the face-state
// adjoints, B takes those through the face-state reverse pass, sums the shares
// that land on each cell and folds the ghost positions of outflow axes.
//
// 1-D grids: the forward step reads primitive states at "extended" cells
// e = i, i in [-1, nx], whose values come from the mapped cells map(e) of the
// boundary conditions; each extended cell builds its face states from itself
// and its two neighbours; every face flux uses the high state of one extended
// cell and the low state of the next.  The reverse pass follows the same
// structure in four kernels, with fixed slots instead of atomics so the result
// is deterministic:
//   1. faces:  recompute the face states of every extended cell -> FS
//   2. hll:    per face, lam' = K^T lam^{n+1} (kick), flux adjoint
//              dt/dx (lam'_{i+1} - lam'_i), HLL vjp -> adjoints of the two face
//              states, each written to its one slot in FSb
//   3. cells:  per extended cell, the vjp of its face-state computation; a
//              wavefront covers 64 consecutive cells and sums self + the right
//              neighbour's left share + the left neighbour's right share by
//              lane shifts into one value per padded position (XS)
//   4. gather: per interior cell, sum the XS of the padded positions that the
//              boundary mapping sends to this cell, chain through W(U) and add
//              lam' itself.
// (The 2-D grids ran this scheme with a y part as five kernels before the
// tiled pass replaced it; its per-cell bodies remain the reference the tiled
// pass is tested against on the CPU.)
//
// The kernels take their workgroup numbers XCD-aware (xcd_block), so tiles or
// rows that share halo cells sit in the same L2.
#include <string>

#include "csh_adjoint.h"
#include "csh_api_util.h"

namespace csh {

// ---- kernels ----------------------------------------------------------------------------------------

template <bool TWOD, int STAGE>
__global__ __launch_bounds__(256) void adjoint_kernel(AdjArgs a)
{
    // cell counts stay below 2^31 (a plane is smaller than 4 GiB): 32-bit index arithmetic
    const unsigned t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (STAGE == 4) {  // interior cells
        if (t >= (unsigned)a.nx * (unsigned)a.ny) return;
        gather_cell<TWOD>(a, (int)(t % (unsigned)a.nx), (int)(t / (unsigned)a.nx));
        return;
    }
    if (t >= (unsigned)a.ex * (unsigned)a.ey) return;  // extended cells
    const int i = (int)(t % (unsigned)a.ex) - 1;
    const int j = TWOD ? (int)(t / (unsigned)a.ex) - 1 : 0;
    if (STAGE == 1) faces_cell<TWOD>(a, i, j);
    if (STAGE == 2) hll_cell<TWOD>(a, i, j);
    if constexpr (STAGE == 3 && TWOD) cells_cell_y(a, i, j);
}

// Stage 5, the x part, summed per padded position: a wavefront covers the
// extended columns base .. base + 63 of one extended row (base = 62 w - 3) and
// writes the padded positions of its lanes 1..62; lanes outside the extended
// range contribute zero.  The summation order is that of a per-position sum of
// slots: self, then the left share of the cell to the right, then the right
// share of the cell to the left.
constexpr int kXsOwned = 62;

template <bool TWOD>
__global__ __launch_bounds__(256) void adjoint_xsum_kernel(AdjArgs a)
{
    const int lane = threadIdx.x & 63;
    const long w = (long)xcd_block(blockIdx.x, gridDim.x) * 4 + wave_in_block();
    const int wpr = (a.nx + 4 + kXsOwned - 1) / kXsOwned;  // wavefronts per extended row
    if (w >= (long)wpr * a.ey) return;                     // uniform per wavefront
    const int j = TWOD ? (int)(w / wpr) - 1 : 0;
    const int i = (int)(w % wpr) * kXsOwned - 3 + lane;
    P b0 = zero_p(), bl = zero_p(), br = zero_p();
    if (i >= -1 && i <= a.nx) cells_x_vjp<TWOD>(a, i, j, b0, bl, br);
    const P l = lane_shift<+1>(bl), r = lane_shift<-1>(br);  // from the cells at i + 1, i - 1
    const P sum = {b0.r + l.r + r.r,       b0.u + l.u + r.u,       b0.v + l.v + r.v,
                   b0.pxx + l.pxx + r.pxx, b0.pxy + l.pxy + r.pxy, b0.pyy + l.pyy + r.pyy};
    if (lane >= 1 && lane <= kXsOwned && i >= -2 && i <= a.nx + 1)
        store_p(a.XS, (size_t)(a.nx + 4) * a.ey, 0, xs_index(a, i, j), sum);
}

// The tiled reverse pass of 2-D grids.  Kernel A: a workgroup per tile of
// 32 x 8 extended cells (one thread each): the states of the tile and a
// ring into LDS, the face states of each cell (its high ones kept in
// registers, its low ones shared through LDS, plus the low ones of the column
// to the right and the row above), then per cell the flux adjoints of its
// high x and y faces through HLL into the face-state adjoints (FSb, device
// memory).  47 KB of LDS: three workgroups per CU.
__global__ __launch_bounds__(kA_THREADS) void adjoint_tileA_kernel(AdjArgs a, int tiles_x)
{
    __shared__ double L[kA_LDS];
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int X0 = -1 + (int)(b % (unsigned)tiles_x) * kA_TX, Y0 = -1 + (int)(b / (unsigned)tiles_x) * kA_TY;
    const int t = threadIdx.x;
    tileA_states(a, X0, Y0, t, L);
    __syncthreads();
    P xhi, yhi;
    tileA_faces(a, t, L, xhi, yhi);
    __syncthreads();
    tileA_fluxes(a, X0, Y0, t, L, xhi, yhi);
}

// Kernel B: a workgroup per tile of 16 x 16 virtual cells (four rows per
// wavefront), outputs its inner 14 x 14: the states of the tile and a ring
// into LDS, per cell the face-state reverse pass from its FSb (its own share
// in registers, the four to its neighbours in LDS), then per position
// everything that lands on it, then per output the folded sum through W(U)
// plus lam'.  77 KB of LDS, two workgroups per CU.
__global__ __launch_bounds__(kB_THREADS) void adjoint_tileB_kernel(AdjArgs a, int tiles_x)
{
    __shared__ double L[kB_LDS];
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int X0 = (int)(b % (unsigned)tiles_x) * kB_OX, Y0 = (int)(b / (unsigned)tiles_x) * kB_OY;
    const int t = threadIdx.x;
    tileB_states(a, X0, Y0, t, L);
    __syncthreads();
    // (loading the face-state adjoints before the staging above, or between it
    // and the barrier, measured slower)
    const P self = tileB_shares(a, X0, Y0, t, L, tileB_face_adjoints(a, X0, Y0, t));
    __syncthreads();
    tileB_put_total(t, tileB_total(t, self, L), L);  // the totals go to a slot no thread reads here
    __syncthreads();
    tileB_gather(a, X0, Y0, t, L);
}

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
    const size_t ey = ny > 1 ? ny + 2 : 1, ne = (size_t)(nx + 2) * ey;
    if (ny > 1) return ne * 6 * 4;  // the tiled pass: the face-state adjoints only
    return ne * 6 * (4 + 4 + 3) + (size_t)(nx + 4) * ey * 6;
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
    set_step_factors(a);
    a.vc2 = v.vc * v.vc;
    a.rc2 = v.rc * v.rc;
    a.x0 = v.x0;
    a.y0 = v.y0;
    a.U = static_cast<const double*>(U);
    a.lam1 = static_cast<const double*>(lam_next);
    a.lam0 = static_cast<double*>(lam);
    const size_t ne = (size_t)a.ex * a.ey;
    if (twod) {
        a.FSb = ws;
        const int tax = (a.ex + kA_TX - 1) / kA_TX, tay = (a.ey + kA_TY - 1) / kA_TY;
        const int tbx = (a.nx + kB_OX - 1) / kB_OX, tby = (a.ny + kB_OY - 1) / kB_OY;
        adjoint_tileA_kernel<<<(unsigned)(tax * tay), kA_THREADS, 0, s>>>(a, tax);
        adjoint_tileB_kernel<<<(unsigned)(tbx * tby), kB_THREADS, 0, s>>>(a, tbx);
    } else {
        a.FS = ws;
        a.FSb = ws + 24 * ne;
        a.Cs = ws + 48 * ne;
        a.XS = ws + 66 * ne;
        const unsigned be = (unsigned)((ne + 255) / 256), bi = (unsigned)(((size_t)v.nx * v.ny + 255) / 256);
        const long xs_waves = (long)((a.nx + 4 + kXsOwned - 1) / kXsOwned) * a.ey;
        const unsigned bx = (unsigned)((xs_waves + 3) / 4);
        adjoint_kernel<false, 1><<<be, 256, 0, s>>>(a);
        adjoint_kernel<false, 2><<<be, 256, 0, s>>>(a);
        adjoint_xsum_kernel<false><<<bx, 256, 0, s>>>(a);
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
