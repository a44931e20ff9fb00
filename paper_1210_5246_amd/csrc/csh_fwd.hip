// Forward sweep kernels of the collisionless-stellar-hydrodynamics scheme
// (Mitchell, Vorobyov & Hensler, arXiv:1210.5246, Sec. 3.3), gfx950.
//
// One sweep = MUSCL-Hancock with characteristic tracing (eqs. (19)-(32)), an
// HLL flux at every face, the dimensionally unsplit conservative update, the
// operator-split external-gravity kick (Sec. 3.3, last paragraph) and the
// fused reduction of the CFL rate of the new state.
//
// Work decomposition (2-D): one wavefront owns a strip of 60 output columns
// and marches up a segment of rows.  Lane l holds column x0 - 2 + l, so the
// two lanes at each edge are the stencil halo.  x neighbours come from lane
// shuffles; the rows r-1, r, r+1 the y slopes need, the flux of the previous
// row and the high y-face state of the cell below stay in registers.  No LDS
// and no second pass: each input cell is read from HBM once per strip it
// belongs to (64/60 columns) and each output cell is written once.
#include "csh_device.h"
#include "csh_internal.h"

namespace csh {

template <typename T>
__device__ __forceinline__ double step_dt(const StepArgs<T>& p, double* t_now)
{
    const Slot& sl = p.slots[p.s_in];
    const double t = sl.t;
    *t_now = t;
    if (!p.dev_dt) return p.dt_in ? *p.dt_in : p.dt;
    const double s = __longlong_as_double((long long)sl.s_bits);
    double dt = p.cfl / s;
    if (p.t_end > 0.0) {
        if (t >= p.t_end) dt = 0.0;
        else if (t + dt > p.t_end) dt = p.t_end - t;
    }
    return dt;
}

template <typename T>
__device__ __forceinline__ void store_face(T* __restrict__ F, size_t plane, size_t idx, const Cons<T>& f)
{
    store_cons(F, plane, idx, f);
}

template <typename T, bool TWOD, bool FLUXES, int RS>
__global__ __launch_bounds__(64 * kWaves) void sweep_kernel(StepArgs<T> p)
{
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (!FLUXES && blockIdx.x == 0 && threadIdx.x == 0) {
        p.slots[p.s_out].t = t_now + dt;
        p.slots[p.s_reset].s_bits = 0ull;
        if (p.dt_log) *p.dt_log = dt;
    }

    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * kWaves + wave_in_block();
    if (wid >= p.nstrips * p.nsegs) return;  // uniform per wavefront
    const int sx = wid % p.nstrips, sy = wid / p.nstrips;
    const int c = sx * kStrip - 2 + lane;  // column of this lane
    const int gc = map_index(c, p.nx, p.bcx);
    const bool own = lane >= 2 && lane < 2 + kStrip && c < p.nx;  // lane owns an output column
    const size_t plane = (size_t)p.nx * p.ny;

    const T kx = T(dt / (2.0 * p.dx)), cx = T(dt / p.dx);
    const double idx = 1.0 / p.dx, idy = TWOD ? 1.0 / p.dy : 0.0;
    double smax = 0.0;
    bool bad = false;

    if constexpr (!TWOD) {
        const Cons<T> U0 = load_cons(p.U, plane, (size_t)gc);
        const Cons<T> F = flux_1d<T, RS>(U0, kx);  // face c + 1/2
        if constexpr (FLUXES) {
            // lanes 1..61 hold faces x0 - 1/2 .. x0 + 59 + 1/2
            if (lane >= 1 && lane <= 1 + kStrip && c >= -1 && c <= p.nx - 1)
                store_face(p.Fx, (size_t)(p.nx + 1), (size_t)(c + 1), F);
            return;
        }
        const Cons<T> Fm = lane_shift<-1>(F);
        Cons<T> Un = update(U0, cx, F, Fm);
        kick(Un, p, dt, c, 0, false);
        if (own) {
            store_cons(p.Unew, plane, (size_t)c, Un);
            const Prim<T> wn = to_prim(Un);
            smax = signal_rate<T, false>(wn, idx, idy);
            bad = !physical(wn);
        }
    } else {
        const T ky = T(dt / (2.0 * p.dy)), cy = T(dt / p.dy);
        const int y0 = sy * p.ty, y1 = min(y0 + p.ty, p.ny);
        const Planes<T> in(p.U, plane);
        const OutPlanes<T> out(p.Unew, plane);
        auto load_row = [&](int r) -> Cons<T> {
            const int gr = map_near(r, p.ny, p.bcy);  // rows y0 - 2 .. y1 + 1, ny >= 2
            return in.load((unsigned)(gr * p.nx + gc));
        };
        // Row window in three rotating register sets: the set holding row r-1
        // is refilled with row r+2, so the window advances without moves.
        Cons<T> Ua = load_row(y0 - 2), Ub = load_row(y0 - 1), Uc = load_row(y0);
        T ia = rcp(Ua.r), ib = rcp(Ub.r), ic = rcp(Uc.r);
        Prim<T> Wa = to_prim(Ua, ia), Wb = to_prim(Ub, ib), Wc = to_prim(Uc, ic);
        Prim<T> yhi_prev{};  // high y-face state of the cell below (primitive, axes not exchanged)
        Cons<T> acc{};       // update of the cell below, all but its high y-face flux
        Prim<T> dly = sub(Wb, Wa);  // y difference below the row: the previous row's upper one

        // one row: (Um, Wm) row r-1 (refilled with row r+2), (U0, W0, ir0) row r, Wp row r+1
        auto row = [&](int r, Cons<T>& Um, Prim<T>& Wm, T& irm, const Cons<T>& U0, const Prim<T>& W0, T ir0,
                       const Prim<T>& Wp) {
            const Cons<T> Unext = load_row(min(r + 2, y1 + 1));  // past the window's end: a row already read

            // face states of (c, r): the x differences from the right neighbour (a lane
            // shift), the left one that of the lane to the left; the y difference below
            // the row carried from the row before
            const Prim<T> drx = sub(lane_shift<+1>(W0), W0), dry = sub(Wp, W0);
            const Faces<T> fs = face_states_d<T, true>(W0, ir0, lane_shift<-1>(drx), drx, dly, dry, kx, ky);
            dly = dry;

            if (r >= y0) {
                // y face r - 1/2 between the cell below (its high state) and this cell (low state)
                const Cons<T> G = swap(riemann_x<RS>(make_face_x(swap(yhi_prev)), make_face_x(swap(fs.ylo))));
                if constexpr (FLUXES) {
                    if (own) store_face(p.Fy, (size_t)p.nx * (p.ny + 1), (size_t)r * p.nx + c, G);
                } else if (r > y0) {  // finish cell (c, r - 1)
                    Cons<T> Un = {acc.r - cy * G.r,     acc.mx - cy * G.mx,   acc.my - cy * G.my,
                                  acc.exx - cy * G.exx, acc.exy - cy * G.exy, acc.eyy - cy * G.eyy};
                    kick(Un, p, dt, c, r - 1, true);
                    if (own) {
                        out.store((unsigned)((r - 1) * p.nx + c), Un);
                        smax = fmax(smax, checked_rate(Un, idx, idy, bad));
                    }
                }
                if (r < y1) {
                    // x faces of row r, then start the update of (c, r) with its low y face
                    const Cons<T> F = riemann_x<RS>(make_face_x(fs.xhi), make_face_x(lane_shift<+1>(fs.xlo)));
                    if constexpr (FLUXES) {
                        if (lane >= 1 && lane <= 1 + kStrip && c >= -1 && c <= p.nx - 1)
                            store_face(p.Fx, (size_t)(p.nx + 1) * p.ny, (size_t)r * (p.nx + 1) + (c + 1), F);
                    } else {
                        const Cons<T> Fm = lane_shift<-1>(F);
                        acc = {U0.r - cx * (F.r - Fm.r) + cy * G.r,
                               U0.mx - cx * (F.mx - Fm.mx) + cy * G.mx,
                               U0.my - cx * (F.my - Fm.my) + cy * G.my,
                               U0.exx - cx * (F.exx - Fm.exx) + cy * G.exx,
                               U0.exy - cx * (F.exy - Fm.exy) + cy * G.exy,
                               U0.eyy - cx * (F.eyy - Fm.eyy) + cy * G.eyy};
                    }
                }
            }
            yhi_prev = fs.yhi;
            Um = Unext;  // row r + 2 takes the place of row r - 1
            irm = rcp(Unext.r);
            Wm = to_prim(Unext, irm);
        };

        for (int r = y0 - 1; r <= y1; r += 3) {
            row(r, Ua, Wa, ia, Ub, Wb, ib, Wc);
            if (r + 1 > y1) break;
            row(r + 1, Ub, Wb, ib, Uc, Wc, ic, Wa);
            if (r + 2 > y1) break;
            row(r + 2, Uc, Wc, ic, Ua, Wa, ia, Wb);
        }
        if constexpr (FLUXES) return;
    }

    smax = wave_max(smax);
    if (lane == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
    if (__any(bad) && lane == 0) atomicOr(p.flag, 1);
}

template <typename T, int RS>
void launch_sweep(const StepArgs<T>& a, bool twod, bool fluxes, dim3 grid, dim3 block, hipStream_t s)
{
    if (twod) {
        if (fluxes) sweep_kernel<T, true, true, RS><<<grid, block, 0, s>>>(a);
        else sweep_kernel<T, true, false, RS><<<grid, block, 0, s>>>(a);
    } else {
        if (fluxes) sweep_kernel<T, false, true, RS><<<grid, block, 0, s>>>(a);
        else sweep_kernel<T, false, false, RS><<<grid, block, 0, s>>>(a);
    }
}

template <typename T>
hipError_t launch_step(const StepArgs<T>& a, bool twod, bool fluxes, int solver, hipStream_t s)
{
    const int nwaves = a.nstrips * a.nsegs;
    const dim3 grid((nwaves + kWaves - 1) / kWaves), block(64 * kWaves);
    if (solver == 1) launch_sweep<T, 1>(a, twod, fluxes, grid, block, s);
    else launch_sweep<T, 0>(a, twod, fluxes, grid, block, s);
    return hipGetLastError();
}

// ---- primitive -> conserved, with validation ------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void init_kernel(const T* __restrict__ W, T* __restrict__ U, int64_t n,
                                                   int* flag)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (c < n) {
        const Prim<T> w = {W[c], W[n + c], W[2 * n + c], W[3 * n + c], W[4 * n + c], W[5 * n + c]};
        bad = !physical(w);
        store_cons(U, (size_t)n, (size_t)c, to_cons(w));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_init(const T* W, T* U, int64_t n, int* flag, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    init_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(W, U, n, flag);
    return hipGetLastError();
}

// ---- standalone CFL-rate reduction ----------------------------------------------------------------

// Two cells per thread and iteration (their loads issued together), a
// workgroup maximum in LDS and one 64-bit atomic per workgroup (a wavefront's
// atomic on the one slot serialises with every other's).
template <typename T>
__global__ __launch_bounds__(256) void maxspeed_kernel(const T* __restrict__ U, int64_t n, int twod,
                                                       double idx, double idy, Slot* slot, int* flag)
{
    double s = 0.0;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += 2 * stride) {
        const int64_t c2 = c + stride;
        const Cons<T> ua = load_cons(U, (size_t)n, (size_t)c);
        const Cons<T> ub = load_cons(U, (size_t)n, (size_t)(c2 < n ? c2 : c));
        const Prim<T> wa = to_prim(ua), wb = to_prim(ub);
        s = fmax(s, twod ? signal_rate<T, true>(wa, idx, idy) : signal_rate<T, false>(wa, idx, idy));
        s = fmax(s, twod ? signal_rate<T, true>(wb, idx, idy) : signal_rate<T, false>(wb, idx, idy));
        bad = bad || !physical(wa) || !physical(wb);
    }
    s = wave_max(s);
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = s;
    if (__any(bad) && lane == 0) atomicOr(flag, 1);
    __syncthreads();
    if (threadIdx.x == 0) atomic_max_pos(&slot->s_bits, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

template <typename T>
hipError_t launch_maxspeed(const T* U, int nx, int ny, double dx, double dy, Slot* slot, int* flag,
                           hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny;
    int64_t blocks = (n + 511) / 512;
    if (blocks > 4096) blocks = 4096;
    maxspeed_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(U, n, ny > 1, 1.0 / dx,
                                                                    ny > 1 ? 1.0 / dy : 0.0, slot, flag);
    return hipGetLastError();
}

__global__ void reset_kernel(Slot* slots, int nslots, double t0)
{
    const int i = threadIdx.x;
    if (i < nslots) {
        slots[i].s_bits = 0ull;
        slots[i].t = t0;
    }
}

hipError_t launch_reset(Slot* slots, int nslots, double t0, hipStream_t s)
{
    reset_kernel<<<1, 64, 0, s>>>(slots, nslots, t0);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void copy_kernel(const T* __restrict__ a, T* __restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    copy_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(src, dst, n);
    return hipGetLastError();
}

#define CSH_INSTANTIATE(T)                                                                         \
    template hipError_t launch_step<T>(const StepArgs<T>&, bool, bool, int, hipStream_t);               \
    template hipError_t launch_init<T>(const T*, T*, int64_t, int*, hipStream_t);                  \
    template hipError_t launch_maxspeed<T>(const T*, int, int, double, double, Slot*, int*,        \
                                           hipStream_t);                                           \
    template hipError_t launch_copy<T>(const T*, T*, int64_t, hipStream_t);

CSH_INSTANTIATE(double)
CSH_INSTANTIATE(float)

}  // namespace csh
