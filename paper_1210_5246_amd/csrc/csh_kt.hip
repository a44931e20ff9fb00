// Kurganov-Tadmor central scheme (Sec. 3.2, eqs. (5)-(8)) on gfx950.
//
// One step = two stages of the Runge-Kutta midpoint rule,
//   U* = U^n + dt/2 L(U^n),   U^{n+1} = U^n + dt L(U*)   (+ the external kick),
// L = -(dH_x/dx + dH_y/dy) with the local-speed flux of eq. (6) at faces
// reconstructed by component-wise MC-limited linear primitive profiles.  On a
// 2-D grid both stages run in one launch with the work decomposition of the
// characteristic sweep (a wavefront per column strip marching up a row
// segment, x neighbours by DPP lane shifts, y neighbours from row register
// sets), U* living in registers only; a 1-D grid takes one launch per stage.
// The kernels carry half slopes (face states w -+ h) and twice the flux (the
// update coefficients take the 1/2).
#include <cstdlib>

#include "csh_device.h"
#include "csh_internal.h"

namespace csh {

template <typename T>
__device__ __forceinline__ double kt_dt(const StepArgs<T>& p, double* t_now)
{
    const Slot& sl = p.slots[p.s_in];
    *t_now = sl.t;
    if (p.dt_in) return *p.dt_in;
    if (!p.dev_dt) return p.dt;
    double dt = p.cfl / __longlong_as_double((long long)sl.s_bits);
    if (p.t_end > 0.0) {
        if (sl.t >= p.t_end) dt = 0.0;
        else if (sl.t + dt > p.t_end) dt = p.t_end - sl.t;
    }
    return dt;
}

template <typename T>
__device__ __forceinline__ Prim<T> plus(const Prim<T>& w, const Prim<T>& d)
{
    return {w.r + d.r, w.u + d.u, w.v + d.v, w.pxx + d.pxx, w.pxy + d.pxy, w.pyy + d.pyy};
}

// 1-D grids: one launch per stage, a wavefront per 60 cells (2 halo lanes per
// side); the first stage records the step's timestep in its input slot for
// the second
template <typename T, bool FINAL>
__global__ __launch_bounds__(64 * kWaves) void kt_kernel(StepArgs<T> p)
{
    double t_now;
    const double dt = kt_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!FINAL) {
            p.slots[p.s_in].dt = dt;
        } else {
            p.slots[p.s_out].t = t_now + dt;
            p.slots[p.s_reset].s_bits = 0ull;
            if (p.dt_log) *p.dt_log = dt;
        }
    }
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * kWaves + wave_in_block();
    if (wid >= p.nstrips) return;  // uniform per wavefront
    const int c = wid * kStrip - 2 + lane;
    const int gc = map_index(c, p.nx, p.bcx);
    const bool own = lane >= 2 && lane < 2 + kStrip && c < p.nx;
    const double h = FINAL ? dt : 0.5 * dt;  // stage length
    const T cx = T(0.5 * h / p.dx);  // the flux below is 2H
    const Planes<T> in(p.U, (size_t)p.nx);
    const OutPlanes<T> out(p.Unew, (size_t)p.nx);
    const Cons<T> C0 = in.load((unsigned)gc);
    const Prim<T> W0 = to_prim(C0);
    const Prim<T> s = mc_half_slope(lane_shift<-1>(W0), W0, lane_shift<+1>(W0));
    const Cons<T> F = kt_flux2_x(plus(W0, s), lane_shift<+1>(sub(W0, s)));
    const Cons<T> Fm = lane_shift<-1>(F);
    Cons<T> Un = update(FINAL ? Planes<T>(p.Ubase, (size_t)p.nx).load((unsigned)gc) : C0, cx, F, Fm);
    double smax = 0.0;
    bool bad = false;
    if (FINAL) kick(Un, p, dt, c, 0, false);
    if (own) {
        out.store((unsigned)c, Un);
        if (FINAL) {
            const Prim<T> wn = to_prim(Un);
            smax = fmax(smax, signal_rate<T, false>(wn, 1.0 / p.dx, 0.0));
            bad |= !physical(wn);
        }
    }
    if (FINAL) {
        smax = wave_max(smax);
        if (lane == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
        if (__any(bad) && lane == 0) atomicOr(p.flag, 1);
    }
}

// ---- both stages in one launch (2-D) ---------------------------------------------------------
//
// The first stage's result U* is never stored: each wavefront forms the U*
// rows its second stage needs and keeps them, in primitive form, in a ring of
// three row register sets.  Stage 1 marches rows y0-3 .. y1+2 (U* rows y0-2 ..
// y1+1, the second stage's stencil) and stage 2 follows two rows behind it, so
// a step reads U^n once (a wavefront keeps its last four input rows in LDS for
// the base of stage 2) and writes U^{n+1} once: 96 B per cell-update instead of
// the 240 B of two launches.  A wavefront owns 56 columns: stage 1 is valid on
// lanes 2..61, stage 2 on lanes 4..59.
//
// Boundaries.  The boundary conditions apply to U* as to any state: at a
// ghost position stage 2 sees U* of the mapped cell.  With periodic
// boundaries the lanes and rows of a wavefront hold a contiguous window of
// the torus, so its own U* at a ghost position is already that value; with
// outflow boundaries the ghost columns take U* of the edge column by a lane
// read, and the ghost rows a copy of the edge row.

constexpr int kFusedStrip = 56;  // owned columns per wavefront of the fused step

// Rows per segment of the fused step: the critical-path rule of the sweep,
// with the fused wavefront's halo (stage 1 re-traces 6 rows, stage 2 2, an
// average of 4 per row of the segment) and its 56-column strips.
int kt_fused_rows(int nx, int ny)
{
    if (const char* e = std::getenv("CSH_KT_ROWS")) {
        const int v = std::atoi(e);
        if (v >= 1) return v;
    }
    const long strips = (nx + kFusedStrip - 1) / kFusedStrip;
    auto waves = [&](int t) { return strips * ((ny + t - 1) / t); };
    const int lo = waves(8) >= 256 ? 8 : 4;
    int best = lo;
    long best_cost = -1;
    for (int t = lo; t <= 96; ++t) {
        const long cost = ((waves(t) + 1023) / 1024) * (t + 4);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}

template <typename T>
__global__ __launch_bounds__(64 * kWaves) void kt_fused_kernel(StepArgs<T> p)
{
    double t_now;
    const double dt = kt_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.slots[p.s_out].t = t_now + dt;
        p.slots[p.s_reset].s_bits = 0ull;
        if (p.dt_log) *p.dt_log = dt;
    }
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * kWaves + wave_in_block();
    if (wid >= p.nstrips * p.nsegs) return;  // uniform per wavefront
    const int sx = wid % p.nstrips, sy = wid / p.nstrips;
    const int c0 = sx * kFusedStrip - 4;  // column of lane 0
    const int c = c0 + lane;
    const int gc = map_index(c, p.nx, p.bcx);
    const bool own = lane >= 4 && lane < 4 + kFusedStrip && c < p.nx;
    // outflow in x: ghost lanes read U* from the lane of the edge column
    const bool xfix = p.bcx != 0 && (c0 < 0 || c0 + 63 >= p.nx);
    const int src = c < 0 ? -c0 : (c >= p.nx ? p.nx - 1 - c0 : lane);
    const size_t plane = (size_t)p.nx * p.ny;
    const double h1 = 0.5 * dt;  // stage lengths; the fluxes below are 2H
    const T cx1 = T(0.5 * h1 / p.dx), cy1 = T(0.5 * h1 / p.dy);
    const T cx2 = T(0.5 * dt / p.dx), cy2 = T(0.5 * dt / p.dy);
    const double idx = 1.0 / p.dx, idy = 1.0 / p.dy;
    const Planes<T> in(p.U, plane);
    const OutPlanes<T> out(p.Unew, plane);
    double smax = 0.0;
    bool bad = false;
    const int y0 = sy * p.ty, y1 = min(y0 + p.ty, p.ny);
    const int a1 = y0 - 2, b1 = y1 + 2;  // U* rows formed here: [a1, b1)
    auto load_row = [&](int r) -> Cons<T> { return in.load((unsigned)(map_index(r, p.ny, p.bcy) * p.nx + gc)); };
    auto fix_x = [&](const Prim<T>& w) -> Prim<T> {
        if (!xfix) return w;
        return {__shfl(w.r, src, 64), __shfl(w.u, src, 64), __shfl(w.v, src, 64), __shfl(w.pxx, src, 64),
                __shfl(w.pxy, src, 64), __shfl(w.pyy, src, 64)};
    };

    // the U^n rows of the last four iterations in LDS, for the base of stage 2
    // (each lane reads and writes only its own column: no barrier)
    __shared__ T ring_lds[kWaves][4][6][64];
    T(*const ring)[6][64] = ring_lds[wave_in_block()];
    auto ring_put = [&](int r, const Cons<T>& U) {
        T(*const q)[64] = ring[(r - y0) & 3];
        q[0][lane] = U.r;
        q[1][lane] = U.mx;
        q[2][lane] = U.my;
        q[3][lane] = U.exx;
        q[4][lane] = U.exy;
        q[5][lane] = U.eyy;
    };
    auto ring_get = [&](int r) -> Cons<T> {
        const T(*const q)[64] = ring[(r - y0) & 3];
        return {q[0][lane], q[1][lane], q[2][lane], q[3][lane], q[4][lane], q[5][lane]};
    };

    Cons<T> Ca = load_row(y0 - 4), Cb = load_row(y0 - 3), Cc = load_row(y0 - 2);
    Prim<T> Wa = to_prim(Ca), Wb = to_prim(Cb), Wc = to_prim(Cc);
    ring_put(y0 - 4, Ca);
    ring_put(y0 - 3, Cb);
    ring_put(y0 - 2, Cc);
    Prim<T> Sa{}, Sb{}, Sc{};  // U* rows (primitive)
    Prim<T> yhi1{}, yhi2{};
    Cons<T> acc1{}, acc2{};

    // stage 1 at row r: Wm, W0, Wp rows r-1, r, r+1 of U^n (Wm refilled with
    // row r+2), C0 row r conserved (Cm refilled); finishes U* row r-1 into Sn
    // (Sm3, Sm2: the ring's rows r-3, r-2)
    auto stage1 = [&](int r, Prim<T>& Wm, const Prim<T>& W0, const Prim<T>& Wp, Cons<T>& Cm, const Cons<T>& C0,
                      Prim<T>& Sn, Prim<T>& Sm3, Prim<T>& Sm2) {
        const Cons<T> Unext = load_row(r + 2);
        const Prim<T> sxv = mc_half_slope(lane_shift<-1>(W0), W0, lane_shift<+1>(W0));
        const Prim<T> syv = mc_half_slope(Wm, W0, Wp);
        if (r >= a1) {
            const Cons<T> G = swap(kt_flux2_x(swap(yhi1), swap(sub(W0, syv))));  // face r - 1/2
            if (r > a1) {
                if (p.bcy != 0 && r - 1 >= p.ny) {
                    Sn = Sm2;  // outflow: the ghost rows above copy row ny - 1
                } else {
                    Sn = fix_x(to_prim(Cons<T>{acc1.r - cy1 * G.r, acc1.mx - cy1 * G.mx, acc1.my - cy1 * G.my,
                                               acc1.exx - cy1 * G.exx, acc1.exy - cy1 * G.exy,
                                               acc1.eyy - cy1 * G.eyy}));
                    if (p.bcy != 0 && r - 1 == 0) Sm2 = Sm3 = Sn;  // outflow: the ghost rows below copy row 0
                }
            }
            if (r < b1) {
                const Cons<T> F = kt_flux2_x(plus(W0, sxv), lane_shift<+1>(sub(W0, sxv)));
                const Cons<T> Fm = lane_shift<-1>(F);
                acc1 = {C0.r - cx1 * (F.r - Fm.r) + cy1 * G.r,         C0.mx - cx1 * (F.mx - Fm.mx) + cy1 * G.mx,
                        C0.my - cx1 * (F.my - Fm.my) + cy1 * G.my,     C0.exx - cx1 * (F.exx - Fm.exx) + cy1 * G.exx,
                        C0.exy - cx1 * (F.exy - Fm.exy) + cy1 * G.exy, C0.eyy - cx1 * (F.eyy - Fm.eyy) + cy1 * G.eyy};
            }
        }
        yhi1 = plus(W0, syv);
        Wm = to_prim(Unext);
        Cm = Unext;
        ring_put(r + 2, Unext);  // into the slot of row r - 2, read before this
    };

    // stage 2 at row q on U* rows q-1, q, q+1; B = row q of U^n
    auto stage2 = [&](int q, const Prim<T>& Wm, const Prim<T>& W0, const Prim<T>& Wp, const Cons<T>& B) {
        const Prim<T> sxv = mc_half_slope(lane_shift<-1>(W0), W0, lane_shift<+1>(W0));
        const Prim<T> syv = mc_half_slope(Wm, W0, Wp);
        if (q >= y0) {
            const Cons<T> G = swap(kt_flux2_x(swap(yhi2), swap(sub(W0, syv))));  // face q - 1/2
            if (q > y0) {
                Cons<T> Un = {acc2.r - cy2 * G.r,     acc2.mx - cy2 * G.mx,   acc2.my - cy2 * G.my,
                              acc2.exx - cy2 * G.exx, acc2.exy - cy2 * G.exy, acc2.eyy - cy2 * G.eyy};
                kick(Un, p, dt, c, q - 1, true);
                if (own) {
                    out.store((unsigned)((q - 1) * p.nx + c), Un);
                    smax = fmax(smax, checked_rate(Un, idx, idy, bad));
                }
            }
            if (q < y1) {
                const Cons<T> F = kt_flux2_x(plus(W0, sxv), lane_shift<+1>(sub(W0, sxv)));
                const Cons<T> Fm = lane_shift<-1>(F);
                acc2 = {B.r - cx2 * (F.r - Fm.r) + cy2 * G.r,         B.mx - cx2 * (F.mx - Fm.mx) + cy2 * G.mx,
                        B.my - cx2 * (F.my - Fm.my) + cy2 * G.my,     B.exx - cx2 * (F.exx - Fm.exx) + cy2 * G.exx,
                        B.exy - cx2 * (F.exy - Fm.exy) + cy2 * G.exy, B.eyy - cx2 * (F.eyy - Fm.eyy) + cy2 * G.eyy};
            }
        }
        yhi2 = plus(W0, syv);
    };

    // one row of the march: stage 1 at r, then stage 2 at q = r - 2 (from the
    // first row whose stencil stage 1 has finished); S0, Sr3, Sr2: the ring
    // slots of U* rows r-1, r-3, r-2
    auto iter = [&](int r, Prim<T>& Wm, const Prim<T>& W0, const Prim<T>& Wp, Cons<T>& Cm, const Cons<T>& C0,
                    Prim<T>& S0, Prim<T>& Sr3, Prim<T>& Sr2) {
        const int q = r - 2;
        const Cons<T> B = ring_get(q);  // row q's U^n (used for q in [y0, y1) only)
        stage1(r, Wm, W0, Wp, Cm, C0, S0, Sr3, Sr2);
        if (q >= y0 - 1) stage2(q, Sr3, Sr2, S0, B);
    };

    for (int r = a1 - 1; r <= b1; r += 3) {
        iter(r, Wa, Wb, Wc, Ca, Cb, Sa, Sb, Sc);
        if (r + 1 > b1) break;
        iter(r + 1, Wb, Wc, Wa, Cb, Cc, Sb, Sc, Sa);
        if (r + 2 > b1) break;
        iter(r + 2, Wc, Wa, Wb, Cc, Ca, Sc, Sa, Sb);
    }

    smax = wave_max(smax);
    if (lane == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
    if (__any(bad) && lane == 0) atomicOr(p.flag, 1);
}

template <typename T>
hipError_t launch_kt_fused(StepArgs<T> a, hipStream_t s)
{
    a.nstrips = (a.nx + kFusedStrip - 1) / kFusedStrip;
    a.ty = kt_fused_rows(a.nx, a.ny);
    a.nsegs = (a.ny + a.ty - 1) / a.ty;
    const int nwaves = a.nstrips * a.nsegs;
    kt_fused_kernel<T><<<dim3((nwaves + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, s>>>(a);
    return hipGetLastError();
}

template hipError_t launch_kt_fused<double>(StepArgs<double>, hipStream_t);
template hipError_t launch_kt_fused<float>(StepArgs<float>, hipStream_t);

template <typename T>
hipError_t launch_kt(const StepArgs<T>& a, bool final_stage, hipStream_t s)
{
    const dim3 grid((a.nstrips + kWaves - 1) / kWaves), block(64 * kWaves);
    if (final_stage) kt_kernel<T, true><<<grid, block, 0, s>>>(a);
    else kt_kernel<T, false><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

template hipError_t launch_kt<double>(const StepArgs<double>&, bool, hipStream_t);
template hipError_t launch_kt<float>(const StepArgs<float>&, bool, hipStream_t);

}  // namespace csh
