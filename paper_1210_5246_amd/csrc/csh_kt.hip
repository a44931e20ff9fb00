// Kurganov-Tadmor central scheme (Sec. 3.2, eqs. (5)-(8)) on gfx950.
//
// One step = two stages of the Runge-Kutta midpoint rule,
//   U* = U^n + dt/2 L(U^n),   U^{n+1} = U^n + dt L(U*)   (+ the external kick),
// L = -(dH_x/dx + dH_y/dy) with the local-speed flux of eq. (6) at faces
// reconstructed by component-wise MC-limited linear primitive profiles.  Each
// stage is one launch with the work decomposition of the characteristic sweep
// (a wavefront per 60-column strip, marching up a row segment, neighbours by
// DPP lane shifts); the first stage records the step's timestep in its input
// slot for the second.  The kernels carry half slopes (face states w -+ h)
// and twice the flux (the update coefficients take the 1/2).
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

template <typename T, bool TWOD, bool FINAL>
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
    if (wid >= p.nstrips * p.nsegs) return;  // uniform per wavefront
    const int sx = wid % p.nstrips, sy = wid / p.nstrips;
    const int c = sx * kStrip - 2 + lane;
    const int gc = map_index(c, p.nx, p.bcx);
    const bool own = lane >= 2 && lane < 2 + kStrip && c < p.nx;
    const size_t plane = (size_t)p.nx * p.ny;
    const double h = FINAL ? dt : 0.5 * dt;  // stage length
    const T cx = T(0.5 * h / p.dx);  // the fluxes below are 2H
    const double idx = 1.0 / p.dx, idy = TWOD ? 1.0 / p.dy : 0.0;
    const Planes<T> in(p.U, plane);
    const Planes<T> base(p.Ubase ? p.Ubase : p.U, plane);
    const OutPlanes<T> out(p.Unew, plane);
    double smax = 0.0;
    bool bad = false;

    auto finish = [&](Cons<T> Un, int i, int j) {
        if (FINAL) kick(Un, p, dt, i, j, TWOD);
        if (own) {
            out.store((unsigned)(j * p.nx + i), Un);
            if constexpr (FINAL && TWOD) {
                smax = fmax(smax, checked_rate(Un, idx, idy, bad));
            } else if constexpr (FINAL) {
                const Prim<T> wn = to_prim(Un);
                smax = fmax(smax, signal_rate<T, TWOD>(wn, idx, idy));
                bad |= !physical(wn);
            }
        }
    };

    if constexpr (!TWOD) {
        const Cons<T> C0 = in.load((unsigned)gc);
        const Prim<T> W0 = to_prim(C0);
        const Prim<T> s = mc_half_slope(lane_shift<-1>(W0), W0, lane_shift<+1>(W0));
        const Cons<T> F = kt_flux2_x(plus(W0, s), lane_shift<+1>(sub(W0, s)));
        const Cons<T> Fm = lane_shift<-1>(F);
        finish(update(FINAL ? base.load((unsigned)gc) : C0, cx, F, Fm), c, 0);
    } else {
        const T cy = T(0.5 * h / p.dy);
        const int y0 = sy * p.ty, y1 = min(y0 + p.ty, p.ny);
        auto load_row = [&](const Planes<T>& P, int r) -> Cons<T> {
            return P.load((unsigned)(map_near(r, p.ny, p.bcy) * p.nx + gc));  // ny >= 2
        };
        // the first stage starts its update from its own input: the conserved
        // rows stay in registers beside their primitive form (no second read)
        constexpr bool kOwnBase = !FINAL;
        Cons<T> Ca = load_row(in, y0 - 2), Cb = load_row(in, y0 - 1), Cc = load_row(in, y0);
        Prim<T> Wa = to_prim(Ca), Wb = to_prim(Cb), Wc = to_prim(Cc);
        Prim<T> yhi_prev{};
        Cons<T> acc{};

        // one row: Wm row r-1 (refilled with row r+2), W0 row r, Wp row r+1;
        // Cm, C0 the conserved forms of rows r-1 and r
        auto row = [&](int r, Prim<T>& Wm, const Prim<T>& W0, const Prim<T>& Wp, Cons<T>& Cm, const Cons<T>& C0) {
            const Cons<T> Unext = load_row(in, min(r + 2, y1 + 1));  // past the end: a row already read
            const Prim<T> sxv = mc_half_slope(lane_shift<-1>(W0), W0, lane_shift<+1>(W0));
            const Prim<T> syv = mc_half_slope(Wm, W0, Wp);
            const Prim<T> ylo = sub(W0, syv);
            if (r >= y0) {
                const Cons<T> G = swap(kt_flux2_x(swap(yhi_prev), swap(ylo)));  // face r - 1/2
                if (r > y0) {
                    finish({acc.r - cy * G.r, acc.mx - cy * G.mx, acc.my - cy * G.my, acc.exx - cy * G.exx,
                            acc.exy - cy * G.exy, acc.eyy - cy * G.eyy},
                           c, r - 1);
                }
                if (r < y1) {
                    const Cons<T> F = kt_flux2_x(plus(W0, sxv), lane_shift<+1>(sub(W0, sxv)));
                    const Cons<T> Fm = lane_shift<-1>(F);
                    const Cons<T> B = kOwnBase ? C0 : load_row(base, r);
                    acc = {B.r - cx * (F.r - Fm.r) + cy * G.r,           B.mx - cx * (F.mx - Fm.mx) + cy * G.mx,
                           B.my - cx * (F.my - Fm.my) + cy * G.my,       B.exx - cx * (F.exx - Fm.exx) + cy * G.exx,
                           B.exy - cx * (F.exy - Fm.exy) + cy * G.exy, B.eyy - cx * (F.eyy - Fm.eyy) + cy * G.eyy};
                }
            }
            yhi_prev = plus(W0, syv);
            Wm = to_prim(Unext);  // row r + 2 takes the place of row r - 1
            if (kOwnBase) Cm = Unext;
        };

        for (int r = y0 - 1; r <= y1; r += 3) {
            row(r, Wa, Wb, Wc, Ca, Cb);
            if (r + 1 > y1) break;
            row(r + 1, Wb, Wc, Wa, Cb, Cc);
            if (r + 2 > y1) break;
            row(r + 2, Wc, Wa, Wb, Cc, Ca);
        }
    }

    if (FINAL) {
        smax = wave_max(smax);
        if (lane == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
        if (__any(bad) && lane == 0) atomicOr(p.flag, 1);
    }
}

// LDS reserved (unused) per workgroup of the 2-D stages: with 160 KB of LDS per
// CU it caps residency at 2 workgroups (2 wavefronts per SIMD).  The stages
// are close to bandwidth-bound and their register count would allow 3
// wavefronts per SIMD; at 3 the 50% more concurrent row streams cost DRAM
// locality (measured on the 4096^2 disc: 0.96 ms per step at 3, 0.91 ms at 2).
constexpr size_t kKtLdsCap = 56 * 1024;

template <typename T>
hipError_t launch_kt(const StepArgs<T>& a, bool twod, bool final_stage, hipStream_t s)
{
    const int nwaves = a.nstrips * a.nsegs;
    const dim3 grid((nwaves + kWaves - 1) / kWaves), block(64 * kWaves);
    if (twod) {
        if (final_stage) kt_kernel<T, true, true><<<grid, block, kKtLdsCap, s>>>(a);
        else kt_kernel<T, true, false><<<grid, block, kKtLdsCap, s>>>(a);
    } else {
        if (final_stage) kt_kernel<T, false, true><<<grid, block, 0, s>>>(a);
        else kt_kernel<T, false, false><<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

template hipError_t launch_kt<double>(const StepArgs<double>&, bool, bool, hipStream_t);
template hipError_t launch_kt<float>(const StepArgs<float>&, bool, bool, hipStream_t);

}  // namespace csh
