// Three-dimensional sweep of the ten-moment system (FP64), gfx950.
//
// Two launches per step:
//   march3_kernel  a wavefront per 60-column strip of one row y (the rows
//                  -1 and ny included, for their y-face states), marching
//                  along z over a segment of planes with two planes of
//                  primitive states in registers; per cell the
//                  characteristic MC slopes along x (lane shifts), y (the
//                  neighbouring rows, loaded) and z, the Hancock predictor
//                  with the transverse terms of the two other axes, the six
//                  face states; the x-face flux by a lane shift and the z-face
//                  flux against the previous plane's high face, so the
//                  partial update U - dt/dx dFx - dt/dz dFz is written to
//                  the output; the two y-face states go to a workspace
//                  [2][10][nz][ny + 2][nx];
//   yflux3_kernel  a thread per (x, z) column marching over a segment of
//                  rows: each y-face HLL flux once, the end of the update and
//                  the fused CFL reduction that sets the next timestep on the
//                  device.
#include "csh3_device.h"
#include "csh_internal.h"
#include "cshydro.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>

namespace csh {
namespace d3 {

struct Args {
    const double* U;   // [10][nz][ny][nx]
    double* Unew;
    double* FS;        // [6][10][ne], ne = (nx + 2)(ny + 2)(nz + 2)
    int n[3], bc[3];
    double h[3];
    double dt;
    int dev_dt;
    const double* dt_in;
    double cfl;
    Slot* slots;
    int s_in, s_out, s_reset;
    double* dt_log;
    int* flag;
};

__device__ __forceinline__ double step_dt(const Args& p, double* t_now)
{
    const Slot& sl = p.slots[p.s_in];
    *t_now = sl.t;
    if (!p.dev_dt) return p.dt_in ? *p.dt_in : p.dt;
    return p.cfl / __longlong_as_double((long long)sl.s_bits);
}

__device__ __forceinline__ V10 load(const double* __restrict__ U, size_t plane, size_t c)
{
    V10 x;
#pragma unroll
    for (int m = 0; m < NV; ++m) x.v[m] = U[m * plane + c];
    return x;
}

__device__ __forceinline__ V10 load_prim(const Args& p, int i, int j, int k)
{
    const int gi = map_index(i, p.n[0], p.bc[0]), gj = map_index(j, p.n[1], p.bc[1]);
    const int gk = map_index(k, p.n[2], p.bc[2]);
    const size_t plane = (size_t)p.n[0] * p.n[1] * p.n[2];
    const V10 U = load(p.U, plane, ((size_t)gk * p.n[1] + gj) * p.n[0] + gi);
    return to_prim(U, rcp(U.v[0]));
}

// wavefront-wide shift of a 10-vector by one lane (zero fill at the end)
template <int D>
__device__ __forceinline__ V10 shift(const V10& x)
{
    V10 y;
#pragma unroll
    for (int m = 0; m < NV; ++m) y.v[m] = lane_shift<D>(x.v[m]);
    return y;
}

struct MArgs {
    Args a;
    double* FY;        // y-face states [2 (lo, hi)][10][nz][ny + 2][nx]
    int nstrips, nsegs, tz;
};

// One wavefront: 60 output columns (64 lanes, 2 halo lanes per side) of one
// row j in [-1, ny] (the two outer rows only supply y-face states), marching
// over planes [z0, z1).  Per plane: characteristic slopes along x (lane
// shifts), y (the neighbouring rows, loaded) and z (three planes in
// registers), the six face states, the x-face flux by a lane shift, the
// z-face flux against the previous plane's high face; the partial update
// U - dt/dx dFx - dt/dz dFz is written to Unew and the two y-face states to FY.
__global__ __launch_bounds__(256) void march3_kernel(MArgs q)
{
    const Args& p = q.a;
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) p.slots[p.s_out].s_bits = 0ull;
    const int lane = threadIdx.x & 63;
    const long wid = (long)blockIdx.x * 4 + wave_in_block();
    const int ey = p.n[1] + 2;
    if (wid >= (long)q.nsegs * q.nstrips * ey) return;  // uniform per wavefront
    const int jj = (int)(wid % ey), sx = (int)((wid / ey) % q.nstrips), sz = (int)(wid / ((long)ey * q.nstrips));
    const int j = jj - 1;
    const bool interior = j >= 0 && j < p.n[1];
    const int c = sx * kStrip - 2 + lane;
    const bool own = lane >= 2 && lane < 2 + kStrip && c < p.n[0];
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int gc = map_index(c, nx, p.bc[0]);
    const int gjm = map_index(j - 1, ny, p.bc[1]), gj0 = map_index(j, ny, p.bc[1]), gjp = map_index(j + 1, ny, p.bc[1]);
    const size_t plane = (size_t)nx * ny, ncell = plane * nz;
    const size_t fplane = (size_t)nx * ey, nf = fplane * nz;
    // with half slopes the tracing coefficients are dt/h (twice dt/2h)
    const double kx2 = dt / p.h[0], ky2 = dt / p.h[1], kz2 = dt / p.h[2];
    const double cx = kx2, cz = kz2;
    const int z0 = sz * q.tz, z1 = min(z0 + q.tz, nz);

    auto cell = [&](int gj, int r) -> size_t {
        return ((size_t)map_index(r, nz, p.bc[2]) * ny + gj) * nx + gc;
    };
    auto ld = [&](int gj, int r) -> V10 { return load(p.U, ncell, cell(gj, r)); };
    auto prim = [](const V10& U) -> V10 { return to_prim(U, rcp(U.v[0])); };

    // Window of the first step (r = z0 - 1): primitive planes z0 - 2 and
    // z0 - 1, the conserved centre of plane z0 - 1, and the loads the step
    // consumes, issued one step ahead (centre of plane r + 1, rows j -+ 1 of
    // plane r): one wavefront per SIMD hides the memory latency this way.
    V10 Wa = prim(ld(gj0, z0 - 2)), C0 = ld(gj0, z0 - 1), Wb = prim(C0);
    V10 Cz = ld(gj0, z0), Cym = ld(gjm, z0 - 1), Cyp = ld(gjp, z0 - 1), zhi_prev, acc;
    V10 Cym1 = ld(gjm, z0), Cyp1 = ld(gjp, z0);  // neighbour rows one plane ahead
#pragma unroll
    for (int m = 0; m < NV; ++m) zhi_prev.v[m] = acc.v[m] = 0.0;

    // plane r: Wm = plane r - 1 (refilled with plane r + 1), W0 = plane r.
    // Ordered so that each slope and face pair dies as early as possible.
    auto plane_step = [&](int r, V10& Wm, const V10& W0) {
        // the next step's loads first
        // the neighbour rows of plane r + 2, loaded with this row's own plane r + 2
        // (the neighbouring wavefronts load them as their own rows in the same step)
        const V10 Cz_n = ld(gj0, r + 2), Cym_n = ld(gjm, r + 2), Cyp_n = ld(gjp, r + 2);
        const double ir = rcp(W0.v[0]);
        double a3[3];  // fast speeds sqrt(3 P_kk / rho)
        auto coef = [&](int k, double k2, double& chi, double& clo) {
            const double ak = a3[k], uk = W0.v[1 + k];
            chi = 1.0 + k2 * fmin(uk + ak, 0.0);
            clo = 1.0 - k2 * fmax(uk - ak, 0.0);
        };
        V10 base = W0, dz, dy, dx;  // half slopes
        {
            const Eig<0> e = eig<0>(W0, ir);
            a3[0] = e.a;
            dx = half_slope<0>(W0, ir, e, shift<-1>(W0), shift<+1>(W0));
            const V10 Ad = jac<0>(W0, ir, dx);
#pragma unroll
            for (int m = 0; m < NV; ++m) base.v[m] -= kx2 * Ad.v[m];
        }
        {
            const Eig<1> e = eig<1>(W0, ir);
            a3[1] = e.a;
            dy = half_slope<1>(W0, ir, e, prim(Cym), prim(Cyp));
            const V10 Ad = jac<1>(W0, ir, dy);
#pragma unroll
            for (int m = 0; m < NV; ++m) base.v[m] -= ky2 * Ad.v[m];
        }
        const V10 Wp = prim(Cz);
        {
            const Eig<2> e = eig<2>(W0, ir);
            a3[2] = e.a;
            dz = half_slope<2>(W0, ir, e, Wm, Wp);
            const V10 Ad = jac<2>(W0, ir, dz);
#pragma unroll
            for (int m = 0; m < NV; ++m) base.v[m] -= kz2 * Ad.v[m];
        }
        double ch, cl;
        if (r >= z0 && r < z1 && own) {  // the y-face states of (c, j, r)
            coef(1, ky2, ch, cl);
            const size_t f = ((size_t)r * ey + jj) * nx + c;
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                q.FY[m * nf + f] = base.v[m] - cl * dy.v[m];
                q.FY[(NV + m) * nf + f] = base.v[m] + ch * dy.v[m];
            }
        }
        coef(2, kz2, ch, cl);
        V10 zhi;
        if (r >= z0) {
            V10 zlo;
#pragma unroll
            for (int m = 0; m < NV; ++m) zlo.v[m] = base.v[m] - cl * dz.v[m];
            const V10 Gz = hll<2>(zhi_prev, zlo);  // face r - 1/2
            if (r > z0 && interior && own) {
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    p.Unew[m * ncell + ((size_t)(r - 1) * ny + j) * nx + c] = acc.v[m] - cz * Gz.v[m];
            }
            if (r < z1) {
#pragma unroll
                for (int m = 0; m < NV; ++m) acc.v[m] = C0.v[m] + cz * Gz.v[m];
            }
        }
#pragma unroll
        for (int m = 0; m < NV; ++m) zhi.v[m] = base.v[m] + ch * dz.v[m];
        zhi_prev = zhi;
        if (r >= z0 && r < z1) {
            coef(0, kx2, ch, cl);
            V10 xlo, xhi;
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                xlo.v[m] = base.v[m] - cl * dx.v[m];
                xhi.v[m] = base.v[m] + ch * dx.v[m];
            }
            const V10 F = hll<0>(xhi, shift<+1>(xlo));  // face c + 1/2
            const V10 Fm = shift<-1>(F);
#pragma unroll
            for (int m = 0; m < NV; ++m) acc.v[m] -= cx * (F.v[m] - Fm.v[m]);
        }
        // advance the window: plane r + 1 takes the place of plane r - 1
        Wm = Wp;
        C0 = Cz;
        Cz = Cz_n;
        Cym = Cym1;
        Cyp = Cyp1;
        Cym1 = Cym_n;
        Cyp1 = Cyp_n;
    };

    for (int r = z0 - 1; r <= z1; r += 2) {
        plane_step(r, Wa, Wb);
        if (r + 1 > z1) break;
        plane_step(r + 1, Wb, Wa);
    }
}

// A thread per (x, z) column marching over a segment of rows: each y face's
// flux once (the previous face's flux carried in registers), the end of the
// update, CFL rate and validity.
__global__ __launch_bounds__(256) void yflux3_kernel(MArgs q, int ty)
{
    const Args& p = q.a;
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.slots[p.s_out].t = t_now + dt;
        p.slots[p.s_reset].s_bits = 0ull;
        if (p.dt_log) *p.dt_log = dt;
    }
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2], ey = ny + 2;
    const int nseg = (ny + ty - 1) / ty;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double smax = 0.0;
    bool bad = false;
    if (t < (size_t)nx * nz * nseg) {
        const int i = (int)(t % nx), k = (int)((t / nx) % nz), sy = (int)(t / ((size_t)nx * nz));
        const int y0 = sy * ty, y1 = min(y0 + ty, ny);
        const size_t ncell = (size_t)nx * ny * nz, nf = (size_t)nx * ey * nz;
        const double cy = dt / p.h[1];
        const double ih[3] = {1.0 / p.h[0], 1.0 / p.h[1], 1.0 / p.h[2]};
        auto fidx = [&](int jj) { return ((size_t)k * ey + jj) * nx + i; };  // jj = j + 1
        const double* FL = q.FY;
        const double* FH = q.FY + (size_t)NV * nf;
        // face y0 - 1/2: high state of row y0 - 1, low state of row y0; the
        // face states of the next face are loaded one row ahead
        V10 Gm = hll<1>(load(FH, nf, fidx(y0)), load(FL, nf, fidx(y0 + 1)));
        V10 hi_n = load(FH, nf, fidx(y0 + 1)), lo_n = load(FL, nf, fidx(y0 + 2));
        for (int j = y0; j < y1; ++j) {
            const V10 hi = hi_n, lo = lo_n;
            if (j + 1 < y1) {
                hi_n = load(FH, nf, fidx(j + 2));
                lo_n = load(FL, nf, fidx(j + 3));
            }
            const size_t c = ((size_t)k * ny + j) * nx + i;
            const V10 A = load(p.Unew, ncell, c);
            const V10 Gp = hll<1>(hi, lo);
            V10 Un;
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                Un.v[m] = A.v[m] - cy * (Gp.v[m] - Gm.v[m]);
                p.Unew[m * ncell + c] = Un.v[m];
            }
            const V10 wn = to_prim(Un, rcp(Un.v[0]));
            smax = fmax(smax, signal_rate(wn, ih));
            bad |= !physical(wn);
            Gm = Gp;
        }
    }
    smax = wave_max(smax);
    if ((threadIdx.x & 63) == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(p.flag, 1);
}

__global__ __launch_bounds__(256) void init3_kernel(const double* __restrict__ W, double* __restrict__ U, int64_t n,
                                                    int* flag)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (c < n) {
        const V10 w = load(W, (size_t)n, (size_t)c);
        bad = !physical(w);
        const V10 u = to_cons(w);
#pragma unroll
        for (int m = 0; m < NV; ++m) U[m * n + c] = u.v[m];
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void maxspeed3_kernel(const double* __restrict__ U, int64_t n, double ih0,
                                                        double ih1, double ih2, Slot* slot, int* flag)
{
    double s = 0.0;
    bool bad = false;
    const double ih[3] = {ih0, ih1, ih2};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const V10 u = load(U, (size_t)n, (size_t)c);
        const V10 w = to_prim(u, rcp(u.v[0]));
        s = fmax(s, signal_rate(w, ih));
        bad |= !physical(w);
    }
    s = wave_max(s);
    if ((threadIdx.x & 63) == 0) atomic_max_pos(&slot->s_bits, s);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace d3
}  // namespace csh

using csh::Slot;
namespace d3 = csh::d3;

struct csh3_grid {
    int n[3] = {0, 0, 0}, bc[3] = {0, 0, 0};
    double h[3] = {1, 1, 1};
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    Slot* slots = nullptr;
    int* flag = nullptr;
    double* FS = nullptr;  // y-face states of the march
    int phase = 0;
    hipGraphExec_t exec = nullptr;
    int g_nsteps = -1;
    double g_cfl = 0;  // arguments the cached graph of csh3_run_cfl was recorded with
    const void *g_U = nullptr, *g_W = nullptr, *g_log = nullptr;
};

namespace {

thread_local std::string g_err3;

int fail3(int code, const std::string& msg)
{
    g_err3 = msg;
    return code;
}

#define CSH3_HIP(x)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return fail3(CSH_ERR_HIP, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t ncell(const csh3_grid* h)
{
    return (size_t)h->n[0] * h->n[1] * h->n[2];
}

// cells of the y-face workspace: the grid plus one row on each side in y
size_t nfy(const csh3_grid* h)
{
    return (size_t)h->n[0] * (h->n[1] + 2) * h->n[2];
}

d3::Args args(csh3_grid* h, const double* U, double* Un, int dev_dt, double dt, double cfl, double* log,
              const double* dt_in)
{
    d3::Args a{};
    a.U = U;
    a.Unew = Un;
    a.FS = h->FS;
    for (int k = 0; k < 3; ++k) {
        a.n[k] = h->n[k];
        a.bc[k] = h->bc[k];
        a.h[k] = h->h[k];
    }
    a.dt = dt;
    a.dev_dt = dev_dt;
    a.dt_in = dt_in;
    a.cfl = cfl;
    a.slots = h->slots;
    a.s_in = h->phase;
    a.s_out = (h->phase + 1) % 3;
    a.s_reset = (h->phase + 2) % 3;
    a.dt_log = log;
    a.flag = h->flag;
    return a;
}

// z-segment length of the march: as for the rows of the 2-D sweep, the length
// that minimises the busiest SIMD's critical path, ceil(wavefronts / 1024) x
// (planes + 2) (one wavefront per SIMD; each re-traces two halo planes), over
// 4..128 planes (measured at 256^3: 37 planes, 3.24 ms per step against 3.36 ms
// for 32 and 3.29-3.45 ms for 24-128).
int planes_per_segment(const csh3_grid* h)
{
    if (const char* e = std::getenv("CSH_PLANES")) {  // tuning override
        const int v = std::atoi(e);
        if (v >= 1) return v;
    }
    const int nz = h->n[2];
    const long per_segment = (long)((h->n[0] + csh::kStrip - 1) / csh::kStrip) * (h->n[1] + 2);
    int best = nz;
    long best_cost = -1;
    for (int t = 4; t <= std::min(nz, 128); ++t) {
        const long waves = per_segment * ((nz + t - 1) / t);
        const long cost = ((waves + 1023) / 1024) * (t + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}

hipError_t enqueue_step3(csh3_grid* h, const double* U, double* Un, int dev_dt, double dt, double cfl, double* log,
                         hipStream_t s)
{
    d3::MArgs m{};
    m.a = args(h, U, Un, dev_dt, dt, cfl, log, nullptr);
    m.FY = h->FS;
    m.nstrips = (h->n[0] + csh::kStrip - 1) / csh::kStrip;
    m.tz = planes_per_segment(h);
    m.nsegs = (h->n[2] + m.tz - 1) / m.tz;
    h->phase = m.a.s_out;
    const long nwaves = (long)m.nsegs * m.nstrips * (h->n[1] + 2);
    const int ty = 32, nsegy = (h->n[1] + ty - 1) / ty;
    const size_t ncol = (size_t)h->n[0] * h->n[2] * nsegy;
    d3::march3_kernel<<<(unsigned)((nwaves + 3) / 4), 256, 0, s>>>(m);
    d3::yflux3_kernel<<<(unsigned)((ncol + 255) / 256), 256, 0, s>>>(m, ty);
    return hipGetLastError();
}

hipError_t enqueue_maxspeed3(csh3_grid* h, const double* U, hipStream_t s)
{
    hipError_t e = csh::launch_reset(h->slots + h->phase, 1, 0.0, s);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)ncell(h);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    d3::maxspeed3_kernel<<<blocks, 256, 0, s>>>(U, n, 1.0 / h->h[0], 1.0 / h->h[1], 1.0 / h->h[2],
                                                h->slots + h->phase, h->flag);
    return hipGetLastError();
}

int read_rate(csh3_grid* h, int slot, double* s)
{
    unsigned long long bits = 0;
    int flag = 0;
    CSH3_HIP(hipMemcpyAsync(&bits, &h->slots[slot].s_bits, sizeof(bits), hipMemcpyDeviceToHost, h->stream));
    CSH3_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    CSH3_HIP(hipStreamSynchronize(h->stream));
    double v;
    memcpy(&v, &bits, sizeof(v));
    *s = v;
    if (flag) return fail3(CSH_ERR_NONPHYSICAL, "a state was not physical");
    return CSH_OK;
}

void drop_graph3(csh3_grid* h)
{
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    h->exec = nullptr;
    h->g_nsteps = -1;
}

}  // namespace

extern "C" const char* csh3_last_error(void)
{
    return g_err3.c_str();
}

extern "C" int csh3_init_state(csh3_grid** out, int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                               int bc_y, int bc_z, const void* W, void* U, void* stream)
{
    if (!out) return fail3(CSH_ERR_ARG, "h is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail3(CSH_ERR_ARG, "nx, ny, nz must be >= 1");
    if ((long long)nx * (ny + 2) * nz * 8 >= (1LL << 32))
        return fail3(CSH_ERR_ARG, "one plane of the state must be smaller than 4 GiB");
    if (!(dx > 0) || !(dy > 0) || !(dz > 0)) return fail3(CSH_ERR_ARG, "cell sizes must be > 0");
    const int bcs[3] = {bc_x, bc_y, bc_z};
    for (int k = 0; k < 3; ++k)
        if (bcs[k] != CSH_BC_PERIODIC && bcs[k] != CSH_BC_OUTFLOW) return fail3(CSH_ERR_ARG, "bad boundary condition");
    if (!W || !U) return fail3(CSH_ERR_ARG, "W and U must be device pointers");
    csh3_grid* h = new csh3_grid;
    h->n[0] = nx;
    h->n[1] = ny;
    h->n[2] = nz;
    h->h[0] = dx;
    h->h[1] = dy;
    h->h[2] = dz;
    for (int k = 0; k < 3; ++k) h->bc[k] = bcs[k];
    h->stream = static_cast<hipStream_t>(stream);
    auto cleanup = [&](int code) {
        csh3_destroy(h);
        return code;
    };
    if (hipMalloc(&h->slots, 3 * sizeof(Slot)) != hipSuccess || hipMalloc(&h->flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&h->FS, sizeof(double) * 2 * d3::NV * nfy(h)) != hipSuccess)
        return cleanup(fail3(CSH_ERR_HIP, "hipMalloc of the handle's buffers failed"));
    if (hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail3(CSH_ERR_HIP, "hipStreamCreate failed"));
    const int64_t n = (int64_t)ncell(h);
    hipError_t e = csh::launch_reset(h->slots, 3, 0.0, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->flag, 0, sizeof(int), h->stream);
    if (e == hipSuccess) {
        d3::init3_kernel<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(static_cast<const double*>(W),
                                                                              static_cast<double*>(U), n, h->flag);
        e = hipGetLastError();
    }
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return cleanup(fail3(CSH_ERR_HIP, std::string("init: ") + hipGetErrorString(e)));
    *out = h;
    if (flag) return fail3(CSH_ERR_NONPHYSICAL, "initial state not physical");
    return CSH_OK;
}

extern "C" int csh3_step(csh3_grid* h, double dt, const void* U, void* U_new)
{
    if (!h || !U || !U_new) return fail3(CSH_ERR_ARG, "NULL argument");
    if (U == U_new) return fail3(CSH_ERR_ARG, "U_new must not alias U");
    if (!(dt >= 0)) return fail3(CSH_ERR_ARG, "dt must be >= 0");
    CSH3_HIP(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    CSH3_HIP(enqueue_step3(h, static_cast<const double*>(U), static_cast<double*>(U_new), 0, dt, 0, nullptr,
                           h->stream));
    int flag = 0;
    CSH3_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    CSH3_HIP(hipStreamSynchronize(h->stream));
    if (flag) return fail3(CSH_ERR_NONPHYSICAL, "the new state is not physical");
    return CSH_OK;
}

extern "C" int csh3_max_signal_speed(csh3_grid* h, const void* U, double* s)
{
    if (!h || !U || !s) return fail3(CSH_ERR_ARG, "NULL argument");
    CSH3_HIP(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    CSH3_HIP(enqueue_maxspeed3(h, static_cast<const double*>(U), h->stream));
    return read_rate(h, h->phase, s);
}

extern "C" int csh3_last_signal_speed(csh3_grid* h, double* s)
{
    if (!h || !s) return fail3(CSH_ERR_ARG, "NULL argument");
    return read_rate(h, h->phase, s);
}

namespace {

// the whole run from phase 0: all slots cleared, the rate of the input into
// slot 0, then the steps (device timestep), a copy back if nsteps is odd
hipError_t enqueue_run3(csh3_grid* h, int nsteps, double cfl, void* U, void* Uw, double* dt_log, hipStream_t s)
{
    h->phase = 0;
    hipError_t e = csh::launch_reset(h->slots, 3, 0.0, s);
    if (e == hipSuccess) e = enqueue_maxspeed3(h, static_cast<const double*>(U), s);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
        const double* in = static_cast<const double*>(k % 2 == 0 ? U : Uw);
        double* outp = static_cast<double*>(k % 2 == 0 ? Uw : U);
        e = enqueue_step3(h, in, outp, 1, 0.0, cfl, dt_log + k, s);
    }
    if (e == hipSuccess && nsteps % 2 == 1)
        e = csh::launch_copy<double>(static_cast<const double*>(Uw), static_cast<double*>(U),
                                     (int64_t)ncell(h) * d3::NV, s);
    return e;
}

}  // namespace

extern "C" int csh3_run_cfl(csh3_grid* h, int nsteps, double cfl, void* U, void* U_work, double* dt_log)
{
    if (!h || !U || !U_work || (nsteps > 0 && !dt_log)) return fail3(CSH_ERR_ARG, "NULL argument");
    if (U == U_work) return fail3(CSH_ERR_ARG, "U and U_work must be distinct");
    if (nsteps < 0 || !(cfl > 0)) return fail3(CSH_ERR_ARG, "nsteps >= 0 and cfl > 0 required");
    if (nsteps == 0) return CSH_OK;
    const bool same = h->exec && h->g_nsteps == nsteps && h->g_cfl == cfl && h->g_U == U && h->g_W == U_work &&
                      h->g_log == dt_log;
    if (!same) {
        drop_graph3(h);
        hipGraph_t graph = nullptr;
        CSH3_HIP(hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_run3(h, nsteps, cfl, U, U_work, dt_log, h->capture);
        hipError_t e2 = hipStreamEndCapture(h->capture, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail3(CSH_ERR_HIP, std::string("capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&h->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            h->exec = nullptr;
            return fail3(CSH_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
        }
        h->g_nsteps = nsteps;
        h->g_cfl = cfl;
        h->g_U = U;
        h->g_W = U_work;
        h->g_log = dt_log;
    }
    CSH3_HIP(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    CSH3_HIP(hipGraphLaunch(h->exec, h->stream));
    h->phase = nsteps % 3;
    int flag = 0;
    CSH3_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    CSH3_HIP(hipStreamSynchronize(h->stream));
    if (flag) return fail3(CSH_ERR_NONPHYSICAL, "a state was not physical");
    return CSH_OK;
}

extern "C" void csh3_destroy(csh3_grid* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graph3(h);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    if (h->slots) (void)hipFree(h->slots);
    if (h->flag) (void)hipFree(h->flag);
    if (h->FS) (void)hipFree(h->FS);
    delete h;
}
