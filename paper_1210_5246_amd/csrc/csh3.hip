// Three-dimensional sweep of the ten-moment system (FP64), gfx950.
//
// Two launches per step:
//   trace3_kernel  one thread per cell of the grid and of a one-cell ring
//                  around it: primitive state and its six neighbours (index
//                  maps of the boundary conditions), characteristic MC slopes
//                  along x, y, z, the Hancock predictor with the transverse
//                  terms of the two other axes, the six face states, stored
//                  as [6 faces][10][ring-extended cells];
//   flux3_kernel   one thread per cell: HLL fluxes of its six faces from its
//                  own face states and its neighbours' (each face is solved by
//                  both cells that share it), the unsplit update and the fused
//                  CFL reduction that sets the next timestep on the device.
// This moves about 1.7 KB per cell-update (the face states are written once
// and read twice) against 160 B for a single-pass kernel.
#include "csh3_device.h"
#include "csh_internal.h"
#include "cshydro.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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

template <int N>
__device__ __forceinline__ void axis_slope(const Args& p, const V10& w, double ir, int i, int j, int k, V10& dw,
                                           V10& base, double kf)
{
    const int di = N == 0, dj = N == 1, dk = N == 2;
    const V10 wm = load_prim(p, i - di, j - dj, k - dk), wp = load_prim(p, i + di, j + dj, k + dk);
    const Eig<N> e = eig<N>(w, ir);
    dw = limited_slope<N>(w, e, wm, wp);
    const V10 Ad = jac<N>(w, ir, dw);
#pragma unroll
    for (int m = 0; m < NV; ++m) base.v[m] -= kf * Ad.v[m];
}

template <int N>
__device__ __forceinline__ void store_faces(const Args& p, size_t ne, size_t e, const V10& w, const V10& base,
                                            const V10& dw, double kf)
{
    const double a = 1.7320508075688772935 * sqrt(w.v[P(N, N)] * rcp(w.v[0]));
    const double chi = 0.5 + kf * fmin(w.v[1 + N] + a, 0.0);
    const double clo = 0.5 - kf * fmax(w.v[1 + N] - a, 0.0);
    double* lo = p.FS + (size_t)(2 * N) * NV * ne + e;
    double* hi = lo + (size_t)NV * ne;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        lo[m * ne] = base.v[m] - clo * dw.v[m];
        hi[m * ne] = base.v[m] + chi * dw.v[m];
    }
}

__global__ __launch_bounds__(256) void trace3_kernel(Args p)
{
    const int ex = p.n[0] + 2, ey = p.n[1] + 2, ez = p.n[2] + 2;
    const size_t ne = (size_t)ex * ey * ez;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (e == 0) p.slots[p.s_out].s_bits = 0ull;  // the flux kernel accumulates the new rate there
    const int i = (int)(e % ex) - 1, j = (int)((e / ex) % ey) - 1, k = (int)(e / ((size_t)ex * ey)) - 1;
    const V10 w = load_prim(p, i, j, k);
    const double ir = rcp(w.v[0]);
    const double kf0 = 0.5 * dt / p.h[0], kf1 = 0.5 * dt / p.h[1], kf2 = 0.5 * dt / p.h[2];
    V10 base = w, d0, d1, d2;
    axis_slope<0>(p, w, ir, i, j, k, d0, base, kf0);
    axis_slope<1>(p, w, ir, i, j, k, d1, base, kf1);
    axis_slope<2>(p, w, ir, i, j, k, d2, base, kf2);
    store_faces<0>(p, ne, e, w, base, d0, kf0);
    store_faces<1>(p, ne, e, w, base, d1, kf1);
    store_faces<2>(p, ne, e, w, base, d2, kf2);
}

__device__ __forceinline__ V10 load_face(const Args& p, size_t ne, int face, size_t e)
{
    return load(p.FS + (size_t)face * NV * ne, ne, e);
}

template <int N>
__device__ __forceinline__ void axis_flux(const Args& p, size_t ne, size_t e, size_t stride, double c, V10& du)
{
    const V10 Fm = hll<N>(load_face(p, ne, 2 * N + 1, e - stride), load_face(p, ne, 2 * N, e));
    const V10 Fp = hll<N>(load_face(p, ne, 2 * N + 1, e), load_face(p, ne, 2 * N, e + stride));
#pragma unroll
    for (int m = 0; m < NV; ++m) du.v[m] -= c * (Fp.v[m] - Fm.v[m]);
}

__global__ __launch_bounds__(256) void flux3_kernel(Args p)
{
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.slots[p.s_out].t = t_now + dt;
        p.slots[p.s_reset].s_bits = 0ull;
        if (p.dt_log) *p.dt_log = dt;
    }
    const size_t ncell = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double smax = 0.0;
    bool bad = false;
    if (c < ncell) {
        const int i = (int)(c % p.n[0]), j = (int)((c / p.n[0]) % p.n[1]), k = (int)(c / ((size_t)p.n[0] * p.n[1]));
        const int ex = p.n[0] + 2, ey = p.n[1] + 2;
        const size_t ne = (size_t)ex * ey * (p.n[2] + 2);
        const size_t e = ((size_t)(k + 1) * ey + (j + 1)) * ex + (i + 1);
        V10 du;
#pragma unroll
        for (int m = 0; m < NV; ++m) du.v[m] = 0.0;
        axis_flux<0>(p, ne, e, 1, dt / p.h[0], du);
        axis_flux<1>(p, ne, e, (size_t)ex, dt / p.h[1], du);
        axis_flux<2>(p, ne, e, (size_t)ex * ey, dt / p.h[2], du);
        const V10 U = load(p.U, ncell, c);
        V10 Un;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            Un.v[m] = U.v[m] + du.v[m];
            p.Unew[m * ncell + c] = Un.v[m];
        }
        const V10 wn = to_prim(Un, rcp(Un.v[0]));
        const double ih[3] = {1.0 / p.h[0], 1.0 / p.h[1], 1.0 / p.h[2]};
        smax = signal_rate(wn, ih);
        bad = !physical(wn);
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
        bad = bad || !physical(w);
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
    double* FS = nullptr;
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

size_t next(const csh3_grid* h)
{
    return (size_t)(h->n[0] + 2) * (h->n[1] + 2) * (h->n[2] + 2);
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

hipError_t enqueue_step3(csh3_grid* h, const double* U, double* Un, int dev_dt, double dt, double cfl, double* log,
                         hipStream_t s)
{
    const d3::Args a = args(h, U, Un, dev_dt, dt, cfl, log, nullptr);
    h->phase = a.s_out;
    const size_t ne = next(h), nc = ncell(h);
    d3::trace3_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(a);
    d3::flux3_kernel<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(a);
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
    if ((long long)(nx + 2) * (ny + 2) * (nz + 2) * 8 >= (1LL << 32))
        return fail3(CSH_ERR_ARG, "one extended plane must be smaller than 4 GiB");
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
        hipMalloc(&h->FS, sizeof(double) * 6 * d3::NV * next(h)) != hipSuccess)
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
