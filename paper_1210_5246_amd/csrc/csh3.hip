// Three-dimensional sweep of the ten-moment system (FP64), gfx950.
//
// One launch per step, sweep3_kernel: a workgroup of four wavefronts, each
// holding two rows y of a 28-column strip (32 lanes per row), marches along z
// with two planes of primitive states in registers; one workgroup per CU, each
// taking an equal share of the (strip, row group, plane) columns.  Per cell:
// the characteristic MC slopes along x (lane shifts), y (neighbouring rows
// shared through LDS) and z, the Hancock predictor with the transverse terms
// of the two other axes, the face states; the HLL fluxes of the x faces (lane
// shift), the y faces (neighbouring rows' states through LDS) and the z faces
// (against the previous plane's high face, carried in registers); the
// conservative update, and the fused CFL reduction that sets the next
// timestep on the device.  Of the eight rows of a workgroup the outer two
// supply slopes and y-face states only, so a quarter of the rows' face states
// are formed twice; in exchange nothing but the state itself crosses HBM.
#include "csh3_device.h"
#include "csh_internal.h"
#include "csh_xcd.h"
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

// Component bases of a state, set on the host: with one opaque base per
// component each load or store takes a scalar base and a 32-bit offset
struct Bases {
    const char* in[NV];
    char* out[NV];
};

// The ten components of cell `cell` (one component < 4 GiB)
__device__ __forceinline__ V10 load32(const Bases& b, unsigned cell)
{
    const unsigned o = cell * (unsigned)sizeof(double);
    V10 x;
#pragma unroll
    for (int m = 0; m < NV; ++m) x.v[m] = *reinterpret_cast<const double*>(b.in[m] + o);
    return x;
}

__device__ __forceinline__ void store32(const Bases& b, unsigned cell, const V10& x)
{
    const unsigned o = cell * (unsigned)sizeof(double);
#pragma unroll
    for (int m = 0; m < NV; ++m) *reinterpret_cast<double*>(b.out[m] + o) = x.v[m];
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

// Workgroup of the sweep: four wavefronts, each holding two rows of one
// 28-column strip (32 lanes per row, two halo lanes per side): wavefront w
// the rows j0 - 1 + 2w (lanes 0-31) and j0 + 2w (lanes 32-63), so that the
// workgroup spans the rows j0 - 1 .. j0 + 6, of which j0 .. j0 + 5 are its
// outputs.  Every wavefront does the same work; wavefront 0 also loads the
// rows j0 - 2 and j0 + 7 that the outer rows' y slopes need.
constexpr int kHalf = 32;             // lanes per row
constexpr int kStrip3 = kHalf - 4;    // output columns per row
constexpr int kWaves = 4;
constexpr int kRows = 2 * kWaves;     // rows j0 - 1 .. j0 + 6 of a workgroup
constexpr int kOut = kRows - 2;       // output rows j0 .. j0 + 5
constexpr int kRowSlots = kRows + 2;  // primitive rows j0 - 2 .. j0 + 7 of a plane

struct SArgs {
    Args a;
    Bases b;
    int nstrips, ngroups;  // strips of kStrip3 columns, groups of kOut rows
    long long units;       // nstrips * ngroups * nz plane-columns
    int max_planes;        // longest run of planes taken in one piece
};

// 10-vectors in LDS as [row slot][component][column]: the 32 lanes of a row
// read or write 32 consecutive doubles
__device__ __forceinline__ void put10(double* L, int slot, int col, const V10& x)
{
#pragma unroll
    for (int m = 0; m < NV; ++m) L[(slot * NV + m) * kHalf + col] = x.v[m];
}

__device__ __forceinline__ V10 get10(const double* L, int slot, int col)
{
    V10 x;
#pragma unroll
    for (int m = 0; m < NV; ++m) x.v[m] = L[(slot * NV + m) * kHalf + col];
    return x;
}

// One pass per step.  The plane-columns (a strip, a group of rows, a plane;
// numbered in the order strip, row group, plane) are dealt to the workgroups
// as below; a workgroup marches along z through each run of planes it is
// given.  Per plane r every lane forms the characteristic MC slopes of its
// cell along x (lane shifts; a shift that crosses from one row to the other
// lands on a halo lane, whose results are not used), y (the neighbouring rows
// from LDS) and z (three planes in registers), the Hancock predictor with the
// transverse terms of the two other axes and the face states; it publishes
// its high y-face state, takes the z-face flux against the previous plane's
// high face and finishes the cell of plane r - 1 (store, CFL rate,
// validity), then the x-face flux.  After a barrier it publishes its row of
// plane r + 1 and the y flux of its low face.  After a second barrier the
// output rows add the y-flux difference.  Each LDS area is written and read
// on opposite sides of one of the two barriers, so one copy of each suffices.
__global__ __launch_bounds__(256) void sweep3_kernel(SArgs q)
{
    __shared__ double R[kRowSlots * NV * kHalf];  // primitive rows of plane r (then r + 1)
    __shared__ double Y[kRows * NV * kHalf];      // high y-face state of each row
    __shared__ double G[kRows * NV * kHalf];      // y flux at the low face of each row
    const Args& p = q.a;
    double t_now;
    const double dt = step_dt(p, &t_now);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.slots[p.s_out].t = t_now + dt;
        p.slots[p.s_reset].s_bits = 0ull;
        if (p.dt_log) *p.dt_log = dt;
    }
    const int lane = threadIdx.x & 63, w = wave_in_block();
    const int half = lane >> 5, col = lane & (kHalf - 1);
    const int ys = 2 * w + half;  // row slot among j0 - 1 .. j0 + 6
    const bool loader = w == 0;   // wave-uniform
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const size_t plane = (size_t)nx * ny, ncell = plane * nz;
    // with half slopes the tracing coefficients are dt/h (twice dt/2h)
    const double kx2 = dt / p.h[0], ky2 = dt / p.h[1], kz2 = dt / p.h[2];
    const double cx = kx2, cy = ky2, cz = kz2;
    const double ih[3] = {1.0 / p.h[0], 1.0 / p.h[1], 1.0 / p.h[2]};
    double smax = 0.0;
    bool bad = false;

    // This workgroup's share of the plane-columns, in two passes.  With at
    // least as many columns (strip, row group) as workgroups, the first pass
    // gives each workgroup one whole column: all march in step, and the
    // XCD-aware numbering puts neighbouring row groups, which read two rows
    // in common, on one L2 at the same planes.  The second pass deals the
    // remaining plane-columns in equal contiguous shares.
    const long long g = xcd_block(blockIdx.x, gridDim.x), nwg = gridDim.x;
    const long long ncols = q.units / nz, full = ncols >= nwg ? nwg : 0;
    const long long rest = q.units - full * nz;
    for (int pass = 0; pass < 2; ++pass) {
        long long u = pass == 0 ? g * nz : full * nz + rest * g / nwg;
        const long long u_end = pass == 0 ? (g < full ? (g + 1) * nz : g * nz) : full * nz + rest * (g + 1) / nwg;
        while (u < u_end) {  // wave-uniform: every wavefront takes the same runs
            const long long cidx = u / nz;
            const int z0 = (int)(u - cidx * nz);
            const int z1 = (int)min((long long)min(nz, z0 + q.max_planes), z0 + (u_end - u));
            u += z1 - z0;
            const int gy = (int)(cidx % q.ngroups), sx = (int)(cidx / q.ngroups);
            const int j0 = kOut * gy, j = j0 - 1 + ys;
            const bool out_row = ys >= 1 && ys <= kOut && j < ny;
            const int c = sx * kStrip3 - 2 + col;
            const bool own = col >= 2 && col < 2 + kStrip3 && c < nx;
            const int gc = map_index(c, nx, p.bc[0]);
            const int gj = map_index(j, ny, p.bc[1]);
            const int gh = map_index(half ? j0 + kOut + 1 : j0 - 2, ny, p.bc[1]);  // wavefront 0's extra rows

            auto ld = [&](int row, int r) -> V10 {
                return load32(q.b, ((unsigned)map_index(r, nz, p.bc[2]) * ny + row) * nx + gc);
            };
            auto prim = [](const V10& U) -> V10 { return to_prim(U, rcp(U.v[0])); };

            // Window of the first step (r = z0 - 1): primitive planes z0 - 2 and
            // z0 - 1, the conserved own row of plane z0 - 1 and of plane z0 (loads
            // run one plane ahead), the extra rows of plane z0 for the loader; the
            // rows of plane z0 - 1 go to LDS before the loop.
            V10 Wa = prim(ld(gj, z0 - 2)), C0 = ld(gj, z0 - 1), Wb = prim(C0), Cz = ld(gj, z0), H{}, zhi_prev{}, acc{};
            if (loader) {
                H = ld(gh, z0);
                put10(R, half ? kRowSlots - 1 : 0, col, prim(ld(gh, z0 - 1)));
            }
            put10(R, ys + 1, col, Wb);
            __syncthreads();

            // plane r: Wm = plane r - 1 (refilled with plane r + 1), W0 = plane r
            auto plane_step = [&](int r, V10& Wm, const V10& W0) {
                const V10 Cz_n = ld(gj, r + 2);  // the next step's loads first
                V10 H_n{};
                if (loader) H_n = ld(gh, r + 2);
                const bool inner = r >= z0 && r < z1;  // a plane of the run (not a halo plane)
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
                    dy = half_slope<1>(W0, ir, e, get10(R, ys, col), get10(R, ys + 2, col));
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
                V10 ylo;
                {
                    double ch, cl;
                    coef(1, ky2, ch, cl);
                    V10 yhi;
#pragma unroll
                    for (int m = 0; m < NV; ++m) {
                        ylo.v[m] = base.v[m] - cl * dy.v[m];
                        yhi.v[m] = base.v[m] + ch * dy.v[m];
                    }
                    if (inner) put10(Y, ys, col, yhi);
                }
                {
                    double ch, cl;
                    coef(2, kz2, ch, cl);
                    if (r >= z0) {
                        V10 zlo;
#pragma unroll
                        for (int m = 0; m < NV; ++m) zlo.v[m] = base.v[m] - cl * dz.v[m];
                        const V10 Gz = hll<2>(zhi_prev, zlo);  // face r - 1/2
                        if (r > z0 && out_row) {  // finish the cell of plane r - 1
                            V10 Un;
#pragma unroll
                            for (int m = 0; m < NV; ++m) Un.v[m] = acc.v[m] - cz * Gz.v[m];
                            if (own) {
                                store32(q.b, ((unsigned)(r - 1) * ny + j) * nx + c, Un);
                                const V10 wn = to_prim(Un, rcp(Un.v[0]));
                                smax = fmax(smax, signal_rate(wn, ih));
                                bad |= !physical(wn);
                            }
                        }
                        if (r < z1) {
#pragma unroll
                            for (int m = 0; m < NV; ++m) acc.v[m] = C0.v[m] + cz * Gz.v[m];
                        }
                    }
#pragma unroll
                    for (int m = 0; m < NV; ++m) zhi_prev.v[m] = base.v[m] + ch * dz.v[m];
                }
                if (inner) {
                    double ch, cl;
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
                __syncthreads();  // the rows of plane r are read, the high y-face states written

                put10(R, ys + 1, col, Wp);  // rows of plane r + 1
                if (loader) put10(R, half ? kRowSlots - 1 : 0, col, prim(H));
                if (inner)  // face j - 1/2 (the first row's is not used)
                    put10(G, ys, col, hll<1>(get10(Y, ys > 0 ? ys - 1 : 0, col), ylo));
                __syncthreads();  // the y fluxes and the rows of plane r + 1 written

                if (inner && out_row) {  // faces j -+ 1/2
                    const V10 Gm = get10(G, ys, col), Gp = get10(G, ys + 1, col);
#pragma unroll
                    for (int m = 0; m < NV; ++m) acc.v[m] -= cy * (Gp.v[m] - Gm.v[m]);
                }
                // advance the window: plane r + 1 takes the place of plane r - 1
                Wm = Wp;
                C0 = Cz;
                Cz = Cz_n;
                H = H_n;
            };

            for (int r = z0 - 1; r <= z1; r += 2) {
                plane_step(r, Wa, Wb);
                if (r + 1 > z1) break;
                plane_step(r + 1, Wb, Wa);
            }
        }
    }

    smax = wave_max(smax);
    if (lane == 0) atomic_max_pos(&p.slots[p.s_out].s_bits, smax);
    if (__any(bad) && lane == 0) atomicOr(p.flag, 1);
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
    int phase = 0;
    int ncu = 256;  // compute units of the device
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

d3::Args args(csh3_grid* h, const double* U, double* Un, int dev_dt, double dt, double cfl, double* log,
              const double* dt_in)
{
    d3::Args a{};
    a.U = U;
    a.Unew = Un;
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

// Workgroups of the sweep: one per CU (four wavefronts at one per SIMD fill
// a CU), each taking whole columns of planes and then an equal share of the
// rest, so that every CU marches the same number of planes (plus two halo
// planes per run).
long long sweep_units(const csh3_grid* h)
{
    const long long nstrips = (h->n[0] + d3::kStrip3 - 1) / d3::kStrip3;
    const long long ngroups = (h->n[1] + d3::kOut - 1) / d3::kOut;
    return nstrips * ngroups * h->n[2];
}

hipError_t enqueue_step3(csh3_grid* h, const double* U, double* Un, int dev_dt, double dt, double cfl, double* log,
                         hipStream_t s)
{
    d3::SArgs m{};
    m.a = args(h, U, Un, dev_dt, dt, cfl, log, nullptr);
    for (int k = 0; k < d3::NV; ++k) {
        m.b.in[k] = reinterpret_cast<const char*>(U + k * ncell(h));
        m.b.out[k] = reinterpret_cast<char*>(Un + k * ncell(h));
    }
    m.nstrips = (h->n[0] + d3::kStrip3 - 1) / d3::kStrip3;
    m.ngroups = (h->n[1] + d3::kOut - 1) / d3::kOut;
    m.units = sweep_units(h);
    m.max_planes = h->n[2];
    if (const char* e = std::getenv("CSH_PLANES")) {  // longest run in one piece (seam tests)
        const int v = std::atoi(e);
        if (v >= 1) m.max_planes = v;
    }
    long long wg = h->ncu;
    if (const char* e = std::getenv("CSH_WG3")) {  // tuning override
        const int v = std::atoi(e);
        if (v >= 1) wg = v;
    }
    wg = std::min(wg, m.units);
    h->phase = m.a.s_out;
    d3::sweep3_kernel<<<(unsigned)wg, d3::kWaves * 64, 0, s>>>(m);
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
    // the kernels index with 64 bits; the limit is that of the 2-D path, kept for
    // symmetry (3-D grids are tested up to 256^3)
    if ((long long)nx * ny * nz * 8 >= (1LL << 32))
        return fail3(CSH_ERR_ARG, "one component of the state must be smaller than 4 GiB");
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
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            h->ncu = ncu;
    }
    auto cleanup = [&](int code) {
        csh3_destroy(h);
        return code;
    };
    if (hipMalloc(&h->slots, 3 * sizeof(Slot)) != hipSuccess || hipMalloc(&h->flag, sizeof(int)) != hipSuccess)
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
    delete h;
}
