// Global Fourier amplitudes of the surface density (Sec. 4.4), gfx950.
//
//   A_m = | sum over cells centred in [-X, X] x [-Y, Y] of rho exp(i m phi) |
//         / sum over all cells of rho
//
// (the cell area cancels).  exp(i m phi) is formed without trigonometry as
// the m-th power of z = (x + i y) / R, one rsqrt per cell and one complex
// multiply per mode.  Two launches, deterministic: a fixed grid of workgroups
// each reduces its rows to 1 + 2 m_max partial sums in a fixed order, then one
// workgroup of one thread per partial row reduces them in a fixed order and
// forms the amplitudes.
// The pass reads one plane (8 B per cell in FP64) and is bound by HBM.
#include <mutex>

#include "csh_device.h"
#include "csh_diag.h"

namespace csh {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// cell-centre coordinate c0 + (k + 1/2) h with the product and the sum rounded
// separately (no fused multiply-add), so that a centre on the origin comes out
// as exactly 0 and is recognised as such
__device__ __forceinline__ double centre(double c0, int k, double h)
{
#pragma clang fp contract(off)
    return c0 + (k + 0.5) * h;
}

// M = m_max (a template argument: registers and loop bounds fixed at compile time)
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void fourier_partials(FourierArgs<T> p)
{
    double mass = 0.0, re[M], im[M];
#pragma unroll
    for (int m = 0; m < M; ++m) re[m] = im[m] = 0.0;

    // one cell's contribution: its mass always, its phasors inside the region
    auto add = [&](double s, int i, double y, bool row_in) {
        mass += s;
        const double x = centre(p.x0, i, p.dx);
        const double r2 = x * x + y * y;
        if (!row_in || fabs(x) > p.X || r2 == 0.0) return;
        const double ir = rsqrt(r2);
        const double zr = x * ir, zi = y * ir;
        double wr = zr, wi = zi;  // exp(i m phi) for m = 1
#pragma unroll
        for (int m = 0; m < M; ++m) {
            re[m] += s * wr;
            im[m] += s * wi;
            const double t = wr * zr - wi * zi;
            wi = wr * zi + wi * zr;
            wr = t;
        }
    };
    constexpr int kU = 4;  // loads issued ahead of the arithmetic
    for (int j = blockIdx.x; j < p.ny; j += gridDim.x) {
        const double y = centre(p.y0, j, p.dy);
        const bool row_in = fabs(y) <= p.Y;
        const T* row = p.rho + (size_t)j * p.nx;
        for (int i0 = threadIdx.x; i0 < p.nx; i0 += kU * kThreads) {
            double s[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * kThreads;
                s[u] = i < p.nx ? double(row[i]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * kThreads;
                if (i < p.nx) add(s[u], i, y, row_in);
            }
        }
    }

    // workgroup reduction in a fixed order: wavefront butterflies, then the
    // four wavefronts' sums added in wavefront order
    __shared__ double part[kThreads / 64][1 + 2 * M];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double ms = wave_sum(mass);
    if (lane == 0) part[wv][0] = ms;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double a = wave_sum(re[m]), b = wave_sum(im[m]);
        if (lane == 0) {
            part[wv][1 + 2 * m] = a;
            part[wv][2 + 2 * m] = b;
        }
    }
    __syncthreads();
    constexpr int nv = 1 + 2 * M;
    if ((int)threadIdx.x < nv) {
        double acc = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) acc += part[w][threadIdx.x];
        p.partials[(size_t)threadIdx.x * kFourierBlocks + blockIdx.x] = acc;  // value-major
    }
}

// one thread per partial row; per value a wavefront butterfly, then the
// wavefronts' sums added in wavefront order (a fixed order).  The partial sums
// are stored value-major, so each value's loads are coalesced; with M fixed
// at compile time the loads of eight values go out together and their
// butterflies interleave.
template <int M>
__global__ __launch_bounds__(kFourierBlocks) void fourier_finish(const double* __restrict__ partials,
                                                                 double* __restrict__ A)
{
    constexpr int kW = kFourierBlocks / 64, nv = 1 + 2 * M;
    __shared__ double part[kW][nv];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int kC = 8;  // values in flight at once (registers stay within the 1024-thread limit)
#pragma unroll
    for (int k0 = 0; k0 < nv; k0 += kC) {
        double v[kC];
#pragma unroll
        for (int k = 0; k < kC; ++k)
            if (k0 + k < nv) v[k] = partials[(size_t)(k0 + k) * kFourierBlocks + threadIdx.x];
#pragma unroll
        for (int k = 0; k < kC; ++k)
            if (k0 + k < nv) v[k] = wave_sum(v[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kC; ++k)
                if (k0 + k < nv) part[wv][k0 + k] = v[k];
        }
    }
    __syncthreads();
    __shared__ double tot[nv];
    if ((int)threadIdx.x < nv) {
        double acc = 0.0;
        for (int w = 0; w < kW; ++w) acc += part[w][threadIdx.x];
        tot[threadIdx.x] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        const double a = tot[1 + 2 * threadIdx.x], b = tot[2 + 2 * threadIdx.x];
        A[threadIdx.x] = sqrt(a * a + b * b) / tot[0];
    }
}

}  // namespace

template <typename T, int M>
void launch_partials(const FourierArgs<T>& a, hipStream_t s)
{
    if constexpr (M > 1) {
        if (a.m_max < M) return launch_partials<T, M - 1>(a, s);
    }
    fourier_partials<T, M><<<kFourierBlocks, kThreads, 0, s>>>(a);
    fourier_finish<M><<<1, kFourierBlocks, 0, s>>>(a.partials, a.A);
}

template <typename T>
hipError_t launch_fourier(const FourierArgs<T>& a, hipStream_t s)
{
    if (a.m_max < 1 || a.m_max > kFourierMaxM) return hipErrorInvalidValue;
    launch_partials<T, kFourierMaxM>(a, s);  // the partial sums and the finishing reduction
    return hipGetLastError();
}

template hipError_t launch_fourier<double>(const FourierArgs<double>&, hipStream_t);
template hipError_t launch_fourier<float>(const FourierArgs<float>&, hipStream_t);

// ---- statically sized partial sums (the allocation-free entry point) ----------------------------

// In host code `scratch` names a host-side stand-in, not device memory: only
// the address hipGetSymbolAddress returns for the current device may be handed
// to a kernel or a copy.
namespace {
constexpr size_t kStaticPartials = (size_t)kFourierBlocks * (1 + 2 * kFourierMaxM);
static __device__ __align__(256) double scratch[kStaticPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t fourier_static_partials(double** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace csh
