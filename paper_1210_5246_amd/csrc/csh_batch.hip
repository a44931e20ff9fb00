// Many independent 1-D problems of uneven length in one persistent launch.
//
// Each workgroup takes a whole tube from a device queue (tubes ordered longest
// first, so the queue hands out work in LPT order) and advances it nsteps
// steps: for every step, its wavefronts sweep the tube in chunks of 60 cells
// (the 1-D device sweep of the plain path), the workgroup reduces the CFL
// rate of the new state, and every thread forms the tube's next timestep
// dt = C / s itself.  Steps alternate between the tube's cells in U and in
// the work buffer; a workgroup barrier separates them.  No host round trip,
// no grid-wide barrier: tubes never interact.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <numeric>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "csh_api_util.h"
#include "csh_device.h"
#include "csh_internal.h"

namespace csh {

struct BatchArgs {
    const int64_t* offsets;  // [ntubes + 1]
    const int* order;        // tubes, longest first
    int* counter;            // queue head
    double* U;               // [6][N]
    double* Uw;              // [6][N]
    double* dt_out;          // [ntubes][nsteps] or null
    int64_t N;
    int ntubes, nsteps;
    double cfl;
    int* flag;
};

// zero-gradient outflow index inside a tube of n cells
__device__ __forceinline__ int clamp_cell(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// Workgroup maximum; red holds two rows used alternately (parity), so a row
// is rewritten only after the barrier of the call in between, when every
// thread has read it: one barrier per call.
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red, int parity)
{
    constexpr int NW = NT / 64;
    double* r = red + parity * NW;
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) r[w] = v;
    __syncthreads();
    double m = r[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) m = fmax(m, r[k]);
    return m;
}

template <int NT>
__global__ __launch_bounds__(NT) void batch_kernel(BatchArgs a)
{
    constexpr int NW = NT / 64;
    __shared__ int s_q;
    __shared__ double red[2 * NW];
    const int lane = threadIdx.x & 63, wave = wave_in_block();  // wave-uniform chunk loop
    const size_t plane = (size_t)a.N;

    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(a.counter, 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= a.ntubes) break;  // uniform: every thread read the same q
        const int k = a.order[q];
        const int64_t off = a.offsets[k];
        const int n = (int)(a.offsets[k + 1] - off);
        const double idx = (double)n;  // dx = 1 / n
        double* A = a.U + off;
        double* B = a.Uw + off;

        // rate of the initial state
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += NT)
            s = fmax(s, signal_rate<double, false>(to_prim(load_cons<double>(A, plane, (size_t)i)), idx, 0.0));
        s = block_max<NT>(s, red, 0);

        bool bad = false;
        for (int step = 0; step < a.nsteps; ++step) {
            const double dt = a.cfl / s;
            if (threadIdx.x == 0 && a.dt_out) a.dt_out[(size_t)k * a.nsteps + step] = dt;
            const double kx = dt * idx * 0.5, cx = dt * idx;
            double smax = 0.0;
            // the next chunk's loads are issued before this chunk's arithmetic
            Cons<double> Unext{};
            if (wave * kStrip < n) Unext = load_cons<double>(A, plane, (size_t)clamp_cell(wave * kStrip - 2 + lane, n));
            for (int base = wave * kStrip; base < n; base += NW * kStrip) {
                const int c = base - 2 + lane;
                const Cons<double> U0 = Unext;
                if (base + NW * kStrip < n)
                    Unext = load_cons<double>(A, plane, (size_t)clamp_cell(base + NW * kStrip - 2 + lane, n));
                const Cons<double> F = flux_1d(U0, kx);
                const Cons<double> Un = update(U0, cx, F, lane_shift<-1>(F));
                if (lane >= 2 && lane < 2 + kStrip && c < n) {
                    store_cons(B, plane, (size_t)c, Un);
                    const Prim<double> wn = to_prim(Un);
                    smax = fmax(smax, signal_rate<double, false>(wn, idx, 0.0));
                    bad |= !physical(wn);
                }
            }
            s = block_max<NT>(smax, red, (step + 1) & 1);  // its barrier also orders this step's stores before the next step's loads
            double* t = A;
            A = B;
            B = t;
        }
        if (a.nsteps % 2 == 1) {  // the state ended in the work buffer: copy it home
            for (int i = threadIdx.x; i < n; i += NT)
                store_cons(a.U + off, plane, (size_t)i, load_cons<double>(A, plane, (size_t)i));
            __syncthreads();
        }
        if (__any(bad) && lane == 0) atomicOr(a.flag, 1);
    }
}

__global__ void queue_reset_kernel(int* counter) { *counter = 0; }

hipError_t launch_batch(const BatchArgs& a, int threads, int blocks, hipStream_t s)
{
    queue_reset_kernel<<<1, 1, 0, s>>>(a.counter);
    switch (threads) {
        case 64: batch_kernel<64><<<blocks, 64, 0, s>>>(a); break;
        case 128: batch_kernel<128><<<blocks, 128, 0, s>>>(a); break;
        case 256: batch_kernel<256><<<blocks, 256, 0, s>>>(a); break;
        case 512: batch_kernel<512><<<blocks, 512, 0, s>>>(a); break;
        case 1024: batch_kernel<1024><<<blocks, 1024, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int resident_blocks(int threads)
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 256;
    hipError_t e = hipErrorInvalidValue;
    switch (threads) {
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<64>, 64, 0); break;
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<128>, 128, 0); break;
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<256>, 256, 0); break;
        case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<512>, 512, 0); break;
        case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<1024>, 1024, 0); break;
    }
    if (e != hipSuccess || per < 1) per = 1;
    return ncu * per;
}

}  // namespace csh

struct csh_batch {
    int ntubes = 0;
    int64_t N = 0;
    hipStream_t stream = nullptr, capture = nullptr;
    int64_t* offsets = nullptr;
    int* order = nullptr;
    int* counter = nullptr;
    int* flag = nullptr;
    int best_threads = 256;
    int max_len = 0;
    hipGraphExec_t exec = nullptr;
    int g_nsteps = -1, g_threads = 0;
    double g_cfl = 0;
    const void *g_U = nullptr, *g_W = nullptr, *g_dt = nullptr;
};

namespace {

bool valid_threads(int t) { return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024; }

csh::BatchArgs batch_args(csh_batch* b, int nsteps, double cfl, void* U, void* Uw, double* dt_out)
{
    csh::BatchArgs a{};
    a.offsets = b->offsets;
    a.order = b->order;
    a.counter = b->counter;
    a.U = static_cast<double*>(U);
    a.Uw = static_cast<double*>(Uw);
    a.dt_out = dt_out;
    a.N = b->N;
    a.ntubes = b->ntubes;
    a.nsteps = nsteps;
    a.cfl = cfl;
    a.flag = b->flag;
    return a;
}

void drop_graph(csh_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->g_nsteps = -1;
}

}  // namespace

extern "C" int csh_batch_init(csh_batch** out, int ntubes, const int64_t* offsets, int dtype, const void* W,
                              void* U, void* stream)
{
    if (!out) return csh_fail(CSH_ERR_ARG, "b is NULL");
    *out = nullptr;
    if (ntubes < 1 || !offsets) return csh_fail(CSH_ERR_ARG, "ntubes >= 1 and offsets required");
    if (dtype != CSH_F64) return csh_fail(CSH_ERR_ARG, "batched tubes are FP64");
    if (!W || !U) return csh_fail(CSH_ERR_ARG, "W and U must be device pointers");
    if (offsets[0] != 0) return csh_fail(CSH_ERR_ARG, "offsets[0] must be 0");
    std::vector<int> len(ntubes);
    for (int k = 0; k < ntubes; ++k) {
        const int64_t l = offsets[k + 1] - offsets[k];
        if (l < 1 || l > (1LL << 30)) return csh_fail(CSH_ERR_ARG, "every tube needs 1 .. 2^30 cells");
        len[k] = (int)l;
    }
    std::vector<int> order(ntubes);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return len[a] > len[c]; });

    csh_batch* b = new csh_batch;
    b->ntubes = ntubes;
    b->N = offsets[ntubes];
    b->max_len = *std::max_element(len.begin(), len.end());
    b->stream = static_cast<hipStream_t>(stream);
    auto cleanup = [&](int code) {
        csh_batch_destroy(b);
        return code;
    };
    if (hipMalloc(&b->offsets, sizeof(int64_t) * (ntubes + 1)) != hipSuccess ||
        hipMalloc(&b->order, sizeof(int) * ntubes) != hipSuccess || hipMalloc(&b->counter, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->flag, sizeof(int)) != hipSuccess)
        return cleanup(csh_fail(CSH_ERR_HIP, "hipMalloc of the batch tables failed"));
    if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
        return cleanup(csh_fail(CSH_ERR_HIP, "hipStreamCreate failed"));
    hipError_t e = hipMemcpyAsync(b->offsets, offsets, sizeof(int64_t) * (ntubes + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->order, order.data(), sizeof(int) * ntubes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, sizeof(int), b->stream);
    if (e == hipSuccess)
        e = csh::launch_init<double>(static_cast<const double*>(W), static_cast<double*>(U), b->N, b->flag, b->stream);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, b->flag, sizeof(int), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return cleanup(csh_fail(CSH_ERR_HIP, std::string("batch init: ") + hipGetErrorString(e)));
    *out = b;
    if (flag) return csh_fail(CSH_ERR_NONPHYSICAL, "initial state not physical");
    return CSH_OK;
}

extern "C" int csh_batch_run(csh_batch* b, int nsteps, double cfl, void* U, void* U_work, double* dt_out, int threads)
{
    if (!b || !U || !U_work) return csh_fail(CSH_ERR_ARG, "NULL argument");
    if (U == U_work) return csh_fail(CSH_ERR_ARG, "U and U_work must be distinct");
    if (nsteps < 0 || !(cfl > 0)) return csh_fail(CSH_ERR_ARG, "nsteps >= 0 and cfl > 0 required");
    if (threads == 0) threads = b->best_threads;
    if (!valid_threads(threads)) return csh_fail(CSH_ERR_ARG, "threads must be 64, 128, 256, 512 or 1024");
    if (nsteps == 0) return CSH_OK;
    const bool same = b->exec && b->g_nsteps == nsteps && b->g_threads == threads && b->g_cfl == cfl &&
                      b->g_U == U && b->g_W == U_work && b->g_dt == dt_out;
    if (!same) {
        drop_graph(b);
        const int blocks = std::min(b->ntubes, csh::resident_blocks(threads));
        const auto a = batch_args(b, nsteps, cfl, U, U_work, dt_out);
        hipGraph_t g = nullptr;
        CSH_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        hipError_t e = csh::launch_batch(a, threads, blocks, b->capture);
        hipError_t e2 = hipStreamEndCapture(b->capture, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return csh_fail(CSH_ERR_HIP, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return csh_fail(CSH_ERR_HIP, std::string("batch instantiate: ") + hipGetErrorString(e));
        }
        b->g_nsteps = nsteps;
        b->g_threads = threads;
        b->g_cfl = cfl;
        b->g_U = U;
        b->g_W = U_work;
        b->g_dt = dt_out;
    }
    CSH_HIP(hipGraphLaunch(b->exec, b->stream));
    return CSH_OK;
}

extern "C" int csh_batch_status(csh_batch* b)
{
    if (!b) return csh_fail(CSH_ERR_ARG, "NULL argument");
    int flag = 0;
    CSH_HIP(hipMemcpyAsync(&flag, b->flag, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    CSH_HIP(hipStreamSynchronize(b->stream));
    if (flag) return csh_fail(CSH_ERR_NONPHYSICAL, "a tube's state was not physical");
    return CSH_OK;
}

namespace {

// ---- persisted choices of the autotuner --------------------------------------------------------
//
// One line per tuned batch shape, "<key> <threads>", key =
// "arch=<gcnArchName>;cus=<compute units>;tubes=<ntubes>;cells=<total cells>;maxlen=<longest tube>".
// The file is CSH_TUNE_CACHE if set ("off" disables the cache), else
// $HOME/.cache/cshydro/batch_autotune.txt.  Unreadable or malformed lines are
// ignored; a failed write loses nothing but the record.

std::string tune_cache_path()
{
    if (const char* e = std::getenv("CSH_TUNE_CACHE")) return std::string(e) == "off" ? std::string() : std::string(e);
    const char* home = std::getenv("HOME");
    if (!home || !*home) return std::string();
    const std::string dir = std::string(home) + "/.cache/cshydro";
    (void)mkdir((std::string(home) + "/.cache").c_str(), 0755);
    (void)mkdir(dir.c_str(), 0755);
    return dir + "/batch_autotune.txt";
}

std::string tune_key(const csh_batch* b)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    char buf[512];
    std::snprintf(buf, sizeof buf, "arch=%s;cus=%d;tubes=%d;cells=%lld;maxlen=%d", prop.gcnArchName,
                  prop.multiProcessorCount, b->ntubes, (long long)b->N, b->max_len);
    return std::string(buf);
}

int tune_lookup(const std::string& path, const std::string& key)
{
    if (path.empty() || key.empty()) return 0;
    std::ifstream f(path);
    std::string line;
    int found = 0;
    while (std::getline(f, line)) {
        if (line.size() > key.size() && line.compare(0, key.size(), key) == 0 && line[key.size()] == ' ') {
            const int t = std::atoi(line.c_str() + key.size() + 1);
            if (valid_threads(t)) found = t;  // the last record wins
        }
    }
    return found;
}

void tune_record(const std::string& path, const std::string& key, int threads)
{
    if (path.empty() || key.empty()) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << threads << '\n';
}

}  // namespace

extern "C" int csh_batch_autotune(csh_batch* b, int probe_steps, double cfl, const void* U, int* best_threads)
{
    if (!b || !U || !best_threads) return csh_fail(CSH_ERR_ARG, "NULL argument");
    if (probe_steps < 1 || !(cfl > 0)) return csh_fail(CSH_ERR_ARG, "probe_steps >= 1 and cfl > 0 required");
    const std::string path = tune_cache_path(), key = tune_key(b);
    if (const int cached = tune_lookup(path, key)) {
        b->best_threads = cached;
        *best_threads = cached;
        return CSH_OK;
    }
    const size_t bytes = sizeof(double) * 6 * (size_t)b->N;
    double *A = nullptr, *B = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (A) (void)hipFree(A);
        if (B) (void)hipFree(B);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&A, bytes) != hipSuccess || hipMalloc(&B, bytes) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        return csh_fail(CSH_ERR_HIP, "autotune: allocation failed");
    }
    const int cands[] = {64, 128, 256, 512, 1024};
    float best_ms = 0;
    int best = 0;
    for (int t : cands) {
        const int blocks = std::min(b->ntubes, csh::resident_blocks(t));
        const auto a = batch_args(b, probe_steps, cfl, A, B, nullptr);
        float ms = 0;
        hipError_t e = hipMemcpyAsync(A, U, bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = csh::launch_batch(a, t, blocks, b->stream);  // warm
        if (e == hipSuccess) e = hipMemcpyAsync(A, U, bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = csh::launch_batch(a, t, blocks, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            release();
            return csh_fail(CSH_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
        }
        if (best == 0 || ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    release();
    b->best_threads = best;
    *best_threads = best;
    tune_record(path, key, best);
    return CSH_OK;
}

extern "C" int csh_batch_destroy(csh_batch* b)
{
    if (!b) return CSH_OK;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->offsets) (void)hipFree(b->offsets);
    if (b->order) (void)hipFree(b->order);
    if (b->counter) (void)hipFree(b->counter);
    if (b->flag) (void)hipFree(b->flag);
    delete b;
    return CSH_OK;
}
