// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace csh {

// Device scalars of the timestep reduction.  Step n reads slot n % 3 (the
// rate s of its input and the time t), accumulates the rate of its output
// into slot (n + 1) % 3 and clears slot (n + 2) % 3 for the step after.
struct Slot {
    unsigned long long s_bits;  // max CFL rate as the bit pattern of a positive double
    double t;                   // simulation time of the state this slot describes
    double dt;                  // timestep a multi-stage step chose in its first stage
    double pad;
};

constexpr int kStrip = 60;  // output columns per wavefront (64 lanes, 2 halo lanes per side)
constexpr int kWaves = 4;   // wavefronts per workgroup of the sweep kernels

template <typename T>
struct StepArgs {
    const T* U;   // input state [6][ny][nx]
    T* Unew;      // output state (step) -- may not alias U
    T* Fx;        // face fluxes (flux mode): [6][ny][nx+1], column i = face i-1/2
    T* Fy;        // [6][ny+1][nx], row j = face j-1/2
    int nx, ny, bcx, bcy;
    double dx, dy;
    int nstrips, nsegs, ty;  // strips of kStrip columns, segments of ty rows
    double dt;               // timestep when dev_dt == 0
    int dev_dt;              // 1: dt = min(cfl / s, t_end - t) from slots[s_in]
    double cfl, t_end;       // t_end <= 0: no end time
    Slot* slots;
    int s_in, s_out, s_reset;
    double* dt_log;          // if set, receives the timestep used
    const double* dt_in;     // if set (and dev_dt == 0), the timestep is read from here
    double vc2, rc2, x0, y0; // external flat-rotation-curve potential (vc2 == 0: none)
    int* flag;               // set to 1 if an output cell is not physical
    const T* Ubase;          // two-stage schemes: state the stage update starts from (null: U)
};

// solver: 0 HLL, 1 HLLC
template <typename T>
hipError_t launch_step(const StepArgs<T>& a, bool twod, bool fluxes, int solver, hipStream_t s);

template <typename T>
hipError_t launch_init(const T* W, T* U, int64_t n, int* flag, hipStream_t s);

template <typename T>
hipError_t launch_maxspeed(const T* U, int nx, int ny, double dx, double dy, Slot* slot, int* flag,
                           hipStream_t s);

hipError_t launch_reset(Slot* slots, int nslots, double t0, hipStream_t s);

// Kurganov-Tadmor stage on a 1-D grid: first (half step into the stage
// buffer, records dt in slots[s_in].dt) or final (full step from Ubase with
// the stage state's fluxes)
template <typename T>
hipError_t launch_kt(const StepArgs<T>& a, bool final_stage, hipStream_t s);

// Kurganov-Tadmor step on a 2-D grid, both stages in one launch (its own
// strips and row segments; the arguments' decomposition fields are ignored)
template <typename T>
hipError_t launch_kt_fused(StepArgs<T> a, hipStream_t s);

template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t s);

}  // namespace csh
