// Declarations of the Fourier-amplitude diagnostic (Sec. 4.4).
#pragma once

#include <hip/hip_runtime.h>

namespace csh {

// Global Fourier amplitudes of the density plane (diagnostic of Sec. 4.4)
constexpr int kFourierMaxM = 16;     // highest mode
constexpr int kFourierBlocks = 1024; // fixed workgroup count: the sums' order does not depend on the device

template <typename T>
struct FourierArgs {
    const T* rho;        // density plane [ny][nx]
    int nx, ny;
    double dx, dy, x0, y0;  // cell (i, j) centred at (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy)
    double X, Y;         // region [-X, X] x [-Y, Y]
    int m_max;
    double* partials;    // [1 + 2 m_max][kFourierBlocks] (value-major)
    double* A;           // [m_max] amplitudes A_1..A_m_max (device)
};

template <typename T>
hipError_t launch_fourier(const FourierArgs<T>& a, hipStream_t s);

// Partial-sum rows of the allocation-free variant: a statically sized device
// array, kFourierBlocks x (1 + 2 kFourierMaxM) doubles per GPU.  Returns its
// address on the current device (looked up once per device), or an error.
hipError_t fourier_static_partials(double** ptr);

}  // namespace csh
