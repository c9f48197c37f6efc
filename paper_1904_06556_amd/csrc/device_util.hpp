// Device helpers shared by the kernel sources of libvts: indexing, the
// penalty-barrier function of Section 3.1, fixed-order block reductions and
// the gather of an element's DOF values.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "vts_internal.hpp"

namespace vts {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t gid() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ int64_t node_id(int i, int j, int k, int NX, int NY) {
    return (int64_t)i + (int64_t)NX * ((int64_t)j + (int64_t)NY * k);
}

// Penalty-barrier function of Ben-Tal and Zibulevsky with tau_hat = -1/2
// (Section 3.1): quadratic for t >= -1/2, logarithmic branch below.
__device__ __forceinline__ double pen_phi(double t) {
    return t >= -0.5 ? t + 0.5 * t * t : -0.25 * log(-2.0 * t) - 0.375;
}
__device__ __forceinline__ double pen_dphi(double t) {
    return t >= -0.5 ? 1.0 + t : -0.25 / t;
}
__device__ __forceinline__ double pen_d2phi(double t) {
    return t >= -0.5 ? 1.0 : 0.25 / (t * t);
}
// phi(t + dt) - phi(t) without subtracting two values of phi when both points
// lie on one branch: dt (1 + t + dt/2) (quadratic), -1/4 log1p(dt/t) (log)
__device__ __forceinline__ double pen_phi_diff(double t, double dt) {
    const double t1 = t + dt;
    if (t >= -0.5 && t1 >= -0.5) return dt * (1.0 + t + 0.5 * dt);
    if (t < -0.5 && t1 < -0.5) return -0.25 * log1p(dt / t);
    return pen_phi(t1) - pen_phi(t);
}

// block-wide sum of NQ values per thread; thread 0 writes partials[q*kRedBlocks + block]
template <int NQ>
__device__ __forceinline__ void block_sum_store(double (&v)[NQ], double* partials, int slot0,
                                                uint32_t maxmask = 0) {
    __shared__ double sh[NQ][kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double x = v[q];
        const bool mx = (maxmask >> q) & 1u;
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(x, off, 64);
            x = mx ? fmax(x, o) : x + o;
        }
        if (lane == 0) sh[q][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const bool mx = (maxmask >> q) & 1u;
            double x = sh[q][0];
            for (int k = 1; k < kThreads / 64; ++k) x = mx ? fmax(x, sh[q][k]) : x + sh[q][k];
            partials[(slot0 + q) * kRedBlocks + blockIdx.x] = x;
        }
    }
}

static inline int red_grid(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    return (int)(b < kRedBlocks ? b : kRedBlocks);
}
static inline int grid1d(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : b);
}

// Sum (or max) of partials[slot*kRedBlocks + b] over b < nb, fixed order.
__device__ __forceinline__ void finalize_body(const double* __restrict__ partials, int nb,
                                              int slot0, uint32_t maxmask,
                                              double* __restrict__ out) {
    const int q = slot0 + blockIdx.x;
    const bool mx = (maxmask >> blockIdx.x) & 1u;
    double x = mx ? -DBL_MAX : 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double v = partials[q * kRedBlocks + b];
        x = mx ? fmax(x, v) : x + v;
    }
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                                  : sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
}

// gather the 24 (masked) DOF values of element (i,j,k)
__device__ __forceinline__ void gather_elem(const double* __restrict__ x,
                                            const uint8_t* __restrict__ fixed, int i, int j,
                                            int k, int NX, int NY, double (&xe)[24]) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int64_t nb = node_id(i + (b & 1), j + ((b >> 1) & 1), k + (b >> 2), NX, NY);
#pragma unroll
        for (int c = 0; c < 3; ++c) xe[3 * b + c] = fixed[3 * nb + c] ? 0.0 : x[3 * nb + c];
    }
}

__device__ __forceinline__ void elem_ijk(int64_t e, int nx, int ny, int& i, int& j, int& k) {
    i = (int)(e % nx);
    const int64_t t = e / nx;
    j = (int)(t % ny);
    k = (int)(t / ny);
}

}  // namespace vts
