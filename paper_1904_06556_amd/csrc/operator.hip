// The element operator K(rho) x = sum_i rho_i K_i x (problem (1.1)) and the
// Schur complement S [x; beta] of eq. (3.12), applied element by element.
//
// Arithmetic: for the cube element, K_e is sparse in the per-direction
// sum/difference basis.  With H8 the 8x8 Hadamard matrix over the nodes
// (node a = ax + 2 ay + 4 az, H8[m][a] = (-1)^(m.a)) and H = H8 x I3,
//     K_e = H Kh H,   Kh = H K_e H / 64,
// and Kh has 45 non-zeros (the constant mode is the rigid translation; the
// linear modes {x, y, z}, the bilinear modes {xy, xz, yz} and the trilinear
// mode xyz do not couple across groups).  One application costs two
// butterflies (72 add/sub each) and 45 multiply-adds instead of 576.
//
// Data movement: a workgroup owns a 15x15 column of nodes and marches along
// z.  Each step stages one node plane of x in LDS (double-buffered); the 256
// threads each process one element column; the top-face outputs of an element
// stay in registers and become the bottom-face contributions of the next
// plane; the four elements around a node meet through per-corner LDS slots
// summed in a fixed order, so results are deterministic without atomics.
#include <hip/hip_runtime.h>

#include "vts_internal.hpp"

namespace vts {

namespace {

constexpr int TXE = 16, TYE = 16;                 // element columns per workgroup
constexpr int NXL = TXE + 1, NYL = TYE + 1;       // nodes per tile row / column
constexpr int kTileThreads = TXE * TYE;

// Kh in closed form.  Cubic symmetry leaves eight distinct coefficients in
// the 45-entry pattern (host_fe.cpp computes Kh from K_e and checks that it has
// exactly this structure):
//   linear modes x=1, y=2, z=4 (index 3*mode + component):
//     normal  n_d = (mode 2^d, comp d):  y(n_d) = A x(n_d) + B sum_{d'!=d} x(n_d')
//     shear   (1,1)-(2,0), (1,2)-(4,0), (2,2)-(4,1): both rows C (x_a + x_b)
//   bilinear modes xy=3, xz=5, yz=6:
//     (3,0)-(6,2), (3,1)-(5,2), (5,0)-(6,1): [[D, E], [E, D]]
//     (3,2), (5,1), (6,0):                   F on the diagonal, G off it
//   trilinear mode 7: H on the diagonal.
template <typename T>
struct KhVals {
    T A, B, C, D, E, F, G, H;
};

// in-place butterflies over the 8 nodes of each component: v <- H v
template <typename T>
__device__ __forceinline__ void hadamard24(T (&v)[24]) {
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if (a & bit) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T p = v[3 * a + c], q = v[3 * (a | bit) + c];
                v[3 * a + c] = p + q;
                v[3 * (a | bit) + c] = p - q;
            }
        }
    }
}

// v <- s * K_e v, in place (keeps one 24-vector live)
template <typename T>
__device__ __forceinline__ void ke_apply(const KhVals<T>& k, T s, T (&v)[24]) {
    hadamard24(v);
#pragma unroll
    for (int q = 3; q < 24; ++q) v[q] *= s;
    v[0] = v[1] = v[2] = T(0);
    // linear modes: normals 3, 7, 14; shears (4,6), (5,12), (8,13)
    const T vol = k.B * (v[3] + v[7] + v[14]);
    const T AmB = k.A - k.B;
    v[3] = AmB * v[3] + vol;
    v[7] = AmB * v[7] + vol;
    v[14] = AmB * v[14] + vol;
    const T sxy = k.C * (v[4] + v[6]);
    const T sxz = k.C * (v[5] + v[12]);
    const T syz = k.C * (v[8] + v[13]);
    v[4] = sxy;
    v[6] = sxy;
    v[5] = sxz;
    v[12] = sxz;
    v[8] = syz;
    v[13] = syz;
    // bilinear pairs (9,20), (10,17), (15,19)
    T p0 = v[9], p1 = v[20];
    v[9] = k.D * p0 + k.E * p1;
    v[20] = k.E * p0 + k.D * p1;
    p0 = v[10];
    p1 = v[17];
    v[10] = k.D * p0 + k.E * p1;
    v[17] = k.E * p0 + k.D * p1;
    p0 = v[15];
    p1 = v[19];
    v[15] = k.D * p0 + k.E * p1;
    v[19] = k.E * p0 + k.D * p1;
    // bilinear triple 11, 16, 18
    const T tri = k.G * (v[11] + v[16] + v[18]);
    const T FmG = k.F - k.G;
    v[11] = FmG * v[11] + tri;
    v[16] = FmG * v[16] + tri;
    v[18] = FmG * v[18] + tri;
    // trilinear
    v[21] *= k.H;
    v[22] *= k.H;
    v[23] *= k.H;
    hadamard24(v);
}

struct TileGeom {
    int nx, ny, nz;
    int tiles_x, tiles_y, kz;     // tiles in x, y; owned node planes per workgroup
};

__device__ __forceinline__ int64_t nid(int i, int j, int k, int NX, int NY) {
    return (int64_t)i + (int64_t)NX * ((int64_t)j + (int64_t)NY * k);
}

// Node plane k of the tile (nodes [X0-1, X0-1+TXE] x [Y0-1, Y0-1+TYE]) of one
// or two vectors into LDS, masked, zero outside the grid.  LDS layout
// [vector][component][node], node = ly*NXL + lx, so lanes reading
// neighbouring nodes hit neighbouring banks.
constexpr int kPlaneNodes = NXL * NYL;
constexpr int kPlaneVals = kPlaneNodes * 3;

constexpr int kPerThread = (kPlaneVals + kTileThreads - 1) / kTileThreads;

template <typename T, int NV>
struct PlaneRegs {
    T v[NV][kPerThread];
};

// issue the global loads of node plane k (masked, zero outside the grid)
template <typename T, int NV>
__device__ __forceinline__ void fetch_plane(const TileGeom& g, int X0, int Y0, int k,
                                            const T* const (&src)[NV],
                                            const uint8_t* __restrict__ fixed,
                                            PlaneRegs<T, NV>& pr) {
    const int NX = g.nx + 1, NY = g.ny + 1;
#pragma unroll
    for (int s = 0; s < kPerThread; ++s) {
        const int q = threadIdx.x + s * kTileThreads;
        const int c = q % 3, nd = q / 3;
        const int lx = nd % NXL, ly = nd / NXL;
        const int i = X0 - 1 + lx, j = Y0 - 1 + ly;
        const bool in = q < kPlaneVals && k >= 0 && k <= g.nz && i >= 0 && i < NX && j >= 0 &&
                        j < NY;
        const int dof = in ? 3 * (i + NX * (j + NY * k)) + c : 0;
        const bool keep = in && fixed[dof] == 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T val = in ? src[v][dof] : T(0);
            pr.v[v][s] = keep ? val : T(0);
        }
    }
}

template <typename T, int NV>
__device__ __forceinline__ void commit_plane(const PlaneRegs<T, NV>& pr, T (*dst)[kPlaneVals]) {
#pragma unroll
    for (int s = 0; s < kPerThread; ++s) {
        const int q = threadIdx.x + s * kTileThreads;
        if (q < kPlaneVals) {
            const int c = q % 3, nd = q / 3;
#pragma unroll
            for (int v = 0; v < NV; ++v) dst[v][c * kPlaneNodes + nd] = pr.v[v][s];
        }
    }
}

// the element's 24 local values of staged vector v: bottom face from plane
// buffer `lo`, top face from `hi`
template <typename T>
__device__ __forceinline__ T elem_val(const T* lo, const T* hi, int tx, int ty, int q) {
    const int a = q / 3, c = q % 3;
    const T* P = (a & 4) ? hi : lo;
    return P[c * kPlaneNodes + (ty + ((a >> 1) & 1)) * NXL + tx + (a & 1)];
}

// Plane contributions of one element column (its 4 nodes (tx+ax, ty+ay), 3
// components each, in v[3*(ax + 2 ay) + c]) are summed into node values.
// x-neighbours meet through a lane shuffle (a tile row is 16 consecutive
// lanes of one wave), y-neighbours through the LDS row buffer `part`
// (one value per node and component).  Fixed order, no atomics.
template <typename T>
__device__ __forceinline__ void combine_store(const T (&v)[12], T* part, int tx, int ty,
                                              bool store, int64_t n,
                                              const uint8_t* __restrict__ fixed,
                                              T* __restrict__ y) {
    T row0[3], row1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // node (tx, ty+ay) gets own ax=0 part and the ax=1 part of lane tx-1
        const T left0 = __shfl_up(v[3 * 1 + c], 1, 16);
        const T left1 = __shfl_up(v[3 * 3 + c], 1, 16);
        row0[c] = v[3 * 0 + c] + (tx >= 1 ? left0 : T(0));
        row1[c] = v[3 * 2 + c] + (tx >= 1 ? left1 : T(0));
        part[c * kPlaneNodes + (ty + 1) * NXL + tx] = row1[c];
    }
    __syncthreads();
    if (store) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T s = row0[c] + part[c * kPlaneNodes + ty * NXL + tx];
            y[3 * n + c] = fixed[3 * n + c] ? T(0) : s;
        }
    }
}

// ---------------------------------------------------------------------------
// y = K(rho) x
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kTileThreads)
k_apply_K_tile(TileGeom g, KhVals<T> kh, const T* __restrict__ x, const T* __restrict__ rho,
               const uint8_t* __restrict__ fixed, T* __restrict__ y) {
    __shared__ T xs[2][1][kPlaneVals];
    __shared__ T part[kPlaneVals];
    const int tx = threadIdx.x % TXE, ty = threadIdx.x / TXE;
    const int b = blockIdx.x;
    const int bx = b % g.tiles_x, by = (b / g.tiles_x) % g.tiles_y, bz = b / (g.tiles_x * g.tiles_y);
    const int X0 = bx * (TXE - 1), Y0 = by * (TYE - 1);
    const int K0 = bz * g.kz;
    const int K1 = min(K0 + g.kz, g.nz + 1);
    const int ex = X0 - 1 + tx, ey = Y0 - 1 + ty;
    const bool col_ok = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
    const int NX = g.nx + 1, NY = g.ny + 1;
    const int i = X0 - 1 + tx, j = Y0 - 1 + ty;
    const bool owner = tx >= 1 && ty >= 1 && i < NX && j < NY;
    const T* const src[1] = {x};

    PlaneRegs<T, 1> pre;
    T topacc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) topacc[q] = T(0);
    fetch_plane<T, 1>(g, X0, Y0, K0 - 1, src, fixed, pre);
    commit_plane<T, 1>(pre, xs[(K0 - 1) & 1]);
    fetch_plane<T, 1>(g, X0, Y0, K0, src, fixed, pre);
    for (int l = K0 - 1; l < K1; ++l) {
        // plane l+1 (top of layer l) to LDS; plane l+2 starts loading
        commit_plane<T, 1>(pre, xs[(l + 1) & 1]);
        if (l + 1 < K1) fetch_plane<T, 1>(g, X0, Y0, l + 2, src, fixed, pre);
        const bool el_ok = col_ok && l >= 0 && l < g.nz;
        const T r = el_ok ? rho[ex + g.nx * (ey + g.ny * l)] : T(0);
        __syncthreads();
        T v[24];
        const T* lo = xs[l & 1][0];
        const T* hi = xs[(l + 1) & 1][0];
#pragma unroll
        for (int q = 0; q < 24; ++q) v[q] = elem_val(lo, hi, tx, ty, q);
        ke_apply(kh, r, v);                    // r = 0 outside the grid
        // plane l: bottom face of layer l + top face of layer l-1
        T face[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            face[q] = v[q] + topacc[q];
            topacc[q] = v[12 + q];
        }
        combine_store(face, part, tx, ty, l >= K0 && owner,
                      (int64_t)i + NX * ((int64_t)j + NY * l), fixed, y);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// S [x; beta] = [K(rho') x + sum_e w_e b_e (b_e^T x - beta); -sum_e w_e (b_e^T x - beta)]
// with b_e = K_e u_e recomputed: y_e = K_e (rho'_e x_e + w_e t_e u_e),
// t_e = (K_e u_e)^T x_e - beta.  Per-block partial sums of w_e t_e.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kTileThreads)
k_apply_S_tile(TileGeom g, KhVals<T> kh, const T* __restrict__ x, const T* __restrict__ u,
               const T* __restrict__ r1, const T* __restrict__ w, const uint8_t* __restrict__ fixed,
               int64_t ndof, T* __restrict__ y, double* __restrict__ partials) {
    __shared__ T xs[2][2][kPlaneVals];
    __shared__ T part[kPlaneVals];
    __shared__ double red[kTileThreads / 64];
    const int tx = threadIdx.x % TXE, ty = threadIdx.x / TXE;
    const int b = blockIdx.x;
    const int bx = b % g.tiles_x, by = (b / g.tiles_x) % g.tiles_y, bz = b / (g.tiles_x * g.tiles_y);
    const int X0 = bx * (TXE - 1), Y0 = by * (TYE - 1);
    const int K0 = bz * g.kz;
    const int K1 = min(K0 + g.kz, g.nz + 1);
    const int ex = X0 - 1 + tx, ey = Y0 - 1 + ty;
    const bool col_ok = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
    const int NX = g.nx + 1, NY = g.ny + 1;
    const int i = X0 - 1 + tx, j = Y0 - 1 + ty;
    const bool owner = tx >= 1 && ty >= 1 && i < NX && j < NY;
    const T beta = x[ndof];
    const T* const src[2] = {x, u};
    double wsum = 0.0;

    PlaneRegs<T, 2> pre;
    T topacc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) topacc[q] = T(0);
    fetch_plane<T, 2>(g, X0, Y0, K0 - 1, src, fixed, pre);
    commit_plane<T, 2>(pre, xs[(K0 - 1) & 1]);
    fetch_plane<T, 2>(g, X0, Y0, K0, src, fixed, pre);
    for (int l = K0 - 1; l < K1; ++l) {
        commit_plane<T, 2>(pre, xs[(l + 1) & 1]);
        if (l + 1 < K1) fetch_plane<T, 2>(g, X0, Y0, l + 2, src, fixed, pre);
        const bool el_ok = col_ok && l >= 0 && l < g.nz;
        const int e = el_ok ? ex + g.nx * (ey + g.ny * l) : 0;
        const T rr = el_ok ? r1[e] : T(0), ww = el_ok ? w[e] : T(0);
        __syncthreads();
        const T* xlo = xs[l & 1][0];
        const T* xhi = xs[(l + 1) & 1][0];
        const T* ulo = xs[l & 1][1];
        const T* uhi = xs[(l + 1) & 1][1];
        T v[24];
        // b_e = K_e u_e, t = b_e . x_e - beta
#pragma unroll
        for (int q = 0; q < 24; ++q) v[q] = elem_val(ulo, uhi, tx, ty, q);
        ke_apply(kh, T(1), v);
        T t = T(0);
#pragma unroll
        for (int q = 0; q < 24; ++q) t += v[q] * elem_val(xlo, xhi, tx, ty, q);
        t -= beta;
        const T wt = ww * t;                   // 0 outside the grid
        // the tile's halo elements are counted by their owning tile
        if (el_ok && tx >= 1 && ty >= 1 && l >= K0) wsum += (double)wt;
#pragma unroll
        for (int q = 0; q < 24; ++q)
            v[q] = rr * elem_val(xlo, xhi, tx, ty, q) + wt * elem_val(ulo, uhi, tx, ty, q);
        ke_apply(kh, T(1), v);
        T face[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            face[q] = v[q] + topacc[q];
            topacc[q] = v[12 + q];
        }
        combine_store(face, part, tx, ty, l >= K0 && owner,
                      (int64_t)i + NX * ((int64_t)j + NY * l), fixed, y);
        __syncthreads();
    }
    // block partial of sum w t
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_down(wsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < kTileThreads / 64; ++q) s += red[q];
        partials[blockIdx.x] = s;
    }
}

// deterministic sum of nb partials into dst (negated: the alpha row of S)
__global__ void k_sum_neg(const double* __restrict__ partials, int nb, double* __restrict__ dst) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) s += partials[q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[0] = -sh[0];
}

TileGeom geom_of(const Ctx& c, int kz) {
    TileGeom g;
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = c.nz;
    g.tiles_x = (c.nx + 1 + TXE - 2) / (TXE - 1);
    g.tiles_y = (c.ny + 1 + TYE - 2) / (TYE - 1);
    g.kz = kz;
    return g;
}

// owned node planes per workgroup: enough workgroups to fill the chip
int choose_kz(const Ctx& c) {
    const int cols = ((c.nx + TXE - 1) / (TXE - 1)) * ((c.ny + TYE - 1) / (TYE - 1));
    int kz = 16;
    while (kz > 2 && (int64_t)cols * ((c.nz + 1 + kz - 1) / kz) < 2048) kz /= 2;
    return kz;
}

}  // namespace

bool tile_ok(const Ctx& c) { return c.kh_ok; }

void launch_apply_K_tile_f64(Ctx& c, const double* rho, const double* x, double* y) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    KhVals<double> kh{c.kh8[0], c.kh8[1], c.kh8[2], c.kh8[3], c.kh8[4], c.kh8[5], c.kh8[6], c.kh8[7]};
    const int nb = g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
    hipLaunchKernelGGL(k_apply_K_tile<double>, dim3(nb), dim3(kTileThreads), 0, c.s, g, kh, x, rho,
                       c.fixed, y);
}

void launch_apply_K_tile_f32(Ctx& c, const float* rho, const float* x, float* y) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    KhVals<float> kh{(float)c.kh8[0], (float)c.kh8[1], (float)c.kh8[2], (float)c.kh8[3],
                     (float)c.kh8[4], (float)c.kh8[5], (float)c.kh8[6], (float)c.kh8[7]};
    const int nb = g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
    hipLaunchKernelGGL(k_apply_K_tile<float>, dim3(nb), dim3(kTileThreads), 0, c.s, g, kh, x, rho,
                       c.fixed, y);
}

int apply_S_tile_blocks(const Ctx& c) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    return g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
}

void launch_apply_S_tile(Ctx& c, const double* x, double* y) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    KhVals<double> kh{c.kh8[0], c.kh8[1], c.kh8[2], c.kh8[3], c.kh8[4], c.kh8[5], c.kh8[6], c.kh8[7]};
    const int nb = g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
    hipLaunchKernelGGL(k_apply_S_tile<double>, dim3(nb), dim3(kTileThreads), 0, c.s, g, kh, x, c.u,
                       c.r1, c.w, c.fixed, c.ndof, y, c.spart);
    hipLaunchKernelGGL(k_sum_neg, dim3(1), dim3(256), 0, c.s, c.spart, nb, y + c.ndof);
}

}  // namespace vts
