// The element operator K(rho) x = sum_i rho_i K_i x (problem (1.1)) and the
// Schur complement S [x; beta] of eq. (3.12), applied element by element.
//
// Arithmetic: for the cube element, K_e is sparse in the per-direction
// sum/difference basis.  With H8 the 8x8 Hadamard matrix over the nodes
// (node a = ax + 2 ay + 4 az, H8[m][a] = (-1)^(m.a)) and H = H8 x I3,
//     K_e = H Kh H,   Kh = H K_e H / 64,
// and Kh has 45 non-zeros (the constant mode is the rigid translation; the
// linear modes {x, y, z}, the bilinear modes {xy, xz, yz} and the trilinear
// mode xyz do not couple across groups).  H8 = Hz x Hy x Hx factors by
// direction, so the x-y part of the transform of a node plane's 2x2 face is
// shared by the element below and the element above that face.
//
// K(rho) x (k_apply_K_plane): a workgroup owns a 15x15 column of nodes and
// marches through a range of node planes.  Node planes are loaded two
// planes ahead into registers and staged through a ring of three LDS
// buffers, so each plane costs one barrier.  Per element: the 2x2 face
// transforms of its bottom face (kept from the previous plane) and top face
// are combined into the 8 modes, multiplied by rho Kh, and split back into
// the two faces; the face sums of two consecutive elements are transformed
// back to nodes once per plane.  x-neighbours meet through a DPP row shift,
// y-neighbours through LDS, in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

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
// y = K(rho) x, plane-marching form
// ---------------------------------------------------------------------------
constexpr int kPN = NXL * NYL;                 // nodes of a staged plane (17 x 17)
constexpr int kPV = 3 * kPN;                   // values of a staged plane
constexpr int kLoads = (kPV + kTileThreads - 1) / kTileThreads;
constexpr int kRing = 3;                       // LDS plane buffers

struct PlaneGeom {
    int nx, ny, nz;                            // elements
    int tiles_x, tiles_y, zblocks, nblocks;    // workgroup tiles (x, y) and z ranges
    int per_xcd;                               // logical blocks per XCD (grid = 8 per_xcd)
};

// consecutive hardware workgroups go to the 8 XCDs in turn; this maps them so
// that each XCD works on a contiguous range of tiles (shared halos stay in
// that XCD's L2).  Returns -1 for the padding workgroups.
__device__ __forceinline__ int logical_block(const PlaneGeom& g) {
    const int b = blockIdx.x;
    const int lb = (b & 7) * g.per_xcd + (b >> 3);
    return lb < g.nblocks ? lb : -1;
}

// DPP row shift right by one lane within rows of 16 lanes (lane 0 of a row gets 0)
__device__ __forceinline__ float row_shr1(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, false));
}
__device__ __forceinline__ double row_shr1(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x111, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x111, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// per-thread part of one staged plane: values q = tid + 256 s (s < kLoads)
// of the 17x17x3 block, row-major over the tile's node rows with xyz per
// node.  The LDS buffer has the same layout, so value q goes to index q.
struct PlaneSlots {
    int goff[kLoads];      // DOF offset within the grid plane
    int noff[kLoads];      // node offset within the grid plane
    uint32_t comp;         // 2 bits per slot: component of the value
    uint32_t valid;        // bit s: the node is inside the grid
};

__device__ __forceinline__ PlaneSlots plane_slots(int X0, int Y0, int NX, int NY) {
    PlaneSlots ps;
    ps.valid = 0;
    ps.comp = 0;
#pragma unroll
    for (int s = 0; s < kLoads; ++s) {
        const int q = threadIdx.x + s * kTileThreads;
        const int row = q / (3 * NXL), col = q - row * (3 * NXL);
        const int lx = col / 3, c = col - 3 * lx;
        const int i = X0 - 1 + lx, j = Y0 - 1 + row;
        const bool in = q < kPV && i >= 0 && i < NX && j >= 0 && j < NY;
        ps.goff[s] = in ? 3 * (j * NX + i) + c : 0;
        ps.noff[s] = in ? j * NX + i : 0;
        ps.comp |= (uint32_t)c << (2 * s);
        ps.valid |= in ? (1u << s) : 0u;
    }
    return ps;
}

template <typename T>
struct PlaneRegsK {
    T v[kLoads];
    uint32_t fx[kLoads];   // node mask bytes
};

template <typename T>
__device__ __forceinline__ void plane_fetch(const PlaneSlots& ps, const T* __restrict__ x,
                                            const uint8_t* __restrict__ nmask, int64_t pnode,
                                            PlaneRegsK<T>& r) {
    const T* xp = x + 3 * pnode;
    const uint8_t* mp = nmask + pnode;
#pragma unroll
    for (int s = 0; s < kLoads; ++s) {
        const bool in = (ps.valid >> s) & 1u;
        r.v[s] = in ? xp[ps.goff[s]] : T(0);
        r.fx[s] = in ? (uint32_t)mp[ps.noff[s]] : 0u;
    }
}

// masked values into LDS buffer `buf`; the node mask bytes into `mb` (one
// per node, by the thread holding the node's x component)
template <typename T>
__device__ __forceinline__ void plane_commit(const PlaneSlots& ps, const PlaneRegsK<T>& r, T* buf,
                                             uint8_t* mb) {
#pragma unroll
    for (int s = 0; s < kLoads; ++s) {
        const int q = threadIdx.x + s * kTileThreads;
        if (s < kLoads - 1 || q < kPV) {
            const uint32_t c = (ps.comp >> (2 * s)) & 3u;
            buf[q] = ((r.fx[s] >> c) & 1u) ? T(0) : r.v[s];
            if (c == 0) mb[q / 3] = (uint8_t)r.fx[s];
        }
    }
}

// 2x2 face transform of the element column's nodes (tx..tx+1, ty..ty+1) of a
// staged plane, per component: F[c][mxy], mxy = 0 (sum), 1 (x), 2 (y), 3 (xy)
template <typename T>
__device__ __forceinline__ void face_fwd(const T* buf, int tx, int ty, T (&F)[3][4]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T* p = buf + 3 * (ty * NXL + tx) + c;
        const T a = p[0], b = p[3], d = p[3 * NXL], e = p[3 * NXL + 3];
        const T s1 = a + b, d1 = a - b, s2 = d + e, d2 = d - e;
        F[c][0] = s1 + s2;
        F[c][1] = d1 + d2;
        F[c][2] = s1 - s2;
        F[c][3] = d1 - d2;
    }
}

// the element's modes from its bottom/top face transforms, rho Kh applied, and
// the result split back into bottom (Gb) and top (Gt) face transforms
template <typename T>
__device__ __forceinline__ void elem_modes(const KhVals<T>& k, T r, const T (&Fb)[3][4],
                                           const T (&Ft)[3][4], T (&Gb)[3][4], T (&Gt)[3][4]) {
    T v[24];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[3 * m + c] = Fb[c][m] + Ft[c][m];
            v[3 * (m + 4) + c] = Fb[c][m] - Ft[c][m];
        }
    const T AmB = r * (k.A - k.B), rB = r * k.B, rC = r * k.C, rD = r * k.D, rE = r * k.E;
    const T FmG = r * (k.F - k.G), rG = r * k.G, rH = r * k.H;
    T y[24];
    y[0] = y[1] = y[2] = T(0);
    const T vol = rB * (v[3] + v[7] + v[14]);
    y[3] = AmB * v[3] + vol;
    y[7] = AmB * v[7] + vol;
    y[14] = AmB * v[14] + vol;
    y[4] = y[6] = rC * (v[4] + v[6]);
    y[5] = y[12] = rC * (v[5] + v[12]);
    y[8] = y[13] = rC * (v[8] + v[13]);
    y[9] = rD * v[9] + rE * v[20];
    y[20] = rE * v[9] + rD * v[20];
    y[10] = rD * v[10] + rE * v[17];
    y[17] = rE * v[10] + rD * v[17];
    y[15] = rD * v[15] + rE * v[19];
    y[19] = rE * v[15] + rD * v[19];
    const T tri = rG * (v[11] + v[16] + v[18]);
    y[11] = FmG * v[11] + tri;
    y[16] = FmG * v[16] + tri;
    y[18] = FmG * v[18] + tri;
    y[21] = rH * v[21];
    y[22] = rH * v[22];
    y[23] = rH * v[23];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Gb[c][m] = y[3 * m + c] + y[3 * (m + 4) + c];
            Gt[c][m] = y[3 * m + c] - y[3 * (m + 4) + c];
        }
}

// plane contributions in face-transform form -> node values of the column's
// row0 node (tx, ty) and row1 node (tx, ty+1), x-neighbours combined
template <typename T>
__device__ __forceinline__ void face_inv_combine(const T (&P)[3][4], T (&row0)[3], T (&row1)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T u0 = P[c][0] + P[c][1], u1 = P[c][0] - P[c][1];
        const T u2 = P[c][2] + P[c][3], u3 = P[c][2] - P[c][3];
        // (ax, ay) = (0,0), (1,0), (0,1), (1,1)
        const T n00 = u0 + u2, n10 = u1 + u3, n01 = u0 - u2, n11 = u1 - u3;
        row0[c] = n00 + row_shr1(n10);
        row1[c] = n01 + row_shr1(n11);
    }
}

template <typename T>
struct KMarch {
    // geometry of this workgroup
    int tx, ty, X0, Y0, K0, K1, NX, NY, ex, ey;
    int64_t plane_nodes;
    bool col_ok, owner;
    PlaneSlots ps;
    // LDS
    T (*ring)[kPV];
    uint8_t (*mring)[kPN];
    T (*part)[3][kTileThreads];
    // registers carried between planes
    PlaneRegsK<T> pre[2];
    T rpre[2];
    T Fb[3][4], Gtp[3][4];
    T pend[3];
    uint32_t omask;

    __device__ __forceinline__ int64_t clamp_plane(int k, int nz) const {
        return (int64_t)(k < 0 ? 0 : (k > nz ? nz : k)) * plane_nodes;
    }
};

// one element layer l of the march (S: register slot of plane l+1)
template <typename T, int S>
__device__ __forceinline__ void k_step(KMarch<T>& M, const PlaneGeom& g, const KhVals<T>& kh,
                                       const T* __restrict__ x, const T* __restrict__ rho,
                                       const uint8_t* __restrict__ nmask, T* __restrict__ y,
                                       int l) {
    const int rel = l + 1 - (M.K0 - 1);                  // relative index of plane l+1
    plane_commit(M.ps, M.pre[S], M.ring[rel % kRing], M.mring[rel % kRing]);
    if (l + 3 <= M.K1) plane_fetch(M.ps, x, nmask, M.clamp_plane(l + 3, g.nz), M.pre[S]);
    const T r = M.rpre[S];
    {
        const int le = l + 2;
        const bool ok = M.col_ok && le >= 0 && le < g.nz;
        M.rpre[S] = ok ? rho[M.ex + (int64_t)g.nx * (M.ey + (int64_t)g.ny * le)] : T(0);
    }
    __syncthreads();
    // plane l-1 complete: y-neighbour part from LDS, store
    if (l - 1 >= M.K0 && M.owner) {
        const T* pp = &M.part[(rel - 2) & 1][0][0];
        const int64_t n = (int64_t)(l - 1) * M.plane_nodes + (int64_t)(M.Y0 - 1 + M.ty) * M.NX +
                          (M.X0 - 1 + M.tx);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T v = M.pend[c] + pp[c * kTileThreads + (M.ty - 1) * TXE + M.tx];
            y[3 * n + c] = ((M.omask >> c) & 1u) ? T(0) : v;
        }
    }
    M.omask = M.mring[(rel - 1) % kRing][M.ty * NXL + M.tx];   // node (tx, ty) of plane l
    T Ft[3][4], Gb[3][4], Gt[3][4];
    face_fwd(M.ring[rel % kRing], M.tx, M.ty, Ft);
    elem_modes(kh, r, M.Fb, Ft, Gb, Gt);
    T P[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            P[c][m] = Gb[c][m] + M.Gtp[c][m];
            M.Gtp[c][m] = Gt[c][m];
            M.Fb[c][m] = Ft[c][m];
        }
    T row0[3], row1[3];
    face_inv_combine(P, row0, row1);
    T* pw = &M.part[(rel - 1) & 1][0][0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pw[c * kTileThreads + M.ty * TXE + M.tx] = row1[c];
        M.pend[c] = row0[c];
    }
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads)
k_apply_K_plane(PlaneGeom g, KhVals<T> kh, const T* __restrict__ x, const T* __restrict__ rho,
                const uint8_t* __restrict__ nmask, T* __restrict__ y) {
    __shared__ T ring[kRing][kPV];
    __shared__ uint8_t mring[kRing][kPN];
    __shared__ T part[2][3][kTileThreads];
    const int lb = logical_block(g);
    if (lb < 0) return;
    KMarch<T> M;
    M.tx = threadIdx.x % TXE;
    M.ty = threadIdx.x / TXE;
    const int bx = lb % g.tiles_x, by = (lb / g.tiles_x) % g.tiles_y;
    const int bz = lb / (g.tiles_x * g.tiles_y);
    M.X0 = bx * (TXE - 1);
    M.Y0 = by * (TYE - 1);
    M.NX = g.nx + 1;
    M.NY = g.ny + 1;
    M.K0 = (int)((int64_t)(g.nz + 1) * bz / g.zblocks);
    M.K1 = (int)((int64_t)(g.nz + 1) * (bz + 1) / g.zblocks);
    M.plane_nodes = (int64_t)M.NX * M.NY;
    M.ex = M.X0 - 1 + M.tx;
    M.ey = M.Y0 - 1 + M.ty;
    M.col_ok = M.ex >= 0 && M.ex < g.nx && M.ey >= 0 && M.ey < g.ny;
    M.owner = M.tx >= 1 && M.ty >= 1 && M.ex < M.NX && M.ey < M.NY;
    M.ps = plane_slots(M.X0, M.Y0, M.NX, M.NY);
    M.ring = ring;
    M.mring = mring;
    M.part = part;
    M.omask = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        M.pend[c] = T(0);
#pragma unroll
        for (int m = 0; m < 4; ++m) M.Gtp[c][m] = T(0);
    }
    // planes K0-1 (slot 0) and K0 (slot 1); rho of layers K0-1 (slot 1), K0 (slot 0)
    plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0 - 1, g.nz), M.pre[0]);
    plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0, g.nz), M.pre[1]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int le = M.K0 - 1 + q;
        const bool ok = M.col_ok && le >= 0 && le < g.nz;
        M.rpre[1 - q] = ok ? rho[M.ex + (int64_t)g.nx * (M.ey + (int64_t)g.ny * le)] : T(0);
    }
    // plane K0-1: commit, refill slot 0 with plane K0+1, bottom face transform
    plane_commit(M.ps, M.pre[0], M.ring[0], M.mring[0]);
    if (M.K0 + 1 <= M.K1) plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0 + 1, g.nz), M.pre[0]);
    __syncthreads();
    face_fwd(M.ring[0], M.tx, M.ty, M.Fb);
    // layers K0-1 .. K1-1 (plane l+1 is in register slot (l - K0) & 1 ^ 1)
    int l = M.K0 - 1;
    for (;;) {
        k_step<T, 1>(M, g, kh, x, rho, nmask, y, l);
        if (++l >= M.K1) break;
        k_step<T, 0>(M, g, kh, x, rho, nmask, y, l);
        if (++l >= M.K1) break;
    }
    // the last plane K1-1
    __syncthreads();
    if (M.owner) {
        const int rel = M.K1 - (M.K0 - 1);               // relative index of plane K1 ... K1-1 is rel-1
        const T* pp = &M.part[(rel - 1) & 1][0][0];
        const int64_t n = (int64_t)(M.K1 - 1) * M.plane_nodes +
                          (int64_t)(M.Y0 - 1 + M.ty) * M.NX + (M.X0 - 1 + M.tx);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T v = M.pend[c] + pp[c * kTileThreads + (M.ty - 1) * TXE + M.tx];
            y[3 * n + c] = ((M.omask >> c) & 1u) ? T(0) : v;
        }
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

PlaneGeom plane_geom(const Ctx& c, int zblocks) {
    PlaneGeom g;
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = c.nz;
    g.tiles_x = (c.nx + 1 + TXE - 2) / (TXE - 1);
    g.tiles_y = (c.ny + 1 + TYE - 2) / (TYE - 1);
    g.zblocks = zblocks < 1 ? 1 : (zblocks > c.nz + 1 ? c.nz + 1 : zblocks);
    g.nblocks = g.tiles_x * g.tiles_y * g.zblocks;
    g.per_xcd = (g.nblocks + 7) / 8;
    return g;
}

// z ranges per tile column: about kPlaneWaves workgroups in total (three
// resident per CU), at least 8 planes per range
constexpr int kPlaneTarget = 768;
int choose_zblocks(const Ctx& c) {
    const int cols = ((c.nx + TXE - 1) / (TXE - 1)) * ((c.ny + TYE - 1) / (TYE - 1));
    int zb = (kPlaneTarget + cols - 1) / cols;
    const int maxzb = (c.nz + 1 + 7) / 8;
    if (zb > maxzb) zb = maxzb;
    return zb < 1 ? 1 : zb;
}

template <typename T>
void launch_plane_K(Ctx& c, const T* rho, const T* x, T* y) {
    const PlaneGeom g = plane_geom(c, choose_zblocks(c));
    const KhVals<T> kh{(T)c.kh8[0], (T)c.kh8[1], (T)c.kh8[2], (T)c.kh8[3],
                       (T)c.kh8[4], (T)c.kh8[5], (T)c.kh8[6], (T)c.kh8[7]};
    hipLaunchKernelGGL(k_apply_K_plane<T>, dim3(8 * g.per_xcd), dim3(kTileThreads), 0, c.s, g, kh,
                       x, rho, c.nmask, y);
}

}  // namespace

bool tile_ok(const Ctx& c) { return c.kh_ok; }

void launch_apply_K_tile_f64(Ctx& c, const double* rho, const double* x, double* y) {
    launch_plane_K<double>(c, rho, x, y);
}

void launch_apply_K_tile_f32(Ctx& c, const float* rho, const float* x, float* y) {
    launch_plane_K<float>(c, rho, x, y);
}

int apply_S_tile_blocks(const Ctx& c) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    return g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
}

void launch_apply_S_tile_ws(Ctx& c, const double* x, double* y, double* partials) {
    const int kz = choose_kz(c);
    TileGeom g = geom_of(c, kz);
    KhVals<double> kh{c.kh8[0], c.kh8[1], c.kh8[2], c.kh8[3], c.kh8[4], c.kh8[5], c.kh8[6], c.kh8[7]};
    const int nb = g.tiles_x * g.tiles_y * ((c.nz + 1 + kz - 1) / kz);
    hipLaunchKernelGGL(k_apply_S_tile<double>, dim3(nb), dim3(kTileThreads), 0, c.s, g, kh, x, c.u,
                       c.r1, c.w, c.fixed, c.ndof, y, partials);
    hipLaunchKernelGGL(k_sum_neg, dim3(1), dim3(256), 0, c.s, partials, nb, y + c.ndof);
}

void launch_apply_S_tile(Ctx& c, const double* x, double* y) {
    launch_apply_S_tile_ws(c, x, y, c.spart);
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free S-apply: the per-workgroup partial sums of
// the alpha row live in this file-scope device array instead of the
// context's buffer.  Each device holds its own copy; host code reaches it
// only through the address hipGetSymbolAddress returns for that device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchPartials];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

vts_status scratch_partials(int device, double** out, std::string& err) {
    if (device < 0 || device >= kMaxScratchDevices) {
        err = "device index beyond the scratch table";
        return VTS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) { err = "hipGetDevice failed"; return VTS_EDEVICE; }
        if (cur != device && hipSetDevice(device) != hipSuccess) {
            err = "hipSetDevice failed";
            return VTS_EDEVICE;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return VTS_EDEVICE;
        }
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return VTS_OK;
}

}  // namespace vts
