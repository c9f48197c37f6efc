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
//
// S [x; beta] (k_apply_S_plane) marches the same way with x and u staged
// together; per element b_e = K_e u_e and t = b_e^T x_e - beta are formed in
// the transformed basis, and y_e = K_e (rho'_e x_e + w_e t u_e) goes through
// Kh once more.  Bottom-face transforms are taken again from the LDS ring
// (not carried in registers) to keep two workgroups resident per CU.
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

// z-stage of the transform: the element's 24 modes v[3 m + c] (m = mxy + 4 mz)
// from the face transforms of its bottom (Fb) and top (Ft) faces
template <typename T>
__device__ __forceinline__ void modes_from_faces(const T (&Fb)[3][4], const T (&Ft)[3][4],
                                                 T (&v)[24]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[3 * m + c] = Fb[c][m] + Ft[c][m];
            v[3 * (m + 4) + c] = Fb[c][m] - Ft[c][m];
        }
}

// y = r Kh v (the constant modes of v are ignored; y's are zero)
template <typename T>
__device__ __forceinline__ void kh_apply(const KhVals<T>& k, T r, const T (&v)[24], T (&y)[24]) {
    const T AmB = r * (k.A - k.B), rB = r * k.B, rC = r * k.C, rD = r * k.D, rE = r * k.E;
    const T FmG = r * (k.F - k.G), rG = r * k.G, rH = r * k.H;
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
}

// inverse z-stage: bottom (Gb) and top (Gt) face transforms of the modes y
template <typename T>
__device__ __forceinline__ void faces_from_modes(const T (&y)[24], T (&Gb)[3][4], T (&Gt)[3][4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Gb[c][m] = y[3 * m + c] + y[3 * (m + 4) + c];
            Gt[c][m] = y[3 * m + c] - y[3 * (m + 4) + c];
        }
}

// the element's modes from its bottom/top face transforms, rho Kh applied, and
// the result split back into bottom (Gb) and top (Gt) face transforms
template <typename T>
__device__ __forceinline__ void elem_modes(const KhVals<T>& k, T r, const T (&Fb)[3][4],
                                           const T (&Ft)[3][4], T (&Gb)[3][4], T (&Gt)[3][4]) {
    T v[24], y[24];
    modes_from_faces(Fb, Ft, v);
    kh_apply(k, r, v, y);
    faces_from_modes(y, Gb, Gt);
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
// S [x; beta] of eq. (3.12), plane-marching form: x and u staged together;
// per element b^ = Kh u^ (b_e = K_e u_e in the transformed basis), t = b^ . x^
// - beta (= b_e^T x_e - beta: H is symmetric and H H = 8 I per direction pair
// folded into Kh), y_e = K_e (rho'_e x_e + w_e t u_e) through Kh once more.
// Per-workgroup partial sums of w t over the elements the tile owns.
// ---------------------------------------------------------------------------
template <typename T>
struct SMarch {
    int tx, ty, K0, K1, NX, NY, ex, ey;   // (ex, ey): this thread's element column = node
    int64_t plane_nodes;
    bool col_ok, owner, own_col;
    PlaneSlots ps;
    T (*rx)[kPV];
    T (*ru)[kPV];
    uint8_t (*mring)[kPN];
    T (*part)[3][kTileThreads];
    PlaneRegsK<T> px[2], pu[2];
    T r1pre[2], wpre[2];
    T Gtp[3][4];
    T pend[3];
    uint32_t omask;
    double wsum;

    __device__ __forceinline__ int64_t clamp_plane(int k, int nz) const {
        return (int64_t)(k < 0 ? 0 : (k > nz ? nz : k)) * plane_nodes;
    }
};

template <typename T>
__device__ __forceinline__ void s_fetch_elem(SMarch<T>& M, const PlaneGeom& g, const T* r1,
                                             const T* w, int le, T& r, T& ww) {
    const bool ok = M.col_ok && le >= 0 && le < g.nz;
    const int64_t e = M.ex + (int64_t)g.nx * (M.ey + (int64_t)g.ny * le);
    r = ok ? r1[e] : T(0);
    ww = ok ? w[e] : T(0);
}

// what a march over (x, u) produces
enum SMode {
    S_APPLY = 0,   // y = S [x; beta] (displacement part), partials of sum w (b.x - beta)
    S_RESID = 1,   // y = r - S [x; beta], partials of acol . x = -sum w b.x
    S_TDOT = 2     // te[e] = b_e . x_e for every element, nothing else
};

template <typename T, int S, int MODE>
__device__ __forceinline__ void s_step(SMarch<T>& M, const PlaneGeom& g, const KhVals<T>& kh,
                                       const T* __restrict__ x, const T* __restrict__ u,
                                       const T* __restrict__ r1, const T* __restrict__ w,
                                       const uint8_t* __restrict__ nmask, T beta,
                                       const T* __restrict__ rr_in, T* __restrict__ y,
                                       T* __restrict__ te, int l) {
    const int rel = l + 1 - (M.K0 - 1);
    plane_commit(M.ps, M.px[S], M.rx[rel % kRing], M.mring[rel % kRing]);
    plane_commit(M.ps, M.pu[S], M.ru[rel % kRing], M.mring[rel % kRing]);
    if (l + 3 <= M.K1) {
        plane_fetch(M.ps, x, nmask, M.clamp_plane(l + 3, g.nz), M.px[S]);
        plane_fetch(M.ps, u, nmask, M.clamp_plane(l + 3, g.nz), M.pu[S]);
    }
    const T rr = M.r1pre[S], ww = M.wpre[S];
    s_fetch_elem(M, g, r1, w, l + 2, M.r1pre[S], M.wpre[S]);
    __syncthreads();
    if (MODE != S_TDOT && l - 1 >= M.K0 && M.owner) {
        const T* pp = &M.part[(rel - 2) & 1][0][0];
        const int64_t n = (int64_t)(l - 1) * M.plane_nodes + (int64_t)M.ey * M.NX + M.ex;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = M.pend[c] + pp[c * kTileThreads + (M.ty - 1) * TXE + M.tx];
            if (MODE == S_RESID) v = rr_in[3 * n + c] - v;
            y[3 * n + c] = ((M.omask >> c) & 1u) ? T(0) : v;
        }
    }
    if (MODE != S_TDOT) M.omask = M.mring[(rel - 1) % kRing][M.ty * NXL + M.tx];
    // bottom faces from the plane still in the ring (keeps registers low)
    T vx[24], vu[24], b[24];
    {
        T Fb[3][4], Ft[3][4];
        face_fwd(M.rx[(rel - 1) % kRing], M.tx, M.ty, Fb);
        face_fwd(M.rx[rel % kRing], M.tx, M.ty, Ft);
        modes_from_faces(Fb, Ft, vx);
        face_fwd(M.ru[(rel - 1) % kRing], M.tx, M.ty, Fb);
        face_fwd(M.ru[rel % kRing], M.tx, M.ty, Ft);
        modes_from_faces(Fb, Ft, vu);
    }
    kh_apply(kh, T(1), vu, b);
    T traw = T(0);
#pragma unroll
    for (int q = 3; q < 24; ++q) traw += b[q] * vx[q];
    const bool own = M.own_col && l >= M.K0 && l < g.nz;  // elements owned by this tile
    if (MODE == S_TDOT) {
        if (own) te[M.ex + (int64_t)g.nx * (M.ey + (int64_t)g.ny * l)] = traw;
        return;
    }
    const T wt = ww * (traw - beta);                      // 0 outside the grid
    if (own) M.wsum += MODE == S_RESID ? -(double)(ww * traw) : (double)wt;
#pragma unroll
    for (int q = 3; q < 24; ++q) vx[q] = rr * vx[q] + wt * vu[q];
    kh_apply(kh, T(1), vx, b);
    T Gb[3][4], Gt[3][4];
    faces_from_modes(b, Gb, Gt);
    T P[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            P[c][m] = Gb[c][m] + M.Gtp[c][m];
            M.Gtp[c][m] = Gt[c][m];
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

// The march over (x, u) for the S-apply (S_APPLY), the finest-level residual
// of the V-cycle (S_RESID: x = z, beta = z_alpha, r_in = r) and the element
// products b_e^T x_e (S_TDOT).  beta is x[ndof].
template <typename T>
struct SPlaneArgs {
    PlaneGeom g;
    KhVals<T> kh;
    const T* x;
    const T* u;
    const T* r1;
    const T* w;
    const uint8_t* nmask;
    int64_t ndof;
    const T* r_in;
    T* y;
    T* te;
    double* partials;
};

template <typename T, int MODE>
__device__ __forceinline__ void s_plane_body(const SPlaneArgs<T>& a) {
    const PlaneGeom g = a.g;
    const KhVals<T> kh = a.kh;
    const T* __restrict__ x = a.x;
    const T* __restrict__ u = a.u;
    const T* __restrict__ r1 = a.r1;
    const T* __restrict__ w = a.w;
    const uint8_t* __restrict__ nmask = a.nmask;
    const int64_t ndof = a.ndof;
    const T* __restrict__ r_in = a.r_in;
    T* __restrict__ y = a.y;
    T* __restrict__ te = a.te;
    double* __restrict__ partials = a.partials;
    __shared__ T rx[kRing][kPV];
    __shared__ T ru[kRing][kPV];
    __shared__ uint8_t mring[kRing][kPN];
    __shared__ T part[2][3][kTileThreads];
    __shared__ double red[kTileThreads / 64];
    const int lb = logical_block(g);
    if (lb < 0) return;
    SMarch<T> M;
    M.tx = threadIdx.x % TXE;
    M.ty = threadIdx.x / TXE;
    const int bx = lb % g.tiles_x, by = (lb / g.tiles_x) % g.tiles_y;
    const int bz = lb / (g.tiles_x * g.tiles_y);
    const int X0 = bx * (TXE - 1), Y0 = by * (TYE - 1);
    M.NX = g.nx + 1;
    M.NY = g.ny + 1;
    M.K0 = (int)((int64_t)(g.nz + 1) * bz / g.zblocks);
    M.K1 = (int)((int64_t)(g.nz + 1) * (bz + 1) / g.zblocks);
    M.plane_nodes = (int64_t)M.NX * M.NY;
    M.ex = X0 - 1 + M.tx;
    M.ey = Y0 - 1 + M.ty;
    M.col_ok = M.ex >= 0 && M.ex < g.nx && M.ey >= 0 && M.ey < g.ny;
    M.owner = M.tx >= 1 && M.ty >= 1 && M.ex < M.NX && M.ey < M.NY;
    M.own_col = M.col_ok && M.tx >= 1 && M.ty >= 1;
    M.ps = plane_slots(X0, Y0, M.NX, M.NY);
    M.rx = rx;
    M.ru = ru;
    M.mring = mring;
    M.part = part;
    M.omask = 0;
    M.wsum = 0.0;
    const T beta = MODE == S_TDOT ? T(0) : x[ndof];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        M.pend[c] = T(0);
#pragma unroll
        for (int m = 0; m < 4; ++m) M.Gtp[c][m] = T(0);
    }
    plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0 - 1, g.nz), M.px[0]);
    plane_fetch(M.ps, u, nmask, M.clamp_plane(M.K0 - 1, g.nz), M.pu[0]);
    plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0, g.nz), M.px[1]);
    plane_fetch(M.ps, u, nmask, M.clamp_plane(M.K0, g.nz), M.pu[1]);
    s_fetch_elem(M, g, r1, w, M.K0 - 1, M.r1pre[1], M.wpre[1]);
    s_fetch_elem(M, g, r1, w, M.K0, M.r1pre[0], M.wpre[0]);
    plane_commit(M.ps, M.px[0], M.rx[0], M.mring[0]);
    plane_commit(M.ps, M.pu[0], M.ru[0], M.mring[0]);
    if (M.K0 + 1 <= M.K1) {
        plane_fetch(M.ps, x, nmask, M.clamp_plane(M.K0 + 1, g.nz), M.px[0]);
        plane_fetch(M.ps, u, nmask, M.clamp_plane(M.K0 + 1, g.nz), M.pu[0]);
    }
    __syncthreads();
    int l = M.K0 - 1;
    for (;;) {
        s_step<T, 1, MODE>(M, g, kh, x, u, r1, w, nmask, beta, r_in, y, te, l);
        if (++l >= M.K1) break;
        s_step<T, 0, MODE>(M, g, kh, x, u, r1, w, nmask, beta, r_in, y, te, l);
        if (++l >= M.K1) break;
    }
    if (MODE == S_TDOT) return;
    __syncthreads();
    if (M.owner) {
        const T* pp = &M.part[(M.K1 - M.K0) & 1][0][0];
        const int64_t n = (int64_t)(M.K1 - 1) * M.plane_nodes + (int64_t)M.ey * M.NX + M.ex;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = M.pend[c] + pp[c * kTileThreads + (M.ty - 1) * TXE + M.tx];
            if (MODE == S_RESID) v = r_in[3 * n + c] - v;
            y[3 * n + c] = ((M.omask >> c) & 1u) ? T(0) : v;
        }
    }
    // block partial (fixed order)
    double ws = M.wsum;
    for (int off = 32; off > 0; off >>= 1) ws += __shfl_down(ws, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int q = 0; q < kTileThreads / 64; ++q) sum += red[q];
        partials[lb] = sum;
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kTileThreads) k_S_plane(SPlaneArgs<T> a) {
    s_plane_body<T, MODE>(a);
}

// the same for problem blockIdx.y of a group launch
template <typename T, int MODE>
__global__ void __launch_bounds__(kTileThreads) k_S_plane_b(const SPlaneArgs<T>* __restrict__ tab) {
    s_plane_body<T, MODE>(tab[blockIdx.y]);
}

// deterministic sum of nb partials into dst (negated: the alpha row of S)
struct SumNegArgs {
    const double* partials;
    int nb;
    double* dst;
};
__device__ __forceinline__ void sum_neg_body(const SumNegArgs& a) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int q = threadIdx.x; q < a.nb; q += blockDim.x) s += a.partials[q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.dst[0] = -sh[0];
}
VTS_KERNEL_PAIR(, 256, k_sum_neg, SumNegArgs, sum_neg_body)

template <typename T, int MODE>
void launch_s_plane(Ctx& c, dim3 grid, const SPlaneArgs<T>& a) {
    vlaunch(c, (const void*)&k_S_plane<T, MODE>, (const void*)&k_S_plane_b<T, MODE>, grid,
            dim3(kTileThreads), a);
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
    return plane_geom(c, choose_zblocks(c)).nblocks;
}

void launch_apply_S_tile_ws(Ctx& c, const double* x, double* y, double* partials) {
    const PlaneGeom g = plane_geom(c, choose_zblocks(c));
    const KhVals<double> kh{c.kh8[0], c.kh8[1], c.kh8[2], c.kh8[3],
                            c.kh8[4], c.kh8[5], c.kh8[6], c.kh8[7]};
    launch_s_plane<double, S_APPLY>(
        c, dim3(8 * g.per_xcd),
        SPlaneArgs<double>{g, kh, x, c.u, c.r1, c.w, c.nmask, c.ndof, (const double*)nullptr, y,
                           (double*)nullptr, partials});
    vlaunch(c, (const void*)&k_sum_neg, (const void*)&k_sum_neg_b, dim3(1), dim3(256),
            SumNegArgs{partials, g.nblocks, y + c.ndof});
}

void launch_apply_S_tile(Ctx& c, const double* x, double* y) {
    launch_apply_S_tile_ws(c, x, y, c.spart);
}

// finest level of the V-cycle, matrix-free (precision T): res = r - S [z; z_a]
// with partial sums of acol . z (one per workgroup) into parts, and the
// element products te = b_e^T z_e
template <typename T>
void launch_fine_resid(Ctx& c, const Level<T>& L, const T* u, const T* r1, const T* w,
                       double* parts) {
    const PlaneGeom g = plane_geom(c, choose_zblocks(c));
    const KhVals<T> kh{(T)c.kh8[0], (T)c.kh8[1], (T)c.kh8[2], (T)c.kh8[3],
                       (T)c.kh8[4], (T)c.kh8[5], (T)c.kh8[6], (T)c.kh8[7]};
    launch_s_plane<T, S_RESID>(c, dim3(8 * g.per_xcd),
                               SPlaneArgs<T>{g, kh, (const T*)L.z, u, r1, w, c.nmask, 3 * L.nn,
                                             (const T*)L.r, L.res, (T*)nullptr, parts});
}

template <typename T>
void launch_fine_tdot(Ctx& c, const Level<T>& L, const T* u, const T* r1, const T* w, T* te) {
    const PlaneGeom g = plane_geom(c, choose_zblocks(c));
    const KhVals<T> kh{(T)c.kh8[0], (T)c.kh8[1], (T)c.kh8[2], (T)c.kh8[3],
                       (T)c.kh8[4], (T)c.kh8[5], (T)c.kh8[6], (T)c.kh8[7]};
    launch_s_plane<T, S_TDOT>(c, dim3(8 * g.per_xcd),
                              SPlaneArgs<T>{g, kh, (const T*)L.z, u, r1, w, c.nmask, 3 * L.nn,
                                            (const T*)nullptr, (T*)nullptr, te,
                                            (double*)nullptr});
}

int fine_resid_blocks(const Ctx& c) { return plane_geom(c, choose_zblocks(c)).nblocks; }

template void launch_fine_resid<float>(Ctx&, const Level<float>&, const float*, const float*,
                                       const float*, double*);
template void launch_fine_resid<double>(Ctx&, const Level<double>&, const double*,
                                        const double*, const double*, double*);
template void launch_fine_tdot<float>(Ctx&, const Level<float>&, const float*, const float*,
                                      const float*, float*);
template void launch_fine_tdot<double>(Ctx&, const Level<double>&, const double*, const double*,
                                       const double*, double*);

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
        if (cur != device) (void)hipSetDevice(cur);
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
