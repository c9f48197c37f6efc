// Geometric multigrid for the reduced Newton matrix S of eq. (3.12)
// (Section 6.1: V-cycle correction scheme, Galerkin coarse operators,
// Gauss-Seidel smoothing; Section 6.2: 27-point trilinear prolongation,
// identity transfer of the scalar alpha).
//
// Each level's displacement block is stored as an assembled 27-point
// stencil of 3x3 blocks in colour-major node order (colour = parity
// (i&1) + 2(j&1) + 4(k&1)), so one Gauss-Seidel colour pass reads its
// nodes' rows with unit stride.  Coarse operators are built element by
// element: E_parent = sum_children Q_c^T E_child Q_c, which equals P^T A P
// because each fine element lies in one coarse element and trilinear
// interpolation restricted to it is the local map Q_c.
#include <hip/hip_runtime.h>

#include <cmath>

#include "vts_internal.hpp"

namespace vts {

namespace {

__device__ __forceinline__ int64_t gidx() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}
inline int grid_of(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : b);
}
inline int red_grid_of(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    return (int)(b < kRedBlocks ? b : kRedBlocks);
}

template <typename T>
__device__ __forceinline__ void cm_decode(const Level<T>& L, int64_t t, int& i, int& j, int& k) {
    int col = 0;
    while (col < 7 && t >= L.coff[col + 1]) ++col;
    int64_t tl = t - L.coff[col];
    const int cx = L.cnx[col], cy = L.cny[col];
    i = 2 * (int)(tl % cx) + (col & 1);
    tl /= cx;
    j = 2 * (int)(tl % cy) + ((col >> 1) & 1);
    k = 2 * (int)(tl / cy) + (col >> 2);
}

__device__ __forceinline__ int64_t nat(int i, int j, int k, int NX, int NY) {
    return (int64_t)i + (int64_t)NX * ((int64_t)j + (int64_t)NY * k);
}

// inverse of the free sub-block of a 3x3 block (identity on fixed components,
// then zeroed there)
__device__ void masked_inverse3(const double (&D0)[9], const bool (&fx)[3], double (&Di)[9]) {
    double D[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double v = D0[r * 3 + c];
            if (fx[r] || fx[c]) v = (r == c) ? 1.0 : 0.0;
            D[r * 3 + c] = v;
        }
    const double c00 = D[4] * D[8] - D[5] * D[7];
    const double c01 = D[5] * D[6] - D[3] * D[8];
    const double c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    const double id = 1.0 / det;
    Di[0] = c00 * id;
    Di[1] = (D[2] * D[7] - D[1] * D[8]) * id;
    Di[2] = (D[1] * D[5] - D[2] * D[4]) * id;
    Di[3] = c01 * id;
    Di[4] = (D[0] * D[8] - D[2] * D[6]) * id;
    Di[5] = (D[2] * D[3] - D[0] * D[5]) * id;
    Di[6] = c02 * id;
    Di[7] = (D[1] * D[6] - D[0] * D[7]) * id;
    Di[8] = (D[0] * D[4] - D[1] * D[3]) * id;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            if (fx[r] || fx[c]) Di[r * 3 + c] = 0.0;
}

// ---------------------------------------------------------------------------
// finest level: stencil of K(rho') + sum_e w_e b_e b_e^T from (rho', w, b),
// its inverse diagonal blocks, and the alpha column -sum_e w_e b_e
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fine_stencil(Level<T> L, const double* __restrict__ Ke, const double* __restrict__ r1,
               const double* __restrict__ w, const double* __restrict__ be) {
    const int64_t t = gidx();
    if (t >= L.nn) return;
    int i, j, k;
    cm_decode(L, t, i, j, k);
    const int64_t n = nat(i, j, k, L.NX, L.NY);
    const int64_t m = L.m;
    double diag[9] = {0};
    for (int s = 0; s < kStencil; ++s) {
        const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const bool inside = (i + dx >= 0 && i + dx < L.NX && j + dy >= 0 && j + dy < L.NY &&
                             k + dz >= 0 && k + dz < L.NZ);
        if (inside) {
            for (int ez = -1; ez <= 0; ++ez)
                for (int ey = -1; ey <= 0; ++ey)
                    for (int ex = -1; ex <= 0; ++ex) {
                        const int ii = i + ex, jj = j + ey, kk = k + ez;
                        if (ii < 0 || ii >= L.nx || jj < 0 || jj >= L.ny || kk < 0 || kk >= L.nz)
                            continue;
                        const int bx = dx - ex, by = dy - ey, bz = dz - ez;
                        if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                        const int64_t e = ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk);
                        const int la = -ex - 2 * ey - 4 * ez, lb = bx + 2 * by + 4 * bz;
                        const double rr = r1[e], ww = w[e];
                        for (int r = 0; r < 3; ++r) {
                            const double wb = ww * be[(3 * la + r) * m + e];
                            for (int c = 0; c < 3; ++c)
                                blk[r * 3 + c] += rr * Ke[(3 * la + r) * 24 + 3 * lb + c] +
                                                  wb * be[(3 * lb + c) * m + e];
                        }
                    }
        }
        for (int q = 0; q < 9; ++q) L.st[(int64_t)(s * 9 + q) * L.nn + t] = (T)blk[q];
        if (s == 13)
            for (int q = 0; q < 9; ++q) diag[q] = blk[q];
    }
    bool fx[3];
    for (int c = 0; c < 3; ++c) fx[c] = L.fixed[3 * n + c] != 0;
    // diagonal from the rounded values so that both precisions smooth with
    // the inverse of the matrix they apply
    double d0[9];
    for (int q = 0; q < 9; ++q) d0[q] = (double)(T)diag[q];
    double di[9];
    masked_inverse3(d0, fx, di);
    for (int q = 0; q < 9; ++q) L.dinv[(int64_t)q * L.nn + t] = (T)di[q];
    double ac[3] = {0, 0, 0};
    for (int ez = -1; ez <= 0; ++ez)
        for (int ey = -1; ey <= 0; ++ey)
            for (int ex = -1; ex <= 0; ++ex) {
                const int ii = i + ex, jj = j + ey, kk = k + ez;
                if (ii < 0 || ii >= L.nx || jj < 0 || jj >= L.ny || kk < 0 || kk >= L.nz) continue;
                const int64_t e = ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk);
                const int la = -ex - 2 * ey - 4 * ez;
                for (int c = 0; c < 3; ++c) ac[c] -= w[e] * be[(3 * la + c) * m + e];
            }
    for (int c = 0; c < 3; ++c) L.acol[3 * n + c] = fx[c] ? T(0) : (T)ac[c];
}

// ---------------------------------------------------------------------------
// finest level without a stored stencil: per node (colour-major t) its 3x3
// diagonal block sum_e rho'_e K_e[a,a] + w_e b_{e,a} b_{e,a}^T (inverted, masked),
// the alpha column -sum_e w_e b_{e,a}, and bc[t][o] = b_{e,a} of the element
// at offset o in {-1,0}^3 (the node is its corner a = o; zero outside the grid)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fine_mf_setup(Level<T> L, const double* __restrict__ Ke, const double* __restrict__ r1,
                const double* __restrict__ w, const double* __restrict__ be, T* __restrict__ bc) {
    const int64_t t = gidx();
    if (t >= L.nn) return;
    int i, j, k;
    cm_decode(L, t, i, j, k);
    const int64_t n = nat(i, j, k, L.NX, L.NY);
    const int64_t m = L.m;
    double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ac[3] = {0, 0, 0};
    for (int o = 0; o < 8; ++o) {
        const int ii = i - (o & 1), jj = j - ((o >> 1) & 1), kk = k - (o >> 2);
        const bool in = ii >= 0 && ii < L.nx && jj >= 0 && jj < L.ny && kk >= 0 && kk < L.nz;
        double bv[3] = {0, 0, 0};
        if (in) {
            const int64_t e = ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk);
            const double rr = r1[e], ww = w[e];
            for (int r = 0; r < 3; ++r) bv[r] = be[(3 * o + r) * m + e];
            for (int r = 0; r < 3; ++r) {
                for (int cc = 0; cc < 3; ++cc)
                    D[r * 3 + cc] += rr * Ke[(3 * o + r) * 24 + 3 * o + cc] + ww * bv[r] * bv[cc];
                ac[r] -= ww * bv[r];
            }
        }
        for (int r = 0; r < 3; ++r) bc[t * 24 + 3 * o + r] = (T)bv[r];
    }
    bool fx[3];
    for (int cc = 0; cc < 3; ++cc) fx[cc] = L.fixed[3 * n + cc] != 0;
    // inverse of the block rounded to T, as for the stored stencil
    double d0[9], di[9];
    for (int q = 0; q < 9; ++q) d0[q] = (double)(T)D[q];
    masked_inverse3(d0, fx, di);
    for (int q = 0; q < 9; ++q) L.dinv[(int64_t)q * L.nn + t] = (T)di[q];
    for (int cc = 0; cc < 3; ++cc) L.acol[3 * n + cc] = fx[cc] ? T(0) : (T)ac[cc];
}

// rho', w (m each) and u (3 nn) in the level precision
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fine_mf_convert(int64_t m, int64_t nu, const double* __restrict__ r1,
                  const double* __restrict__ w, const double* __restrict__ u, T* __restrict__ r1f,
                  T* __restrict__ wf, T* __restrict__ uf) {
    const int64_t t = gidx();
    if (t < m) {
        r1f[t] = (T)r1[t];
        wf[t] = (T)w[t];
    }
    if (t < nu) uf[t] = (T)u[t];
}

// g_e = Q_{c(e)}^T b_e: the element force seen from the parent element's nodes
__global__ void k_child_g(int nx, int ny, int nz, const double* __restrict__ Q,
                          const double* __restrict__ be, double* __restrict__ gch) {
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t e = gidx();
    if (e >= m) return;
    const int i = (int)(e % nx);
    const int64_t tt = e / nx;
    const int j = (int)(tt % ny), k = (int)(tt / ny);
    const int c = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    for (int A = 0; A < 8; ++A)
        for (int comp = 0; comp < 3; ++comp) {
            double s = 0.0;
            for (int a = 0; a < 8; ++a) s += Q[(c * 8 + a) * 8 + A] * be[(3 * a + comp) * m + e];
            gch[(3 * A + comp) * m + e] = s;
        }
}

// first coarse level: E_C = sum_c rho'_c M_c + w_c g_c g_c^T, one row per thread
template <typename T>
__global__ void k_coarse_first(Level<T> C, int fnx, int fny, int fnz, const double* __restrict__ Mc,
                               const double* __restrict__ r1, const double* __restrict__ w,
                               const double* __restrict__ gch) {
    const int64_t t = gidx();
    if (t >= C.m * 24) return;
    const int64_t ec = t / 24;
    const int R = (int)(t % 24);
    const int I = (int)(ec % C.nx);
    const int64_t tt = ec / C.nx;
    const int J = (int)(tt % C.ny), K = (int)(tt / C.ny);
    const int64_t mf = (int64_t)fnx * fny * fnz;
    double row[24];
    for (int q = 0; q < 24; ++q) row[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int64_t ef = (2 * I + (c & 1)) + (int64_t)fnx * ((2 * J + ((c >> 1) & 1)) +
                                                                (int64_t)fny * (2 * K + (c >> 2)));
        const double rr = r1[ef];
        const double wg = w[ef] * gch[(int64_t)R * mf + ef];
        const double* M = Mc + c * 576 + R * 24;
        for (int q = 0; q < 24; ++q) row[q] += rr * M[q] + wg * gch[(int64_t)q * mf + ef];
    }
    T* out = C.E + ec * 576 + R * 24;
    for (int q = 0; q < 24; ++q) out[q] = (T)row[q];
}

// TQ_e = E_e (Q_c x I3) for every element e of level F (its parent is on the
// next coarser level); one row per thread
template <typename T>
__global__ void k_coarsen_tq(Level<T> F, const double* __restrict__ Q) {
    const int64_t t = gidx();
    if (t >= F.m * 24) return;
    const int64_t e = t / 24;
    const int r = (int)(t % 24);
    const int i = (int)(e % F.nx);
    const int64_t tt = e / F.nx;
    const int j = (int)(tt % F.ny), k = (int)(tt / F.ny);
    const int c = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    const T* Er = F.E + e * 576 + r * 24;
    double x[24];
    for (int q = 0; q < 24; ++q) x[q] = (double)Er[q];
    T* out = F.TQ + e * 576 + r * 24;
    for (int A = 0; A < 8; ++A)
        for (int comp = 0; comp < 3; ++comp) {
            double s = 0.0;
            for (int a = 0; a < 8; ++a) s += x[3 * a + comp] * Q[(c * 8 + a) * 8 + A];
            out[3 * A + comp] = (T)s;
        }
}

// E_C[R, :] = sum_c sum_a Q_c[a][A] TQ_c[3a+comp, :],  R = 3A + comp
template <typename T>
__global__ void k_coarsen_e(Level<T> C, Level<T> F, const double* __restrict__ Q) {
    const int64_t t = gidx();
    if (t >= C.m * 24) return;
    const int64_t ec = t / 24;
    const int R = (int)(t % 24);
    const int A = R / 3, comp = R % 3;
    const int I = (int)(ec % C.nx);
    const int64_t tt = ec / C.nx;
    const int J = (int)(tt % C.ny), K = (int)(tt / C.ny);
    double row[24];
    for (int q = 0; q < 24; ++q) row[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int64_t ef = (2 * I + (c & 1)) + (int64_t)F.nx * ((2 * J + ((c >> 1) & 1)) +
                                                                 (int64_t)F.ny * (2 * K + (c >> 2)));
        for (int a = 0; a < 8; ++a) {
            const double qa = Q[(c * 8 + a) * 8 + A];
            if (qa == 0.0) continue;
            const T* src = F.TQ + ef * 576 + (3 * a + comp) * 24;
            for (int q = 0; q < 24; ++q) row[q] += qa * (double)src[q];
        }
    }
    T* out = C.E + ec * 576 + R * 24;
    for (int q = 0; q < 24; ++q) out[q] = (T)row[q];
}

// coarse level stencil and inverse diagonal blocks from element matrices
template <typename T>
__global__ void __launch_bounds__(kThreads) k_elem_stencil(Level<T> L) {
    const int64_t t = gidx();
    if (t >= L.nn) return;
    int i, j, k;
    cm_decode(L, t, i, j, k);
    const int64_t n = nat(i, j, k, L.NX, L.NY);
    double diag[9] = {0};
    for (int s = 0; s < kStencil; ++s) {
        const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int ez = -1; ez <= 0; ++ez)
            for (int ey = -1; ey <= 0; ++ey)
                for (int ex = -1; ex <= 0; ++ex) {
                    const int ii = i + ex, jj = j + ey, kk = k + ez;
                    if (ii < 0 || ii >= L.nx || jj < 0 || jj >= L.ny || kk < 0 || kk >= L.nz)
                        continue;
                    const int bx = dx - ex, by = dy - ey, bz = dz - ez;
                    if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                    const int64_t e = ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk);
                    const int la = -ex - 2 * ey - 4 * ez, lb = bx + 2 * by + 4 * bz;
                    const T* Ee = L.E + e * 576;
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c)
                            blk[r * 3 + c] += (double)Ee[(3 * la + r) * 24 + 3 * lb + c];
                }
        for (int q = 0; q < 9; ++q) L.st[(int64_t)(s * 9 + q) * L.nn + t] = (T)blk[q];
        if (s == 13)
            for (int q = 0; q < 9; ++q) diag[q] = blk[q];
    }
    bool fx[3];
    for (int c = 0; c < 3; ++c) fx[c] = L.fixed[3 * n + c] != 0;
    double d0[9];
    for (int q = 0; q < 9; ++q) d0[q] = (double)(T)diag[q];
    double di[9];
    masked_inverse3(d0, fx, di);
    for (int q = 0; q < 9; ++q) L.dinv[(int64_t)q * L.nn + t] = (T)di[q];
}

// ---------------------------------------------------------------------------
// smoothing and residual
// ---------------------------------------------------------------------------
// partial sums of acol . z
template <typename T>
struct AcolDotArgs {
    Level<T> L;
    const T* z;
    double* partials;
};

template <typename T>
__device__ __forceinline__ void acol_dot_body(const AcolDotArgs<T>& a_) {
    const Level<T>& L = a_.L;
    const T* const z = a_.z;
    double* const partials = a_.partials;
    double acc = 0.0;
    for (int64_t q = gidx(); q < 3 * L.nn; q += (int64_t)gridDim.x * blockDim.x)
        acc += (double)L.acol[q] * (double)z[q];
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[SL_AUX * kRedBlocks + blockIdx.x] = sh[0];
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_acol_dot, AcolDotArgs<T>, acol_dot_body<T>)

// The alpha step of k_alpha_fin inside another kernel, by the first kThreads
// threads of the block (every thread of the block must call it: it holds
// barriers).  Same partial-sum order and the same operations as k_alpha_fin,
// so the result is bitwise the same: returns v = r_a - (T)(sum partials) - d z_a.
template <typename T>
__device__ __forceinline__ T alpha_residual(const double* __restrict__ parts, int nb, double d,
                                            T ra, T za, double* sh) {
    if ((int)threadIdx.x < kThreads) {
        double x = 0.0;
        for (int b = threadIdx.x; b < nb; b += kThreads) x += parts[b];
        sh[threadIdx.x] = x;
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const T td = (T)d;
    const T dot = (T)sh[0];
    const T v = ra - dot - td * za;
    __syncthreads();
    return v;
}

// Sum the partials, then either the Gauss-Seidel update of alpha
// (mode 0: z_a += (r_a - acol.z - d z_a)/d) or the alpha residual
// (mode 1: res_a = r_a - acol.z - d z_a).
template <typename T>
struct AlphaFinArgs {
    const double* partials;
    int nb;
    int64_t nn;
    double d;
    const T* r;
    T* z;
    T* res;
    int mode;
};

template <typename T>
__device__ __forceinline__ void alpha_fin_body(const AlphaFinArgs<T>& a_) {
    const double* const partials = a_.partials;
    const int nb = a_.nb;
    const int64_t nn = a_.nn;
    const double d = a_.d;
    const T* const r = a_.r;
    T* const z = a_.z;
    T* const res = a_.res;
    const int mode = a_.mode;
    __shared__ double sh[kThreads];
    double x = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) x += partials[SL_AUX * kRedBlocks + b];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const T td = (T)d;
        const T dot = (T)sh[0];
        const T v = r[3 * nn] - dot - td * z[3 * nn];
        if (mode == 0)
            z[3 * nn] += v / td;
        else
            res[3 * nn] = v;
    }
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_alpha_fin, AlphaFinArgs<T>, alpha_fin_body<T>)

// ---------------------------------------------------------------------------
// transfers (Section 6.2): trilinear prolongation P, restriction P^T,
// identity on alpha
// ---------------------------------------------------------------------------
// restriction P^T; with_alpha: the alpha entry by identity.  With nb > 0 the
// parent's alpha residual res_a = r_a - acol.z - d z_a is formed here first
// (block 0, from the nb partial sums parts of acol . z of the residual kernel) and
// becomes the coarse alpha entry.
template <typename T>
struct RestrictArgs {
    Level<T> F;
    Level<T> C;
    const T* rf;
    T* rc;
    int with_alpha;
    const double* parts;
    int nb;
    double d;
};

template <typename T>
__device__ __forceinline__ void restrict_body(const RestrictArgs<T>& a_) {
    const Level<T>& F = a_.F;
    const Level<T>& C = a_.C;
    const T* const rf = a_.rf;
    T* const rc = a_.rc;
    const int with_alpha = a_.with_alpha;
    const double* const parts = a_.parts;
    const int nb = a_.nb;
    const double d = a_.d;
    __shared__ double sh[kThreads];
    if (nb > 0 && blockIdx.x == 0) {
        const T v = alpha_residual<T>(parts, nb, d, F.r[3 * F.nn], F.z[3 * F.nn], sh);
        if (threadIdx.x == 0) {
            F.res[3 * F.nn] = v;
            rc[3 * C.nn] = v;
        }
    }
    const int64_t N = gidx();
    if (N >= C.nn) return;
    const int I = (int)(N % C.NX);
    const int64_t tt = N / C.NX;
    const int J = (int)(tt % C.NY), K = (int)(tt / C.NY);
    T a0 = 0, a1 = 0, a2 = 0;
    for (int dk = -1; dk <= 1; ++dk) {
        const int k = 2 * K + dk;
        if (k < 0 || k >= F.NZ) continue;
        const T wk = dk ? T(0.5) : T(1);
        for (int dj = -1; dj <= 1; ++dj) {
            const int j = 2 * J + dj;
            if (j < 0 || j >= F.NY) continue;
            const T wj = dj ? T(0.5) : T(1);
            for (int di = -1; di <= 1; ++di) {
                const int i = 2 * I + di;
                if (i < 0 || i >= F.NX) continue;
                const T wgt = wk * wj * (di ? T(0.5) : T(1));
                const int64_t n = nat(i, j, k, F.NX, F.NY);
                a0 += wgt * rf[3 * n];
                a1 += wgt * rf[3 * n + 1];
                a2 += wgt * rf[3 * n + 2];
            }
        }
    }
    rc[3 * N] = C.fixed[3 * N] ? T(0) : a0;
    rc[3 * N + 1] = C.fixed[3 * N + 1] ? T(0) : a1;
    rc[3 * N + 2] = C.fixed[3 * N + 2] ? T(0) : a2;
    if (with_alpha && nb <= 0 && N == 0) rc[3 * C.nn] = rf[3 * F.nn];
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_restrict, RestrictArgs<T>, restrict_body<T>)

template <typename T>
struct ProlongArgs {
    Level<T> C;
    Level<T> F;
    const T* zc;
    T* zf;
};

template <typename T>
__device__ __forceinline__ void prolong_add_body(const ProlongArgs<T>& a_) {
    const Level<T>& C = a_.C;
    const Level<T>& F = a_.F;
    const T* const zc = a_.zc;
    T* const zf = a_.zf;
    const int64_t n = gidx();
    if (n >= F.nn) return;
    const int i = (int)(n % F.NX);
    const int64_t tt = n / F.NX;
    const int j = (int)(tt % F.NY), k = (int)(tt / F.NY);
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1,
              k1 = (k + 1) >> 1;
    const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
    T a0 = 0, a1 = 0, a2 = 0;
    for (int b = 0; b < 8; ++b) {
        const int I = (b & 1) ? i1 : i0, J = ((b >> 1) & 1) ? j1 : j0, K = (b >> 2) ? k1 : k0;
        // an even index has a single parent: count it once
        if ((b & 1) && !(i & 1)) continue;
        if (((b >> 1) & 1) && !(j & 1)) continue;
        if ((b >> 2) && !(k & 1)) continue;
        const int64_t N = nat(I, J, K, C.NX, C.NY);
        const T wgt = wi * wj * wk;
        a0 += wgt * zc[3 * N];
        a1 += wgt * zc[3 * N + 1];
        a2 += wgt * zc[3 * N + 2];
    }
    if (!F.fixed[3 * n]) zf[3 * n] += a0;
    if (!F.fixed[3 * n + 1]) zf[3 * n + 1] += a1;
    if (!F.fixed[3 * n + 2]) zf[3 * n + 2] += a2;
    if (n == 0) zf[3 * F.nn] += zc[3 * C.nn];
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_prolong_add, ProlongArgs<T>, prolong_add_body<T>)

// ---------------------------------------------------------------------------
// coarsest level: dense S_1 on (free DOFs, alpha), Cholesky, solve (FP64)
// ---------------------------------------------------------------------------
__global__ void k_zero(double* a, int64_t n) {
    const int64_t t = gidx();
    if (t < n) a[t] = 0.0;
}

template <typename T>
__global__ void k_coarse_assemble(Level<T> L, const int* __restrict__ cmap, int nc, double d,
                                  double* __restrict__ A) {
    const int64_t g = gidx();
    if (g >= L.nn * kStencil) return;
    const int64_t t = g / kStencil;
    const int s = (int)(g % kStencil);
    int i, j, k;
    cm_decode(L, t, i, j, k);
    const int64_t n = nat(i, j, k, L.NX, L.NY);
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    if (ii >= 0 && ii < L.NX && jj >= 0 && jj < L.NY && kk >= 0 && kk < L.NZ) {
        const int64_t mm = nat(ii, jj, kk, L.NX, L.NY);
        for (int r = 0; r < 3; ++r) {
            const int row = cmap[3 * n + r];
            if (row < 0) continue;
            for (int c = 0; c < 3; ++c) {
                const int col = cmap[3 * mm + c];
                if (col < 0) continue;
                A[(int64_t)row * nc + col] = (double)L.st[(int64_t)(s * 9 + r * 3 + c) * L.nn + t];
            }
        }
    }
    if (s == 0) {
        for (int r = 0; r < 3; ++r) {
            const int row = cmap[3 * n + r];
            if (row < 0) continue;
            const double v = (double)L.acol[3 * n + r];
            A[(int64_t)row * nc + nc - 1] = v;
            A[(int64_t)(nc - 1) * nc + row] = v;
        }
    }
    if (g == 0) A[(int64_t)(nc - 1) * nc + nc - 1] = d;
}

// in-place lower Cholesky, one block; flag = 1 on a non-positive pivot
__global__ void __launch_bounds__(1024) k_cholesky(double* __restrict__ A, int nc, int* flag) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        if (threadIdx.x == 0) {
            const double akk = A[(int64_t)k * nc + k];
            if (!(akk > 0.0)) {
                bad = 1;
                A[(int64_t)k * nc + k] = 1.0;
            } else {
                A[(int64_t)k * nc + k] = sqrt(akk);
            }
        }
        __syncthreads();
        const double dkk = A[(int64_t)k * nc + k];
        for (int i = k + 1 + threadIdx.x; i < nc; i += blockDim.x) A[(int64_t)i * nc + k] /= dkk;
        __syncthreads();
        const int T = nc - k - 1;
        for (int p = threadIdx.x; p < T * T; p += blockDim.x) {
            const int i = k + 1 + p / T, j = k + 1 + p % T;
            if (j <= i) A[(int64_t)i * nc + j] -= A[(int64_t)i * nc + k] * A[(int64_t)j * nc + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *flag = bad;
}

template <typename T>
struct CoarseSolveArgs {
    const double* A;
    int nc;
    const int* cmap;
    int64_t nn;
    const T* r;
    T* z;
};

template <typename T>
__device__ __forceinline__ void coarse_solve_body(const CoarseSolveArgs<T>& a_) {
    const double* const A = a_.A;
    const int nc = a_.nc;
    const int* const cmap = a_.cmap;
    const int64_t nn = a_.nn;
    const T* const r = a_.r;
    T* const z = a_.z;
    __shared__ double x[kMaxCoarse];
    for (int64_t q = threadIdx.x; q < 3 * nn; q += blockDim.x) {
        const int c = cmap[q];
        if (c >= 0) x[c] = (double)r[q];
    }
    if (threadIdx.x == 0) x[nc - 1] = (double)r[3 * nn];
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        if (threadIdx.x == 0) x[k] /= A[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = k + 1 + threadIdx.x; i < nc; i += blockDim.x) x[i] -= A[(int64_t)i * nc + k] * xk;
        __syncthreads();
    }
    for (int k = nc - 1; k >= 0; --k) {
        if (threadIdx.x == 0) x[k] /= A[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] -= A[(int64_t)k * nc + i] * xk;
        __syncthreads();
    }
    for (int64_t q = threadIdx.x; q < 3 * nn; q += blockDim.x) {
        const int c = cmap[q];
        z[q] = c >= 0 ? (T)x[c] : T(0);
    }
    if (threadIdx.x == 0) z[3 * nn] = (T)x[nc - 1];
}

VTS_KERNEL_PAIR(template <typename T>, 1024, k_coarse_solve, CoarseSolveArgs<T>, coarse_solve_body<T>)


// ---------------------------------------------------------------------------
// fused entry steps of a level: the level's right-hand side (conversion of
// the finest input, or restriction of the parent's residual) together with
// its first forward colour, which with z = 0 reduces to z = D^-1 r on the
// colour-0 nodes and z = 0 elsewhere
// ---------------------------------------------------------------------------
// colour-major index of natural node (i, j, k)
template <typename T>
__device__ __forceinline__ int64_t cm_index(const Level<T>& L, int i, int j, int k) {
    const int col = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
    return L.coff[col] + (i >> 1) + (int64_t)L.cnx[col] * ((j >> 1) + (int64_t)L.cny[col] * (k >> 1));
}

// the first forward colour with z = 0: z = D^-1 r on colour-0 nodes, zero
// elsewhere
template <typename T>
__device__ __forceinline__ void first_colour(const Level<T>& L, int64_t N, int i, int j, int k,
                                               T r0, T r1, T r2) {
    T z0 = 0, z1 = 0, z2 = 0;
    if (((i | j | k) & 1) == 0) {
        const int64_t t = cm_index(L, i, j, k);
        T D[9];
        for (int q = 0; q < 9; ++q) D[q] = L.dinv[(int64_t)q * L.nn + t];
        // b = r - acol z_a - S z with z = 0
        z0 = T(0) + (D[0] * r0 + D[1] * r1 + D[2] * r2);
        z1 = T(0) + (D[3] * r0 + D[4] * r1 + D[5] * r2);
        z2 = T(0) + (D[6] * r0 + D[7] * r1 + D[8] * r2);
    }
    L.z[3 * N] = z0;
    L.z[3 * N + 1] = z1;
    L.z[3 * N + 2] = z2;
}

// finest level: r (FP64 S-vector) into the level's precision, then the first colour
template <typename T>
struct TopInitArgs {
    Level<T> L;
    const double* rin;
};

template <typename T>
__device__ __forceinline__ void top_init_body(const TopInitArgs<T>& a_) {
    const Level<T>& L = a_.L;
    const double* const rin = a_.rin;
    const int64_t N = gidx();
    if (N < L.nn) {
        const int i = (int)(N % L.NX);
        const int64_t tt = N / L.NX;
        const int j = (int)(tt % L.NY), k = (int)(tt / L.NY);
        const T r0 = (T)rin[3 * N], r1 = (T)rin[3 * N + 1], r2 = (T)rin[3 * N + 2];
        L.r[3 * N] = r0;
        L.r[3 * N + 1] = r1;
        L.r[3 * N + 2] = r2;
        first_colour(L, N, i, j, k, r0, r1, r2);
    }
    if (N == 0) {
        L.r[3 * L.nn] = (T)rin[3 * L.nn];
        L.z[3 * L.nn] = T(0);
    }
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_top_init, TopInitArgs<T>, top_init_body<T>)

// restriction P^T of the parent's residual (alpha by identity), then the
// child's first colour
template <typename T>
struct RestrictInitArgs {
    Level<T> F;
    Level<T> C;
    const T* rf;
    const double* parts;
    int nb;
    double d;
};

template <typename T>
__device__ __forceinline__ void restrict_init_body(const RestrictInitArgs<T>& a_) {
    const Level<T>& F = a_.F;
    const Level<T>& C = a_.C;
    const T* const rf = a_.rf;
    const double* const parts = a_.parts;
    const int nb = a_.nb;
    const double d = a_.d;
    __shared__ double sh[kThreads];
    T va = T(0);
    if (blockIdx.x == 0)
        va = alpha_residual<T>(parts, nb, d, F.r[3 * F.nn], F.z[3 * F.nn], sh);
    const int64_t N = gidx();
    if (N < C.nn) {
        const int I = (int)(N % C.NX);
        const int64_t tt = N / C.NX;
        const int J = (int)(tt % C.NY), K = (int)(tt / C.NY);
        T a0 = 0, a1 = 0, a2 = 0;
        for (int dk = -1; dk <= 1; ++dk) {
            const int k = 2 * K + dk;
            if (k < 0 || k >= F.NZ) continue;
            const T wk = dk ? T(0.5) : T(1);
            for (int dj = -1; dj <= 1; ++dj) {
                const int j = 2 * J + dj;
                if (j < 0 || j >= F.NY) continue;
                const T wj = dj ? T(0.5) : T(1);
                for (int di = -1; di <= 1; ++di) {
                    const int i = 2 * I + di;
                    if (i < 0 || i >= F.NX) continue;
                    const T wgt = wk * wj * (di ? T(0.5) : T(1));
                    const int64_t n = nat(i, j, k, F.NX, F.NY);
                    a0 += wgt * rf[3 * n];
                    a1 += wgt * rf[3 * n + 1];
                    a2 += wgt * rf[3 * n + 2];
                }
            }
        }
        const T r0 = C.fixed[3 * N] ? T(0) : a0;
        const T r1 = C.fixed[3 * N + 1] ? T(0) : a1;
        const T r2 = C.fixed[3 * N + 2] ? T(0) : a2;
        C.r[3 * N] = r0;
        C.r[3 * N + 1] = r1;
        C.r[3 * N + 2] = r2;
        first_colour(C, N, I, J, K, r0, r1, r2);
    }
    if (N == 0) {
        F.res[3 * F.nn] = va;
        C.r[3 * C.nn] = va;
        C.z[3 * C.nn] = T(0);
    }
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_restrict_init, RestrictInitArgs<T>, restrict_init_body<T>)

// ---------------------------------------------------------------------------
// finest level without a stored stencil: one Gauss-Seidel colour pass, eight
// lanes per node of the colour, lane o for the element at offset o (bit set =
// element on the low side; the node is that element's corner a = o).  Lane o
// forms its element's share of the node's row of S z,
// rho'_e (K_e z_e)_a + w_e b_{e,a} (b_e^T z_e), with b_e^T z_e = te kept
// current by the passes themselves; the eight shares meet in a butterfly
// over the lane group (the same tree, hence the same sum, in every lane).
// After the node's update each lane adds b_{e,a} . dz to its element's te;
// every element has exactly one node of each colour, so each te has one
// writer per pass.
// ---------------------------------------------------------------------------
constexpr int kMfBlock = 256;   // 32 nodes of 8 lanes

// The rows of K_e at corner a follow from those at corner 0 by the cube's
// reflections: K_e[3a+r][3b+c] = s_r(a) s_c(a) K0[a^b][r][c], s_r(a) = -1 if
// bit r of a is set (reflecting axis r maps corner a to a ^ 2^r and flips the
// r components).  K0[d][r][c] = K_e[r][3d+c]: 72 numbers for all corners.
// With d = a ^ b the block K0[d] is the same for every lane, and node b of
// the element sits at offset d_x (1 - 2 a_x) (and likewise in y, z) from the
// node itself.
template <typename T>
struct KeRows0 {
    T v[8 * 9];
};

template <typename T>
struct GsMfArgs {
    Level<T> L;
    int col;
    KeRows0<T> K0;
    const T* r1;
    const T* w;
    const T* bc;
    T* te;
};

template <typename T>
__device__ __forceinline__ void gs_mf_body(const GsMfArgs<T>& a_) {
    const Level<T>& L = a_.L;
    const int col = a_.col;
    const KeRows0<T>& K0 = a_.K0;
    const T* const r1 = a_.r1;
    const T* const w = a_.w;
    const T* const bc = a_.bc;
    T* const te = a_.te;
    const int64_t g = gidx();
    const uint32_t tl = (uint32_t)(g >> 3);
    const int o = (int)(g & 7);
    const uint32_t cnt = (uint32_t)(L.coff[col + 1] - L.coff[col]);
    if (tl >= cnt) return;   // whole lane groups leave together
    const int64_t tcm = L.coff[col] + tl;
    const uint32_t cnx = (uint32_t)L.cnx[col], cny = (uint32_t)L.cny[col];
    const uint32_t q1 = tl / cnx, q2 = q1 / cny;
    const int i = 2 * (int)(tl - q1 * cnx) + (col & 1);
    const int j = 2 * (int)(q1 - q2 * cny) + ((col >> 1) & 1);
    const int k = 2 * (int)q2 + (col >> 2);
    const int64_t n = nat(i, j, k, L.NX, L.NY);
    const int ax = o & 1, ay = (o >> 1) & 1, az = o >> 2;
    const int ii = i - ax, jj = j - ay, kk = k - az;
    const bool in = ii >= 0 && ii < L.nx && jj >= 0 && jj < L.ny && kk >= 0 && kk < L.nz;
    const int64_t e = in ? ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk) : 0;
    const T* __restrict__ bb = bc + tcm * 24 + 3 * o;
    const T bb0 = bb[0], bb1 = bb[1], bb2 = bb[2];
    const T rr = in ? r1[e] : T(0);
    const T tv = in ? te[e] : T(0);
    const T wt = in ? w[e] * tv : T(0);
    T* __restrict__ z = L.z;
    // K0[d] z_b summed over the element's nodes, per (row, column) pair
    T A[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) A[q] = T(0);
    T zc0 = 0, zc1 = 0, zc2 = 0;
    if (in) {
        const int64_t sy = L.NX, sz = (int64_t)L.NX * L.NY;
        const int64_t ox = 1 - 2 * ax, oy = sy * (1 - 2 * ay), oz = sz * (1 - 2 * az);
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int64_t mm = n + ((d & 1) ? ox : 0) + ((d & 2) ? oy : 0) + ((d & 4) ? oz : 0);
            const T x0 = z[3 * mm], x1 = z[3 * mm + 1], x2 = z[3 * mm + 2];
            if (d == 0) {
                zc0 = x0;
                zc1 = x1;
                zc2 = x2;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                A[3 * r] += K0.v[d * 9 + 3 * r] * x0;
                A[3 * r + 1] += K0.v[d * 9 + 3 * r + 1] * x1;
                A[3 * r + 2] += K0.v[d * 9 + 3 * r + 2] * x2;
            }
        }
    } else {
        zc0 = z[3 * n];
        zc1 = z[3 * n + 1];
        zc2 = z[3 * n + 2];
    }
    // this element's share of -(S z)_a: -rho' s_r(a) sum_c s_c(a) A[r][c] - w t b_a
    const T sx = ax ? T(-1) : T(1), sy_ = ay ? T(-1) : T(1), sz_ = az ? T(-1) : T(1);
    const T y0 = sx * A[0] + sy_ * A[1] + sz_ * A[2];
    const T y1 = sx * A[3] + sy_ * A[4] + sz_ * A[5];
    const T y2 = sx * A[6] + sy_ * A[7] + sz_ * A[8];
    T p0 = -(rr * sx) * y0 - wt * bb0;
    T p1 = -(rr * sy_) * y1 - wt * bb1;
    T p2 = -(rr * sz_) * y2 - wt * bb2;
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        p0 += __shfl_xor(p0, off, 8);
        p1 += __shfl_xor(p1, off, 8);
        p2 += __shfl_xor(p2, off, 8);
    }
    const T za = z[3 * L.nn];
    const T b0 = (L.r[3 * n] - L.acol[3 * n] * za) + p0;
    const T b1 = (L.r[3 * n + 1] - L.acol[3 * n + 1] * za) + p1;
    const T b2 = (L.r[3 * n + 2] - L.acol[3 * n + 2] * za) + p2;
    T D[9];
#pragma unroll
    for (int q9 = 0; q9 < 9; ++q9) D[q9] = L.dinv[(int64_t)q9 * L.nn + tcm];
    const T d0 = D[0] * b0 + D[1] * b1 + D[2] * b2;
    const T d1 = D[3] * b0 + D[4] * b1 + D[5] * b2;
    const T d2 = D[6] * b0 + D[7] * b1 + D[8] * b2;
    if (o == 0) {
        z[3 * n] = zc0 + d0;
        z[3 * n + 1] = zc1 + d1;
        z[3 * n + 2] = zc2 + d2;
    }
    if (in) te[e] = tv + (bb0 * d0 + bb1 * d1 + bb2 * d2);
}

VTS_KERNEL_PAIR(template <typename T>, kMfBlock, k_gs_mf, GsMfArgs<T>, gs_mf_body<T>)

// finest level without a stored stencil: r (FP64 S-vector) into T, the first
// colour (z = D^-1 r on colour-0 nodes, zero elsewhere), and te = b_e^T z_e,
// written by each element's colour-0 node
template <typename T>
struct TopInitMfArgs {
    Level<T> L;
    const double* rin;
    const T* bc;
    T* te;
};

template <typename T>
__device__ __forceinline__ void top_init_mf_body(const TopInitMfArgs<T>& a_) {
    const Level<T>& L = a_.L;
    const double* const rin = a_.rin;
    const T* const bc = a_.bc;
    T* const te = a_.te;
    const int64_t N = gidx();
    if (N < L.nn) {
        const int i = (int)(N % L.NX);
        const int64_t tt = N / L.NX;
        const int j = (int)(tt % L.NY), k = (int)(tt / L.NY);
        const T r0 = (T)rin[3 * N], r1 = (T)rin[3 * N + 1], r2 = (T)rin[3 * N + 2];
        L.r[3 * N] = r0;
        L.r[3 * N + 1] = r1;
        L.r[3 * N + 2] = r2;
        first_colour(L, N, i, j, k, r0, r1, r2);
        if (((i | j | k) & 1) == 0) {
            const int64_t t = cm_index(L, i, j, k);
            const T z0 = L.z[3 * N], z1 = L.z[3 * N + 1], z2 = L.z[3 * N + 2];
            for (int o = 0; o < 8; ++o) {
                const int ii = i - (o & 1), jj = j - ((o >> 1) & 1), kk = k - (o >> 2);
                if (ii < 0 || ii >= L.nx || jj < 0 || jj >= L.ny || kk < 0 || kk >= L.nz) continue;
                const T* bb = bc + t * 24 + 3 * o;
                te[ii + (int64_t)L.nx * (jj + (int64_t)L.ny * kk)] =
                    bb[0] * z0 + bb[1] * z1 + bb[2] * z2;
            }
        }
    }
    if (N == 0) {
        L.r[3 * L.nn] = (T)rin[3 * L.nn];
        L.z[3 * L.nn] = T(0);
    }
}

VTS_KERNEL_PAIR(template <typename T>, kThreads, k_top_init_mf, TopInitMfArgs<T>, top_init_mf_body<T>)

// ---------------------------------------------------------------------------
// large levels: one colour pass / residual with 9 waves per 64 nodes; wave g
// sums the three neighbours of row (dy, dz) = (g%3 - 1, g/3 - 1), the partial
// sums are combined in LDS in a fixed order
// ---------------------------------------------------------------------------
constexpr int kRowWaves = 9;
constexpr int kBlk9 = 64 * kRowWaves;

template <typename T>
__device__ __forceinline__ void row_partial(const Level<T>& L, int64_t t, int i, int j, int k,
                                            int g, const T* __restrict__ z, T& a0, T& a1, T& a2) {
    const int dy = g % 3 - 1, dz = g / 3 - 1;
    const int jj = j + dy, kk = k + dz;
    a0 = a1 = a2 = T(0);
    if (jj < 0 || jj >= L.NY || kk < 0 || kk >= L.NZ) return;
    const int64_t N = L.nn;
    for (int dx = -1; dx <= 1; ++dx) {
        const int ii = i + dx;
        if (ii < 0 || ii >= L.NX) continue;
        const int s = (dx + 1) + 3 * g;
        const int64_t mm = nat(ii, jj, kk, L.NX, L.NY);
        const T x0 = z[3 * mm], x1 = z[3 * mm + 1], x2 = z[3 * mm + 2];
        const T* S = L.st + (int64_t)(s * 9) * N + t;
        a0 += S[0] * x0 + S[N] * x1 + S[2 * N] * x2;
        a1 += S[3 * N] * x0 + S[4 * N] * x1 + S[5 * N] * x2;
        a2 += S[6 * N] * x0 + S[7 * N] * x1 + S[8 * N] * x2;
    }
}

// TOP = finest level (a separate instantiation so profiles tell them apart)
template <typename T>
struct GsColor9Args {
    Level<T> L;
    int col;
    const T* r;
    T* z;
};

template <typename T>
__device__ __forceinline__ void gs_color9_body(const GsColor9Args<T>& a_) {
    const Level<T>& L = a_.L;
    const int col = a_.col;
    const T* const r = a_.r;
    T* const z = a_.z;
    __shared__ T part[kRowWaves][3][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t cnt = L.coff[col + 1] - L.coff[col];
    const int64_t tl = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = tl < cnt;
    int i = 0, j = 0, k = 0;
    int64_t t = 0;
    T a0 = 0, a1 = 0, a2 = 0;
    int64_t n = 0;
    T b0 = 0, b1 = 0, b2 = 0, z0 = 0, z1 = 0, z2 = 0, D[9];
    if (valid) {
        t = L.coff[col] + tl;
        int64_t q = tl;
        i = 2 * (int)(q % L.cnx[col]) + (col & 1);
        q /= L.cnx[col];
        j = 2 * (int)(q % L.cny[col]) + ((col >> 1) & 1);
        k = 2 * (int)(q / L.cny[col]) + (col >> 2);
        n = nat(i, j, k, L.NX, L.NY);
        if (g == 0) {
            // operands of the update, loaded while the rows are summed
            const T za = z[3 * L.nn];
            b0 = r[3 * n] - L.acol[3 * n] * za;
            b1 = r[3 * n + 1] - L.acol[3 * n + 1] * za;
            b2 = r[3 * n + 2] - L.acol[3 * n + 2] * za;
            z0 = z[3 * n];
            z1 = z[3 * n + 1];
            z2 = z[3 * n + 2];
            for (int q9 = 0; q9 < 9; ++q9) D[q9] = L.dinv[(int64_t)q9 * L.nn + t];
        }
        row_partial(L, t, i, j, k, g, z, a0, a1, a2);
    }
    part[g][0][lane] = a0;
    part[g][1][lane] = a1;
    part[g][2][lane] = a2;
    __syncthreads();
    if (g == 0 && valid) {
        for (int h = 0; h < kRowWaves; ++h) {
            b0 -= part[h][0][lane];
            b1 -= part[h][1][lane];
            b2 -= part[h][2][lane];
        }
        z0 += D[0] * b0 + D[1] * b1 + D[2] * b2;
        z1 += D[3] * b0 + D[4] * b1 + D[5] * b2;
        z2 += D[6] * b0 + D[7] * b1 + D[8] * b2;
        z[3 * n] = z0;
        z[3 * n + 1] = z1;
        z[3 * n + 2] = z2;
    }
}

// TOP = finest level (a separate instantiation so profiles tell them apart)
template <typename T, bool TOP>
__global__ void __launch_bounds__(kBlk9) k_gs_color9(GsColor9Args<T> a) {
    gs_color9_body<T>(a);
}
template <typename T, bool TOP>
__global__ void __launch_bounds__(kBlk9) k_gs_color9_b(const GsColor9Args<T>* __restrict__ tab) {
    gs_color9_body<T>(tab[blockIdx.y]);
}

// res = r - S z (displacement part, masked) and per-block partial sums of
// acol . z (slot SL_STAT).  First the alpha step that ends the forward sweep,
// z_a += (r_a - acol.z - d z_a)/d from the nb partial sums of k_acol_dot
// (slot SL_AUX): every block forms it (identical value, fixed order) and
// block 0 stores it.  The level entered the sweep with z = 0 and the colour
// passes leave z_a alone, so z_a is 0 before this step and the blocks never
// read the location block 0 writes.
template <typename T>
struct Resid9Args {
    Level<T> L;
    const T* r;
    T* z;
    T* res;
    double* partials;
    int nb;
    double d;
};

template <typename T>
__device__ __forceinline__ void resid9_body(const Resid9Args<T>& a_) {
    const Level<T>& L = a_.L;
    const T* const r = a_.r;
    T* const z = a_.z;
    T* const res = a_.res;
    double* const partials = a_.partials;
    const int nb = a_.nb;
    const double d = a_.d;
    // row partial sums, double-buffered: the buffer of chunk q is rewritten
    // in chunk q + 2, after every wave has passed the barrier of chunk q + 1,
    // which wave 0 reaches only once it has read chunk q's sums
    __shared__ T part[2][kRowWaves][3][64];
    __shared__ double sh[kThreads];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const T za = T(0) + alpha_residual<T>(partials + SL_AUX * kRedBlocks, nb, d, r[3 * L.nn], T(0),
                                          sh) / (T)d;
    if (blockIdx.x == 0 && threadIdx.x == 0) z[3 * L.nn] = za;
    double acc = 0.0;
    int buf = 0;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < L.nn;
         base += (int64_t)gridDim.x * 64, buf ^= 1) {
        const int64_t t = base + lane;
        const bool valid = t < L.nn;
        int i = 0, j = 0, k = 0;
        int64_t n = 0;
        T a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
        if (valid) {
            cm_decode(L, t, i, j, k);
            if (g == 0) {
                // operands of the update, loaded while the rows are summed
                n = nat(i, j, k, L.NX, L.NY);
                b0 = r[3 * n] - L.acol[3 * n] * za;
                b1 = r[3 * n + 1] - L.acol[3 * n + 1] * za;
                b2 = r[3 * n + 2] - L.acol[3 * n + 2] * za;
            }
            row_partial(L, t, i, j, k, g, z, a0, a1, a2);
        }
        part[buf][g][0][lane] = a0;
        part[buf][g][1][lane] = a1;
        part[buf][g][2][lane] = a2;
        __syncthreads();
        if (g == 0 && valid) {
            for (int h = 0; h < kRowWaves; ++h) {
                b0 -= part[buf][h][0][lane];
                b1 -= part[buf][h][1][lane];
                b2 -= part[buf][h][2][lane];
            }
            res[3 * n] = L.fixed[3 * n] ? T(0) : b0;
            res[3 * n + 1] = L.fixed[3 * n + 1] ? T(0) : b1;
            res[3 * n + 2] = L.fixed[3 * n + 2] ? T(0) : b2;
            acc += (double)L.acol[3 * n] * z[3 * n] + (double)L.acol[3 * n + 1] * z[3 * n + 1] +
                   (double)L.acol[3 * n + 2] * z[3 * n + 2];
        }
    }
    if (g == 0) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) partials[SL_STAT * kRedBlocks + blockIdx.x] = acc;
    }
}

template <typename T, bool TOP>
__global__ void __launch_bounds__(kBlk9) k_resid9(Resid9Args<T> a) {
    resid9_body<T>(a);
}
template <typename T, bool TOP>
__global__ void __launch_bounds__(kBlk9) k_resid9_b(const Resid9Args<T>* __restrict__ tab) {
    resid9_body<T>(tab[blockIdx.y]);
}

// ---------------------------------------------------------------------------
// small levels: the whole V-cycle below a level in one workgroup (phases
// separated by barriers), ending in the coarsest solve by the explicit inverse
// ---------------------------------------------------------------------------
template <typename T>
struct SmallArgs {
    Level<T> lev[kMaxSmallLevels];
    int ks;                  // top level handled here
    double d;                // alpha diagonal
    const double* Ainv;
    int nc;
    const int* cinv;
};

// One workgroup of 1024 threads.  A colour pass splits each node's 9 neighbour
// rows over G lanes (G = 9, 3 or 1, the largest that lets one pass cover the
// colour); partial sums meet in LDS in a fixed order.
constexpr int kSmallThreads = 1024;

template <typename T>
struct SmallShared {
    T part[3][kSmallThreads];
};

template <typename T>
__device__ void blk_gs_color(const Level<T>& L, int col, const T* r, T* z, SmallShared<T>& sh,
                             bool first) {
    const int64_t cnt = L.coff[col + 1] - L.coff[col];
    const int G = cnt * 9 <= kSmallThreads ? 9 : (cnt * 3 <= kSmallThreads ? 3 : 1);
    const int slots = kSmallThreads / G;
    const int slot = threadIdx.x % slots, g = threadIdx.x / slots;
    const bool lane_on = g < G;
    const T za = first ? T(0) : z[3 * L.nn];
    for (int64_t base = 0; base < cnt; base += slots) {
        const int64_t tl = base + slot;
        const bool valid = lane_on && tl < cnt;
        int i = 0, j = 0, k = 0;
        int64_t t = 0, n = 0;
        T a0 = 0, a1 = 0, a2 = 0;
        T c0 = 0, c1 = 0, c2 = 0, y0 = 0, y1 = 0, y2 = 0, D[9];
        if (valid) {
            t = L.coff[col] + tl;
            int64_t q = tl;
            i = 2 * (int)(q % L.cnx[col]) + (col & 1);
            q /= L.cnx[col];
            j = 2 * (int)(q % L.cny[col]) + ((col >> 1) & 1);
            k = 2 * (int)(q / L.cny[col]) + (col >> 2);
            n = nat(i, j, k, L.NX, L.NY);
            if (g == 0) {
                c0 = r[3 * n] - L.acol[3 * n] * za;
                c1 = r[3 * n + 1] - L.acol[3 * n + 1] * za;
                c2 = r[3 * n + 2] - L.acol[3 * n + 2] * za;
                if (!first) {
                    y0 = z[3 * n];
                    y1 = z[3 * n + 1];
                    y2 = z[3 * n + 2];
                }
                for (int q9 = 0; q9 < 9; ++q9) D[q9] = L.dinv[(int64_t)q9 * L.nn + t];
            }
            if (!first) {
                const int per = kRowWaves / G;
                for (int h = g * per; h < (g + 1) * per; ++h) {
                    T b0, b1, b2;
                    row_partial(L, t, i, j, k, h, z, b0, b1, b2);
                    a0 += b0;
                    a1 += b1;
                    a2 += b2;
                }
            }
        }
        if (G > 1) {
            if (lane_on) {
                sh.part[0][threadIdx.x] = a0;
                sh.part[1][threadIdx.x] = a1;
                sh.part[2][threadIdx.x] = a2;
            }
            __syncthreads();
        }
        if (valid && g == 0) {
            for (int h = 1; h < G; ++h) {
                a0 += sh.part[0][h * slots + slot];
                a1 += sh.part[1][h * slots + slot];
                a2 += sh.part[2][h * slots + slot];
            }
            const T b0 = c0 - a0, b1 = c1 - a1, b2 = c2 - a2;
            z[3 * n] = y0 + (D[0] * b0 + D[1] * b1 + D[2] * b2);
            z[3 * n + 1] = y1 + (D[3] * b0 + D[4] * b1 + D[5] * b2);
            z[3 * n + 2] = y2 + (D[6] * b0 + D[7] * b1 + D[8] * b2);
        }
        __syncthreads();
    }
}

// mode 0: z_a += (r_a - acol.z - d z_a)/d ; mode 1: res_a = r_a - acol.z - d z_a
template <typename T>
__device__ void blk_alpha(const Level<T>& L, const T* r, T* z, T* res, double d, double* red,
                          int mode) {
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < 3 * L.nn; q += blockDim.x)
        acc += (double)L.acol[q] * (double)z[q];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
        const T td = (T)d;
        const T v = r[3 * L.nn] - (T)sum - td * z[3 * L.nn];
        if (mode == 0)
            z[3 * L.nn] += v / td;
        else
            res[3 * L.nn] = v;
    }
    __syncthreads();
}

template <typename T>
__device__ void blk_resid(const Level<T>& L, const T* r, const T* z, T* res) {
    const T za = z[3 * L.nn];
    for (int64_t t = threadIdx.x; t < L.nn; t += blockDim.x) {
        int i, j, k;
        cm_decode(L, t, i, j, k);
        const int64_t n = nat(i, j, k, L.NX, L.NY);
        T b0 = r[3 * n] - L.acol[3 * n] * za;
        T b1 = r[3 * n + 1] - L.acol[3 * n + 1] * za;
        T b2 = r[3 * n + 2] - L.acol[3 * n + 2] * za;
        for (int h = 0; h < kRowWaves; ++h) {
            T a0, a1, a2;
            row_partial(L, t, i, j, k, h, z, a0, a1, a2);
            b0 -= a0;
            b1 -= a1;
            b2 -= a2;
        }
        res[3 * n] = L.fixed[3 * n] ? T(0) : b0;
        res[3 * n + 1] = L.fixed[3 * n + 1] ? T(0) : b1;
        res[3 * n + 2] = L.fixed[3 * n + 2] ? T(0) : b2;
    }
    __syncthreads();
}

template <typename T>
__device__ void blk_restrict(const Level<T>& F, const Level<T>& C, const T* rf, T* rc) {
    for (int64_t N = threadIdx.x; N < C.nn; N += blockDim.x) {
        const int I = (int)(N % C.NX);
        const int64_t tt = N / C.NX;
        const int J = (int)(tt % C.NY), K = (int)(tt / C.NY);
        T a0 = 0, a1 = 0, a2 = 0;
        for (int dk = -1; dk <= 1; ++dk) {
            const int k = 2 * K + dk;
            if (k < 0 || k >= F.NZ) continue;
            const T wk = dk ? T(0.5) : T(1);
            for (int dj = -1; dj <= 1; ++dj) {
                const int j = 2 * J + dj;
                if (j < 0 || j >= F.NY) continue;
                const T wj = dj ? T(0.5) : T(1);
                for (int di = -1; di <= 1; ++di) {
                    const int i = 2 * I + di;
                    if (i < 0 || i >= F.NX) continue;
                    const T wgt = wk * wj * (di ? T(0.5) : T(1));
                    const int64_t n = nat(i, j, k, F.NX, F.NY);
                    a0 += wgt * rf[3 * n];
                    a1 += wgt * rf[3 * n + 1];
                    a2 += wgt * rf[3 * n + 2];
                }
            }
        }
        rc[3 * N] = C.fixed[3 * N] ? T(0) : a0;
        rc[3 * N + 1] = C.fixed[3 * N + 1] ? T(0) : a1;
        rc[3 * N + 2] = C.fixed[3 * N + 2] ? T(0) : a2;
    }
    if (threadIdx.x == 0) rc[3 * C.nn] = rf[3 * F.nn];
    __syncthreads();
}

template <typename T>
__device__ void blk_prolong(const Level<T>& C, const Level<T>& F, const T* zc, T* zf) {
    for (int64_t n = threadIdx.x; n < F.nn; n += blockDim.x) {
        const int i = (int)(n % F.NX);
        const int64_t tt = n / F.NX;
        const int j = (int)(tt % F.NY), k = (int)(tt / F.NY);
        const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1,
                  k1 = (k + 1) >> 1;
        const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1),
                wk = (k & 1) ? T(0.5) : T(1);
        T a0 = 0, a1 = 0, a2 = 0;
        for (int b = 0; b < 8; ++b) {
            if ((b & 1) && !(i & 1)) continue;
            if (((b >> 1) & 1) && !(j & 1)) continue;
            if ((b >> 2) && !(k & 1)) continue;
            const int I = (b & 1) ? i1 : i0, J = ((b >> 1) & 1) ? j1 : j0, K = (b >> 2) ? k1 : k0;
            const int64_t N = nat(I, J, K, C.NX, C.NY);
            const T wgt = wi * wj * wk;
            a0 += wgt * zc[3 * N];
            a1 += wgt * zc[3 * N + 1];
            a2 += wgt * zc[3 * N + 2];
        }
        if (!F.fixed[3 * n]) zf[3 * n] += a0;
        if (!F.fixed[3 * n + 1]) zf[3 * n + 1] += a1;
        if (!F.fixed[3 * n + 2]) zf[3 * n + 2] += a2;
    }
    if (threadIdx.x == 0) zf[3 * F.nn] += zc[3 * C.nn];
    __syncthreads();
}

template <typename T>
struct VSmallArgs {
    SmallArgs<T> a;
};

template <typename T>
__device__ __forceinline__ void vcycle_small_body(const VSmallArgs<T>& a_) {
    const SmallArgs<T>& a = a_.a;
    __shared__ double red[kSmallThreads / 64];
    __shared__ double xs[kSmallCoarse];
    __shared__ SmallShared<T> sh;
    // restriction phase: levels ks .. 1
    for (int k = a.ks; k >= 1; --k) {
        const Level<T>& L = a.lev[k];
        // z = 0 except colour 0, which the first pass sets to D^{-1} r
        for (int64_t t = L.coff[1] + threadIdx.x; t < L.nn; t += blockDim.x) {
            int i, j, kk;
            cm_decode(L, t, i, j, kk);
            const int64_t n = nat(i, j, kk, L.NX, L.NY);
            L.z[3 * n] = T(0);
            L.z[3 * n + 1] = T(0);
            L.z[3 * n + 2] = T(0);
        }
        if (threadIdx.x == 0) L.z[3 * L.nn] = T(0);
        blk_gs_color(L, 0, L.r, L.z, sh, true);
        for (int col = 1; col < 8; ++col) blk_gs_color(L, col, L.r, L.z, sh, false);
        blk_alpha(L, L.r, L.z, L.res, a.d, red, 0);
        blk_resid(L, L.r, L.z, L.res);
        blk_alpha(L, L.r, L.z, L.res, a.d, red, 1);
        blk_restrict(L, a.lev[k - 1], L.res, a.lev[k - 1].r);
    }
    // coarsest level: z0 = S_0^{-1} r0 with the explicit inverse
    {
        const Level<T>& L = a.lev[0];
        const int nc = a.nc;
        for (int q = threadIdx.x; q < nc - 1; q += blockDim.x) xs[q] = (double)L.r[a.cinv[q]];
        if (threadIdx.x == 0) xs[nc - 1] = (double)L.r[3 * L.nn];
        for (int64_t q = threadIdx.x; q < 3 * L.nn + 1; q += blockDim.x) L.z[q] = T(0);
        __syncthreads();
        for (int row = threadIdx.x; row < nc; row += blockDim.x) {
            const double* Ar = a.Ainv + (int64_t)row * nc;
            double y = 0.0;
            for (int col = 0; col < nc; ++col) y += Ar[col] * xs[col];
            if (row < nc - 1)
                L.z[a.cinv[row]] = (T)y;
            else
                L.z[3 * L.nn] = (T)y;
        }
        __syncthreads();
    }
    // prolongation phase: levels 1 .. ks
    for (int k = 1; k <= a.ks; ++k) {
        const Level<T>& L = a.lev[k];
        blk_prolong(a.lev[k - 1], L, a.lev[k - 1].z, L.z);
        blk_alpha(L, L.r, L.z, L.res, a.d, red, 0);
        for (int col = 7; col >= 0; --col) blk_gs_color(L, col, L.r, L.z, sh, false);
    }
}

VTS_KERNEL_PAIR(template <typename T>, 1024, k_vcycle_small, VSmallArgs<T>, vcycle_small_body<T>)

// column j of the inverse of L L^T (Cholesky factor in A), one block per column
__global__ void __launch_bounds__(256)
k_chol_inverse(const double* __restrict__ A, int nc, double* __restrict__ Ainv) {
    __shared__ double x[kMaxCoarse];
    const int jcol = blockIdx.x;
    for (int q = threadIdx.x; q < nc; q += blockDim.x) x[q] = (q == jcol) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        if (threadIdx.x == 0) x[k] /= A[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = k + 1 + threadIdx.x; i < nc; i += blockDim.x) x[i] -= A[(int64_t)i * nc + k] * xk;
        __syncthreads();
    }
    for (int k = nc - 1; k >= 0; --k) {
        if (threadIdx.x == 0) x[k] /= A[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] -= A[(int64_t)k * nc + i] * xk;
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nc; q += blockDim.x) Ainv[(int64_t)q * nc + jcol] = x[q];
}

template <typename Tin, typename Tout>
struct ConvertArgs {
    const Tin* a;
    Tout* b;
    int64_t n;
};

template <typename Tin, typename Tout>
__device__ __forceinline__ void convert_body(const ConvertArgs<Tin, Tout>& a_) {
    const Tin* const a = a_.a;
    Tout* const b = a_.b;
    const int64_t n = a_.n;
    const int64_t t = gidx();
    if (t < n) b[t] = (Tout)a[t];
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kThreads) k_convert(ConvertArgs<Tin, Tout> a) {
    convert_body<Tin, Tout>(a);
}
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kThreads) k_convert_b(const ConvertArgs<Tin, Tout>* __restrict__ tab) {
    convert_body<Tin, Tout>(tab[blockIdx.y]);
}

template <typename T>
__global__ void k_zero_t(T* a, int64_t n) {
    const int64_t t = gidx();
    if (t < n) a[t] = T(0);
}

}  // namespace

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
template <typename T>
void mg_build(Ctx& c, Hierarchy<T>& H) {
    const int L = (int)H.lev.size();
    Level<T>& fine = H.lev[L - 1];
    if (H.mf) {
        hipLaunchKernelGGL(k_fine_mf_setup<T>, dim3(grid_of(fine.nn)), dim3(kThreads), 0, c.s,
                           fine, c.Ke, c.r1, c.w, c.be, H.bc);
        if (sizeof(T) == 4)
            hipLaunchKernelGGL(k_fine_mf_convert<T>,
                               dim3(grid_of(std::max<int64_t>(fine.m, 3 * fine.nn))),
                               dim3(kThreads), 0, c.s, fine.m, 3 * fine.nn, c.r1, c.w, c.u, H.r1f,
                               H.wf, H.uf);
    } else {
        hipLaunchKernelGGL(k_fine_stencil<T>, dim3(grid_of(fine.nn)), dim3(kThreads), 0, c.s,
                           fine, c.Ke, c.r1, c.w, c.be);
    }
    if (L >= 2) {
        hipLaunchKernelGGL(k_child_g, dim3(grid_of(c.m)), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz,
                           c.Qc, c.be, c.gch);
        Level<T>& C = H.lev[L - 2];
        hipLaunchKernelGGL(k_coarse_first<T>, dim3(grid_of(C.m * 24)), dim3(kThreads), 0, c.s, C,
                           c.nx, c.ny, c.nz, c.Mc, c.r1, c.w, c.gch);
        for (int k = L - 3; k >= 0; --k) {
            Level<T>& F = H.lev[k + 1];
            Level<T>& Cc = H.lev[k];
            hipLaunchKernelGGL(k_coarsen_tq<T>, dim3(grid_of(F.m * 24)), dim3(kThreads), 0, c.s, F,
                               c.Qc);
            hipLaunchKernelGGL(k_coarsen_e<T>, dim3(grid_of(Cc.m * 24)), dim3(kThreads), 0, c.s, Cc,
                               F, c.Qc);
        }
        for (int k = L - 2; k >= 0; --k) {
            Level<T>& Lk = H.lev[k];
            hipLaunchKernelGGL(k_elem_stencil<T>, dim3(grid_of(Lk.nn)), dim3(kThreads), 0, c.s, Lk);
            hipLaunchKernelGGL(k_restrict<T>, dim3(grid_of(Lk.nn)), dim3(kThreads), 0, c.s,
                               RestrictArgs<T>{H.lev[k + 1], Lk, H.lev[k + 1].acol, Lk.acol, 0,
                                               (const double*)nullptr, 0, 0.0});
        }
    }
    Level<T>& L0 = H.lev[0];
    const int64_t nA = (int64_t)H.nc * H.nc;
    hipLaunchKernelGGL(k_zero, dim3(grid_of(nA)), dim3(kThreads), 0, c.s, H.A, nA);
    hipLaunchKernelGGL(k_coarse_assemble<T>, dim3(grid_of(L0.nn * kStencil)), dim3(kThreads), 0,
                       c.s, L0, H.cmap, H.nc, c.sum_w, H.A);
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, c.s, H.A, H.nc, H.flag);
    if (H.ksmall >= 0)
        hipLaunchKernelGGL(k_chol_inverse, dim3(H.nc), dim3(256), 0, c.s, H.A, H.nc, H.Ainv);
}

// Gauss-Seidel colour passes of one sweep: forward colours 1..7 (colour 0
// was applied by the kernel that set up the level's r and z; the alpha
// update that follows is fused into the residual kernel), or backward
// colours 7..0.  On the finest level the colour passes are optionally
// bracketed by the profiling events of the context (kernel class
// VTS_PROF_GS_FINE), one event pair per sweep.
// a launch through vlaunch (issued, or recorded for a group launch)
template <class A, class K1, class K2>
static inline void vl(Ctx& c, K1 k, K2 kb, dim3 g, dim3 b, const A& a) {
    vlaunch(c, reinterpret_cast<const void*>(k), reinterpret_cast<const void*>(kb), g, b, a);
}

template <typename T>
static void gs_sweep(Ctx& c, Level<T>& Lk, bool forward, bool top) {
    const bool prof = top && prof_begin(c, VTS_PROF_GS_FINE);
    double bytes = 0.0;
    int launches = 0;
    for (int q = forward ? 1 : 0; q < 8; ++q) {
        const int col = forward ? q : 7 - q;
        const int64_t cnt = Lk.coff[col + 1] - Lk.coff[col];
        if (cnt == 0) continue;
        const dim3 grid((unsigned)((cnt + 63) / 64));
        const GsColor9Args<T> a{Lk, col, (const T*)Lk.r, Lk.z};
        if (top)
            vl(c, k_gs_color9<T, true>, k_gs_color9_b<T, true>, grid, dim3(kBlk9), a);
        else
            vl(c, k_gs_color9<T, false>, k_gs_color9_b<T, false>, grid, dim3(kBlk9), a);
        bytes += gs_color_bytes(Lk, col, sizeof(T));
        ++launches;
    }
    if (prof) prof_end(c, bytes, launches);
}

// the same sweep on the finest level without a stored stencil
template <typename T>
static void gs_sweep_mf(Ctx& c, Hierarchy<T>& H, Level<T>& Lk, bool forward) {
    const bool prof = prof_begin(c, VTS_PROF_GS_FINE);
    KeRows0<T> K0;
    for (int d = 0; d < 8; ++d)
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) K0.v[d * 9 + r * 3 + q] = (T)c.ke_host[r * 24 + 3 * d + q];
    double bytes = 0.0;
    int launches = 0;
    for (int q = forward ? 1 : 0; q < 8; ++q) {
        const int col = forward ? q : 7 - q;
        const int64_t cnt = Lk.coff[col + 1] - Lk.coff[col];
        if (cnt == 0) continue;
        vl(c, k_gs_mf<T>, k_gs_mf_b<T>, dim3((unsigned)((8 * cnt + kMfBlock - 1) / kMfBlock)),
           dim3(kMfBlock),
           GsMfArgs<T>{Lk, col, K0, (const T*)H.r1f, (const T*)H.wf, (const T*)H.bc, H.te});
        bytes += gs_mf_color_bytes(Lk, col, sizeof(T));
        ++launches;
    }
    if (prof) prof_end(c, bytes, launches);
}

// per-block partial sums of acol . z into SL_AUX; returns the block count
template <typename T>
static int acol_partials(Ctx& c, Level<T>& Lk) {
    const int gr = red_grid_of(3 * Lk.nn);
    vl(c, k_acol_dot<T>, k_acol_dot_b<T>, dim3(gr), dim3(kThreads),
       AcolDotArgs<T>{Lk, (const T*)Lk.z, c.partials});
    return gr;
}

// z_a += (r_a - acol . z - d z_a) / d
template <typename T>
static void alpha_update(Ctx& c, Level<T>& Lk) {
    const int gr = acol_partials(c, Lk);
    vl(c, k_alpha_fin<T>, k_alpha_fin_b<T>, dim3(1), dim3(kThreads),
       AlphaFinArgs<T>{c.partials, gr, Lk.nn, c.sum_w, (const T*)Lk.r, Lk.z, Lk.res, 0});
}

// V-cycle below level k.  On entry a multi-workgroup level (k > ksmall,
// k > 0) holds its r and z after the first forward colour.
template <typename T>
static void vcycle_level(Ctx& c, Hierarchy<T>& H, int k) {
    Level<T>& Lk = H.lev[k];
    const bool top = k == (int)H.lev.size() - 1;
    if (k <= H.ksmall) {
        SmallArgs<T> a;
        for (int q = 0; q <= k; ++q) a.lev[q] = H.lev[q];
        a.ks = k;
        a.d = c.sum_w;
        a.Ainv = H.Ainv;
        a.nc = H.nc;
        a.cinv = H.cinv;
        vl(c, k_vcycle_small<T>, k_vcycle_small_b<T>, dim3(1), dim3(1024), VSmallArgs<T>{a});
        return;
    }
    if (k == 0) {
        vl(c, k_coarse_solve<T>, k_coarse_solve_b<T>, dim3(1), dim3(1024),
           CoarseSolveArgs<T>{H.A, H.nc, H.cmap, Lk.nn, Lk.r, Lk.z});
        return;
    }
    const double d = c.sum_w;
    if (top && H.mf) {
        // finest level without a stored stencil: forward sweep, alpha update,
        // residual with the partial sums of acol . z (one per workgroup of the
        // residual kernel), restriction, coarse correction, prolongation, the
        // element products b_e^T z_e of the corrected z, alpha, backward sweep
        gs_sweep_mf(c, H, Lk, true);
        alpha_update(c, Lk);
        launch_fine_resid<T>(c, Lk, H.uf, H.r1f, H.wf, c.spart);
        const int nbr = fine_resid_blocks(c);
        Level<T>& Lc = H.lev[k - 1];
        if (k - 1 <= H.ksmall || k - 1 == 0)
            vl(c, k_restrict<T>, k_restrict_b<T>, dim3(grid_of(Lc.nn)), dim3(kThreads),
               RestrictArgs<T>{Lk, Lc, (const T*)Lk.res, Lc.r, 1, (const double*)c.spart, nbr, d});
        else
            vl(c, k_restrict_init<T>, k_restrict_init_b<T>, dim3(grid_of(Lc.nn)), dim3(kThreads),
               RestrictInitArgs<T>{Lk, Lc, (const T*)Lk.res, (const double*)c.spart, nbr, d});
        vcycle_level(c, H, k - 1);
        vl(c, k_prolong_add<T>, k_prolong_add_b<T>, dim3(grid_of(Lk.nn)), dim3(kThreads),
           ProlongArgs<T>{Lc, Lk, (const T*)Lc.z, Lk.z});
        launch_fine_tdot<T>(c, Lk, H.uf, H.r1f, H.wf, H.te);
        alpha_update(c, Lk);
        gs_sweep_mf(c, H, Lk, false);
        return;
    }
    // forward sweep (colours 1..7) and the partial sums for its alpha update
    gs_sweep(c, Lk, true, top);
    const int gr = acol_partials(c, Lk);
    // alpha update and residual; alpha residual and restriction; coarse
    // correction; prolongation
    int64_t chunks = (Lk.nn + 63) / 64;
    const int grr = (int)(chunks < kRedBlocks ? chunks : kRedBlocks);
    const Resid9Args<T> ra{Lk, (const T*)Lk.r, Lk.z, Lk.res, c.partials, gr, d};
    if (top)
        vl(c, k_resid9<T, true>, k_resid9_b<T, true>, dim3(grr), dim3(kBlk9), ra);
    else
        vl(c, k_resid9<T, false>, k_resid9_b<T, false>, dim3(grr), dim3(kBlk9), ra);
    Level<T>& Lc = H.lev[k - 1];
    if (k - 1 <= H.ksmall || k - 1 == 0)
        vl(c, k_restrict<T>, k_restrict_b<T>, dim3(grid_of(Lc.nn)), dim3(kThreads),
           RestrictArgs<T>{Lk, Lc, (const T*)Lk.res, Lc.r, 1,
                           (const double*)c.partials + SL_STAT * kRedBlocks, grr, d});
    else
        vl(c, k_restrict_init<T>, k_restrict_init_b<T>, dim3(grid_of(Lc.nn)), dim3(kThreads),
           RestrictInitArgs<T>{Lk, Lc, (const T*)Lk.res,
                               (const double*)c.partials + SL_STAT * kRedBlocks, grr, d});
    vcycle_level(c, H, k - 1);
    vl(c, k_prolong_add<T>, k_prolong_add_b<T>, dim3(grid_of(Lk.nn)), dim3(kThreads),
       ProlongArgs<T>{Lc, Lk, (const T*)Lc.z, Lk.z});
    // backward sweep: alpha, then colours 7..0
    alpha_update(c, Lk);
    gs_sweep(c, Lk, false, top);
}

template <typename T>
void mg_vcycle(Ctx& c, Hierarchy<T>& H, const double* r, double* z) {
    const int L = (int)H.lev.size();
    Level<T>& fine = H.lev[L - 1];
    const int64_t nv = 3 * fine.nn + 1;
    if (L - 1 <= H.ksmall || L == 1)
        vl(c, k_convert<double, T>, k_convert_b<double, T>, dim3(grid_of(nv)), dim3(kThreads),
           ConvertArgs<double, T>{r, fine.r, nv});
    else if (H.mf)
        vl(c, k_top_init_mf<T>, k_top_init_mf_b<T>, dim3(grid_of(fine.nn)), dim3(kThreads),
           TopInitMfArgs<T>{fine, r, (const T*)H.bc, H.te});
    else
        vl(c, k_top_init<T>, k_top_init_b<T>, dim3(grid_of(fine.nn)), dim3(kThreads),
           TopInitArgs<T>{fine, r});
    vcycle_level(c, H, L - 1);
    vl(c, k_convert<T, double>, k_convert_b<T, double>, dim3(grid_of(nv)), dim3(kThreads),
       ConvertArgs<T, double>{(const T*)fine.z, z, nv});
}

template <typename T>
int mg_check_factor(Ctx& c, Hierarchy<T>& H) {
    int flag = 0;
    hipMemcpyAsync(&flag, H.flag, sizeof(int), hipMemcpyDeviceToHost, c.s);
    hipStreamSynchronize(c.s);
    return flag;
}

template void mg_build<double>(Ctx&, Hierarchy<double>&);
template void mg_build<float>(Ctx&, Hierarchy<float>&);
template void mg_vcycle<double>(Ctx&, Hierarchy<double>&, const double*, double*);
template void mg_vcycle<float>(Ctx&, Hierarchy<float>&, const double*, double*);
template int mg_check_factor<double>(Ctx&, Hierarchy<double>&);
template int mg_check_factor<float>(Ctx&, Hierarchy<float>&);

}  // namespace vts
