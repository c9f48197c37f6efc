// Multi-load kernels (gfx950, wave64): several load cases f_1..f_k on one
// density, the summed compliance.  Problem (1.1) for the stacked displacement
// U = (u_1, ..., u_k) with element matrices blockdiag(K_i, ..., K_i): the
// PBM of Section 3.2 keeps its form with
//   e_i = sum_l 1/2 u_l^T K_i u_l,   b_i = (K_i u_1; ...; K_i u_k),
//   res_1 = (K(rho') u_l - f_l)_l,
// and the Newton matrix (3.12) S = [[I (x) K(rho') + B W B^T, -B w], [., sum w]]
// whose rank-one element terms couple the cases.
//
// Layouts: a stacked vector holds case l's all-DOF vector at [l n_dof,
// (l+1) n_dof) and alpha at k n_dof; per-element 24-vectors of case l at
// be[(24 l + j) m + e].  The multigrid (Section 6) takes node blocks of
// NB = 3k unknowns (a node over all cases): block row R = 3 l + c of node n
// is entry l (3 nn) + 3 n + c of the level's stacked vector.  Its stencils
// are assembled on every level, A[((q NB + R) NB + S) nn + p] with q the
// neighbour offset (dx+1) + 3 (dy+1) + 9 (dz+1) and p the node's position in
// colour-major order (the nodes of parity colour 0, then 1, ...), so that a
// colour pass reads each row of its nodes as one contiguous segment.  The
// finest stencil comes from (rho', w, b); coarse ones by Galerkin products
// with the trilinear prolongation per case; block Gauss-Seidel in the eight
// parity colours, alpha last (first) in the forward (backward) sweep; the
// coarsest level by a dense Cholesky inverse.  Everything is FP64.  K(rho)
// on the k cases is the single-load operator once per case: a fused
// k-case element kernel would need k times the registers of that kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <string>
#include <vector>

#include "device_util.hpp"
#include "vts_internal.hpp"

namespace vts {

struct MlLevel {
    int nx = 0, ny = 0, nz = 0;   // elements
    int64_t nn = 0;               // nodes
    uint8_t* fixed = nullptr;     // 3 nn, the same for every case
    double* A = nullptr;          // 27 NB^2 nn
    double* ac = nullptr;         // NB nn: alpha column
    double* Dinv = nullptr;       // NB^2 nn: inverse diagonal blocks
    double* r = nullptr;          // NB nn + 1 (coarse levels)
    double* z = nullptr;          // NB nn + 1 (coarse levels)
    double* t = nullptr;          // NB nn + 1: residual
};

struct MlHierarchy {
    int nl = 1, NB = 3, L = 1;
    std::vector<MlLevel> lv;      // 0 = coarsest
    int nc = 0;                   // dense coarsest size (free DOFs of all cases + alpha)
    int* cmap = nullptr;          // NB nn0 + 1 -> dense index or -1
    int* rows = nullptr;          // nc -> stacked index
    double* A0 = nullptr;         // nc^2: Cholesky factor after the build
    double* A0inv = nullptr;      // nc^2
    int* flag = nullptr;
    double* part = nullptr;       // private reduction partials (kRedBlocks)
    double* red = nullptr;        // private reduction results
};

namespace {

__global__ void k_ml_fin(const double* __restrict__ partials, int nb, int slot0,
                         uint32_t maxmask, double* __restrict__ out) {
    finalize_body(partials, nb, slot0, maxmask, out);
}

__global__ void k_ml_fill(double* __restrict__ a, double v, int64_t n) {
    const int64_t t = gid();
    if (t < n) a[t] = v;
}

__global__ void k_ml_store_neg(const double* __restrict__ red, int slot, double* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = -red[slot];
}

void fin(Ctx& c, int g, int slot0, int nq, uint32_t maxmask) {
    hipLaunchKernelGGL(k_ml_fin, dim3(nq), dim3(kThreads), 0, c.s, c.partials, g, slot0, maxmask,
                       c.red);
}

// ---------------------------------------------------------------------------
// element evaluation (Section 3.2 on the stacked problem)
// ---------------------------------------------------------------------------
struct MlEvalArgs {
    int nx, ny, nz, nl;
    int64_t ndof;
    double alpha;
    const double *Ke, *u, *nlo, *nhi, *rho, *mlo, *mhi, *p, *qlo, *qhi, *rlo, *rhi;
    const uint8_t* fixed;
    double *e, *be, *r1, *r2, *l2, *h2, *g3, *g4, *w, *zc, *partials;
};

__global__ void __launch_bounds__(kThreads) k_ml_eval(MlEvalArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double en = 0.0;
        for (int l = 0; l < a.nl; ++l) {
            double ue[24];
            gather_elem(a.u + l * a.ndof, a.fixed, i, j, k, a.nx + 1, a.ny + 1, ue);
            for (int r = 0; r < 24; ++r) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < 24; ++q) s += a.Ke[r * 24 + q] * ue[q];
                a.be[((int64_t)l * 24 + r) * m + e] = s;
                en += ue[r] * s;
            }
        }
        en *= 0.5;
        a.e[e] = en;
        const double pe = a.p[e], ql = a.qlo[e], qh = a.qhi[e];
        const double s = (en - a.alpha + a.nlo[e] - a.nhi[e]) / pe;
        const double tl = -a.nlo[e] / ql, th = -a.nhi[e] / qh;
        const double rh = a.rho[e], ml = a.mlo[e], mh = a.mhi[e];
        const double r1 = rh * pen_dphi(s), r2 = rh / pe * pen_d2phi(s);
        const double ml1 = ml * pen_dphi(tl), ml2 = ml / ql * pen_d2phi(tl);
        const double mh1 = mh * pen_dphi(th), mh2 = mh / qh * pen_d2phi(th);
        const double g3 = -a.rlo[e] + r1 - ml1;
        const double g4 = a.rhi[e] - r1 - mh1;
        const double det = r2 * (ml2 + mh2) + ml2 * mh2;
        const double w = r2 * ml2 * mh2 / det;
        const double z = r2 * (mh2 * g3 - ml2 * g4) / det;
        a.r1[e] = r1;
        a.r2[e] = r2;
        a.l2[e] = ml2;
        a.h2[e] = mh2;
        a.g3[e] = g3;
        a.g4[e] = g4;
        a.w[e] = w;
        a.zc[e] = z;
        acc[0] += r1;
        acc[1] += z;
        acc[2] += w;
        acc[3] += g3 * g3;
        acc[4] += g4 * g4;
    }
    block_sum_store<5>(acc, a.partials, SL_SUM_R1);
}

// res_1 of every case, K(rho') u_l - f_l = sum_e rho'_e b_{e,l} - f_l, and the
// reduced right-hand side f_l - sum_e (rho'_e - z_e) b_{e,l} (masked)
__global__ void __launch_bounds__(kThreads)
k_ml_grad(int nx, int ny, int nz, int nl, int64_t ndof, const double* __restrict__ be,
          const double* __restrict__ r1, const double* __restrict__ zc,
          const double* __restrict__ f, const uint8_t* __restrict__ fixed,
          double* __restrict__ g1, double* __restrict__ rhs, double* partials) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t m = (int64_t)nx * ny * nz;
    double acc[1] = {0.0};
    for (int64_t n = gid(); n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(n % NX);
        const int64_t t = n / NX;
        const int j = (int)(t % NY), k = (int)(t / NY);
        for (int l = 0; l < nl; ++l) {
            double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            for (int ez = -1; ez <= 0; ++ez) {
                const int kk = k + ez;
                if (kk < 0 || kk >= nz) continue;
                for (int ey = -1; ey <= 0; ++ey) {
                    const int jj = j + ey;
                    if (jj < 0 || jj >= ny) continue;
                    for (int ex = -1; ex <= 0; ++ex) {
                        const int ii = i + ex;
                        if (ii < 0 || ii >= nx) continue;
                        const int64_t e = ii + (int64_t)nx * (jj + (int64_t)ny * kk);
                        const int la = -ex - 2 * ey - 4 * ez;
                        const double w1 = r1[e], w2 = r1[e] - zc[e];
                        for (int c = 0; c < 3; ++c) {
                            const double bv = be[((int64_t)l * 24 + 3 * la + c) * m + e];
                            a[c] += w1 * bv;
                            b[c] += w2 * bv;
                        }
                    }
                }
            }
            for (int c = 0; c < 3; ++c) {
                const int64_t q = l * ndof + 3 * n + c;
                const bool fx = fixed[3 * n + c];
                const double gv = fx ? 0.0 : a[c] - f[q];
                g1[q] = gv;
                rhs[q] = fx ? 0.0 : f[q] - b[c];
                acc[0] += gv * gv;
            }
        }
    }
    block_sum_store<1>(acc, partials, SL_G1SQ);
}

// The rank-one part of the stacked S-apply, added to y (masked):
//   y_l += sum_e wt_e b_{e,l} at each node (one thread per node, every case).
template <int NL>
__global__ void __launch_bounds__(kThreads)
k_ml_rank1(int nx, int ny, int nz, int64_t ndof, const double* __restrict__ be,
           const double* __restrict__ wt, const uint8_t* __restrict__ fixed,
           double* __restrict__ y) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t n = gid();
    if (n >= nn) return;
    const int i = (int)(n % NX);
    const int64_t t = n / NX;
    const int j = (int)(t % NY), k = (int)(t / NY);
    double acc[NL][3];
#pragma unroll
    for (int l = 0; l < NL; ++l) acc[l][0] = acc[l][1] = acc[l][2] = 0.0;
    for (int ez = -1; ez <= 0; ++ez) {
        const int kk = k + ez;
        if (kk < 0 || kk >= nz) continue;
        for (int ey = -1; ey <= 0; ++ey) {
            const int jj = j + ey;
            if (jj < 0 || jj >= ny) continue;
            for (int ex = -1; ex <= 0; ++ex) {
                const int ii = i + ex;
                if (ii < 0 || ii >= nx) continue;
                const int64_t e = ii + (int64_t)nx * (jj + (int64_t)ny * kk);
                const int la = -ex - 2 * ey - 4 * ez;
                const double q = wt[e];
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    const double* bl = be + ((int64_t)l * 24 + 3 * la) * m + e;
                    acc[l][0] += q * bl[0];
                    acc[l][1] += q * bl[m];
                    acc[l][2] += q * bl[2 * m];
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l)
        for (int c = 0; c < 3; ++c)
            if (!fixed[3 * n + c]) y[l * ndof + 3 * n + c] += acc[l][c];
}

// S pass 1: wt_e = w_e (sum_l b_{e,l}^T x_{l,e} - beta), partial sums of wt
__global__ void __launch_bounds__(kThreads)
k_ml_tdot(int nx, int ny, int nz, int nl, int64_t ndof, const double* __restrict__ be,
          const double* __restrict__ w, const double* __restrict__ x,
          const uint8_t* __restrict__ fixed, double* __restrict__ wt, double* partials) {
    const int64_t m = (int64_t)nx * ny * nz;
    const double beta = x[nl * ndof];
    double acc[1] = {0.0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, nx, ny, i, j, k);
        double t = 0.0;
        for (int l = 0; l < nl; ++l) {
            double xe[24];
            gather_elem(x + l * ndof, fixed, i, j, k, nx + 1, ny + 1, xe);
#pragma unroll
            for (int q = 0; q < 24; ++q) t += be[((int64_t)l * 24 + q) * m + e] * xe[q];
        }
        const double v = w[e] * (t - beta);
        wt[e] = v;
        acc[0] += v;
    }
    block_sum_store<1>(acc, partials, SL_WT);
}

// Delta nu of eq. (3.14) with tau_e = sum_l b_{e,l}^T du_{l,e} - dalpha, and the
// line-search coefficients c1 = sum_l b_{e,l}^T du_{l,e}, c2 = e_e(dU)
struct MlDnuArgs {
    int nx, ny, nz, nl;
    int64_t ndof;
    const double *Ke, *be, *dy, *r2, *l2, *h2, *g3, *g4;
    const uint8_t* fixed;
    double *c1, *c2, *dnl, *dnh, *partials;
};

__global__ void __launch_bounds__(kThreads) k_ml_dnu(MlDnuArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    const double da = a.dy[a.nl * a.ndof];
    double acc[1] = {0.0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double t = 0.0, q2 = 0.0;
        for (int l = 0; l < a.nl; ++l) {
            double de[24];
            gather_elem(a.dy + l * a.ndof, a.fixed, i, j, k, a.nx + 1, a.ny + 1, de);
            for (int r = 0; r < 24; ++r) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < 24; ++q) s += a.Ke[r * 24 + q] * de[q];
                q2 += de[r] * s;
                t += a.be[((int64_t)l * 24 + r) * m + e] * de[r];
            }
        }
        a.c1[e] = t;
        a.c2[e] = 0.5 * q2;
        const double tau = t - da;
        const double r2 = a.r2[e], l2 = a.l2[e], h2 = a.h2[e], g3 = a.g3[e], g4 = a.g4[e];
        const double det = r2 * (l2 + h2) + l2 * h2;
        const double dl = -((r2 + h2) * g3 + r2 * g4 + r2 * h2 * tau) / det;
        const double dh = -(r2 * g3 + (r2 + l2) * g4 - r2 * l2 * tau) / det;
        a.dnl[e] = dl;
        a.dnh[e] = dh;
        acc[0] += g3 * dl + g4 * dh;
    }
    block_sum_store<1>(acc, a.partials, SL_SLOPE_NU);
}

// e_e = sum_l 1/2 u_{l,e}^T K_e u_{l,e}
__global__ void __launch_bounds__(kThreads)
k_ml_energy(int nx, int ny, int nz, int nl, int64_t ndof, const double* __restrict__ Ke,
            const double* __restrict__ u, const uint8_t* __restrict__ fixed,
            double* __restrict__ eout) {
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t e = gid();
    if (e >= m) return;
    int i, j, k;
    elem_ijk(e, nx, ny, i, j, k);
    double en = 0.0;
    for (int l = 0; l < nl; ++l) {
        double ue[24];
        gather_elem(u + l * ndof, fixed, i, j, k, nx + 1, ny + 1, ue);
        for (int r = 0; r < 24; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 24; ++q) s += Ke[r * 24 + q] * ue[q];
            en += ue[r] * s;
        }
    }
    eout[e] = 0.5 * en;
}

__global__ void k_ml_update(int64_t nvec, int64_t m, double kappa, double* __restrict__ u,
                            const double* __restrict__ dy, double* __restrict__ nlo,
                            double* __restrict__ nhi, const double* __restrict__ dnl,
                            const double* __restrict__ dnh) {
    const int64_t t = gid();
    if (t < nvec) u[t] += kappa * dy[t];
    if (t < m) {
        nlo[t] += kappa * dnl[t];
        nhi[t] += kappa * dnh[t];
    }
}

// ---------------------------------------------------------------------------
// multigrid with node blocks over all cases
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t vidx(int R, int64_t n, int64_t nn) {
    return (int64_t)(R / 3) * 3 * nn + 3 * n + (R % 3);
}

__device__ __forceinline__ void node_ijk(int64_t n, int NX, int NY, int& i, int& j, int& k) {
    i = (int)(n % NX);
    const int64_t t = n / NX;
    j = (int)(t % NY);
    k = (int)(t / NY);
}

// nodes of parity colour c = (i&1) + 2 (j&1) + 4 (k&1) on a grid of NX x NY x NZ nodes
__device__ __forceinline__ int64_t colour_count(int c, int NX, int NY, int NZ) {
    return (int64_t)((NX - (c & 1) + 1) / 2) * ((NY - ((c >> 1) & 1) + 1) / 2) *
           ((NZ - (c >> 2) + 1) / 2);
}

// colour-major position of node (i, j, k): the nodes of the lower colours,
// then (i, j, k)'s index within its colour (x fastest)
__device__ __forceinline__ int64_t cm_index(int i, int j, int k, int NX, int NY, int NZ) {
    const int c = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
    int64_t off = 0;
    for (int q = 0; q < c; ++q) off += colour_count(q, NX, NY, NZ);
    const int mx = (NX - (c & 1) + 1) / 2, my = (NY - ((c >> 1) & 1) + 1) / 2;
    return off + (i >> 1) + (int64_t)mx * ((j >> 1) + (int64_t)my * (k >> 1));
}

// finest stencil: one thread per (node, neighbour offset q, block row R)
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_stencil(int nx, int ny, int nz, const double* __restrict__ Ke,
             const double* __restrict__ r1, const double* __restrict__ w,
             const double* __restrict__ be, const uint8_t* __restrict__ fixed,
             double* __restrict__ A) {
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t t = gid();
    if (t >= nn * 27 * NB) return;
    // node fastest: a wave reads and writes consecutive nodes
    const int64_t n = t % nn;
    const int64_t t2 = t / nn;
    const int q = (int)(t2 % 27);
    const int R = (int)(t2 / 27);
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    int i, j, k;
    node_ijk(n, NX, NY, i, j, k);
    const int i2 = i + dx, j2 = j + dy, k2 = k + dz;
    double acc[NB];
#pragma unroll
    for (int S = 0; S < NB; ++S) acc[S] = 0.0;
    const int lR = R / 3, cR = R % 3;
    const bool inside = i2 >= 0 && i2 < NX && j2 >= 0 && j2 < NY && k2 >= 0 && k2 < NZ;
    if (inside && !fixed[3 * n + cR]) {
        const int64_t n2 = node_id(i2, j2, k2, NX, NY);
        for (int ez = max(k, k2) - 1; ez <= min(k, k2); ++ez) {
            if (ez < 0 || ez >= nz) continue;
            for (int ey = max(j, j2) - 1; ey <= min(j, j2); ++ey) {
                if (ey < 0 || ey >= ny) continue;
                for (int ex = max(i, i2) - 1; ex <= min(i, i2); ++ex) {
                    if (ex < 0 || ex >= nx) continue;
                    const int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                    const int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
                    const int b = (i2 - ex) + 2 * (j2 - ey) + 4 * (k2 - ez);
                    const double re = r1[e], we = w[e];
                    const double bR = be[((int64_t)lR * 24 + 3 * a + cR) * m + e];
#pragma unroll
                    for (int S = 0; S < NB; ++S) {
                        const int lS = S / 3, cS = S % 3;
                        double v = we * bR * be[((int64_t)lS * 24 + 3 * b + cS) * m + e];
                        if (lS == lR) v += re * Ke[(3 * a + cR) * 24 + 3 * b + cS];
                        acc[S] += v;
                    }
                }
            }
        }
#pragma unroll
        for (int S = 0; S < NB; ++S)
            if (fixed[3 * n2 + S % 3]) acc[S] = 0.0;
    }
    const int64_t pn = cm_index(i, j, k, NX, NY, NZ);
#pragma unroll
    for (int S = 0; S < NB; ++S) A[(((int64_t)q * NB + R) * NB + S) * nn + pn] = acc[S];
}

// finest alpha column: -sum_e w_e b_{e,l} at the node (masked)
__global__ void __launch_bounds__(kThreads)
k_ml_acol_fine(int nx, int ny, int nz, int NB, const double* __restrict__ w,
               const double* __restrict__ be, const uint8_t* __restrict__ fixed,
               double* __restrict__ ac) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t t = gid();
    if (t >= nn * NB) return;
    const int R = (int)(t / nn);
    const int64_t n = t % nn;
    int i, j, k;
    node_ijk(n, NX, NY, i, j, k);
    const int l = R / 3, c = R % 3;
    double s = 0.0;
    if (!fixed[3 * n + c]) {
        for (int ez = -1; ez <= 0; ++ez) {
            const int kk = k + ez;
            if (kk < 0 || kk >= nz) continue;
            for (int ey = -1; ey <= 0; ++ey) {
                const int jj = j + ey;
                if (jj < 0 || jj >= ny) continue;
                for (int ex = -1; ex <= 0; ++ex) {
                    const int ii = i + ex;
                    if (ii < 0 || ii >= nx) continue;
                    const int64_t e = ii + (int64_t)nx * (jj + (int64_t)ny * kk);
                    const int la = -ex - 2 * ey - 4 * ez;
                    s -= w[e] * be[((int64_t)l * 24 + 3 * la + c) * m + e];
                }
            }
        }
    }
    ac[(int64_t)R * nn + cm_index(i, j, k, NX, NY, nz + 1)] = s;
}

// Galerkin coarse stencil P^T A P: one thread per (coarse node I, offset q,
// block row R).  Fine node 2I + a (a in {-1,0,1}^3) has weight prod (a_d ? 1/2 : 1)
// toward I; the pairs (a, b) with fine offset 2 delta + b - a in {-1,0,1}^3 are
// enumerated dimension by dimension.
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_galerkin(int cnx, int cny, int cnz, const double* __restrict__ Af,
              const uint8_t* __restrict__ cfixed, double* __restrict__ Ac) {
    const int CX = cnx + 1, CY = cny + 1, CZ = cnz + 1;
    const int FX = 2 * cnx + 1, FY = 2 * cny + 1, FZ = 2 * cnz + 1;
    const int64_t nnc = (int64_t)CX * CY * CZ;
    const int64_t nnf = (int64_t)FX * FY * FZ;
    const int64_t t = gid();
    if (t >= nnc * 27 * NB) return;
    // coarse node fastest: a wave writes consecutive nodes
    const int64_t I = t % nnc;
    const int64_t t2 = t / nnc;
    const int q = (int)(t2 % 27);
    const int R = (int)(t2 / 27);
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    int ci, cj, ck;
    node_ijk(I, CX, CY, ci, cj, ck);
    const int ci2 = ci + dx, cj2 = cj + dy, ck2 = ck + dz;
    double acc[NB];
#pragma unroll
    for (int S = 0; S < NB; ++S) acc[S] = 0.0;
    const bool inside = ci2 >= 0 && ci2 < CX && cj2 >= 0 && cj2 < CY && ck2 >= 0 && ck2 < CZ;
    if (inside && !cfixed[3 * I + R % 3]) {
        for (int az = -1; az <= 1; ++az) {
            const int fk = 2 * ck + az;
            if (fk < 0 || fk >= FZ) continue;
            for (int bz = -1; bz <= 1; ++bz) {
                const int fk2 = 2 * ck2 + bz;
                const int oz = fk2 - fk;
                if (fk2 < 0 || fk2 >= FZ || oz < -1 || oz > 1) continue;
                const double wz = (az ? 0.5 : 1.0) * (bz ? 0.5 : 1.0);
                for (int ay = -1; ay <= 1; ++ay) {
                    const int fj = 2 * cj + ay;
                    if (fj < 0 || fj >= FY) continue;
                    for (int by = -1; by <= 1; ++by) {
                        const int fj2 = 2 * cj2 + by;
                        const int oy = fj2 - fj;
                        if (fj2 < 0 || fj2 >= FY || oy < -1 || oy > 1) continue;
                        const double wy = wz * (ay ? 0.5 : 1.0) * (by ? 0.5 : 1.0);
                        for (int ax = -1; ax <= 1; ++ax) {
                            const int fi = 2 * ci + ax;
                            if (fi < 0 || fi >= FX) continue;
                            for (int bx = -1; bx <= 1; ++bx) {
                                const int fi2 = 2 * ci2 + bx;
                                const int ox = fi2 - fi;
                                if (fi2 < 0 || fi2 >= FX || ox < -1 || ox > 1) continue;
                                const double wgt = wy * (ax ? 0.5 : 1.0) * (bx ? 0.5 : 1.0);
                                const int qf = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
                                const int64_t pf = cm_index(fi, fj, fk, FX, FY, FZ);
                                const double* row = Af + (((int64_t)qf * NB + R) * NB) * nnf + pf;
#pragma unroll
                                for (int S = 0; S < NB; ++S) acc[S] += wgt * row[(int64_t)S * nnf];
                            }
                        }
                    }
                }
            }
        }
        const int64_t J = node_id(ci2, cj2, ck2, CX, CY);
#pragma unroll
        for (int S = 0; S < NB; ++S)
            if (cfixed[3 * J + S % 3]) acc[S] = 0.0;
    }
    const int64_t pI = cm_index(ci, cj, ck, CX, CY, CZ);
#pragma unroll
    for (int S = 0; S < NB; ++S) Ac[(((int64_t)q * NB + R) * NB + S) * nnc + pI] = acc[S];
}

// coarse alpha column P^T c (masked)
__global__ void __launch_bounds__(kThreads)
k_ml_acol_coarse(int cnx, int cny, int cnz, int NB, const double* __restrict__ acf,
                 const uint8_t* __restrict__ cfixed, double* __restrict__ acc_) {
    const int CX = cnx + 1, CY = cny + 1, CZ = cnz + 1;
    const int FX = 2 * cnx + 1, FY = 2 * cny + 1, FZ = 2 * cnz + 1;
    const int64_t nnc = (int64_t)CX * CY * CZ;
    const int64_t nnf = (int64_t)FX * FY * FZ;
    const int64_t t = gid();
    if (t >= nnc * NB) return;
    const int R = (int)(t / nnc);
    const int64_t I = t % nnc;
    int ci, cj, ck;
    node_ijk(I, CX, CY, ci, cj, ck);
    double s = 0.0;
    if (!cfixed[3 * I + R % 3]) {
        for (int az = -1; az <= 1; ++az) {
            const int fk = 2 * ck + az;
            if (fk < 0 || fk >= FZ) continue;
            for (int ay = -1; ay <= 1; ++ay) {
                const int fj = 2 * cj + ay;
                if (fj < 0 || fj >= FY) continue;
                for (int ax = -1; ax <= 1; ++ax) {
                    const int fi = 2 * ci + ax;
                    if (fi < 0 || fi >= FX) continue;
                    const double wgt = (az ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (ax ? 0.5 : 1.0);
                    s += wgt * acf[(int64_t)R * nnf + cm_index(fi, fj, fk, FX, FY, FZ)];
                }
            }
        }
    }
    acc_[(int64_t)R * nnc + cm_index(ci, cj, ck, CX, CY, CZ)] = s;
}

// inverse of each node's diagonal block (identity on fixed components), by
// Gauss-Jordan elimination without pivoting (the free block is positive
// definite); flag = 1 on a non-positive pivot
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_blockinv(int nx, int ny, int nz, const double* __restrict__ A,
              const uint8_t* __restrict__ fixed, double* __restrict__ Dinv,
              int* __restrict__ flag) {
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    const int64_t n = gid();
    if (n >= nn) return;
    int i, j, k;
    node_ijk(n, NX, NY, i, j, k);
    const int64_t pn = cm_index(i, j, k, NX, NY, NZ);
    double D[NB][NB], X[NB][NB];
    for (int R = 0; R < NB; ++R) {
        const bool fr = fixed[3 * n + R % 3];
        for (int S = 0; S < NB; ++S) {
            const bool fs = fixed[3 * n + S % 3];
            double v = A[(((int64_t)13 * NB + R) * NB + S) * nn + pn];
            if (fr || fs) v = (R == S) ? 1.0 : 0.0;
            D[R][S] = v;
            X[R][S] = (R == S) ? 1.0 : 0.0;
        }
    }
    bool bad = false;
    for (int p = 0; p < NB; ++p) {
        const double piv = D[p][p];
        if (!(piv > 0.0)) bad = true;
        const double ip = 1.0 / piv;
        for (int S = 0; S < NB; ++S) {
            D[p][S] *= ip;
            X[p][S] *= ip;
        }
        for (int R = 0; R < NB; ++R) {
            if (R == p) continue;
            const double f = D[R][p];
            for (int S = 0; S < NB; ++S) {
                D[R][S] -= f * D[p][S];
                X[R][S] -= f * X[p][S];
            }
        }
    }
    if (bad) *flag = 1;
    for (int R = 0; R < NB; ++R)
        for (int S = 0; S < NB; ++S) Dinv[((int64_t)R * NB + S) * nn + pn] = X[R][S];
}

// dense coarsest matrix: row p (free DOF rows[p]) from the stencil, alpha last
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_dense(int nx, int ny, int nz, const double* __restrict__ A, const double* __restrict__ ac,
           const int* __restrict__ cmap, const int* __restrict__ rows, int nc, double d,
           double* __restrict__ A0) {
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    const int p = (int)gid();
    if (p >= nc) return;
    if (p == nc - 1) {
        A0[(int64_t)p * nc + p] = d;
        return;
    }
    const int64_t v = rows[p];
    const int l = (int)(v / (3 * nn));
    const int64_t rem = v % (3 * nn);
    const int64_t n = rem / 3;
    const int R = 3 * l + (int)(rem % 3);
    int i, j, k;
    node_ijk(n, NX, NY, i, j, k);
    const int64_t pn = cm_index(i, j, k, NX, NY, NZ);
    for (int q = 0; q < 27; ++q) {
        const int i2 = i + q % 3 - 1, j2 = j + (q / 3) % 3 - 1, k2 = k + q / 9 - 1;
        if (i2 < 0 || i2 >= NX || j2 < 0 || j2 >= NY || k2 < 0 || k2 >= NZ) continue;
        const int64_t n2 = node_id(i2, j2, k2, NX, NY);
        for (int S = 0; S < NB; ++S) {
            const int col = cmap[vidx(S, n2, nn)];
            if (col < 0) continue;
            A0[(int64_t)p * nc + col] = A[(((int64_t)q * NB + R) * NB + S) * nn + pn];
        }
    }
    const double a = ac[(int64_t)R * nn + pn];
    A0[(int64_t)p * nc + nc - 1] = a;
    A0[(int64_t)(nc - 1) * nc + p] = a;
}

// in-place lower Cholesky factor of the dense matrix, one workgroup
__global__ void __launch_bounds__(1024) k_ml_cholesky(double* __restrict__ A, int nc,
                                                      int* __restrict__ flag) {
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
        for (int64_t p = threadIdx.x; p < (int64_t)T * T; p += blockDim.x) {
            const int i = k + 1 + (int)(p / T), j = k + 1 + (int)(p % T);
            if (j <= i) A[(int64_t)i * nc + j] -= A[(int64_t)i * nc + k] * A[(int64_t)j * nc + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && bad) *flag = 1;
}

// column jcol of (L L^T)^{-1}: one workgroup per column, the column in LDS
__global__ void __launch_bounds__(256) k_ml_chol_inv(const double* __restrict__ L, int nc,
                                                     double* __restrict__ Ainv) {
    extern __shared__ double x[];
    const int jcol = blockIdx.x;
    for (int q = threadIdx.x; q < nc; q += blockDim.x) x[q] = (q == jcol) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        if (threadIdx.x == 0) x[k] /= L[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = k + 1 + threadIdx.x; i < nc; i += blockDim.x) x[i] -= L[(int64_t)i * nc + k] * xk;
        __syncthreads();
    }
    for (int k = nc - 1; k >= 0; --k) {
        if (threadIdx.x == 0) x[k] /= L[(int64_t)k * nc + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] -= L[(int64_t)k * nc + i] * xk;
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nc; q += blockDim.x) Ainv[(int64_t)q * nc + jcol] = x[q];
}

// z = A0^{-1} r on the coarsest level's free DOFs and alpha (z is zero elsewhere)
__global__ void __launch_bounds__(kThreads)
k_ml_dense_apply(const double* __restrict__ Ainv, const int* __restrict__ rows, int nc,
                 const double* __restrict__ r, double* __restrict__ z) {
    const int p = (int)gid();
    if (p >= nc) return;
    double s = 0.0;
    for (int q = 0; q < nc; ++q) s += Ainv[(int64_t)p * nc + q] * r[rows[q]];
    z[rows[p]] = s;
}

// One colour of block Gauss-Seidel on the nodes of parity colour `col`.  A
// workgroup takes kMlGsNodes consecutive nodes of the colour (consecutive in
// the colour-major arrays) and NB block rows: thread (R, slot) forms row R of
// its node's residual r - A z - ac z_alpha, so the threads of one row read
// one contiguous segment per coefficient; the rows meet in LDS for the block
// solve dz = Dinv res, and thread (R, slot) adds row R of dz.  TOP marks the
// finest level's instantiation (the same code; a kernel of its own for the
// profiler).
constexpr int kMlGsNodes = 32;

template <int NB, bool TOP>
__global__ void __launch_bounds__(kMlGsNodes * 12)
k_ml_gs(int nx, int ny, int nz, int col, const double* __restrict__ A,
        const double* __restrict__ ac, const double* __restrict__ Dinv,
        const double* __restrict__ r, double* __restrict__ z) {
    __shared__ double sres[NB][kMlGsNodes];
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    const int cx = col & 1, cy = (col >> 1) & 1, cz = col >> 2;
    const int mx = (NX - cx + 1) / 2, my = (NY - cy + 1) / 2, mz = (NZ - cz + 1) / 2;
    const int slot = (int)(threadIdx.x % kMlGsNodes);
    const int R = (int)(threadIdx.x / kMlGsNodes);
    const int64_t g = (int64_t)blockIdx.x * kMlGsNodes + slot;
    const bool act = g < (int64_t)mx * my * mz;
    int64_t off = 0;
    for (int q = 0; q < col; ++q) off += colour_count(q, NX, NY, NZ);
    const int64_t pn = off + g;
    int i = 0, j = 0, k = 0;
    int64_t n = 0;
    double res = 0.0;
    if (act) {
        i = 2 * (int)(g % mx) + cx;
        const int64_t g2 = g / mx;
        j = 2 * (int)(g2 % my) + cy;
        k = 2 * (int)(g2 / my) + cz;
        n = node_id(i, j, k, NX, NY);
        res = r[vidx(R, n, nn)] - ac[(int64_t)R * nn + pn] * z[(int64_t)NB * nn];
        for (int q = 0; q < 27; ++q) {
            const int i2 = i + q % 3 - 1, j2 = j + (q / 3) % 3 - 1, k2 = k + q / 9 - 1;
            if (i2 < 0 || i2 >= NX || j2 < 0 || j2 >= NY || k2 < 0 || k2 >= NZ) continue;
            const int64_t n2 = node_id(i2, j2, k2, NX, NY);
            const double* row = A + (((int64_t)q * NB + R) * NB) * nn + pn;
            double s = 0.0;
#pragma unroll
            for (int S = 0; S < NB; ++S) s += row[(int64_t)S * nn] * z[vidx(S, n2, nn)];
            res -= s;
        }
    }
    sres[R][slot] = res;
    __syncthreads();
    if (act) {
        double d = 0.0;
#pragma unroll
        for (int S = 0; S < NB; ++S) d += Dinv[((int64_t)R * NB + S) * nn + pn] * sres[S][slot];
        z[vidx(R, n, nn)] += d;
    }
}

// t = r - A z - ac z_alpha, one thread per (node, block row), node fastest
// in the natural order (z read and t written in runs; the coefficients of
// consecutive nodes come from the two colour-major ranges of the row's two
// x parities)
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_resid(int nx, int ny, int nz, const double* __restrict__ A, const double* __restrict__ ac,
           const double* __restrict__ r, const double* __restrict__ z, double* __restrict__ t_) {
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    const int64_t t = gid();
    if (t >= nn * NB) return;
    const int64_t n = t % nn;
    const int R = (int)(t / nn);
    int i, j, k;
    node_ijk(n, NX, NY, i, j, k);
    const int64_t pn = cm_index(i, j, k, NX, NY, NZ);
    double res = r[vidx(R, n, nn)] - ac[(int64_t)R * nn + pn] * z[(int64_t)NB * nn];
    for (int q = 0; q < 27; ++q) {
        const int i2 = i + q % 3 - 1, j2 = j + (q / 3) % 3 - 1, k2 = k + q / 9 - 1;
        if (i2 < 0 || i2 >= NX || j2 < 0 || j2 >= NY || k2 < 0 || k2 >= NZ) continue;
        const int64_t n2 = node_id(i2, j2, k2, NX, NY);
        const double* row = A + (((int64_t)q * NB + R) * NB) * nn + pn;
        double s = 0.0;
#pragma unroll
        for (int S = 0; S < NB; ++S) s += row[(int64_t)S * nn] * z[vidx(S, n2, nn)];
        res -= s;
    }
    t_[vidx(R, n, nn)] = res;
}

// partial sums of ac^T z (the alpha row without its diagonal)
__global__ void __launch_bounds__(kThreads)
k_ml_acol_dot(int nx, int ny, int nz, int NB, const double* __restrict__ ac,
              const double* __restrict__ z, double* partials) {
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int64_t nn = (int64_t)NX * NY * NZ;
    double acc[1] = {0.0};
    for (int64_t t = gid(); t < nn * NB; t += (int64_t)gridDim.x * blockDim.x) {
        const int R = (int)(t / nn);
        const int64_t n = t % nn;
        int i, j, k;
        node_ijk(n, NX, NY, i, j, k);
        acc[0] += ac[(int64_t)R * nn + cm_index(i, j, k, NX, NY, NZ)] * z[vidx(R, n, nn)];
    }
    block_sum_store<1>(acc, partials, 0);
}

// alpha row: update z_alpha (mode 0) or store the residual in t_alpha (mode 1)
__global__ void k_ml_alpha(int64_t ia, double d, const double* __restrict__ red,
                           const double* __restrict__ r, double* __restrict__ z,
                           double* __restrict__ t_, int mode) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double res = r[ia] - red[0] - d * z[ia];
    if (mode == 0)
        z[ia] += res / d;
    else
        t_[ia] = res;
}

// rc = P^T t (masked), alpha by identity
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_restrict(int cnx, int cny, int cnz, const double* __restrict__ tf,
              const uint8_t* __restrict__ cfixed, double* __restrict__ rc) {
    const int CX = cnx + 1, CY = cny + 1, CZ = cnz + 1;
    const int FX = 2 * cnx + 1, FY = 2 * cny + 1, FZ = 2 * cnz + 1;
    const int64_t nnc = (int64_t)CX * CY * CZ;
    const int64_t nnf = (int64_t)FX * FY * FZ;
    const int64_t I = gid();
    if (I == 0) rc[(int64_t)NB * nnc] = tf[(int64_t)NB * nnf];
    if (I >= nnc) return;
    int ci, cj, ck;
    node_ijk(I, CX, CY, ci, cj, ck);
    double acc[NB];
#pragma unroll
    for (int R = 0; R < NB; ++R) acc[R] = 0.0;
    for (int az = -1; az <= 1; ++az) {
        const int fk = 2 * ck + az;
        if (fk < 0 || fk >= FZ) continue;
        for (int ay = -1; ay <= 1; ++ay) {
            const int fj = 2 * cj + ay;
            if (fj < 0 || fj >= FY) continue;
            for (int ax = -1; ax <= 1; ++ax) {
                const int fi = 2 * ci + ax;
                if (fi < 0 || fi >= FX) continue;
                const double wgt = (az ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (ax ? 0.5 : 1.0);
                const int64_t nf = node_id(fi, fj, fk, FX, FY);
#pragma unroll
                for (int R = 0; R < NB; ++R) acc[R] += wgt * tf[vidx(R, nf, nnf)];
            }
        }
    }
#pragma unroll
    for (int R = 0; R < NB; ++R) rc[vidx(R, I, nnc)] = cfixed[3 * I + R % 3] ? 0.0 : acc[R];
}

// z_f += P z_c (masked), alpha by identity
template <int NB>
__global__ void __launch_bounds__(kThreads)
k_ml_prolong(int cnx, int cny, int cnz, const double* __restrict__ zc,
             const uint8_t* __restrict__ ffixed, double* __restrict__ zf) {
    const int CX = cnx + 1, CY = cny + 1;
    const int FX = 2 * cnx + 1, FY = 2 * cny + 1, FZ = 2 * cnz + 1;
    const int64_t nnc = (int64_t)CX * CY * (cnz + 1);
    const int64_t nnf = (int64_t)FX * FY * FZ;
    const int64_t n = gid();
    if (n == 0) zf[(int64_t)NB * nnf] += zc[(int64_t)NB * nnc];
    if (n >= nnf) return;
    int fi, fj, fk;
    node_ijk(n, FX, FY, fi, fj, fk);
    double acc[NB];
#pragma unroll
    for (int R = 0; R < NB; ++R) acc[R] = 0.0;
    // coarse parents per dimension: the coincident node (weight 1) or the two
    // neighbours (1/2 each)
    const int x0 = fi / 2, x1 = (fi + 1) / 2, y0 = fj / 2, y1 = (fj + 1) / 2;
    const int z0 = fk / 2, z1 = (fk + 1) / 2;
    for (int cz = z0; cz <= z1; ++cz) {
        const double wz = (z0 == z1) ? 1.0 : 0.5;
        for (int cy = y0; cy <= y1; ++cy) {
            const double wy = wz * ((y0 == y1) ? 1.0 : 0.5);
            for (int cx = x0; cx <= x1; ++cx) {
                const double wgt = wy * ((x0 == x1) ? 1.0 : 0.5);
                const int64_t I = node_id(cx, cy, cz, CX, CY);
#pragma unroll
                for (int R = 0; R < NB; ++R) acc[R] += wgt * zc[vidx(R, I, nnc)];
            }
        }
    }
#pragma unroll
    for (int R = 0; R < NB; ++R)
        if (!ffixed[3 * n + R % 3]) zf[vidx(R, n, nnf)] += acc[R];
}

inline int grid_of(int64_t n) { return grid1d(n); }

template <int NB>
void build_levels(Ctx& c, MlHierarchy& H) {
    MlLevel& F = H.lv[H.L - 1];
    const int64_t nnf = F.nn;
    hipLaunchKernelGGL(k_ml_stencil<NB>, dim3(grid_of(nnf * 27 * NB)), dim3(kThreads), 0, c.s,
                       F.nx, F.ny, F.nz, c.Ke, c.r1, c.w, c.be, F.fixed, F.A);
    hipLaunchKernelGGL(k_ml_acol_fine, dim3(grid_of(nnf * NB)), dim3(kThreads), 0, c.s, F.nx,
                       F.ny, F.nz, NB, c.w, c.be, F.fixed, F.ac);
    for (int k = H.L - 1; k > 0; --k) {
        MlLevel& Fk = H.lv[k];
        MlLevel& C = H.lv[k - 1];
        hipLaunchKernelGGL(k_ml_galerkin<NB>, dim3(grid_of(C.nn * 27 * NB)), dim3(kThreads), 0,
                           c.s, C.nx, C.ny, C.nz, Fk.A, C.fixed, C.A);
        hipLaunchKernelGGL(k_ml_acol_coarse, dim3(grid_of(C.nn * NB)), dim3(kThreads), 0, c.s,
                           C.nx, C.ny, C.nz, NB, Fk.ac, C.fixed, C.ac);
    }
    for (int k = 1; k < H.L; ++k) {
        MlLevel& Lk = H.lv[k];
        hipLaunchKernelGGL(k_ml_blockinv<NB>, dim3(grid_of(Lk.nn)), dim3(kThreads), 0, c.s, Lk.nx,
                           Lk.ny, Lk.nz, Lk.A, Lk.fixed, Lk.Dinv, H.flag);
    }
    MlLevel& C0 = H.lv[0];
    const int64_t n0 = (int64_t)H.nc * H.nc;
    hipLaunchKernelGGL(k_ml_fill, dim3(grid_of(n0)), dim3(kThreads), 0, c.s, H.A0, 0.0, n0);
    hipLaunchKernelGGL(k_ml_dense<NB>, dim3(grid_of(H.nc)), dim3(kThreads), 0, c.s, C0.nx, C0.ny,
                       C0.nz, C0.A, C0.ac, H.cmap, H.rows, H.nc, c.sum_w, H.A0);
    hipLaunchKernelGGL(k_ml_cholesky, dim3(1), dim3(1024), 0, c.s, H.A0, H.nc, H.flag);
    hipLaunchKernelGGL(k_ml_chol_inv, dim3(H.nc), dim3(256), (size_t)H.nc * sizeof(double), c.s,
                       H.A0, H.nc, H.A0inv);
}

void alpha_row(Ctx& c, MlHierarchy& H, const MlLevel& Lv, const double* r, double* z, double* t,
               int mode) {
    const int64_t n = Lv.nn * H.NB;
    const int g = red_grid(n);
    hipLaunchKernelGGL(k_ml_acol_dot, dim3(g), dim3(kThreads), 0, c.s, Lv.nx, Lv.ny, Lv.nz, H.NB,
                       Lv.ac, z, H.part);
    hipLaunchKernelGGL(k_ml_fin, dim3(1), dim3(kThreads), 0, c.s, H.part, g, 0, 0u, H.red);
    hipLaunchKernelGGL(k_ml_alpha, dim3(1), dim3(64), 0, c.s, (int64_t)H.NB * Lv.nn, c.sum_w,
                       H.red, r, z, t, mode);
}

template <int NB>
void vcycle_level(Ctx& c, MlHierarchy& H, int k, const double* r, double* z) {
    const MlLevel& Lv = H.lv[k];
    const int64_t nv = (int64_t)NB * Lv.nn + 1;
    hipLaunchKernelGGL(k_ml_fill, dim3(grid_of(nv)), dim3(kThreads), 0, c.s, z, 0.0, nv);
    if (k == 0) {
        hipLaunchKernelGGL(k_ml_dense_apply, dim3(grid_of(H.nc)), dim3(kThreads), 0, c.s, H.A0inv,
                           H.rows, H.nc, r, z);
        return;
    }
    const int NX = Lv.nx + 1, NY = Lv.ny + 1, NZ = Lv.nz + 1;
    auto colour_nodes = [&](int col) {
        const int cx = col & 1, cy = (col >> 1) & 1, cz = col >> 2;
        return (int64_t)((NX - cx + 1) / 2) * ((NY - cy + 1) / 2) * ((NZ - cz + 1) / 2);
    };
    // the finest level's colour passes are one kernel class of the profiler:
    // algorithmic bytes = the colour's stencil rows, inverse blocks, r, alpha
    // column and z (read and written), and the z of every other node
    const bool top = k == H.L - 1;
    auto gs = [&](int col) {
        const int64_t cnt = colour_nodes(col);
        const bool prof = top && prof_begin(c, VTS_PROF_GS_FINE);
        const dim3 grid((unsigned)((cnt + kMlGsNodes - 1) / kMlGsNodes)), block(kMlGsNodes * NB);
        if (top)
            hipLaunchKernelGGL((k_ml_gs<NB, true>), grid, block, 0, c.s, Lv.nx, Lv.ny, Lv.nz, col,
                               Lv.A, Lv.ac, Lv.Dinv, r, z);
        else
            hipLaunchKernelGGL((k_ml_gs<NB, false>), grid, block, 0, c.s, Lv.nx, Lv.ny, Lv.nz, col,
                               Lv.A, Lv.ac, Lv.Dinv, r, z);
        if (prof)
            prof_end(c, 8.0 * ((double)cnt * (28.0 * NB * NB + 4.0 * NB) +
                               (double)NB * (double)(Lv.nn - cnt)), 1);
    };
    for (int col = 0; col < 8; ++col) gs(col);
    alpha_row(c, H, Lv, r, z, nullptr, 0);
    hipLaunchKernelGGL(k_ml_resid<NB>, dim3(grid_of(Lv.nn * NB)), dim3(kThreads), 0, c.s, Lv.nx,
                       Lv.ny, Lv.nz, Lv.A, Lv.ac, r, z, Lv.t);
    alpha_row(c, H, Lv, r, z, Lv.t, 1);
    const MlLevel& C = H.lv[k - 1];
    hipLaunchKernelGGL(k_ml_restrict<NB>, dim3(grid_of(C.nn)), dim3(kThreads), 0, c.s, C.nx, C.ny,
                       C.nz, Lv.t, C.fixed, C.r);
    vcycle_level<NB>(c, H, k - 1, C.r, C.z);
    hipLaunchKernelGGL(k_ml_prolong<NB>, dim3(grid_of(Lv.nn)), dim3(kThreads), 0, c.s, C.nx,
                       C.ny, C.nz, C.z, Lv.fixed, z);
    alpha_row(c, H, Lv, r, z, nullptr, 0);
    for (int col = 7; col >= 0; --col) gs(col);
}

}  // namespace

// ---------------------------------------------------------------------------
// host entry points (declared in vts_internal.hpp)
// ---------------------------------------------------------------------------
#define ML_HIPCHK(expr)                                                        \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            c.err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
            return VTS_EDEVICE;                                                \
        }                                                                      \
    } while (0)

void ml_launch_eval(Ctx& c) {
    MlEvalArgs a{c.nx, c.ny, c.nz, c.nl, c.ndof, c.alpha, c.Ke, c.u, c.nlo, c.nhi, c.rho, c.mlo,
                 c.mhi, c.p, c.qlo, c.qhi, c.rlo, c.rhi, c.fixed, c.e, c.be, c.r1, c.r2, c.l2,
                 c.h2, c.g3, c.g4, c.w, c.zc, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_ml_eval, dim3(g), dim3(kThreads), 0, c.s, a);
    fin(c, g, SL_SUM_R1, 5, 0u);
}

void ml_launch_grad(Ctx& c) {
    const int g = red_grid(c.nn);
    hipLaunchKernelGGL(k_ml_grad, dim3(g), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.nl, c.ndof,
                       c.be, c.r1, c.zc, c.f, c.fixed, c.g1, c.rhs, c.partials);
    fin(c, g, SL_G1SQ, 1, 0u);
}

// K(coef) on the k cases: the single-load operator (the plane-marching
// element kernel) once per case
void ml_apply_K(Ctx& c, const double* coef, const double* x, double* y) {
    for (int l = 0; l < c.nl; ++l) launch_apply_K_case(c, coef, x + l * c.ndof, y + l * c.ndof);
}

// S [x; beta]: t_e (coupling the cases) and its sum, K(rho') x_l per case,
// then the rank-one terms added, and the alpha entry -sum wt
void ml_apply_S(Ctx& c, const double* x, double* y) {
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_ml_tdot, dim3(g), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.nl, c.ndof,
                       c.be, c.w, x, c.fixed, c.wt, c.partials);
    ml_apply_K(c, c.r1, x, y);
    const dim3 gn(grid_of(c.nn));
    switch (c.nl) {
        case 2:
            hipLaunchKernelGGL(k_ml_rank1<2>, gn, dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.ndof,
                               c.be, c.wt, c.fixed, y);
            break;
        case 3:
            hipLaunchKernelGGL(k_ml_rank1<3>, gn, dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.ndof,
                               c.be, c.wt, c.fixed, y);
            break;
        default:
            hipLaunchKernelGGL(k_ml_rank1<4>, gn, dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.ndof,
                               c.be, c.wt, c.fixed, y);
            break;
    }
    fin(c, g, SL_WT, 1, 0u);
    hipLaunchKernelGGL(k_ml_store_neg, dim3(1), dim3(64), 0, c.s, c.red, (int)SL_WT, y + c.nvec);
}

void ml_launch_dnu(Ctx& c) {
    MlDnuArgs a{c.nx, c.ny, c.nz, c.nl, c.ndof, c.Ke, c.be, c.dy, c.r2, c.l2, c.h2, c.g3, c.g4,
                c.fixed, c.c1, c.c2, c.dnl, c.dnh, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_ml_dnu, dim3(g), dim3(kThreads), 0, c.s, a);
    fin(c, g, SL_SLOPE_NU, 1, 0u);
}

void ml_launch_energy(Ctx& c, const double* u, double* e) {
    hipLaunchKernelGGL(k_ml_energy, dim3(grid_of(c.m)), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz,
                       c.nl, c.ndof, c.Ke, u, c.fixed, e);
}

void ml_launch_update(Ctx& c, double kappa) {
    const int64_t n = std::max(c.nvec, c.m);
    hipLaunchKernelGGL(k_ml_update, dim3(grid_of(n)), dim3(kThreads), 0, c.s, c.nvec, c.m, kappa,
                       c.u, c.dy, c.nlo, c.nhi, c.dnl, c.dnh);
}

vts_status ml_create(Ctx& c, const std::vector<uint8_t>& fine_mask) {
    MlHierarchy* H = new MlHierarchy();
    c.mlh = H;
    H->nl = c.nl;
    H->NB = 3 * c.nl;
    H->L = c.L;
    H->lv.resize(c.L);
    // every level's DOF mask, kept until the copies below have completed
    std::vector<std::vector<uint8_t>> masks(c.L);
    masks[c.L - 1] = fine_mask;
    for (int k = c.L - 1, nx = c.nx, ny = c.ny, nz = c.nz; k > 0; --k, nx /= 2, ny /= 2, nz /= 2)
        masks[k - 1] = ml_coarsen(masks[k], nx, ny, nz);
    const std::vector<uint8_t>& mk = masks[0];
    int nx = c.nx, ny = c.ny, nz = c.nz;
    for (int k = c.L - 1; k >= 0; --k) {
        MlLevel& Lv = H->lv[k];
        Lv.nx = nx;
        Lv.ny = ny;
        Lv.nz = nz;
        Lv.nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
        const int64_t nb = H->NB;
        vts_status st;
        if ((st = ml_alloc(c, (void**)&Lv.fixed, 3 * Lv.nn)) != VTS_OK) return st;
        ML_HIPCHK(hipMemcpyAsync(Lv.fixed, masks[k].data(), 3 * Lv.nn, hipMemcpyHostToDevice, c.s));
        if ((st = ml_alloc(c, (void**)&Lv.A, 27 * nb * nb * Lv.nn * 8)) != VTS_OK) return st;
        if ((st = ml_alloc(c, (void**)&Lv.ac, nb * Lv.nn * 8)) != VTS_OK) return st;
        if (k > 0 && (st = ml_alloc(c, (void**)&Lv.Dinv, nb * nb * Lv.nn * 8)) != VTS_OK) return st;
        if (k < c.L - 1) {
            if ((st = ml_alloc(c, (void**)&Lv.r, (nb * Lv.nn + 1) * 8)) != VTS_OK) return st;
            if ((st = ml_alloc(c, (void**)&Lv.z, (nb * Lv.nn + 1) * 8)) != VTS_OK) return st;
        }
        if (k > 0 && (st = ml_alloc(c, (void**)&Lv.t, (nb * Lv.nn + 1) * 8)) != VTS_OK) return st;
        if (k > 0) {
            nx /= 2;
            ny /= 2;
            nz /= 2;
        }
    }
    // the coarsest level's dense numbering: free DOFs case by case, alpha last
    const MlLevel& C0 = H->lv[0];
    std::vector<int> cmap(H->NB * C0.nn + 1, -1), rows;
    for (int l = 0; l < c.nl; ++l)
        for (int64_t q = 0; q < 3 * C0.nn; ++q)
            if (!mk[q]) {
                cmap[l * 3 * C0.nn + q] = (int)rows.size();
                rows.push_back((int)(l * 3 * C0.nn + q));
            }
    cmap[H->NB * C0.nn] = (int)rows.size();
    rows.push_back((int)(H->NB * C0.nn));
    H->nc = (int)rows.size();
    if (H->nc > kMlMaxCoarse) {
        c.err = "coarsest multigrid level too large for the dense solver (" +
                std::to_string(H->nc) + ")";
        return VTS_EINVAL;
    }
    vts_status st;
    if ((st = ml_alloc(c, (void**)&H->cmap, cmap.size() * sizeof(int))) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->rows, rows.size() * sizeof(int))) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->A0, (size_t)H->nc * H->nc * 8)) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->A0inv, (size_t)H->nc * H->nc * 8)) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->flag, sizeof(int))) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->part, (size_t)kRedBlocks * 8)) != VTS_OK) return st;
    if ((st = ml_alloc(c, (void**)&H->red, 8 * 8)) != VTS_OK) return st;
    ML_HIPCHK(hipMemcpyAsync(H->cmap, cmap.data(), cmap.size() * sizeof(int), hipMemcpyHostToDevice,
                          c.s));
    ML_HIPCHK(hipMemcpyAsync(H->rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice,
                          c.s));
    ML_HIPCHK(hipStreamSynchronize(c.s));
    return VTS_OK;
}

void ml_destroy(Ctx& c) {
    delete c.mlh;     // the device buffers are in c.allocs
    c.mlh = nullptr;
}

// assemble every level, factor the coarsest; returns 1 if a diagonal block or
// the coarsest matrix is not positive definite (synchronizes the stream)
int ml_mg_build(Ctx& c) {
    MlHierarchy& H = *c.mlh;
    int zero = 0;
    (void)hipMemcpyAsync(H.flag, &zero, sizeof(int), hipMemcpyHostToDevice, c.s);
    switch (H.NB) {
        case 3: build_levels<3>(c, H); break;
        case 6: build_levels<6>(c, H); break;
        case 9: build_levels<9>(c, H); break;
        default: build_levels<12>(c, H); break;
    }
    int flag = 0;
    (void)hipMemcpyAsync(&flag, H.flag, sizeof(int), hipMemcpyDeviceToHost, c.s);
    (void)hipStreamSynchronize(c.s);
    return flag;
}

void ml_vcycle(Ctx& c, const double* r, double* z) {
    MlHierarchy& H = *c.mlh;
    switch (H.NB) {
        case 3: vcycle_level<3>(c, H, H.L - 1, r, z); break;
        case 6: vcycle_level<6>(c, H, H.L - 1, r, z); break;
        case 9: vcycle_level<9>(c, H, H.L - 1, r, z); break;
        default: vcycle_level<12>(c, H, H.L - 1, r, z); break;
    }
}

}  // namespace vts
