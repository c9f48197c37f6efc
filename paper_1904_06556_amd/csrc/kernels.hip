// HIP kernels of libvts for CDNA4 (gfx950), wave64.
//
// Layouts (see include/vts.h): all-DOF displacement vectors, node-major xyz;
// per-element arrays in element order; per-element 24-vectors stored
// component-major ([j][e]) so that a wave reads them coalesced.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cfloat>
#include <cmath>

#include "device_util.hpp"
#include "vts_internal.hpp"

namespace vts {

__global__ void k_finalize(const double* __restrict__ partials, int nb, int slot0,
                           uint32_t maxmask, double* __restrict__ out) {
    finalize_body(partials, nb, slot0, maxmask, out);
}

// ---------------------------------------------------------------------------
// K(rho) x : one thread per node gathers the contributions of its <= 8
// elements (problem (1.1), K(rho) = sum rho_i K_i); deterministic, no atomics.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_apply_K(int nx, int ny, int nz, const T* __restrict__ Ke, const T* __restrict__ rho,
          const T* __restrict__ x, const uint8_t* __restrict__ fixed, T* __restrict__ y) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t n = gid();
    if (n >= nn) return;
    const int i = (int)(n % NX);
    const int64_t t = n / NX;
    const int j = (int)(t % NY), k = (int)(t / NY);
    T a0 = 0, a1 = 0, a2 = 0;
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
                const T* K0 = Ke + (3 * la) * 24;
                T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int64_t nb = node_id(ii + (b & 1), jj + ((b >> 1) & 1), kk + (b >> 2), NX, NY);
                    const T x0 = fixed[3 * nb] ? T(0) : x[3 * nb];
                    const T x1 = fixed[3 * nb + 1] ? T(0) : x[3 * nb + 1];
                    const T x2 = fixed[3 * nb + 2] ? T(0) : x[3 * nb + 2];
                    s0 += K0[3 * b] * x0 + K0[3 * b + 1] * x1 + K0[3 * b + 2] * x2;
                    s1 += K0[24 + 3 * b] * x0 + K0[24 + 3 * b + 1] * x1 + K0[24 + 3 * b + 2] * x2;
                    s2 += K0[48 + 3 * b] * x0 + K0[48 + 3 * b + 1] * x1 + K0[48 + 3 * b + 2] * x2;
                }
                const T r = rho[e];
                a0 += r * s0;
                a1 += r * s1;
                a2 += r * s2;
            }
        }
    }
    y[3 * n] = fixed[3 * n] ? T(0) : a0;
    y[3 * n + 1] = fixed[3 * n + 1] ? T(0) : a1;
    y[3 * n + 2] = fixed[3 * n + 2] ? T(0) : a2;
}

void launch_apply_K_f64(Ctx& c, const double* rho, const double* x, double* y) {
    if (c.nl > 1) {
        ml_apply_K(c, rho, x, y);
        return;
    }
    launch_apply_K_case(c, rho, x, y);
}

// K(rho) x on one all-DOF vector (one load case)
void launch_apply_K_case(Ctx& c, const double* rho, const double* x, double* y) {
    if (tile_ok(c)) {
        // algorithmic bytes: read x and rho, write y (8 B each entry); the
        // Dirichlet data (one mask byte per node) are not counted
        const bool prof = prof_begin(c, VTS_PROF_APPLY_K);
        launch_apply_K_tile_f64(c, rho, x, y);
        if (prof) prof_end(c, 16.0 * c.ndof + 8.0 * c.m);
        return;
    }
    hipLaunchKernelGGL(k_apply_K<double>, dim3(grid1d(c.nn)), dim3(kThreads), 0, c.s,
                       c.nx, c.ny, c.nz, c.Ke, rho, x, c.fixed, y);
}
void launch_apply_K_f32(Ctx& c, const float* rho, const float* x, float* y) {
    if (tile_ok(c)) {
        launch_apply_K_tile_f32(c, rho, x, y);
        return;
    }
    hipLaunchKernelGGL(k_apply_K<float>, dim3(grid1d(c.nn)), dim3(kThreads), 0, c.s,
                       c.nx, c.ny, c.nz, c.Kef, rho, x, c.fixed, y);
}

// e_i = 1/2 u_e^T K_e u_e
__global__ void __launch_bounds__(kThreads)
k_energy(int nx, int ny, int nz, const double* __restrict__ Ke, const double* __restrict__ u,
         const uint8_t* __restrict__ fixed, double* __restrict__ eout) {
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t e = gid();
    if (e >= m) return;
    int i, j, k;
    elem_ijk(e, nx, ny, i, j, k);
    double ue[24];
    gather_elem(u, fixed, i, j, k, nx + 1, ny + 1, ue);
    double en = 0.0;
    for (int r = 0; r < 24; ++r) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 24; ++q) s += Ke[r * 24 + q] * ue[q];
        en += ue[r] * s;
    }
    eout[e] = 0.5 * en;
}

void launch_energy(Ctx& c, const double* u, double* e) {
    if (c.nl > 1) {
        ml_launch_energy(c, u, e);
        return;
    }
    hipLaunchKernelGGL(k_energy, dim3(grid1d(c.m)), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz,
                       c.Ke, u, c.fixed, e);
}

// ---------------------------------------------------------------------------
// Evaluation at the current state (Section 3.2): energies, forces b_e = K_e u_e,
// s_i, rho', rho'', mu', mu'', res_3, res_4, Schur weight w and rhs weight z.
// Partial sums: sum rho', sum z, sum w, ||res3||^2, ||res4||^2.
// ---------------------------------------------------------------------------
struct EvalArgs {
    int nx, ny, nz;
    double alpha;
    const double *Ke, *u, *nlo, *nhi, *rho, *mlo, *mhi, *p, *qlo, *qhi, *rlo, *rhi;
    const uint8_t* fixed;
    double *e, *be, *r1, *r2, *l2, *h2, *g3, *g4, *w, *zc, *partials;
};

__global__ void __launch_bounds__(kThreads) k_eval(EvalArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double ue[24];
        gather_elem(a.u, a.fixed, i, j, k, a.nx + 1, a.ny + 1, ue);
        double en = 0.0;
        for (int r = 0; r < 24; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 24; ++q) s += a.Ke[r * 24 + q] * ue[q];
            a.be[r * m + e] = s;
            en += ue[r] * s;
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
        // 2x2 block of (nu_lo, nu_hi): det with the rho''^2 terms cancelled
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

void launch_eval(Ctx& c) {
    if (c.nl > 1) {
        ml_launch_eval(c);
        return;
    }
    EvalArgs a{c.nx, c.ny, c.nz, c.alpha, c.Ke, c.u, c.nlo, c.nhi, c.rho, c.mlo, c.mhi, c.p,
               c.qlo, c.qhi, c.rlo, c.rhi, c.fixed, c.e, c.be, c.r1, c.r2, c.l2, c.h2,
               c.g3, c.g4, c.w, c.zc, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_eval, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(5), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_SUM_R1,
                       0u, c.red);
}

// res_1 = K(rho')u - f = sum_e rho'_e b_e - f and the reduced right-hand side
// rhs_u = -res_1 + sum_e z_e b_e = f - sum_e (rho'_e - z_e) b_e (masked).
__global__ void __launch_bounds__(kThreads)
k_grad(int nx, int ny, int nz, const double* __restrict__ be, const double* __restrict__ r1,
       const double* __restrict__ zc, const double* __restrict__ f,
       const uint8_t* __restrict__ fixed, double* __restrict__ g1, double* __restrict__ rhs,
       double* partials) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t m = (int64_t)nx * ny * nz;
    double acc[1] = {0.0};
    for (int64_t n = gid(); n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(n % NX);
        const int64_t t = n / NX;
        const int j = (int)(t % NY), k = (int)(t / NY);
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
                        const double bv = be[(3 * la + c) * m + e];
                        a[c] += w1 * bv;
                        b[c] += w2 * bv;
                    }
                }
            }
        }
        for (int c = 0; c < 3; ++c) {
            const bool fx = fixed[3 * n + c];
            const double gv = fx ? 0.0 : a[c] - f[3 * n + c];
            g1[3 * n + c] = gv;
            rhs[3 * n + c] = fx ? 0.0 : f[3 * n + c] - b[c];
            acc[0] += gv * gv;
        }
    }
    block_sum_store<1>(acc, partials, SL_G1SQ);
}

void launch_grad(Ctx& c) {
    if (c.nl > 1) {
        ml_launch_grad(c);
        return;
    }
    const int g = red_grid(c.nn);
    hipLaunchKernelGGL(k_grad, dim3(g), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.be, c.r1,
                       c.zc, c.f, c.fixed, c.g1, c.rhs, c.partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_G1SQ,
                       0u, c.red);
}

// ---------------------------------------------------------------------------
// S [x; beta] of eq. (3.12), matrix-free in FP64:
//   pass 1 (elements): wt_e = w_e (b_e^T x_e - beta), partial sum of wt
//   pass 2 (nodes):    y_n = sum_e rho'_e (K_e x_e)_n + wt_e (b_e)_n
//   y_alpha = -sum_e wt_e
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_S_pass1(int nx, int ny, int nz, const double* __restrict__ be, const double* __restrict__ w,
          const double* __restrict__ x, int64_t ndof, const uint8_t* __restrict__ fixed,
          double* __restrict__ wt, double* partials) {
    const int64_t m = (int64_t)nx * ny * nz;
    const double beta = x[ndof];
    double acc[1] = {0.0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, nx, ny, i, j, k);
        double xe[24];
        gather_elem(x, fixed, i, j, k, nx + 1, ny + 1, xe);
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 24; ++q) t += be[q * m + e] * xe[q];
        const double v = w[e] * (t - beta);
        wt[e] = v;
        acc[0] += v;
    }
    block_sum_store<1>(acc, partials, SL_WT);
}

__global__ void __launch_bounds__(kThreads)
k_S_pass2(int nx, int ny, int nz, const double* __restrict__ Ke, const double* __restrict__ r1,
          const double* __restrict__ be, const double* __restrict__ wt,
          const double* __restrict__ x, const uint8_t* __restrict__ fixed,
          double* __restrict__ y) {
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nn = (int64_t)NX * NY * (nz + 1);
    const int64_t m = (int64_t)nx * ny * nz;
    const int64_t n = gid();
    if (n >= nn) return;
    const int i = (int)(n % NX);
    const int64_t t = n / NX;
    const int j = (int)(t % NY), k = (int)(t / NY);
    double a0 = 0, a1 = 0, a2 = 0;
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
                const double* K0 = Ke + (3 * la) * 24;
                double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int64_t nb = node_id(ii + (b & 1), jj + ((b >> 1) & 1), kk + (b >> 2), NX, NY);
                    const double x0 = fixed[3 * nb] ? 0.0 : x[3 * nb];
                    const double x1 = fixed[3 * nb + 1] ? 0.0 : x[3 * nb + 1];
                    const double x2 = fixed[3 * nb + 2] ? 0.0 : x[3 * nb + 2];
                    s0 += K0[3 * b] * x0 + K0[3 * b + 1] * x1 + K0[3 * b + 2] * x2;
                    s1 += K0[24 + 3 * b] * x0 + K0[24 + 3 * b + 1] * x1 + K0[24 + 3 * b + 2] * x2;
                    s2 += K0[48 + 3 * b] * x0 + K0[48 + 3 * b + 1] * x1 + K0[48 + 3 * b + 2] * x2;
                }
                const double r = r1[e], q = wt[e];
                a0 += r * s0 + q * be[(3 * la) * m + e];
                a1 += r * s1 + q * be[(3 * la + 1) * m + e];
                a2 += r * s2 + q * be[(3 * la + 2) * m + e];
            }
        }
    }
    y[3 * n] = fixed[3 * n] ? 0.0 : a0;
    y[3 * n + 1] = fixed[3 * n + 1] ? 0.0 : a1;
    y[3 * n + 2] = fixed[3 * n + 2] ? 0.0 : a2;
}

__global__ void k_store_neg(const double* __restrict__ red, int slot, double* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = -red[slot];
}

void launch_apply_S(Ctx& c, const double* x, double* y) {
    if (c.nl > 1) {
        ml_apply_S(c, x, y);
        return;
    }
    if (tile_ok(c)) {
        // algorithmic bytes: x, u, y, rho', w and the DOF mask
        const bool prof = prof_begin(c, VTS_PROF_APPLY_S);
        launch_apply_S_tile(c, x, y);
        if (prof) prof_end(c, 24.0 * c.ndof + 16.0 * c.m + c.ndof);
        return;
    }
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_S_pass1, dim3(g), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz, c.be, c.w,
                       x, c.ndof, c.fixed, c.wt, c.partials);
    hipLaunchKernelGGL(k_S_pass2, dim3(grid1d(c.nn)), dim3(kThreads), 0, c.s, c.nx, c.ny, c.nz,
                       c.Ke, c.r1, c.be, c.wt, x, c.fixed, y);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_WT, 0u,
                       c.red);
    hipLaunchKernelGGL(k_store_neg, dim3(1), dim3(64), 0, c.s, c.red, (int)SL_WT, y + c.ndof);
}

// ---------------------------------------------------------------------------
// Newton completion: Delta nu of eq. (3.14) (multiplied out), and the line
// search coefficients c1 = b_e^T du_e, c2 = 1/2 du_e^T K_e du_e so that
// e_i(u + k du) = e_i + k c1 + k^2 c2 exactly.
// ---------------------------------------------------------------------------
struct DnuArgs {
    int nx, ny, nz;
    int64_t ndof;
    const double *Ke, *be, *dy, *r2, *l2, *h2, *g3, *g4;
    const uint8_t* fixed;
    double *c1, *c2, *dnl, *dnh, *partials;
};

__global__ void __launch_bounds__(kThreads) k_dnu(DnuArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    const double da = a.dy[a.ndof];
    double acc[1] = {0.0};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double de[24];
        gather_elem(a.dy, a.fixed, i, j, k, a.nx + 1, a.ny + 1, de);
        double t = 0.0, q2 = 0.0;
        for (int r = 0; r < 24; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 24; ++q) s += a.Ke[r * 24 + q] * de[q];
            q2 += de[r] * s;
            t += a.be[r * m + e] * de[r];
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

void launch_dnu(Ctx& c) {
    if (c.nl > 1) {
        ml_launch_dnu(c);
        return;
    }
    DnuArgs a{c.nx, c.ny, c.nz, c.ndof, c.Ke, c.be, c.dy, c.r2, c.l2, c.h2, c.g3, c.g4,
              c.fixed, c.c1, c.c2, c.dnl, c.dnh, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_dnu, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g,
                       (int)SL_SLOPE_NU, 0u, c.red);
}

// Elementwise part of L(xi + k dxi) - L(xi), eq. (3.9), formed along the ray:
// the argument of each phi changes by k (c1 + k c2 - dalpha + dnu_lo - dnu_hi)/p
// (resp. -k dnu/q), phi's change comes from its branch-wise difference, and
//   rho p dphi(s) + mu_lo q_lo dphi(t_lo) + mu_hi q_hi dphi(t_hi)
//   - k rho_lo dnu_lo + k rho_hi dnu_hi
// is summed; the linear terms in alpha and u are added on the host.
struct LsArgs {
    int64_t m;
    double kappa, alpha, dalpha;
    const double *e, *c1, *c2, *nlo, *nhi, *dnl, *dnh, *rho, *mlo, *mhi, *p, *qlo, *qhi, *rlo,
        *rhi;
    double* partials;
};

__global__ void __launch_bounds__(kThreads) k_linesearch(LsArgs a) {
    double acc[1] = {0.0};
    const double k = a.kappa;
    for (int64_t e = gid(); e < a.m; e += (int64_t)gridDim.x * blockDim.x) {
        const double pe = a.p[e], ql = a.qlo[e], qh = a.qhi[e];
        const double nl0 = a.nlo[e], nh0 = a.nhi[e], dl = a.dnl[e], dh = a.dnh[e];
        const double s0 = (a.e[e] - a.alpha + nl0 - nh0) / pe;
        const double ds = k * (a.c1[e] + k * a.c2[e] - a.dalpha + dl - dh) / pe;
        double v = a.rho[e] * pe * pen_phi_diff(s0, ds);
        v += a.mlo[e] * ql * pen_phi_diff(-nl0 / ql, -k * dl / ql);
        v += a.mhi[e] * qh * pen_phi_diff(-nh0 / qh, -k * dh / qh);
        v += k * (-a.rlo[e] * dl + a.rhi[e] * dh);
        acc[0] += v;
    }
    block_sum_store<1>(acc, a.partials, SL_LS);
}

void launch_linesearch(Ctx& c, double kappa, double dalpha) {
    LsArgs a{c.m, kappa, c.alpha, dalpha, c.e, c.c1, c.c2, c.nlo, c.nhi, c.dnl, c.dnh, c.rho,
             c.mlo, c.mhi, c.p, c.qlo, c.qhi, c.rlo, c.rhi, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_linesearch, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_LS, 0u,
                       c.red);
}

__global__ void k_update(int64_t ndof, int64_t m, double kappa, double* __restrict__ u,
                         const double* __restrict__ dy, double* __restrict__ nlo,
                         double* __restrict__ nhi, const double* __restrict__ dnl,
                         const double* __restrict__ dnh) {
    const int64_t t = gid();
    if (t < ndof) u[t] += kappa * dy[t];
    if (t < m) {
        nlo[t] += kappa * dnl[t];
        nhi[t] += kappa * dnh[t];
    }
}

void launch_update(Ctx& c, double kappa) {
    // u holds every load case (nvec entries)
    const int64_t n = c.nvec > c.m ? c.nvec : c.m;
    hipLaunchKernelGGL(k_update, dim3(grid1d(n)), dim3(kThreads), 0, c.s, c.nvec, c.m, kappa, c.u,
                       c.dy, c.nlo, c.nhi, c.dnl, c.dnh);
}

// ---------------------------------------------------------------------------
// PBM outer step (Algorithm 1): gap (2.6) and dual objective parts, the
// candidate rho+ = clip(rho phi'(s)) and its stationarity estimate.
// ---------------------------------------------------------------------------
struct OuterArgs {
    int64_t m;
    double alpha, beta;
    const double *e, *nlo, *nhi, *rho, *p, *rlo, *rhi;
    double* partials;
};

__global__ void __launch_bounds__(kThreads) k_outer(OuterArgs a) {
    // slots: GAP (sum min), NLO (rlo.nlo), NHI (rhi.nhi), STAT (max), SUM_RHO
    double acc[5] = {0, 0, 0, -DBL_MAX, 0};
    for (int64_t e = gid(); e < a.m; e += (int64_t)gridDim.x * blockDim.x) {
        const double d = a.alpha - a.e[e];
        acc[0] += fmin(a.rlo[e] * d, a.rhi[e] * d);
        acc[1] += a.rlo[e] * a.nlo[e];
        acc[2] += a.rhi[e] * a.nhi[e];
        const double s = (a.e[e] - a.alpha + a.nlo[e] - a.nhi[e]) / a.p[e];
        const double r = a.rho[e];
        const double rp = fmin(fmax(r * pen_dphi(s), a.beta * r), r / a.beta);
        const double proj = fmin(fmax(rp + (a.e[e] - a.alpha) / a.alpha, a.rlo[e]), a.rhi[e]);
        acc[3] = fmax(acc[3], fabs(rp - proj) / a.rhi[e]);
        acc[4] += r;
    }
    block_sum_store<5>(acc, a.partials, SL_GAP, 1u << 3);
}

void launch_outer_eval(Ctx& c) {
    OuterArgs a{c.m, c.alpha, c.opt.beta, c.e, c.nlo, c.nhi, c.rho, c.p, c.rlo, c.rhi, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_outer, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(5), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_GAP,
                       1u << 3, c.red);
}

// KKT residual of (rho, u, lam) by its definition, from Ku = K(rho)u and
// e = e(u): the sums ||Ku - f||^2 and sum rho, and the maxima of
// |rho - clip(rho + (e - lam)/lam)| / hi, of the bound violation and of hi.
__global__ void __launch_bounds__(kThreads)
k_kkt(int64_t ndof, int64_t m, double lam, const double* __restrict__ Ku,
      const double* __restrict__ f, const double* __restrict__ rho, const double* __restrict__ e,
      const double* __restrict__ lo, const double* __restrict__ hi, double* partials) {
    // slots: STAT (max), SUM_RHO, WT (= ||Ku - f||^2), AUX (box, max), MRALPHA (max hi)
    double acc[5] = {-DBL_MAX, 0.0, 0.0, 0.0, -DBL_MAX};
    const int64_t n = ndof > m ? ndof : m;
    for (int64_t t = gid(); t < n; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < ndof) {
            const double d = Ku[t] - f[t];
            acc[2] += d * d;
        }
        if (t < m) {
            const double r = rho[t], l = lo[t], h = hi[t];
            const double proj = fmin(fmax(r + (e[t] - lam) / lam, l), h);
            acc[0] = fmax(acc[0], fabs(r - proj) / h);
            acc[1] += r;
            acc[3] = fmax(acc[3], fmax(l - r, r - h));
            acc[4] = fmax(acc[4], h);
        }
    }
    block_sum_store<5>(acc, partials, SL_STAT, 0x19u);
}

void launch_kkt(Ctx& c, double lam, double* Ku) {
    launch_apply_K_f64(c, c.rho, c.u, Ku);
    launch_energy(c, c.u, c.e);
    const int64_t n = c.nvec > c.m ? c.nvec : c.m;
    const int g = red_grid(n);
    hipLaunchKernelGGL(k_kkt, dim3(g), dim3(kThreads), 0, c.s, c.nvec, c.m, lam, Ku, c.f, c.rho,
                       c.e, c.rlo, c.rhi, c.partials);
    hipLaunchKernelGGL(k_finalize, dim3(5), dim3(kThreads), 0, c.s, c.partials, g, (int)SL_STAT,
                       0x19u, c.red);
}

// Multiplier update of Algorithm 1 with the safeguard beta x <= x+ <= x/beta.
__global__ void k_mult(int64_t m, double alpha, double beta, int rho_only,
                       const double* __restrict__ e, const double* __restrict__ nlo,
                       const double* __restrict__ nhi, const double* __restrict__ p,
                       const double* __restrict__ qlo, const double* __restrict__ qhi,
                       double* __restrict__ rho, double* __restrict__ mlo,
                       double* __restrict__ mhi) {
    const int64_t t = gid();
    if (t >= m) return;
    const double s = (e[t] - alpha + nlo[t] - nhi[t]) / p[t];
    const double r = rho[t];
    rho[t] = fmin(fmax(r * pen_dphi(s), beta * r), r / beta);
    if (rho_only) return;
    const double a = mlo[t], b = mhi[t];
    mlo[t] = fmin(fmax(a * pen_dphi(-nlo[t] / qlo[t]), beta * a), a / beta);
    mhi[t] = fmin(fmax(b * pen_dphi(-nhi[t] / qhi[t]), beta * b), b / beta);
}

void launch_mult_update(Ctx& c, int rho_only) {
    hipLaunchKernelGGL(k_mult, dim3(grid1d(c.m)), dim3(kThreads), 0, c.s, c.m, c.alpha,
                       c.opt.beta, rho_only, c.e, c.nlo, c.nhi, c.p, c.qlo, c.qhi, c.rho, c.mlo,
                       c.mhi);
}

__global__ void k_penalty(int64_t m, double gamma, double pmin, double qmin,
                          double* __restrict__ p, double* __restrict__ qlo,
                          double* __restrict__ qhi) {
    const int64_t t = gid();
    if (t >= m) return;
    p[t] = fmax(gamma * p[t], pmin);
    qlo[t] = fmax(gamma * qlo[t], qmin);
    qhi[t] = fmax(gamma * qhi[t], qmin);
}

void launch_penalty_update(Ctx& c) {
    // floors of p and q relative to the energy scale |alpha| unless asked otherwise
    const bool rel = c.opt.p_min_relative && c.alpha != 0.0;
    const double pfloor = rel ? c.opt.p_min * fabs(c.alpha) : c.opt.p_min;
    const double qfloor = rel ? c.opt.q_min * fabs(c.alpha) : c.opt.q_min;
    hipLaunchKernelGGL(k_penalty, dim3(grid1d(c.m)), dim3(kThreads), 0, c.s, c.m, c.opt.gamma,
                       pfloor, qfloor, c.p, c.qlo, c.qhi);
}

__global__ void k_init(int64_t ndof, int64_t m, double rho0, double* u, double* nlo,
                       double* nhi, double* rho, double* mlo, double* mhi, double* p,
                       double* qlo, double* qhi) {
    const int64_t t = gid();
    if (t < ndof) u[t] = 0.0;
    if (t < m) {
        nlo[t] = 1.0; nhi[t] = 1.0; rho[t] = rho0; mlo[t] = 1.0; mhi[t] = 1.0;
        p[t] = 1.0; qlo[t] = 1.0; qhi[t] = 1.0;
    }
}

void launch_init_state(Ctx& c) {
    const int64_t n = c.nvec > c.m ? c.nvec : c.m;
    hipLaunchKernelGGL(k_init, dim3(grid1d(n)), dim3(kThreads), 0, c.s, c.nvec, c.m,
                       c.V / (double)c.m, c.u, c.nlo, c.nhi, c.rho, c.mlo, c.mhi, c.p, c.qlo,
                       c.qhi);
}

__global__ void k_round(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t t = gid();
    if (t < m) b[t] = (float)a[t];
}
void launch_round_rho(Ctx& c) {
    hipLaunchKernelGGL(k_round, dim3(grid1d(c.m)), dim3(kThreads), 0, c.s, c.m, c.rho, c.rhof);
}

// ---------------------------------------------------------------------------
// vector kernels (MINRES)
// ---------------------------------------------------------------------------
struct DotArgs {
    const double* x;
    const double* y;
    int64_t n;
    int slot;
    double* partials;
};
__device__ __forceinline__ void dot_body(const DotArgs& a) {
    double acc[1] = {0.0};
    for (int64_t t = gid(); t < a.n; t += (int64_t)gridDim.x * blockDim.x)
        acc[0] += a.x[t] * a.y[t];
    block_sum_store<1>(acc, a.partials, a.slot);
}
VTS_KERNEL_PAIR(, kThreads, k_dot, DotArgs, dot_body)

struct FinArgs {
    const double* partials;
    int nb, slot;
    double* out;
};
__device__ __forceinline__ void fin_body(const FinArgs& a) {
    finalize_body(a.partials, a.nb, a.slot, 0u, a.out);
}
VTS_KERNEL_PAIR(, kThreads, k_dot_fin, FinArgs, fin_body)

void launch_dot(Ctx& c, const double* x, const double* y, int64_t n, int slot) {
    const int g = red_grid(n);
    vlaunch(c, (const void*)&k_dot, (const void*)&k_dot_b, dim3(g), dim3(kThreads),
            DotArgs{x, y, n, slot, c.partials});
    vlaunch(c, (const void*)&k_dot_fin, (const void*)&k_dot_fin_b, dim3(1), dim3(kThreads),
            FinArgs{c.partials, g, slot, c.red});
}

__global__ void k_copy1(const double* __restrict__ src, double* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}
void launch_copy1(Ctx& c, const double* src, double* dst) {
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, c.s, src, dst);
}

__global__ void k_set(double* dst, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = v;
}
void launch_set(Ctx& c, double* dst, double v) {
    hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, c.s, dst, v);
}

struct FillArgs {
    double* d;
    double v;
    int64_t n;
};
__device__ __forceinline__ void fill_body(const FillArgs& a) {
    const int64_t t = gid();
    if (t < a.n) a.d[t] = a.v;
}
VTS_KERNEL_PAIR(, kThreads, k_fill, FillArgs, fill_body)
void launch_fill(Ctx& c, double* dst, double v, int64_t n) {
    vlaunch(c, (const void*)&k_fill, (const void*)&k_fill_b, dim3(grid1d(n)), dim3(kThreads),
            FillArgs{dst, v, n});
}

struct ScaleArgs {
    double* d;
    const double* s;
    double a;
    int64_t n;
};
__device__ __forceinline__ void scale_body(const ScaleArgs& a) {
    const int64_t t = gid();
    if (t < a.n) a.d[t] = a.a * a.s[t];
}
VTS_KERNEL_PAIR(, kThreads, k_scale, ScaleArgs, scale_body)
void launch_scale(Ctx& c, double* dst, const double* src, double a, int64_t n) {
    vlaunch(c, (const void*)&k_scale, (const void*)&k_scale_b, dim3(grid1d(n)), dim3(kThreads),
            ScaleArgs{dst, src, a, n});
}

struct AxpyArgs {
    double* y;
    double a;
    const double* x;
    int64_t n;
};
__device__ __forceinline__ void axpy_body(const AxpyArgs& a) {
    const int64_t t = gid();
    if (t < a.n) a.y[t] += a.a * a.x[t];
}
VTS_KERNEL_PAIR(, kThreads, k_axpy, AxpyArgs, axpy_body)
void launch_axpy(Ctx& c, double* y, double a, const double* x, int64_t n) {
    vlaunch(c, (const void*)&k_axpy, (const void*)&k_axpy_b, dim3(grid1d(n)), dim3(kThreads),
            AxpyArgs{y, a, x, n});
}

struct AxpyRedArgs {
    double* y;
    const double* red;
    int slot;
    double div;
    const double* x;
    int64_t n;
};
__device__ __forceinline__ void axpy_red_body(const AxpyRedArgs& a) {
    const int64_t t = gid();
    const double f = -(a.red[a.slot] / a.div);
    if (t < a.n) a.y[t] += f * a.x[t];
}
VTS_KERNEL_PAIR(, kThreads, k_axpy_red, AxpyRedArgs, axpy_red_body)
void launch_axpy_red(Ctx& c, double* y, int slot, double div, const double* x, int64_t n) {
    vlaunch(c, (const void*)&k_axpy_red, (const void*)&k_axpy_red_b, dim3(grid1d(n)),
            dim3(kThreads), AxpyRedArgs{y, c.red, slot, div, x, n});
}

// ---------------------------------------------------------------------------
// damped optimality criteria (Algorithm 4)
// ---------------------------------------------------------------------------
// K(rho) as the Schur operator with rho' = rho, w = 0 (no rank-one terms, no
// alpha coupling) and right-hand side [f; 0]
__global__ void k_doc_setup(int64_t m, int64_t nbe, int64_t nvec, const double* __restrict__ rho,
                            const double* __restrict__ f, double* __restrict__ r1,
                            double* __restrict__ w, double* __restrict__ be,
                            double* __restrict__ rhs) {
    const int64_t t = gid();
    if (t < m) {
        r1[t] = rho[t];
        w[t] = 0.0;
    }
    if (t < nbe) be[t] = 0.0;
    if (t < nvec) rhs[t] = f[t];
    if (t == 0) rhs[nvec] = 0.0;
}
void launch_doc_setup(Ctx& c) {
    // every load case: be of all cases, f and rhs stacked
    const int64_t nbe = 24 * c.m * c.nl;
    hipLaunchKernelGGL(k_doc_setup, dim3(grid1d(std::max<int64_t>(nbe, c.nvec + 1))),
                       dim3(kThreads), 0, c.s, c.m, nbe, c.nvec, c.rho, c.f, c.r1, c.w, c.be,
                       c.rhs);
}

__device__ __forceinline__ double doc_candidate(double rho, double e, double lo, double hi,
                                                double q, double alpha) {
    // rho (u^T K_i u)^q / alpha, clamped to the bounds
    return fmin(fmax(rho * pow(2.0 * e, q) / alpha, lo), hi);
}

// partial sums of the candidate volume sum_i rho+_i(alpha)
__global__ void __launch_bounds__(kThreads)
k_doc_volume(int64_t m, double q, double alpha, const double* __restrict__ rho,
             const double* __restrict__ e, const double* __restrict__ lo,
             const double* __restrict__ hi, double* partials) {
    double acc[1] = {0.0};
    for (int64_t t = gid(); t < m; t += (int64_t)gridDim.x * blockDim.x)
        acc[0] += doc_candidate(rho[t], e[t], lo[t], hi[t], q, alpha);
    block_sum_store<1>(acc, partials, SL_SUM_RHO);
}
void launch_doc_volume(Ctx& c, double q, double alpha) {
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_doc_volume, dim3(g), dim3(kThreads), 0, c.s, c.m, q, alpha, c.rho, c.e,
                       c.rlo, c.rhi, c.partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g,
                       (int)SL_SUM_RHO, 0u, c.red);
}

// rho+ (alpha) into out and the partial maxima of |rho+ - rho|
__global__ void __launch_bounds__(kThreads)
k_doc_candidate(int64_t m, double q, double alpha, const double* __restrict__ rho,
                const double* __restrict__ e, const double* __restrict__ lo,
                const double* __restrict__ hi, double* __restrict__ out, double* partials) {
    double acc[1] = {0.0};
    for (int64_t t = gid(); t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const double r = doc_candidate(rho[t], e[t], lo[t], hi[t], q, alpha);
        out[t] = r;
        acc[0] = fmax(acc[0], fabs(r - rho[t]));
    }
    block_sum_store<1>(acc, partials, SL_STAT, 1u);
}
void launch_doc_candidate(Ctx& c, double q, double alpha, double* out) {
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_doc_candidate, dim3(g), dim3(kThreads), 0, c.s, c.m, q, alpha, c.rho,
                       c.e, c.rlo, c.rhi, out, c.partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c.s, c.partials, g,
                       (int)SL_STAT, 1u, c.red);
}

// ---------------------------------------------------------------------------
// primal-dual interior point method (Section 4, Algorithm 3)
//
// The reduced system (eq. S_IP) is solved in the form of the PBM Schur
// operator with rho' = rho, w = W and the alpha unknown negated
// (beta = -dalpha): that turns the coupling vector [b_i; 1] of S_IP into the
// [b_i; -1] of the S-apply and the V-cycle.  With dlo = rho - rho_lo,
// dhi = rho_hi - rho:
//   W = (nu_lo/dlo + nu_hi/dhi)^-1 = dlo dhi / (nu_lo dhi + nu_hi dlo)
//   X = res_3 - res_4/dlo + res_5/dhi = e + alpha + r/dlo - s/dhi
//   rhs = [-res_1 - sum W X b_i ; res_2 + sum W X]    (alpha row negated)
// so the PBM right-hand side kernel applies with z = -W X.
// ---------------------------------------------------------------------------
struct IpEvalArgs {
    int nx, ny, nz;
    double alpha, r, s;
    const double *Ke, *u, *nlo, *nhi, *rho, *rlo, *rhi;
    const uint8_t* fixed;
    double *e, *be, *r1, *w, *zc, *g3, *g4, *partials;
};

// reduction (kIpEvalQ quantities from slot kIpEvalSlot): sums of rho, z, W,
// res_3^2, the gap term, nu_lo dlo, nu_hi dhi, nu_lo^2, nu_hi^2; maxima of
// the complementarity products and of max(-dlo, -dhi, -nu_lo, -nu_hi)
// (>= 0 once a variable has reached its bound)
__global__ void __launch_bounds__(kThreads) k_ip_eval(IpEvalArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    double acc[kIpEvalQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0, -DBL_MAX, -DBL_MAX};
    const double lam = -a.alpha;
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double ue[24];
        gather_elem(a.u, a.fixed, i, j, k, a.nx + 1, a.ny + 1, ue);
        double en = 0.0;
        for (int r = 0; r < 24; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 24; ++q) s += a.Ke[r * 24 + q] * ue[q];
            a.be[r * m + e] = s;
            en += ue[r] * s;
        }
        en *= 0.5;
        a.e[e] = en;
        const double rh = a.rho[e], nl = a.nlo[e], nh = a.nhi[e];
        const double lo = a.rlo[e], hi = a.rhi[e];
        const double dlo = rh - lo, dhi = hi - rh;
        const double res3 = en + a.alpha + nl - nh;
        const double W = dlo * dhi / (nl * dhi + nh * dlo);
        const double X = en + a.alpha + a.r / dlo - a.s / dhi;
        const double z = -W * X;
        a.r1[e] = rh;
        a.w[e] = W;
        a.zc[e] = z;
        a.g3[e] = res3;
        a.g4[e] = X;
        const double gl = lam - en;                       // gap (2.6) at lambda = -alpha
        const double cl = nl * dlo, ch = nh * dhi;
        acc[0] += rh;
        acc[1] += z;
        acc[2] += W;
        acc[3] += res3 * res3;
        acc[4] += gl >= 0.0 ? lo * gl : hi * gl;
        acc[5] += cl;
        acc[6] += ch;
        acc[7] += nl * nl;
        acc[8] += nh * nh;
        acc[9] = fmax(acc[9], fmax(fabs(cl), fabs(ch)));
        acc[10] = fmax(acc[10], fmax(fmax(-dlo, -dhi), fmax(-nl, -nh)));
    }
    block_sum_store<kIpEvalQ>(acc, a.partials, kIpEvalSlot, kIpEvalMax);
}

void launch_ip_eval(Ctx& c, double r, double s) {
    IpEvalArgs a{c.nx, c.ny, c.nz, c.alpha, r, s, c.Ke, c.u, c.nlo, c.nhi, c.rho, c.rlo, c.rhi,
                 c.fixed, c.e, c.be, c.r1, c.w, c.zc, c.g3, c.g4, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_ip_eval, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(kIpEvalQ), dim3(kThreads), 0, c.s, c.partials, g,
                       kIpEvalSlot, kIpEvalMax, c.red);
}

// Increments from the solution dy = [du; -dalpha] of the reduced system:
//   t = b_i^T du + dalpha,  drho = W (t + X)                      (eq. Delta_rho)
//   dnu_hi = (dlo t - (nu_lo - nu_hi) drho - (res_4 + res_5 - dlo res_3))
//            / (rho_hi - rho_lo)                                    (eq. Delta_onu)
//   dnu_lo = dnu_hi - t - res_3                                     (eq. Delta_unu)
// and the partial maxima of -(step to the boundary) for rho, nu_lo, nu_hi.
struct IpDirArgs {
    int nx, ny, nz;
    int64_t ndof;
    double r, s;
    const double *be, *dy, *w, *g3, *g4, *rho, *nlo, *nhi, *rlo, *rhi;
    const uint8_t* fixed;
    double *drho, *dnl, *dnh, *partials;
};

__global__ void __launch_bounds__(kThreads) k_ip_dir(IpDirArgs a) {
    const int64_t m = (int64_t)a.nx * a.ny * a.nz;
    const double dalpha = -a.dy[a.ndof];
    double acc[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        elem_ijk(e, a.nx, a.ny, i, j, k);
        double de[24];
        gather_elem(a.dy, a.fixed, i, j, k, a.nx + 1, a.ny + 1, de);
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 24; ++q) t += a.be[q * m + e] * de[q];
        t += dalpha;
        const double rh = a.rho[e], nl = a.nlo[e], nh = a.nhi[e];
        const double lo = a.rlo[e], hi = a.rhi[e];
        const double dlo = rh - lo, dhi = hi - rh;
        const double res3 = a.g3[e];
        const double res4 = nl * dlo - a.r, res5 = nh * dhi - a.s;
        const double dr = a.w[e] * (t + a.g4[e]);
        const double dh = (dlo * t - (nl - nh) * dr - (res4 + res5 - dlo * res3)) / (hi - lo);
        const double dl = dh - t - res3;
        a.drho[e] = dr;
        a.dnl[e] = dl;
        a.dnh[e] = dh;
        if (dr > 0.0) acc[0] = fmax(acc[0], -(dhi / dr));
        if (dr < 0.0) acc[0] = fmax(acc[0], -((lo - rh) / dr));
        if (dl < 0.0) acc[1] = fmax(acc[1], -(-nl / dl));
        if (dh < 0.0) acc[2] = fmax(acc[2], -(-nh / dh));
    }
    block_sum_store<3>(acc, a.partials, SL_SUM_R1, 0x7u);
}

void launch_ip_dir(Ctx& c, double r, double s) {
    IpDirArgs a{c.nx, c.ny, c.nz, c.ndof, r, s, c.be, c.dy, c.w, c.g3, c.g4, c.rho, c.nlo,
                c.nhi, c.rlo, c.rhi, c.fixed, c.c1, c.dnl, c.dnh, c.partials};
    const int g = red_grid(c.m);
    hipLaunchKernelGGL(k_ip_dir, dim3(g), dim3(kThreads), 0, c.s, a);
    hipLaunchKernelGGL(k_finalize, dim3(3), dim3(kThreads), 0, c.s, c.partials, g,
                       (int)SL_SUM_R1, 0x7u, c.red);
}

__global__ void k_ip_update(int64_t ndof, int64_t m, double ku, double kl, double kh,
                            double* __restrict__ u, const double* __restrict__ dy,
                            double* __restrict__ rho, const double* __restrict__ drho,
                            double* __restrict__ nlo, const double* __restrict__ dnl,
                            double* __restrict__ nhi, const double* __restrict__ dnh) {
    const int64_t t = gid();
    if (t < ndof) u[t] += ku * dy[t];
    if (t < m) {
        rho[t] += ku * drho[t];
        nlo[t] += kl * dnl[t];
        nhi[t] += kh * dnh[t];
    }
}

void launch_ip_update(Ctx& c, double ku, double kl, double kh) {
    const int64_t n = c.ndof > c.m ? c.ndof : c.m;
    hipLaunchKernelGGL(k_ip_update, dim3(grid1d(n)), dim3(kThreads), 0, c.s, c.ndof, c.m, ku, kl,
                       kh, c.u, c.dy, c.rho, c.c1, c.nlo, c.dnl, c.nhi, c.dnh);
}

// w = (v - eps_old w1 - delta w2) / gamma ; x += phi w
struct MinresWArgs {
    double* w;
    const double* v;
    const double* w1;
    const double* w2;
    double eps_old, delta, inv_gamma;
    double* x;
    double phi;
    int64_t n;
};
__device__ __forceinline__ void minres_w_body(const MinresWArgs& a) {
    const int64_t t = gid();
    if (t >= a.n) return;
    const double wn = (a.v[t] - a.eps_old * a.w1[t] - a.delta * a.w2[t]) * a.inv_gamma;
    a.w[t] = wn;
    a.x[t] += a.phi * wn;
}
VTS_KERNEL_PAIR(, kThreads, k_minres_w, MinresWArgs, minres_w_body)
void launch_minres_w(Ctx& c, double* w, const double* v, const double* w1, const double* w2,
                     double eps_old, double delta, double inv_gamma, double* x, double phi,
                     int64_t n) {
    vlaunch(c, (const void*)&k_minres_w, (const void*)&k_minres_w_b, dim3(grid1d(n)),
            dim3(kThreads), MinresWArgs{w, v, w1, w2, eps_old, delta, inv_gamma, x, phi, n});
}

}  // namespace vts
