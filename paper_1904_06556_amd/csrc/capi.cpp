// C ABI of libvts: problem validation, device allocation, and the host-side
// control flow of Algorithm 1 (PBM), Algorithm 2 (PBM NEWTON) and MINRES.
// Every per-element and per-DOF step runs in the kernels of kernels.hip and
// mg.hip; the host only reads the scalars that decide the next branch.
#include <hip/hip_runtime.h>

#include <cstdarg>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vts_internal.hpp"

using namespace vts;

namespace {

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            c.err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            return VTS_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

struct Dims {
    int nx, ny, nz;
};

int64_t nodes_of(const Dims& d) { return (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1); }

// sizes of every device allocation of a problem (bytes), in allocation order
struct Plan {
    std::vector<size_t> bytes;
    size_t total() const {
        size_t s = 0;
        for (size_t b : bytes) s += (b + 255) / 256 * 256;
        return s;
    }
};

vts_status validate(const vts_problem* pr, std::string& err) {
    if (!pr) { err = "null problem"; return VTS_EINVAL; }
    if (pr->nx < 1 || pr->ny < 1 || pr->nz < 1 || pr->levels < 1 || pr->levels > 12) {
        err = "grid dimensions and levels must be positive";
        return VTS_EINVAL;
    }
    const int s = 1 << (pr->levels - 1);
    if (pr->nx % s || pr->ny % s || pr->nz % s) {
        err = "nx, ny, nz must be divisible by 2^(levels-1)";
        return VTS_EINVAL;
    }
    if (!pr->fixed_host || !pr->f_host) { err = "fixed and f are required"; return VTS_EINVAL; }
    if (!(pr->E > 0) || !(pr->nu > -1.0 && pr->nu < 0.5) || !(pr->h > 0)) {
        err = "material constants out of range";
        return VTS_EINVAL;
    }
    if (pr->precision != VTS_FP64 && pr->precision != VTS_MIXED) {
        err = "unknown precision";
        return VTS_EINVAL;
    }
    if (pr->nload < 0 || pr->nload > kMaxLoads) {
        err = "nload must be 0..4";
        return VTS_EINVAL;
    }
    if (pr->nload > 1 && pr->precision != VTS_FP64) {
        err = "several load cases need precision VTS_FP64";
        return VTS_EINVAL;
    }
    return VTS_OK;
}

int load_cases(const vts_problem* pr) { return pr->nload > 1 ? pr->nload : 1; }

template <typename T>
void fill_level_geom(Level<T>& L, const Dims& d) {
    L.nx = d.nx; L.ny = d.ny; L.nz = d.nz;
    L.NX = d.nx + 1; L.NY = d.ny + 1; L.NZ = d.nz + 1;
    L.nn = nodes_of(d);
    L.m = (int64_t)d.nx * d.ny * d.nz;
    L.coff[0] = 0;
    for (int col = 0; col < 8; ++col) {
        const int px = col & 1, py = (col >> 1) & 1, pz = col >> 2;
        L.cnx[col] = (L.NX - px + 1) / 2;
        L.cny[col] = (L.NY - py + 1) / 2;
        L.cnz[col] = (L.NZ - pz + 1) / 2;
        L.coff[col + 1] = L.coff[col] + (int64_t)L.cnx[col] * L.cny[col] * L.cnz[col];
    }
}

// coarse mask by injection: coarse DOF fixed iff the coincident fine DOF is
std::vector<uint8_t> coarsen_mask(const std::vector<uint8_t>& fm, const Dims& f) {
    const Dims c{f.nx / 2, f.ny / 2, f.nz / 2};
    std::vector<uint8_t> cm(3 * nodes_of(c));
    const int64_t FX = f.nx + 1, FY = f.ny + 1, CX = c.nx + 1, CY = c.ny + 1;
    for (int K = 0; K <= c.nz; ++K)
        for (int J = 0; J <= c.ny; ++J)
            for (int I = 0; I <= c.nx; ++I) {
                const int64_t N = I + CX * (J + CY * K);
                const int64_t n = 2 * I + FX * (2 * J + FY * 2 * K);
                for (int q = 0; q < 3; ++q) cm[3 * N + q] = fm[3 * n + q];
            }
    return cm;
}

// every fixed fine DOF must interpolate from fixed coarse DOFs only
bool nested(const std::vector<uint8_t>& fm, const Dims& f, const std::vector<uint8_t>& cm) {
    const int64_t FX = f.nx + 1, FY = f.ny + 1, CX = f.nx / 2 + 1, CY = f.ny / 2 + 1;
    for (int k = 0; k <= f.nz; ++k)
        for (int j = 0; j <= f.ny; ++j)
            for (int i = 0; i <= f.nx; ++i) {
                const int64_t n = i + FX * (j + FY * k);
                for (int q = 0; q < 3; ++q) {
                    if (!fm[3 * n + q]) continue;
                    const int is[2] = {i >> 1, (i + 1) >> 1}, js[2] = {j >> 1, (j + 1) >> 1},
                              ks[2] = {k >> 1, (k + 1) >> 1};
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int cc = 0; cc < 2; ++cc) {
                                const int64_t N = is[a] + CX * (js[b] + CY * ks[cc]);
                                if (!cm[3 * N + q]) return false;
                            }
                }
            }
    return true;
}

// the finest level keeps no stencil when it is too large for the one-workgroup
// V-cycle (its Gauss-Seidel rows are formed from the element data instead)
bool fine_matrix_free(int levels, int64_t fine_nodes) {
    return levels >= 2 && fine_nodes > kSmallNodes;
}

Plan make_plan(const vts_problem* pr) {
    Plan p;
    const Dims d{pr->nx, pr->ny, pr->nz};
    const int64_t nn = nodes_of(d), ndof = 3 * nn, m = (int64_t)d.nx * d.ny * d.nz;
    auto add = [&](size_t b) { p.bytes.push_back(b); };
    add(576 * 8); add(576 * 4); add(8 * 576 * 8); add(512 * 8);     // Ke, Kef, Mc, Qc
    add(ndof); add(nn); add(ndof * 8);                               // fixed, nmask, f
    add(m * 8); add(m * 8);                                          // bounds
    add(ndof * 8);                                                   // u
    for (int q = 0; q < 8; ++q) add(m * 8);                          // nlo..qhi
    add(m * 4);                                                      // rhof
    add(m * 8); add(24 * m * 8);                                     // e, be
    for (int q = 0; q < 8; ++q) add(m * 8);                          // r1 r2 l2 h2 g3 g4 w zc
    add(24 * m * 8);                                                 // gch
    add(ndof * 8); add((ndof + 1) * 8); add((ndof + 1) * 8);         // g1 rhs dy
    for (int q = 0; q < 5; ++q) add(m * 8);                          // dnl dnh c1 c2 wt
    for (int q = 0; q < 8; ++q) add((ndof + 1) * 8);                 // MINRES
    add(kRedSlots * kRedBlocks * 8); add(kRedSlots * 8);             // partials, red
    {
        Ctx t;                                                       // tiled S partials
        t.nx = d.nx; t.ny = d.ny; t.nz = d.nz;
        add(8 * (size_t)apply_S_tile_blocks(t));
    }
    const size_t ts = pr->precision == VTS_MIXED ? 4 : 8;
    Dims dl = d;
    for (int k = pr->levels - 1; k >= 0; --k) {
        const int64_t lnn = nodes_of(dl), lm = (int64_t)dl.nx * dl.ny * dl.nz;
        add(3 * lnn);                                                // fixed
        if (k == pr->levels - 1 && fine_matrix_free(pr->levels, lnn)) {
            add(24 * lnn * ts); add(lm * ts);                        // bc, te
            if (ts == 4) { add(lm * 4); add(lm * 4); add(3 * lnn * 4); }   // r1f, wf, uf
        } else {
            add(kStencilVals * lnn * ts);                            // stencil
        }
        add(9 * lnn * ts); add(3 * lnn * ts);                        // dinv, acol
        if (k < pr->levels - 1) {
            add(576 * lm * ts);                                      // E
            if (k > 0) add(576 * lm * ts);                           // TQ (levels with a parent)
        }
        for (int q = 0; q < 3; ++q) add((3 * lnn + 1) * ts);         // r z res
        if (k == 0) {
            // dense coarsest system and its inverse, DOF maps, flag (bounded
            // by an all-free coarsest level)
            const size_t nc = (size_t)(3 * lnn + 1);
            add(nc * nc * 8); add(nc * nc * 8);
            add(3 * lnn * 4); add(nc * 4); add(4);
        }
        dl = Dims{dl.nx / 2, dl.ny / 2, dl.nz / 2};
    }
    return p;
}

// device buffer of `count` elements: from the context's arena if it has one
// (256-byte granules, no hipMalloc), else hipMalloc
template <typename T>
vts_status alloc_t(Ctx& c, T** ptr, int64_t count) {
    const size_t b = ((size_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    void* q = nullptr;
    if (c.arena) {
        if (c.arena_used + b > c.arena_size) {
            c.err = "device arena exhausted (" + std::to_string(c.arena_used + b) + " > " +
                    std::to_string(c.arena_size) + " bytes)";
            return VTS_ENOMEM;
        }
        q = c.arena + c.arena_used;
        c.arena_used += b;
    } else {
        if (hipMalloc(&q, b) != hipSuccess) {
            c.err = "hipMalloc failed (" + std::to_string(b) + " bytes)";
            return VTS_ENOMEM;
        }
        c.allocs.push_back(q);
    }
    c.alloc_bytes += b;
    *ptr = (T*)q;
    return VTS_OK;
}

#define ALLOC(ptr, count)                                  \
    do {                                                   \
        vts_status s_ = alloc_t(c, &(ptr), (count));       \
        if (s_ != VTS_OK) return s_;                       \
    } while (0)

template <typename T>
vts_status build_hierarchy(Ctx& c, Hierarchy<T>& H, const std::vector<uint8_t>& fine_mask) {
    const int L = c.L;
    H.lev.resize(L);
    std::vector<std::vector<uint8_t>> masks(L);
    std::vector<Dims> dims(L);
    masks[L - 1] = fine_mask;
    dims[L - 1] = Dims{c.nx, c.ny, c.nz};
    for (int k = L - 2; k >= 0; --k) {
        dims[k] = Dims{dims[k + 1].nx / 2, dims[k + 1].ny / 2, dims[k + 1].nz / 2};
        masks[k] = coarsen_mask(masks[k + 1], dims[k + 1]);
        if (!nested(masks[k + 1], dims[k + 1], masks[k])) {
            c.err = "fixed DOFs are not nested across multigrid levels";
            return VTS_EINVAL;
        }
    }
    for (int k = 0; k < L; ++k) {
        Level<T>& Lk = H.lev[k];
        std::memset(&Lk, 0, sizeof(Lk));
        fill_level_geom(Lk, dims[k]);
        ALLOC(Lk.fixed, 3 * Lk.nn);
        HIPCHK(hipMemcpyAsync(Lk.fixed, masks[k].data(), 3 * Lk.nn, hipMemcpyHostToDevice, c.s));
        if (k == L - 1 && fine_matrix_free(L, Lk.nn)) {
            H.mf = true;
            ALLOC(H.bc, 24 * Lk.nn);
            ALLOC(H.te, Lk.m);
            if (sizeof(T) == 4) {
                ALLOC(H.r1f, Lk.m);
                ALLOC(H.wf, Lk.m);
                ALLOC(H.uf, 3 * Lk.nn);
            } else {
                // FP64 levels read the context's own vectors
                H.r1f = (T*)c.r1;
                H.wf = (T*)c.w;
                H.uf = (T*)c.u;
            }
        } else {
            ALLOC(Lk.st, (int64_t)kStencilVals * Lk.nn);
        }
        ALLOC(Lk.dinv, 9 * Lk.nn);
        ALLOC(Lk.acol, 3 * Lk.nn);
        if (k < L - 1) {
            ALLOC(Lk.E, 576 * Lk.m);
            if (k > 0) ALLOC(Lk.TQ, 576 * Lk.m);
        }
        ALLOC(Lk.r, 3 * Lk.nn + 1);
        ALLOC(Lk.z, 3 * Lk.nn + 1);
        ALLOC(Lk.res, 3 * Lk.nn + 1);
    }
    // the scratch TQ of level k is written from level k's E (k >= 1); level L-1 has none
    std::vector<int> cmap(3 * H.lev[0].nn, -1);
    int nc = 0;
    for (size_t q = 0; q < cmap.size(); ++q)
        if (!masks[0][q]) cmap[q] = nc++;
    nc += 1;  // alpha
    if (nc > kMaxCoarse) {
        c.err = "coarsest level too large for the dense solver (" + std::to_string(nc) + ")";
        return VTS_EINVAL;
    }
    if (nc < 2) {
        c.err = "coarsest level has no free DOF";
        return VTS_EINVAL;
    }
    H.nc = nc;
    ALLOC(H.A, (int64_t)nc * nc);
    ALLOC(H.cmap, (int64_t)cmap.size());
    HIPCHK(hipMemcpyAsync(H.cmap, cmap.data(), cmap.size() * sizeof(int), hipMemcpyHostToDevice,
                          c.s));
    std::vector<int> cinv(nc - 1);
    for (size_t q = 0; q < cmap.size(); ++q)
        if (cmap[q] >= 0) cinv[cmap[q]] = (int)q;
    ALLOC(H.cinv, nc - 1);
    HIPCHK(hipMemcpyAsync(H.cinv, cinv.data(), (nc - 1) * sizeof(int), hipMemcpyHostToDevice,
                          c.s));
    ALLOC(H.flag, 1);
    // levels small enough for the one-workgroup V-cycle (needs the inverse)
    H.ksmall = -1;
    if (nc <= kSmallCoarse) {
        for (int k = 0; k < L && k < kMaxSmallLevels; ++k) {
            if (H.lev[k].nn > kSmallNodes) break;
            H.ksmall = k;
        }
    }
    if (H.ksmall >= 0) ALLOC(H.Ainv, (int64_t)nc * nc);
    // the host masks and maps above go out of scope: finish their copies
    HIPCHK(hipStreamSynchronize(c.s));
    return VTS_OK;
}

vts_status sync_red(Ctx& c) {
    HIPCHK(hipMemcpyAsync(c.red_host, c.red, kRedSlots * sizeof(double), hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    return VTS_OK;
}

// evaluation at the current state: energies, coefficients, gradient, rhs
vts_status evaluate(Ctx& c) {
    launch_eval(c);
    launch_grad(c);
    vts_status st = sync_red(c);
    if (st != VTS_OK) return st;
    const double* r = c.red_host;
    c.sum_r1 = r[SL_SUM_R1];
    c.sum_z = r[SL_SUM_Z];
    c.sum_w = r[SL_SUM_W];
    c.n_g3 = std::sqrt(r[SL_G3SQ]);
    c.n_g4 = std::sqrt(r[SL_G4SQ]);
    c.n_g1 = std::sqrt(r[SL_G1SQ]);
    c.g2 = c.V - c.sum_r1;
    launch_set(c, c.rhs + c.nvec, -c.g2 - c.sum_z);
    if (!std::isfinite(c.n_g1) || !std::isfinite(c.sum_w) || !std::isfinite(c.n_g3)) {
        c.err = "non-finite value in the gradient";
        return VTS_EINVAL;
    }
    c.eval_valid = true;
    c.setup_valid = false;
    return VTS_OK;
}

double res_pbm(const Ctx& c) {
    return c.n_g1 / c.norm_f + std::fabs(c.g2) / c.V + c.n_g3 / c.norm_bounds;
}
double res4_term(const Ctx& c) { return c.n_g4 / c.norm_bounds; }

// drop the captured V-cycles (the stream must be idle: build_mg has synchronized)
void drop_graphs(Ctx& c) {
    for (auto& g : c.vgraphs) hipGraphExecDestroy(g.exec);
    c.vgraphs.clear();
}

vts_status build_mg(Ctx& c) {
    int flag = 0;
    if (c.mlh) {
        flag = ml_mg_build(c);
    } else if (c.h64) {
        mg_build(c, *c.h64);
        flag = mg_check_factor(c, *c.h64);
    } else {
        mg_build(c, *c.h32);
        flag = mg_check_factor(c, *c.h32);
    }
    // mg_check_factor synchronized the stream: no captured V-cycle is in flight
    drop_graphs(c);
    HIPCHK(hipGetLastError());
    if (flag) {
        c.err = "coarsest multigrid matrix is not positive definite";
        return VTS_ENONSPD;
    }
    c.setup_valid = true;
    return VTS_OK;
}

vts_status setup(Ctx& c) {
    if (!c.eval_valid) {
        vts_status st = evaluate(c);
        if (st != VTS_OK) return st;
    }
    if (!c.setup_valid) return build_mg(c);
    return VTS_OK;
}

void vcycle_launches(Ctx& c, const double* r, double* z) {
    if (c.mlh)
        ml_vcycle(c, r, z);
    else if (c.h64)
        mg_vcycle(c, *c.h64, r, z);
    else
        mg_vcycle(c, *c.h32, r, z);
}

// One V-cycle from a captured graph; false if graphs are unavailable (the
// caller then launches the kernels directly).  The capture records the same
// launches on a private stream; nothing runs during the capture.
bool precond_graph(Ctx& c, const double* r, double* z) {
    for (const auto& g : c.vgraphs)
        if (g.r == r && g.z == z && g.d == c.sum_w) return hipGraphLaunch(g.exec, c.s) == hipSuccess;
    if (!c.cap_stream && hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c.cap_stream = nullptr;
        c.opt.use_graphs = 0;
        return false;
    }
    hipStream_t s0 = c.s;
    c.s = c.cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        vcycle_launches(c, r, z);
        e = hipStreamEndCapture(c.s, &graph);
    }
    c.s = s0;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c.opt.use_graphs = 0;
        return false;
    }
    if (c.vgraphs.size() >= 4) {
        // the oldest entry may still be in flight on s: finish it first
        hipStreamSynchronize(c.s);
        hipGraphExecDestroy(c.vgraphs.front().exec);
        c.vgraphs.erase(c.vgraphs.begin());
    }
    c.vgraphs.push_back({r, z, c.sum_w, exec});
    return hipGraphLaunch(exec, c.s) == hipSuccess;
}

void precond(Ctx& c, const double* r, double* z) {
    // graphs only outside server pools (instantiation may allocate) and
    // while no kernel class is being timed
    if (c.opt.use_graphs && !c.arena && !c.rec && c.prof_class == 0 && precond_graph(c, r, z)) return;
    vcycle_launches(c, r, z);
}

// Preconditioned MINRES (Paige-Saunders), x0 = 0: Lanczos in the M-inner
// product with M^{-1} one V-cycle, Givens QR of the tridiagonal, stop when the
// M^{-1}-norm estimate phi_bar of the residual is <= eps * beta_1.  A
// negative M^{-1}-norm means the V-cycle is not positive definite in floating
// point: VTS_ENONSPD, or with stop_indef the iterate reached so far is kept.
//
// The solve is split into steps between its synchronizations so that a group
// runner can advance several solves together: mr_issue_* queue the device
// work of one step (issued on c.s, or recorded while c.rec is set), the
// reductions land in c.red_host after the stream is synchronized, and
// mr_after_* read them.  minres() runs the steps for one context.
}  // namespace

namespace vts {

void mr_init(Ctx& c, MrState& m, double eps, int maxit, bool stop_indef) {
    m = MrState{};
    m.eps = eps;
    m.maxit = maxit < 0 ? c.opt.max_minres : maxit;
    m.stop_indef = stop_indef;
    m.n = c.nvec + 1;
    m.x = c.mv[0];
    m.r1 = c.mv[1];
    m.r2 = c.mv[2];
    m.y = c.mv[3];
    m.v = c.mv[4];
    m.wb[0] = c.mv[5];
    m.wb[1] = c.mv[6];
    m.wb[2] = c.mv[7];
}

static void mr_red_copy(Ctx& c) {
    (void)vmemcpy(c, c.red_host, c.red, kRedSlots * sizeof(double), hipMemcpyDeviceToHost);
}

void mr_issue_start(Ctx& c, MrState& m) {
    launch_fill(c, m.x, 0.0, m.n);
    (void)vmemcpy(c, m.r1, c.rhs, m.n * sizeof(double), hipMemcpyDeviceToDevice);
    precond(c, m.r1, m.y);
    launch_dot(c, m.r1, m.y, m.n, SL_DOT);
    mr_red_copy(c);
}

void mr_after_start(Ctx& c, MrState& m) {
    const double b1sq = c.red_host[SL_DOT];
    const bool indef0 = m.stop_indef && b1sq < 0;
    if (!indef0 && (!(b1sq >= 0) || !std::isfinite(b1sq))) {
        c.err = "MINRES: preconditioner not positive definite";
        m.st = VTS_ENONSPD;
        m.phase = MrState::kDone;
        return;
    }
    m.rel = indef0 ? 1.0 : 0.0;
    if (!(b1sq > 0) || m.maxit <= 0) {
        m.phase = MrState::kFinish;
        return;
    }
    m.beta1 = std::sqrt(b1sq);
    m.beta = m.beta1;
    m.beta_old = 0.0;
    (void)vmemcpy(c, m.r2, m.r1, m.n * sizeof(double), hipMemcpyDeviceToDevice);
    launch_fill(c, m.wb[0], 0.0, m.n);
    launch_fill(c, m.wb[1], 0.0, m.n);
    launch_fill(c, m.wb[2], 0.0, m.n);
    m.iw = 0;
    m.iw1 = 1;
    m.iw2 = 2;
    m.cs = -1.0;
    m.sn = 0.0;
    m.dbar = 0.0;
    m.eps_l = 0.0;
    m.phibar = m.beta1;
    m.phase = MrState::kIterate;
}

void mr_issue_iter(Ctx& c, MrState& m) {
    ++m.it;
    launch_scale(c, m.v, m.y, 1.0 / m.beta, m.n);
    launch_apply_S(c, m.v, m.y);
    if (m.it >= 2) launch_axpy(c, m.y, -m.beta / m.beta_old, m.r1, m.n);
    // alpha = v . S v stays on the device for the next update; the host
    // reads it with beta^2 after one synchronization
    launch_dot(c, m.v, m.y, m.n, SL_MRALPHA);
    launch_axpy_red(c, m.y, SL_MRALPHA, m.beta, m.r2, m.n);
    std::swap(m.r1, m.r2);
    std::swap(m.r2, m.y);
    precond(c, m.r2, m.y);
    launch_dot(c, m.r2, m.y, m.n, SL_DOT);
    mr_red_copy(c);
}

void mr_after_iter(Ctx& c, MrState& m) {
    const double alpha = c.red_host[SL_MRALPHA];
    const double bsq = c.red_host[SL_DOT];
    if (m.stop_indef && bsq < 0) {
        m.rel = m.phibar / m.beta1;
        m.phase = MrState::kFinish;
        return;
    }
    if (!(bsq >= 0) || !std::isfinite(bsq)) {
        c.err = "MINRES: preconditioner not positive definite";
        m.st = VTS_ENONSPD;
        m.phase = MrState::kDone;
        return;
    }
    m.beta_old = m.beta;
    m.beta = std::sqrt(bsq);
    const double eps_old = m.eps_l;
    const double delta = m.cs * m.dbar + m.sn * alpha;
    const double gbar = m.sn * m.dbar - m.cs * alpha;
    m.eps_l = m.sn * m.beta;
    m.dbar = -m.cs * m.beta;
    double gamma = std::hypot(gbar, m.beta);
    gamma = std::max(gamma, 2.220446049250313e-16);
    m.cs = gbar / gamma;
    m.sn = m.beta / gamma;
    const double phi = m.cs * m.phibar;
    m.phibar = m.sn * m.phibar;
    // w1 <- w2, w2 <- w, w <- (v - eps_old w1 - delta w2)/gamma
    const int old_w1 = m.iw1;
    m.iw1 = m.iw2;
    m.iw2 = m.iw;
    m.iw = old_w1;
    launch_minres_w(c, m.wb[m.iw], m.v, m.wb[m.iw1], m.wb[m.iw2], eps_old, delta, 1.0 / gamma,
                    m.x, phi, m.n);
    m.rel = m.phibar / m.beta1;
    if (m.phibar <= m.eps * m.beta1 || m.it >= m.maxit) m.phase = MrState::kFinish;
}

// the result into c.dy, counters; c.mv keeps the rotated buffers for the next call
void mr_finish(Ctx& c, MrState& m, vts_linstats* out) {
    (void)vmemcpy(c, c.dy, m.x, m.n * sizeof(double), hipMemcpyDeviceToDevice);
    c.mv[1] = m.r1;
    c.mv[2] = m.r2;
    c.mv[3] = m.y;
    c.minres_total += m.it;
    if (out) {
        out->iterations = m.it;
        out->rel_residual = m.rel;
    }
    m.phase = MrState::kDone;
}

}  // namespace vts

namespace {

vts_status minres(Ctx& c, double eps, vts_linstats* out, int maxit = -1,
                  bool stop_indef = false) {
    if (c.group && !stop_indef && c.prof_class == 0 && tile_ok(c))
        return group_minres(c, eps, out, maxit < 0 ? c.opt.max_minres : maxit);
    MrState m;
    mr_init(c, m, eps, maxit, stop_indef);
    mr_issue_start(c, m);
    HIPCHK(hipStreamSynchronize(c.s));
    mr_after_start(c, m);
    while (m.phase == MrState::kIterate) {
        mr_issue_iter(c, m);
        HIPCHK(hipStreamSynchronize(c.s));
        mr_after_iter(c, m);
    }
    if (m.phase == MrState::kFinish) mr_finish(c, m, out);
    HIPCHK(hipGetLastError());
    return m.st;
}

vts_status newton_step(Ctx& c, vts_newtonstats* out, bool final_call) {
    vts_status st = setup(c);
    if (st != VTS_OK) return st;
    vts_linstats ls{0, 0.0};
    double slope = 0.0, dalpha = 0.0;
    for (int tries = 0;; ++tries) {
        if ((st = minres(c, c.eps_mr, &ls)) != VTS_OK) return st;
        launch_dnu(c);
        launch_dot(c, c.g1, c.dy, c.nvec, SL_DOT);
        launch_copy1(c, c.dy + c.nvec, c.red + SL_AUX);
        if ((st = sync_red(c)) != VTS_OK) return st;
        dalpha = c.red_host[SL_AUX];
        slope = c.red_host[SL_DOT] + c.g2 * dalpha + c.red_host[SL_SLOPE_NU];
        if (slope < 0 || tries >= 1) break;
        // a non-descent direction: tighten the MINRES tolerance once
        c.eps_mr = std::max(0.1 * c.eps_mr, c.opt.eps_mr_min);
    }
    if (!(slope < 0)) {
        c.err = "Newton direction is not a descent direction";
        return VTS_ENONDESCENT;
    }
    // f^T du for the linear part of the Lagrangian change
    launch_dot(c, c.f, c.dy, c.nvec, SL_DOT);
    if ((st = sync_red(c)) != VTS_OK) return st;
    const double fdu = c.red_host[SL_DOT];
    double kappa = 1.0;
    for (;;) {
        launch_linesearch(c, kappa, dalpha);
        if ((st = sync_red(c)) != VTS_OK) return st;
        const double dL = kappa * dalpha * c.V - kappa * fdu + c.red_host[SL_LS];
        if (dL <= c.opt.armijo_c1 * kappa * slope) break;
        kappa *= 0.5;
        if (kappa < c.opt.armijo_min) {
            c.err = "Armijo line search stalled";
            return VTS_ENONDESCENT;
        }
    }
    launch_update(c, kappa);
    c.alpha += kappa * dalpha;
    c.eval_valid = false;
    if ((st = evaluate(c)) != VTS_OK) return st;
    const double res = res_pbm(c), r4 = res4_term(c);
    if (c.res_prev >= 0 && res > 0.9 * c.res_prev)
        c.eps_mr = std::max(0.1 * c.eps_mr, c.opt.eps_mr_min);
    c.res_prev = res;
    c.newton_total += 1;
    if (out) {
        out->res_pbm = res;
        out->res4 = r4;
        out->kappa = kappa;
        out->slope = slope;
        out->eps_mr = c.eps_mr;
        out->minres_its = ls.iterations;
    }
    (void)final_call;
    return VTS_OK;
}

// one line of the context's JSON-lines log (no-op without a log path)
void log_line(Ctx& c, const char* fmt, ...) {
    if (c.log_path.empty()) return;
    if (!c.log) {
        c.log = std::fopen(c.log_path.c_str(), "a");
        if (!c.log) {
            c.log_path.clear();   // cannot be opened: no log
            return;
        }
    }
    va_list ap;
    va_start(ap, fmt);
    std::vfprintf(c.log, fmt, ap);
    va_end(ap);
    std::fputc('\n', c.log);
    std::fflush(c.log);
}

vts_status newton(Ctx& c, double eps_nwt, bool final_call, vts_newtonstats* last, int* its) {
    c.res_prev = -1.0;
    vts_newtonstats ns{};
    int k = 0;
    vts_status st = VTS_OK;
    double best = HUGE_VAL;
    int since = 0;
    bool stalled = false;
    for (k = 0; k < c.opt.max_newton; ++k) {
        st = newton_step(c, &ns, final_call);
        if (st != VTS_OK) break;
        log_line(c,
                 "{\"event\": \"newton\", \"outer\": %d, \"final\": %d, \"step\": %d, "
                 "\"res_pbm\": %.17g, \"res4\": %.17g, \"kappa\": %.17g, \"slope\": %.17g, "
                 "\"eps_mr\": %.17g, \"minres\": %d}",
                 c.outer, final_call ? 1 : 0, k, ns.res_pbm, ns.res4, ns.kappa, ns.slope,
                 ns.eps_mr, ns.minres_its);
        const double crit = (final_call && c.opt.final_res4) ? ns.res_pbm + ns.res4 : ns.res_pbm;
        if (crit < eps_nwt) break;
        if (crit < 0.9 * best) {
            best = crit;
            since = 0;
        } else {
            ++since;
        }
        if (c.opt.stall_steps > 0 && since >= c.opt.stall_steps) {
            stalled = true;
            break;
        }
    }
    if (last) *last = ns;
    if (its) *its = k + (st == VTS_OK ? 1 : 0);
    // a call before the last one that stalls is taken as the minimizer (the
    // rounding floor of res_PBM lies above its tolerance); the outer loop's
    // multiplier update and tests go on from there
    if (st == VTS_OK && stalled && !final_call) return VTS_OK;
    if (st == VTS_OK && stalled) {
        c.err = "Newton stalled";
        return VTS_ENOTCONV;
    }
    if (st == VTS_OK && k >= c.opt.max_newton) {
        c.err = "Newton iteration limit";
        return VTS_ENOTCONV;
    }
    return st;
}

vts_status pbm_iterate(Ctx& c, vts_pbmstats* out) {
    const int mr0 = c.minres_total;
    int nits = 0;
    vts_newtonstats ns{};
    vts_status st = newton(c, c.eps_nwt, false, &ns, &nits);
    if (st != VTS_OK) return st;
    launch_outer_eval(c);
    launch_dot(c, c.f, c.u, c.nvec, SL_DOT);
    if ((st = sync_red(c)) != VTS_OK) return st;
    const double* r = c.red_host;
    const double fu = r[SL_DOT];
    const double gap = -0.5 * fu + c.alpha * c.V - r[SL_GAP];
    const double dual = c.alpha * c.V - fu - r[SL_NLO] + r[SL_NHI];
    const double ratio = std::fabs(gap / dual);
    const double stat = r[SL_STAT];
    c.outer += 1;
    const bool gap_ok = ratio < c.opt.eps_pbm;
    bool stat_ok = c.eps_stat <= 0 || stat < c.eps_stat;
    if (gap_ok && !stat_ok && c.opt.stall_steps > 0 && stat < 10.0 * c.eps_stat) {
        // the stationarity term is this library's addition to the gap test;
        // once the gap test holds and the term, within 10x of its target,
        // stops decreasing, the outer loop ends and the final Newton call
        // and the KKT check decide
        if (c.stat_since < 0 || stat < 0.9 * c.stat_best) {
            c.stat_best = stat;
            c.stat_since = 0;
        } else if (++c.stat_since >= c.opt.stall_steps) {
            stat_ok = true;
        }
    }
    const bool stop = gap_ok && stat_ok;
    log_line(c,
             "{\"event\": \"outer\", \"outer\": %d, \"ratio\": %.17g, \"gap\": %.17g, "
             "\"stat\": %.17g, \"eps_nwt\": %.17g, \"sum_rho\": %.17g, \"newton\": %d, "
             "\"minres\": %d, \"stop\": %d}",
             c.outer, ratio, gap, stat, c.eps_nwt, r[SL_SUM_RHO], nits, c.minres_total - mr0,
             stop ? 1 : 0);
    if (out) {
        out->gap = gap;
        out->dual = dual;
        out->ratio = ratio;
        out->stat = c.eps_stat > 0 ? stat : 0.0;
        out->eps_nwt = c.eps_nwt;
        out->sum_rho = r[SL_SUM_RHO];
        out->newton_its = nits;
        out->minres_its = c.minres_total - mr0;
        out->converged = stop ? 1 : 0;
    }
    if (stop) {
        c.converged = true;
        return VTS_OK;
    }
    launch_mult_update(c, 0);
    launch_penalty_update(c);
    c.eps_nwt = std::max(std::min(100.0 * ratio, c.eps_nwt), c.opt.eps_nwt_min);
    c.eval_valid = false;
    c.setup_valid = false;
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

// The state equation K(rho) u = f for the context's rho: MINRES with one
// V-cycle of blockdiag(K(rho), 1) (the Schur operator with rho' = rho, no
// rank-one terms, alpha decoupled), u <- solution.  Used after the last rho
// update of Algorithm 1 so that (rho, u) satisfy the equilibrium condition
// to the solver's accuracy; the Newton iterate u is only near it.
vts_status state_solve(Ctx& c, double eps) {
    c.eval_valid = false;
    c.setup_valid = false;
    launch_doc_setup(c);
    c.sum_w = 1.0;
    vts_status st = build_mg(c);
    if (st != VTS_OK) return st;
    vts_linstats ls{0, 0.0};
    if ((st = minres(c, eps, &ls)) != VTS_OK) return st;
    HIPCHK(hipMemcpyAsync(c.u, c.dy, c.nvec * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    c.eval_valid = false;
    c.setup_valid = false;
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

// ---------------------------------------------------------------------------
// primal-dual interior point method (Section 4, Algorithm 3)
// ---------------------------------------------------------------------------
// evaluation at the current point with the current barrier parameters: the
// reduced system's weights and right-hand side (alpha row negated, see
// kernels.hip), the gap and feasibility sums, the complementarity measures
vts_status ip_evaluate(Ctx& c) {
    launch_ip_eval(c, c.ip.r, c.ip.s);
    launch_grad(c);                           // res_1 = K(rho) u - f, rhs_u, ||res_1||^2
    launch_dot(c, c.f, c.u, c.ndof, SL_SUM_R1);
    vts_status st = sync_red(c);
    if (st != VTS_OK) return st;
    const double* q = c.red_host + kIpEvalSlot;
    c.ip.sum_rho = q[0];
    c.sum_z = q[1];
    c.sum_w = q[2];
    c.ip.n_res3 = std::sqrt(q[3]);
    c.ip.gap_sum = q[4];
    c.ip.cl = q[5];
    c.ip.ch = q[6];
    c.ip.n_nl = std::sqrt(q[7]);
    c.ip.n_nh = std::sqrt(q[8]);
    c.ip.dmax = q[9];
    c.ip.viol = q[10];
    c.n_g1 = std::sqrt(c.red_host[SL_G1SQ]);
    c.ip.fu = c.red_host[SL_SUM_R1];
    c.g2 = c.V - c.ip.sum_rho;
    launch_set(c, c.rhs + c.ndof, -c.g2 - c.sum_z);
    // the PBM evaluation buffers now hold the IP system
    c.eval_valid = false;
    c.setup_valid = false;
    if (!(c.ip.viol < 0)) {
        c.err = "interior point iterate reached a bound";
        return VTS_ENOTCONV;
    }
    if (!std::isfinite(c.n_g1) || !std::isfinite(c.sum_w) || !std::isfinite(c.ip.n_res3)) {
        c.err = "non-finite value in the interior point residual";
        return VTS_EINVAL;
    }
    return VTS_OK;
}

vts_status ip_init(Ctx& c, const vts_ip_options* opt) {
    vts_ip_options o;
    vts_ip_default_options(&o);
    if (opt) o = *opt;
    if (!(o.eps_ip > 0) || !(o.sigma_r > 0 && o.sigma_r < 1) || !(o.sigma_s > 0 && o.sigma_s < 1) ||
        !(o.r0 > 0) || !(o.s0 > 0) || !(o.step_frac > 0 && o.step_frac < 1) || !(o.eps_mr0 > 0) ||
        !(o.eps_mr_min > 0) || o.max_iter < 1 || o.max_minres < 1) {
        c.err = "invalid interior point options";
        return VTS_EINVAL;
    }
    c.ip = Ctx::Ip{};
    c.ip.o = o;
    launch_init_state(c);
    launch_round_rho(c);
    c.alpha = 1.0;
    c.ip.r = o.r0;
    c.ip.s = o.s0;
    c.ip.eps_mr = o.eps_mr0;
    c.converged = false;
    vts_status st = ip_evaluate(c);
    if (st != VTS_OK) return st;
    // the first shifted update, from the initial point
    c.ip.r_plus = o.sigma_r * c.ip.cl / (double)c.m;
    c.ip.s_plus = o.sigma_s * c.ip.ch / (double)c.m;
    c.ip.ready = true;
    return VTS_OK;
}

vts_status ip_step(Ctx& c, vts_ipstats* out) {
    if (!c.ip.ready) {
        c.err = "vts_ip_step before vts_ip_init";
        return VTS_ESTATE;
    }
    const vts_ip_options& o = c.ip.o;
    // the system at the current point (the same values as the evaluation
    // that ended the previous iteration; repeated because other calls on the
    // context may have used the evaluation buffers since)
    vts_status st = ip_evaluate(c);
    if (st != VTS_OK) return st;
    if ((st = build_mg(c)) != VTS_OK) return st;
    vts_linstats ls{0, 0.0};
    const double eps_mr = c.ip.eps_mr;
    if ((st = minres(c, eps_mr, &ls, o.max_minres, true)) != VTS_OK) return st;
    const double r_used = c.ip.r, s_used = c.ip.s;
    launch_ip_dir(c, r_used, s_used);
    launch_copy1(c, c.dy + c.ndof, c.red + SL_AUX);
    if ((st = sync_red(c)) != VTS_OK) return st;
    const double dalpha = -c.red_host[SL_AUX];
    // step lengths: maxima of -(step to the boundary), -DBL_MAX where no
    // component moves towards a bound
    const double k_u = std::min(o.step_frac * -c.red_host[SL_SUM_R1], 1.0);
    const double k_l = std::min(o.step_frac * -c.red_host[SL_SUM_R1 + 1], 1.0);
    const double k_h = std::min(o.step_frac * -c.red_host[SL_SUM_R1 + 2], 1.0);
    // the barrier shift: this iteration's update values become current
    c.ip.r = c.ip.r_plus;
    c.ip.s = c.ip.s_plus;
    launch_ip_update(c, k_u, k_l, k_h);
    c.alpha += dalpha;
    HIPCHK(hipGetLastError());
    st = ip_evaluate(c);
    c.newton_total += 1;
    if (out) {
        *out = vts_ipstats{};
        out->r = r_used;
        out->s = s_used;
        out->kappa_u = k_u;
        out->kappa_nu_lo = k_l;
        out->kappa_nu_hi = k_h;
        out->eps_mr = eps_mr;
        out->minres_its = ls.iterations;
        out->alpha = c.alpha;
        out->iterations = 1;
    }
    if (st != VTS_OK) return st;
    const double m = (double)c.m;
    const double obj = 0.5 * c.ip.fu;
    const double gap = -0.5 * c.ip.fu + (-c.alpha) * c.V - c.ip.gap_sum;
    const double res_ip = c.n_g1 / c.norm_f + std::fabs(c.ip.sum_rho - c.V) / c.V +
                          c.ip.n_res3 / (c.ip.n_nl + c.ip.n_nh) +
                          std::fabs(c.ip.cl - m * c.ip.r) / m + std::fabs(c.ip.ch - m * c.ip.s) / m;
    const double ratio = obj != 0.0 ? gap / obj : HUGE_VAL;
    const bool conv = (o.eps_ip > ratio && ratio > -0.1 * o.eps_ip) && res_ip < 10.0 * o.eps_ip;
    c.converged = conv;
    // shifted barrier update values and the MINRES tolerance rule
    c.ip.r_plus = o.sigma_r * c.ip.cl / m;
    c.ip.s_plus = o.sigma_s * c.ip.ch / m;
    const double cand = std::max(100.0 * c.ip.dmax, o.eps_mr_min);
    if (cand < c.ip.eps_mr) c.ip.eps_mr = cand;
    if (out) {
        out->gap_ratio = ratio;
        out->res_ip = res_ip;
        out->compliance = obj;
        out->converged = conv ? 1 : 0;
    }
    return VTS_OK;
}

// host-side checks of the data (assumptions after problem (1.1)) and the
// cleaned host arrays: the DOF mask as 0/1, loads zeroed at fixed DOFs, the
// bounds expanded to m entries; nested supports and the coarsest size
struct HostData {
    std::vector<uint8_t> mask;
    std::vector<double> f, lo, hi;
    int64_t nfree = 0;
    double norm_f = 0.0, norm_bounds = 0.0, lo_min = 0.0;
};

vts_status prepare_host(const vts_problem* pr, HostData& hd, std::string& err) {
    const Dims d0{pr->nx, pr->ny, pr->nz};
    const int64_t ndof = 3 * nodes_of(d0), m = (int64_t)pr->nx * pr->ny * pr->nz;
    const int nl = load_cases(pr);
    hd.mask.assign(pr->fixed_host, pr->fixed_host + ndof);
    hd.f.assign(pr->f_host, pr->f_host + nl * ndof);
    int64_t nfixed = 0;
    double nf2 = 0.0;
    for (int64_t q = 0; q < ndof; ++q) {
        hd.mask[q] = hd.mask[q] ? 1 : 0;
        nfixed += hd.mask[q];
    }
    for (int l = 0; l < nl; ++l)
        for (int64_t q = 0; q < ndof; ++q) {
            double& fq = hd.f[l * ndof + q];
            if (hd.mask[q]) fq = 0.0;
            if (!std::isfinite(fq)) { err = "load vector is not finite"; return VTS_EINVAL; }
            nf2 += fq * fq;
        }
    if (nfixed == 0) { err = "no fixed DOF: K(rho) is singular"; return VTS_EINVAL; }
    if (nf2 == 0.0) { err = "zero load"; return VTS_EINVAL; }
    hd.nfree = ndof - nfixed;
    hd.norm_f = std::sqrt(nf2);
    hd.lo.resize(m);
    hd.hi.resize(m);
    double slo = 0, shi = 0, nlo2 = 0, nhi2 = 0;
    for (int64_t e = 0; e < m; ++e) {
        const double lo = pr->rho_lo_host ? pr->rho_lo_host[e] : pr->rho_lo_s;
        const double hi = pr->rho_hi_host ? pr->rho_hi_host[e] : pr->rho_hi_s;
        if (!(hi > lo) || lo < 0) { err = "need 0 <= rho_lo < rho_hi"; return VTS_EINVAL; }
        hd.lo[e] = lo;
        hd.hi[e] = hi;
        slo += lo; shi += hi; nlo2 += lo * lo; nhi2 += hi * hi;
    }
    if (!(slo < pr->V && pr->V < shi)) { err = "volume not strictly feasible"; return VTS_EINVAL; }
    hd.norm_bounds = std::sqrt(nlo2) + std::sqrt(nhi2);
    hd.lo_min = *std::min_element(hd.lo.begin(), hd.lo.end());
    std::vector<uint8_t> mk = hd.mask;
    Dims dk = d0;
    for (int k = pr->levels - 1; k > 0; --k) {
        std::vector<uint8_t> mc = coarsen_mask(mk, dk);
        if (!nested(mk, dk, mc)) {
            err = "fixed DOFs are not nested across multigrid levels";
            return VTS_EINVAL;
        }
        mk.swap(mc);
        dk = Dims{dk.nx / 2, dk.ny / 2, dk.nz / 2};
    }
    int64_t nc = 1;
    for (uint8_t v : mk) nc += v ? 0 : nl;
    if (nc > (nl > 1 ? kMlMaxCoarse : kMaxCoarse)) {
        err = "coarsest level too large for the dense solver (" + std::to_string(nc) + ")";
        return VTS_EINVAL;
    }
    return VTS_OK;
}

vts_status ctx_create(Ctx& c, const vts_problem* pr, const vts_options* opt, void* stream) {
    c.nx = pr->nx; c.ny = pr->ny; c.nz = pr->nz; c.L = pr->levels;
    c.nn = nodes_of(Dims{c.nx, c.ny, c.nz});
    c.ndof = 3 * c.nn;
    c.m = (int64_t)c.nx * c.ny * c.nz;
    c.E = pr->E; c.nu = pr->nu; c.h = pr->h; c.V = pr->V;
    c.prec = pr->precision;
    c.nl = load_cases(pr);
    c.nvec = c.nl * c.ndof;
    if (opt) c.opt = *opt; else vts_default_options(&c.opt);
    if (c.nl > 1) c.opt.use_graphs = 0;
    // the log path is the caller's string: keep a copy, not the pointer
    c.log_path = c.opt.log_path ? c.opt.log_path : "";
    c.opt.log_path = nullptr;
    c.s = (hipStream_t)stream;

    HostData hd;
    {
        vts_status st0 = prepare_host(pr, hd, c.err);
        if (st0 != VTS_OK) return st0;
    }
    std::vector<uint8_t>& mask = hd.mask;
    std::vector<double>& f = hd.f;
    std::vector<double>& lo = hd.lo;
    std::vector<double>& hi = hd.hi;
    c.nfree = hd.nfree;
    c.norm_f = hd.norm_f;
    c.norm_bounds = hd.norm_bounds;
    c.lo_min = hd.lo_min;
    HIPCHK(hipGetDevice(&c.device));

    // constants
    double Ke[576], Q[512], Mc[8 * 576];
    float Kef[576];
    element_stiffness(c.E, c.nu, c.h, Ke);
    std::memcpy(c.ke_host, Ke, sizeof(Ke));
    child_interp(Q);
    galerkin_child_matrices(Ke, Q, Mc);
    for (int q = 0; q < 576; ++q) Kef[q] = (float)Ke[q];
    c.kh_ok = walsh_form(Ke, c.kh8) && c.ndof < (int64_t(1) << 31);
    ALLOC(c.Ke, 576); ALLOC(c.Kef, 576); ALLOC(c.Mc, 8 * 576); ALLOC(c.Qc, 512);
    HIPCHK(hipMemcpyAsync(c.Ke, Ke, sizeof(Ke), hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.Kef, Kef, sizeof(Kef), hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.Mc, Mc, sizeof(Mc), hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.Qc, Q, sizeof(Q), hipMemcpyHostToDevice, c.s));

    ALLOC(c.fixed, c.ndof); ALLOC(c.nmask, c.nn); ALLOC(c.f, c.nvec); ALLOC(c.rlo, c.m);
    ALLOC(c.rhi, c.m);
    HIPCHK(hipMemcpyAsync(c.fixed, mask.data(), c.ndof, hipMemcpyHostToDevice, c.s));
    std::vector<uint8_t> nmask(c.nn);
    for (int64_t q = 0; q < c.nn; ++q)
        nmask[q] = (uint8_t)(mask[3 * q] | (mask[3 * q + 1] << 1) | (mask[3 * q + 2] << 2));
    HIPCHK(hipMemcpyAsync(c.nmask, nmask.data(), c.nn, hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.f, f.data(), c.nvec * 8, hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.rlo, lo.data(), c.m * 8, hipMemcpyHostToDevice, c.s));
    HIPCHK(hipMemcpyAsync(c.rhi, hi.data(), c.m * 8, hipMemcpyHostToDevice, c.s));
    ALLOC(c.u, c.nvec);
    ALLOC(c.nlo, c.m); ALLOC(c.nhi, c.m); ALLOC(c.rho, c.m); ALLOC(c.mlo, c.m);
    ALLOC(c.mhi, c.m); ALLOC(c.p, c.m); ALLOC(c.qlo, c.m); ALLOC(c.qhi, c.m);
    ALLOC(c.rhof, c.m);
    ALLOC(c.e, c.m); ALLOC(c.be, 24 * c.m * c.nl);
    ALLOC(c.r1, c.m); ALLOC(c.r2, c.m); ALLOC(c.l2, c.m); ALLOC(c.h2, c.m);
    ALLOC(c.g3, c.m); ALLOC(c.g4, c.m); ALLOC(c.w, c.m); ALLOC(c.zc, c.m);
    ALLOC(c.gch, 24 * c.m);
    ALLOC(c.g1, c.nvec); ALLOC(c.rhs, c.nvec + 1); ALLOC(c.dy, c.nvec + 1);
    ALLOC(c.dnl, c.m); ALLOC(c.dnh, c.m); ALLOC(c.c1, c.m); ALLOC(c.c2, c.m); ALLOC(c.wt, c.m);
    for (int q = 0; q < 8; ++q) ALLOC(c.mv[q], c.nvec + 1);
    ALLOC(c.partials, kRedSlots * kRedBlocks);
    ALLOC(c.spart, apply_S_tile_blocks(c));
    ALLOC(c.red, kRedSlots);
    {
        void* hp = nullptr;
        HIPCHK(hipHostMalloc(&hp, kRedSlots * sizeof(double), hipHostMallocDefault));
        c.red_host = (double*)hp;
        std::memset(c.red_host, 0, kRedSlots * sizeof(double));
    }
    vts_status st;
    if (c.nl > 1) {
        st = ml_create(c, mask);
    } else if (c.prec == VTS_FP64) {
        c.h64 = new Hierarchy<double>();
        st = build_hierarchy(c, *c.h64, mask);
    } else {
        c.h32 = new Hierarchy<float>();
        st = build_hierarchy(c, *c.h32, mask);
    }
    if (st != VTS_OK) return st;

    launch_init_state(c);
    launch_round_rho(c);
    c.alpha = 1.0;
    c.eps_nwt = c.opt.eps_nwt0;
    c.eps_mr = c.opt.eps_mr0 > 0 ? c.opt.eps_mr0 : 1e-4 * std::sqrt((double)c.nl * c.nfree);
    c.eps_stat = c.opt.eps_stat;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.s));
    return VTS_OK;
}

void ctx_free(Ctx& c) {
    if (c.log) fclose(c.log);
    c.log = nullptr;
    if (c.s) hipStreamSynchronize(c.s);
    else hipDeviceSynchronize();
    drop_graphs(c);
    if (c.cap_stream) hipStreamDestroy(c.cap_stream);
    c.cap_stream = nullptr;
    for (hipEvent_t e : c.prof_ev) hipEventDestroy(e);
    c.prof_ev.clear();
    for (void* p : c.allocs) hipFree(p);
    c.allocs.clear();
    if (c.red_host) hipHostFree(c.red_host);
    c.red_host = nullptr;
    delete c.h64;
    delete c.h32;
    c.h64 = nullptr;
    c.h32 = nullptr;
    ml_destroy(c);
}

thread_local std::string g_create_err;

}  // namespace

namespace vts {

// EINVAL for calls that one load case only supports
bool several_loads(Ctx& c, const char* what) {
    if (c.nl <= 1) return false;
    c.err = std::string(what) + " supports one load case only";
    return true;
}

vts_status ml_alloc(Ctx& c, void** ptr, size_t bytes) {
    uint8_t* q = nullptr;
    const vts_status st = alloc_t(c, &q, (int64_t)bytes);
    *ptr = q;
    return st;
}

std::vector<uint8_t> ml_coarsen(const std::vector<uint8_t>& fine_mask, int nx, int ny, int nz) {
    return coarsen_mask(fine_mask, Dims{nx, ny, nz});
}

bool prof_begin(Ctx& c, int cls) {
    if (c.prof_class != cls) return false;
    const size_t need = 2 * (c.prof_n + 1);
    while (c.prof_ev.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        c.prof_ev.push_back(e);
    }
    hipEventRecord(c.prof_ev[2 * c.prof_n], c.s);
    return true;
}

vts_status check_problem(const vts_problem* pr, std::string& err) {
    vts_status st = validate(pr, err);
    if (st != VTS_OK) return st;
    HostData hd;
    return prepare_host(pr, hd, err);
}

vts_status create_in(const vts_problem* pr, const vts_options* opt, void* stream, void* arena,
                     size_t arena_bytes, vts_ctx** out, std::string& err) {
    if (!out) return VTS_EINVAL;
    *out = nullptr;
    vts_status st = validate(pr, err);
    if (st != VTS_OK) return st;
    vts_ctx* c = new (std::nothrow) vts_ctx();
    if (!c) return VTS_ENOMEM;
    c->arena = (char*)arena;
    c->arena_size = arena ? arena_bytes : 0;
    st = ctx_create(*c, pr, opt, stream);
    if (st != VTS_OK) {
        err = c->err;
        ctx_free(*c);
        delete c;
        return st;
    }
    *out = c;
    return VTS_OK;
}

void prof_end(Ctx& c, double bytes, int launches) {
    hipEventRecord(c.prof_ev[2 * c.prof_n + 1], c.s);
    c.prof_n += 1;
    c.prof_launches += launches;
    c.prof_bytes += bytes;
}

}  // namespace vts

extern "C" {

void vts_default_options(vts_options* o) {
    if (!o) return;
    o->beta = 0.3;
    o->gamma = 0.3;
    o->p_min = 1e-3;
    o->q_min = 1e-8;
    o->eps_pbm = 1e-8;
    o->eps_nwt0 = 1.0;
    o->eps_nwt_min = 1e-5;
    o->eps_nwt_final = 5e-7;
    o->eps_stat = 5e-7;
    o->accept_stall = 1e-6;
    o->eps_mr0 = 0.0;
    o->eps_mr_min = 1e-9;
    o->armijo_c1 = 1e-4;
    o->armijo_min = 9.313225746154785e-10;   // 2^-30
    o->max_outer = 500;
    o->max_newton = 100;
    o->max_minres = 500;
    o->final_res4 = 1;
    o->p_min_relative = 1;
    o->stall_steps = 10;
    o->use_graphs = 0;
    o->kkt_tol = 1e-6;
    o->eps_state = 1e-10;
    o->log_path = nullptr;
}

vts_status vts_create(const vts_problem* pr, const vts_options* opt, void* stream, vts_ctx** out) {
    std::string err;
    vts_status st = create_in(pr, opt, stream, nullptr, 0, out, err);
    if (st != VTS_OK) g_create_err = err;
    return st;
}

size_t vts_allocated_bytes(const vts_ctx* c) { return c ? c->alloc_bytes : 0; }

vts_status vts_reset(vts_ctx* cp) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    launch_init_state(c);
    launch_round_rho(c);
    c.alpha = 1.0;
    c.eps_nwt = c.opt.eps_nwt0;
    c.eps_mr = c.opt.eps_mr0 > 0 ? c.opt.eps_mr0 : 1e-4 * std::sqrt((double)c.nl * c.nfree);
    c.res_prev = -1.0;
    c.outer = c.newton_total = c.minres_total = 0;
    c.converged = false;
    c.stat_since = -1;
    c.eps_stat = c.opt.eps_stat;
    c.kkt_resumes = 0;
    c.eval_valid = c.setup_valid = false;
    c.status = VTS_OK;
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

void vts_destroy(vts_ctx* c) {
    if (!c) return;
    ctx_free(*c);
    delete c;
}

size_t vts_footprint_bytes(const vts_problem* pr, const vts_options* opt) {
    (void)opt;
    std::string err;
    if (validate(pr, err) != VTS_OK || pr->nload > 1) return 0;
    return make_plan(pr).total();
}

vts_status vts_sizes(const vts_ctx* c, int64_t* n_dof, int64_t* m, int64_t* n_free,
                     int32_t* levels) {
    if (!c) return VTS_EINVAL;
    if (n_dof) *n_dof = c->ndof;
    if (m) *m = c->m;
    if (n_free) *n_free = c->nfree;
    if (levels) *levels = c->L;
    return VTS_OK;
}

vts_status vts_set_rho(vts_ctx* cp, const double* rho_dev) {
    if (!cp || !rho_dev) return VTS_EINVAL;
    Ctx& c = *cp;
    HIPCHK(hipMemcpyAsync(c.rho, rho_dev, c.m * 8, hipMemcpyDeviceToDevice, c.s));
    launch_round_rho(c);
    c.eval_valid = false;
    c.setup_valid = false;
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_apply_K(vts_ctx* cp, const double* x, double* y) {
    if (!cp || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    launch_apply_K_f64(c, c.rho, x, y);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_apply_K_f32(vts_ctx* cp, const float* x, float* y) {
    if (!cp || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    if (several_loads(c, "vts_apply_K_f32")) return VTS_EINVAL;
    launch_apply_K_f32(c, c.rhof, x, y);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_apply_K_rho(vts_ctx* cp, const double* rho, const double* x, double* y) {
    if (!cp || !rho || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    launch_apply_K_f64(c, rho, x, y);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_apply_K_rho_f32(vts_ctx* cp, const float* rho, const float* x, float* y) {
    if (!cp || !rho || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    if (several_loads(c, "vts_apply_K_rho_f32")) return VTS_EINVAL;
    launch_apply_K_f32(c, rho, x, y);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_element_energy(vts_ctx* cp, const double* u, double* e) {
    if (!cp || !u || !e) return VTS_EINVAL;
    Ctx& c = *cp;
    launch_energy(c, u, e);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_newton_setup(vts_ctx* cp) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    c.eval_valid = false;
    return setup(c);
}

vts_status vts_apply_S(vts_ctx* cp, const double* x, double* y) {
    if (!cp || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    if (!c.eval_valid) { c.err = "apply_S before newton_setup"; return VTS_ESTATE; }
    launch_apply_S(c, x, y);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_apply_S_noalloc(vts_ctx* cp, const double* x, double* y) {
    if (!cp || !x || !y || x == y) return VTS_EINVAL;
    Ctx& c = *cp;
    if (several_loads(c, "vts_apply_S_noalloc")) return VTS_EINVAL;
    if (!c.eval_valid) { c.err = "apply_S before newton_setup"; return VTS_ESTATE; }
    if (!tile_ok(c)) {
        c.err = "allocation-free S-apply needs the tiled operator (cube element)";
        return VTS_EINVAL;
    }
    const int nb = apply_S_tile_blocks(c);
    if (nb > kScratchPartials) {
        c.err = "grid needs " + std::to_string(nb) + " partial sums; the workspace holds " +
                std::to_string(kScratchPartials);
        return VTS_EINVAL;
    }
    double* ws = nullptr;
    const vts_status st = scratch_partials(c.device, &ws, c.err);
    if (st != VTS_OK) return st;
    launch_apply_S_tile_ws(c, x, y, ws);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_precondition(vts_ctx* cp, const double* r, double* z) {
    if (!cp || !r || !z || r == z) return VTS_EINVAL;
    Ctx& c = *cp;
    if (!c.setup_valid) { c.err = "precondition before newton_setup"; return VTS_ESTATE; }
    precond(c, r, z);
    HIPCHK(hipGetLastError());
    return VTS_OK;
}

vts_status vts_solve_newton(vts_ctx* cp, double eps_mr, vts_linstats* stats) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    if (!c.setup_valid) { c.err = "solve before newton_setup"; return VTS_ESTATE; }
    return minres(c, eps_mr, stats);
}

vts_status vts_newton_step(vts_ctx* cp, vts_newtonstats* stats) {
    if (!cp) return VTS_EINVAL;
    return newton_step(*cp, stats, false);
}

vts_status vts_newton(vts_ctx* cp, double eps_nwt, int32_t final_call, vts_newtonstats* last) {
    if (!cp) return VTS_EINVAL;
    return newton(*cp, eps_nwt, final_call != 0, last, nullptr);
}

vts_status vts_pbm_iterate(vts_ctx* cp, vts_pbmstats* stats) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    if (c.converged) { c.err = "already converged"; return VTS_ESTATE; }
    return pbm_iterate(c, stats);
}

vts_status vts_pbm_solve(vts_ctx* cp, vts_result* res) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    vts_status st = VTS_OK;
    vts_newtonstats ns{};
    bool kkt_done = false;
    double kk[5] = {0, 0, 0, 0, 0};   // kkt, r_eq, r_vol, r_box, r_stat
    for (;;) {
        st = VTS_OK;
        kkt_done = false;
        while (!c.converged && c.outer < c.opt.max_outer) {
            st = pbm_iterate(c, nullptr);
            if (st != VTS_OK) break;
        }
        if (st == VTS_OK && !c.converged) st = VTS_ENOTCONV;
        if (st == VTS_OK) {
            st = newton(c, c.opt.eps_nwt_final, true, &ns, nullptr);
            // a stalled final Newton (no progress, or no descent step) goes on to the
            // rho update; device, argument and definiteness errors never do
            const bool stall = st == VTS_ENOTCONV || st == VTS_ENONDESCENT;
            const bool by_kkt = c.opt.kkt_tol > 0;
            if (stall && (by_kkt || (c.res_prev >= 0 && c.res_prev < c.opt.accept_stall)))
                st = by_kkt ? VTS_ENOTCONV : VTS_OK;
            if (st == VTS_OK || (by_kkt && stall)) {
                vts_status s2 = VTS_OK;
                // the last accepted state was evaluated; make sure of it before the rho update
                if (!c.eval_valid) s2 = evaluate(c);
                if (s2 == VTS_OK) {
                    launch_mult_update(c, 1);
                    launch_round_rho(c);
                    c.eval_valid = false;
                    c.setup_valid = false;
                    // with a zero lower bound K(rho) may be singular on a void region,
                    // where the state equation leaves u free; the dual iterate is then
                    // the displacement that meets the optimality conditions
                    if (c.opt.eps_state > 0 && c.lo_min > 0) s2 = state_solve(c, c.opt.eps_state);
                }
                if (s2 == VTS_OK) {
                    launch_kkt(c, c.alpha, c.g1);
                    s2 = sync_red(c);
                }
                if (s2 != VTS_OK) {
                    st = s2;
                } else {
                    const double* r = c.red_host;
                    kk[1] = std::sqrt(r[SL_WT]) / c.norm_f;
                    kk[2] = std::fabs(r[SL_SUM_RHO] - c.V) / c.V;
                    kk[3] = std::max(0.0, r[SL_AUX]) / r[SL_MRALPHA];
                    kk[4] = r[SL_STAT];
                    kk[0] = std::max(std::max(kk[1], kk[2]), std::max(kk[3], kk[4]));
                    kkt_done = true;
                    if (by_kkt) {
                        st = kk[0] <= c.opt.kkt_tol ? VTS_OK : VTS_ENOTCONV;
                        if (st != VTS_OK) c.err = "KKT residual above kkt_tol";
                    }
                }
            }
        }
        // the returned state misses the KKT target (the final Newton call moved
        // the stationarity term past it): the outer loop goes on from that state
        // with half the stationarity target, a bounded number of times
        if (kkt_done && c.opt.kkt_tol > 0 && kk[0] > c.opt.kkt_tol &&
            c.kkt_resumes < kKktResumes && c.outer < c.opt.max_outer) {
            ++c.kkt_resumes;
            c.eps_stat *= 0.5;
            c.converged = false;
            c.stat_since = -1;
            log_line(c, "{\"event\": \"resume\", \"outer\": %d, \"kkt\": %.17g, \"eps_stat\": %.17g}",
                     c.outer, kk[0], c.eps_stat);
            continue;
        }
        break;
    }
    if (res) {
        launch_dot(c, c.f, c.u, c.nvec, SL_DOT);
        launch_outer_eval(c);
        vts_status s3 = sync_red(c);
        if (s3 != VTS_OK && st == VTS_OK) st = s3;
        res->compliance = 0.5 * c.red_host[SL_DOT];
        res->alpha = c.alpha;
        res->sum_rho = c.red_host[SL_SUM_RHO];
        res->res_pbm = c.res_prev;
        res->outer = c.outer;
        res->newton = c.newton_total;
        res->minres = c.minres_total;
        res->status = st;
        res->kkt = kkt_done ? kk[0] : 0.0;
        res->r_eq = kkt_done ? kk[1] : 0.0;
        res->r_vol = kkt_done ? kk[2] : 0.0;
        res->r_box = kkt_done ? kk[3] : 0.0;
        res->r_stat = kkt_done ? kk[4] : 0.0;
    }
    log_line(c,
             "{\"event\": \"result\", \"status\": %d, \"outer\": %d, \"newton\": %d, "
             "\"minres\": %d, \"res_pbm\": %.17g, \"kkt\": %.17g, \"r_eq\": %.17g, "
             "\"r_vol\": %.17g, \"r_box\": %.17g, \"r_stat\": %.17g}",
             (int)st, c.outer, c.newton_total, c.minres_total, c.res_prev, kkt_done ? kk[0] : 0.0,
             kkt_done ? kk[1] : 0.0, kkt_done ? kk[2] : 0.0, kkt_done ? kk[3] : 0.0,
             kkt_done ? kk[4] : 0.0);
    c.status = st;
    return st;
}

vts_status vts_doc_step(vts_ctx* cp, double q, double tau, double eps_doc, double eps_mr,
                        vts_docstats* out) {
    if (!cp || !(q > 0) || !(tau > 0)) return VTS_EINVAL;
    Ctx& c = *cp;
    if (several_loads(c, "vts_doc_step")) return VTS_EINVAL;
    // the state equation: MINRES with the V-cycle on blockdiag(K(rho), 1)
    c.eval_valid = false;
    c.setup_valid = false;
    launch_doc_setup(c);
    c.sum_w = 1.0;
    vts_status st = build_mg(c);
    if (st != VTS_OK) return st;
    vts_linstats ls{0, 0.0};
    if ((st = minres(c, eps_mr, &ls)) != VTS_OK) return st;
    HIPCHK(hipMemcpyAsync(c.u, c.dy, c.ndof * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    launch_energy(c, c.u, c.e);
    launch_dot(c, c.f, c.u, c.ndof, SL_DOT);
    // bisection on alpha (Algorithm 4)
    double lo = 0.0, hi = 1e4, alpha = 0.5 * (lo + hi);
    int steps = 0;
    while ((hi - lo) / (hi + lo) > tau) {
        alpha = 0.5 * (hi + lo);
        launch_doc_volume(c, q, alpha);
        if ((st = sync_red(c)) != VTS_OK) return st;
        if (c.red_host[SL_SUM_RHO] > c.V)
            lo = alpha;
        else
            hi = alpha;
        ++steps;
    }
    launch_doc_candidate(c, q, alpha, c.c1);
    launch_doc_volume(c, q, alpha);
    if ((st = sync_red(c)) != VTS_OK) return st;
    const double change = c.red_host[SL_STAT];
    const bool conv = eps_doc > 0 && change <= eps_doc;
    if (!conv)
        HIPCHK(hipMemcpyAsync(c.rho, c.c1, c.m * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.s));
    c.minres_total += ls.iterations;
    if (out) {
        out->change = change;
        out->alpha = alpha;
        out->compliance = 0.5 * c.red_host[SL_DOT];
        out->volume = c.red_host[SL_SUM_RHO];
        out->bisection_steps = steps;
        out->minres_its = ls.iterations;
        out->converged = conv ? 1 : 0;
        out->iterations = 1;
    }
    return VTS_OK;
}

vts_status vts_doc_solve(vts_ctx* cp, double q, double eps_doc, double eps_mr, int32_t max_iter,
                         vts_docstats* out) {
    if (!cp || !(eps_doc > 0) || max_iter < 1) return VTS_EINVAL;
    vts_docstats s{};
    int32_t minres = 0;
    for (int32_t k = 0; k < max_iter; ++k) {
        vts_status st = vts_doc_step(cp, q, 0.1 * eps_doc, eps_doc, eps_mr, &s);
        if (st != VTS_OK) return st;
        minres += s.minres_its;
        s.iterations = k + 1;
        if (s.converged) break;
    }
    s.minres_its = minres;
    if (out) *out = s;
    return s.converged ? VTS_OK : VTS_ENOTCONV;
}

void vts_ip_default_options(vts_ip_options* o) {
    if (!o) return;
    o->eps_ip = 1e-5;
    o->sigma_r = 0.2;
    o->sigma_s = 0.2;
    o->r0 = 1e-2;
    o->s0 = 1e-2;
    o->step_frac = 0.9;
    o->eps_mr0 = 1e-2;
    o->eps_mr_min = 1e-9;
    o->max_iter = 300;
    o->max_minres = 3000;
}

vts_status vts_ip_init(vts_ctx* cp, const vts_ip_options* opt) {
    if (!cp) return VTS_EINVAL;
    if (several_loads(*cp, "vts_ip_init")) return VTS_EINVAL;
    return ip_init(*cp, opt);
}

vts_status vts_ip_step(vts_ctx* cp, vts_ipstats* stats) {
    if (!cp) return VTS_EINVAL;
    if (several_loads(*cp, "vts_ip_step")) return VTS_EINVAL;
    return ip_step(*cp, stats);
}

vts_status vts_ip_solve(vts_ctx* cp, const vts_ip_options* opt, vts_ipstats* stats) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    if (several_loads(c, "vts_ip_solve")) return VTS_EINVAL;
    vts_status st = ip_init(c, opt);
    if (st != VTS_OK) return st;
    vts_ipstats s{};
    int32_t minres = 0, k = 0;
    for (k = 0; k < c.ip.o.max_iter; ++k) {
        st = ip_step(c, &s);
        minres += s.minres_its;
        if (st != VTS_OK || s.converged) break;
    }
    s.iterations = std::min(k + 1, c.ip.o.max_iter);
    s.minres_its = minres;
    if (stats) *stats = s;
    if (st != VTS_OK) return st;
    return s.converged ? VTS_OK : VTS_ENOTCONV;
}

vts_status vts_get_vector(const vts_ctx* cp, int32_t which, double* dst) {
    if (!cp || !dst) return VTS_EINVAL;
    Ctx& c = const_cast<vts_ctx&>(*cp);
    const double* src = nullptr;
    int64_t n = 0;
    switch (which) {
        case VTS_VEC_U: src = c.u; n = c.nvec; break;
        case VTS_VEC_RHO: src = c.rho; n = c.m; break;
        case VTS_VEC_ENERGY: src = c.e; n = c.m; break;
        case VTS_VEC_RHS: src = c.rhs; n = c.nvec + 1; break;
        case VTS_VEC_DY: src = c.dy; n = c.nvec + 1; break;
        case VTS_VEC_G1: src = c.g1; n = c.nvec; break;
        case VTS_VEC_DNU_LO: src = c.dnl; n = c.m; break;
        case VTS_VEC_DNU_HI: src = c.dnh; n = c.m; break;
        case VTS_VEC_RHO1: src = c.r1; n = c.m; break;
        case VTS_VEC_W: src = c.w; n = c.m; break;
        default: c.err = "unknown vector"; return VTS_EINVAL;
    }
    if ((which == VTS_VEC_ENERGY || which == VTS_VEC_RHS || which == VTS_VEC_G1 ||
         which == VTS_VEC_RHO1 || which == VTS_VEC_W) && !c.eval_valid) {
        c.err = "state not evaluated (call vts_newton_setup)";
        return VTS_ESTATE;
    }
    HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToDevice, c.s));
    return VTS_OK;
}

// checkpoint layout (FP64): header {magic, version, n_dof, m}, u, alpha, the
// eight m-vectors, eps_nwt, eps_mr, and the outer / Newton / MINRES counters
constexpr double kStateMagic = 5657683.0;   // "VTS" as a number
constexpr double kStateVersion = 2.0;
constexpr int kStateHead = 4, kStateTail = 5;

size_t state_bytes(const Ctx& c) {
    return (size_t)(kStateHead + c.nvec + 1 + 8 * c.m + kStateTail) * 8;
}

vts_status vts_get_state(const vts_ctx* cp, void* buf, size_t* bytes) {
    if (!cp || !bytes) return VTS_EINVAL;
    Ctx& c = const_cast<vts_ctx&>(*cp);
    const size_t need = state_bytes(c);
    if (!buf || *bytes < need) {
        *bytes = need;
        return buf ? VTS_EINVAL : VTS_OK;
    }
    double* b = (double*)buf;
    *b++ = kStateMagic;
    *b++ = kStateVersion;
    *b++ = (double)c.nvec;
    *b++ = (double)c.m;
    HIPCHK(hipMemcpyAsync(b, c.u, c.nvec * 8, hipMemcpyDeviceToHost, c.s));
    b += c.nvec;
    *b++ = c.alpha;
    double* arr[8] = {c.nlo, c.nhi, c.rho, c.mlo, c.mhi, c.p, c.qlo, c.qhi};
    for (int q = 0; q < 8; ++q) {
        HIPCHK(hipMemcpyAsync(b, arr[q], c.m * 8, hipMemcpyDeviceToHost, c.s));
        b += c.m;
    }
    *b++ = c.eps_nwt;
    *b++ = c.eps_mr;
    *b++ = (double)c.outer;
    *b++ = (double)c.newton_total;
    *b++ = (double)c.minres_total;
    HIPCHK(hipStreamSynchronize(c.s));
    *bytes = need;
    return VTS_OK;
}

vts_status vts_set_state(vts_ctx* cp, const void* buf, size_t bytes) {
    if (!cp || !buf) return VTS_EINVAL;
    Ctx& c = *cp;
    const size_t need = state_bytes(c);
    if (bytes != need) { c.err = "state size mismatch"; return VTS_EINVAL; }
    const double* b = (const double*)buf;
    if (b[0] != kStateMagic || b[1] != kStateVersion || b[2] != (double)c.nvec ||
        b[3] != (double)c.m) {
        c.err = "state header does not match this context (magic, version, load cases x n_dof, m)";
        return VTS_EINVAL;
    }
    const double* t = b + kStateHead + c.nvec + 1 + 8 * c.m;
    for (int q = 2; q < kStateTail; ++q)
        if (!(t[q] >= 0 && t[q] < 2147483647.0 && t[q] == std::floor(t[q]))) {
            c.err = "state counters out of range";
            return VTS_EINVAL;
        }
    b += kStateHead;
    HIPCHK(hipMemcpyAsync(c.u, b, c.nvec * 8, hipMemcpyHostToDevice, c.s));
    b += c.nvec;
    c.alpha = *b++;
    double* arr[8] = {c.nlo, c.nhi, c.rho, c.mlo, c.mhi, c.p, c.qlo, c.qhi};
    for (int q = 0; q < 8; ++q) {
        HIPCHK(hipMemcpyAsync(arr[q], b, c.m * 8, hipMemcpyHostToDevice, c.s));
        b += c.m;
    }
    c.eps_nwt = *b++;
    c.eps_mr = *b++;
    c.outer = (int)*b++;
    c.newton_total = (int)*b++;
    c.minres_total = (int)*b++;
    HIPCHK(hipStreamSynchronize(c.s));
    launch_round_rho(c);
    c.eval_valid = false;
    c.setup_valid = false;
    c.converged = false;
    c.stat_since = -1;
    return VTS_OK;
}

vts_status vts_profile_start(vts_ctx* cp, int32_t cls) {
    if (!cp || cls < VTS_PROF_NONE || cls > VTS_PROF_APPLY_S) return VTS_EINVAL;
    Ctx& c = *cp;
    HIPCHK(hipStreamSynchronize(c.s));
    c.prof_class = cls;
    c.prof_n = 0;
    c.prof_launches = 0;
    c.prof_bytes = 0.0;
    return VTS_OK;
}

vts_status vts_profile_stop(vts_ctx* cp, double* total_ms, int64_t* launches, double* bytes) {
    if (!cp) return VTS_EINVAL;
    Ctx& c = *cp;
    HIPCHK(hipStreamSynchronize(c.s));
    double ms = 0.0;
    for (size_t q = 0; q < c.prof_n; ++q) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, c.prof_ev[2 * q], c.prof_ev[2 * q + 1]));
        ms += t;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = c.prof_launches;
    if (bytes) *bytes = c.prof_bytes;
    c.prof_class = 0;
    c.prof_n = 0;
    c.prof_launches = 0;
    c.prof_bytes = 0.0;
    return VTS_OK;
}

const char* vts_last_error(const vts_ctx* c) {
    if (!c) return g_create_err.c_str();
    return c->err.c_str();
}

}  // extern "C"
