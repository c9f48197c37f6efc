// Internal declarations of libvts (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vts.h"

namespace vts {

constexpr int kThreads = 256;          // block size of every 1D launch
constexpr int kRedBlocks = 1024;       // max blocks of a reduction launch
constexpr int kRedSlots = 17;          // quantities per reduction buffer
constexpr int kMaxCoarse = 4096;       // largest dense coarsest system
constexpr int kMaxLoads = 4;           // load cases of one problem
constexpr int kMlMaxCoarse = 4096;     // largest dense coarsest system with several cases
constexpr int kKktResumes = 3;         // outer-loop resumptions after a missed KKT target

// Block of 27 neighbours: offset (dx,dy,dz) in {-1,0,1}^3 -> s = (dx+1) + 3(dy+1) + 9(dz+1).
constexpr int kStencil = 27;
constexpr int kStencilVals = 27 * 9;   // 3x3 block per neighbour

// One multigrid level (all sizes for that level's grid).  Device pointers.
template <typename T>
struct Level {
    int nx, ny, nz;            // elements
    int NX, NY, NZ;            // nodes per direction
    int64_t nn, m;             // nodes, elements
    int cnx[8], cny[8], cnz[8];// nodes per colour and direction
    int64_t coff[9];           // colour offsets in colour-major order
    uint8_t* fixed;            // 3*nn DOF mask
    T* st;                     // 243*nn stencil, [value][colour-major node]
    T* dinv;                   // 9*nn inverse diagonal block, [value][colour-major node]
    T* acol;                   // 3*nn alpha column, natural order
    T* E;                      // 576*m element matrices (coarse levels), [e][row][col]
    T* TQ;                     // 576*m scratch for the Galerkin product
    T* r;                      // S-vectors (3*nn + 1)
    T* z;
    T* res;
};

// Device operations of one context recorded instead of issued: a group of
// contexts with the same launch sequence then runs each recorded launch as
// one launch over all of them (problem = blockIdx.y, arguments from a table).
struct RecOp {
    const void* k = nullptr;    // single-problem kernel: takes Args by value
    const void* kb = nullptr;   // batched kernel: takes const Args* table
    dim3 grid, block;
    uint32_t asize = 0;         // bytes of the argument struct (0: a copy)
    size_t aoff = 0;            // offset of the argument bytes in Recorder::bytes
    void* dst = nullptr;        // copy
    const void* src = nullptr;
    size_t nbytes = 0;
    hipMemcpyKind kind = hipMemcpyDeviceToDevice;
};

struct Recorder {
    std::vector<RecOp> ops;
    std::vector<uint8_t> bytes;
    void clear() {
        ops.clear();
        bytes.clear();
    }
    void kernel(const void* k, const void* kb, dim3 g, dim3 b, const void* args, uint32_t n) {
        RecOp o;
        o.k = k;
        o.kb = kb;
        o.grid = g;
        o.block = b;
        o.asize = n;
        o.aoff = bytes.size();
        bytes.insert(bytes.end(), (const uint8_t*)args, (const uint8_t*)args + n);
        ops.push_back(o);
    }
    void copy(void* dst, const void* src, size_t n, hipMemcpyKind k) {
        RecOp o;
        o.dst = dst;
        o.src = src;
        o.nbytes = n;
        o.kind = k;
        ops.push_back(o);
    }
};

template <typename T>
struct Hierarchy {
    std::vector<Level<T>> lev;   // 0 = coarsest
    double* A = nullptr;         // dense coarsest matrix / Cholesky factor, nc x nc
    double* Ainv = nullptr;      // explicit inverse of the coarsest matrix, nc x nc
    int nc = 0;
    int* cmap = nullptr;         // 3*nn_0 -> dense index or -1
    int* cinv = nullptr;         // dense index -> DOF of level 0 (nc-1 entries)
    int* flag = nullptr;         // device: 1 if the factorization met a non-positive pivot
    int ksmall = -1;             // levels 0..ksmall run in one workgroup (-1: none)
    // finest level without a stored stencil (when it is not one of the small
    // levels): the Gauss-Seidel rows are formed from the element data
    bool mf = false;
    T* bc = nullptr;             // 24 per node (colour-major): b_e rows at the node, per element
    T* te = nullptr;             // m: b_e^T z_e of the current z
    T* r1f = nullptr;            // m: rho' in T (aliases Ctx::r1 when T is double)
    T* wf = nullptr;             // m: w in T (aliases Ctx::w when T is double)
    T* uf = nullptr;             // 3 nn: u in T (aliases Ctx::u when T is double)
};

constexpr int kSmallNodes = 512;    // largest level handled by the one-workgroup V-cycle
constexpr int kSmallCoarse = 2048;  // largest coarsest system for that kernel
constexpr int kMaxSmallLevels = 6;

struct Ctx {
    // problem
    int nx, ny, nz, L;
    int64_t nn, ndof, m, nfree;
    double E, nu, h, V;
    int prec;
    vts_options opt;
    hipStream_t s = nullptr;
    Recorder* rec = nullptr;        // non-null: device operations are recorded (group solves)
    std::string log_path;           // JSON-lines log of Newton steps, outer iterations, results
    FILE* log = nullptr;
    struct GroupRunner* group = nullptr;  // non-null: Newton-system MINRES runs in this group
    int device = 0;

    // constants (device)
    double* Ke = nullptr;        // 576
    float* Kef = nullptr;        // 576
    double* Mc = nullptr;        // 8 x 576: Q_c^T K_e Q_c
    double* Qc = nullptr;        // 8 x 8 x 8: Q_c[a][A] nodal interpolation weights
    double ke_host[576] = {};    // K_e on the host (rows of corner 0 feed the smoother)
    double kh8[8] = {};          // the 8 coefficients of H K_e H / 64 (sum/difference basis)
    bool kh_ok = false;          // K_e has the cube's structure in that basis
    double* spart = nullptr;     // per-workgroup partial sums of the tiled S-apply

    // problem data (device)
    uint8_t* fixed = nullptr;    // ndof
    uint8_t* nmask = nullptr;    // nn: bit c set if DOF 3 node + c is fixed
    double* f = nullptr;         // ndof
    double* rlo = nullptr;       // m
    double* rhi = nullptr;       // m
    double norm_f = 0, norm_bounds = 0;
    double lo_min = 0;             // smallest lower bound of rho

    // PBM state (device)
    double* u = nullptr;         // ndof
    double alpha = 1.0;
    double* nlo = nullptr;       // nu_lo, m
    double* nhi = nullptr;
    double* rho = nullptr;
    double* mlo = nullptr;
    double* mhi = nullptr;
    double* p = nullptr;
    double* qlo = nullptr;
    double* qhi = nullptr;
    float* rhof = nullptr;       // rho rounded to FP32 (for vts_apply_K_f32)

    // evaluation at the current state (device)
    double* e = nullptr;         // m
    double* be = nullptr;        // 24*m, [j][e]
    double* r1 = nullptr;        // rho'
    double* r2 = nullptr;        // rho''
    double* l2 = nullptr;        // mu_lo''
    double* h2 = nullptr;        // mu_hi''
    double* g3 = nullptr;
    double* g4 = nullptr;
    double* w = nullptr;
    double* zc = nullptr;        // z of the right-hand side
    double* gch = nullptr;       // 24*m, Q_c^T b_e (Galerkin helper)
    double* g1 = nullptr;        // ndof
    double* rhs = nullptr;       // ndof+1
    double* dy = nullptr;        // ndof+1
    double* dnl = nullptr;       // m
    double* dnh = nullptr;
    double* c1 = nullptr;        // b_e^T du_e
    double* c2 = nullptr;        // 1/2 du_e^T K_e du_e
    double* wt = nullptr;        // scratch per element (S-apply)
    double g2 = 0, sum_w = 0, sum_z = 0, sum_r1 = 0, n_g1 = 0, n_g3 = 0, n_g4 = 0;
    bool setup_valid = false;
    bool eval_valid = false;

    // MINRES vectors (device), each ndof+1
    double* mv[8] = {};

    // reductions
    double* partials = nullptr;  // kRedSlots * kRedBlocks
    double* red = nullptr;       // kRedSlots results (device)
    double* red_host = nullptr;  // pinned mirror

    // multigrid
    Hierarchy<double>* h64 = nullptr;
    Hierarchy<float>* h32 = nullptr;

    // load cases: u, f, g1 and the u-part of every Newton-system vector hold
    // nl all-DOF vectors one after another (nvec = nl n_dof entries); with
    // nl > 1 the multi-load kernels and their multigrid (mlh) serve the
    // context
    int nl = 1;
    int64_t nvec = 0;
    struct MlHierarchy* mlh = nullptr;

    // algorithm state (host)
    double eps_nwt = 1.0, eps_mr = 0.0, res_prev = -1.0;
    int outer = 0, newton_total = 0, minres_total = 0;
    int status = VTS_OK;
    bool converged = false;
    double eps_stat = 0;            // the outer loop's stationarity target (halved on a resumption)
    int kkt_resumes = 0;            // resumptions after a final KKT check above kkt_tol
    double stat_best = 0;           // smallest stationarity term since the gap test first held
    int stat_since = -1;            // outer iterations since it last fell below 0.9 x best
                                    // (-1: the gap test has not held yet)
    std::string err;

    // interior point method (Algorithm 3): options, barrier parameters and
    // the scalars of the last evaluation
    struct Ip {
        vts_ip_options o{};
        double r = 0, s = 0, r_plus = 0, s_plus = 0, eps_mr = 0;
        double sum_rho = 0, n_res3 = 0, gap_sum = 0, cl = 0, ch = 0, n_nl = 0, n_nh = 0;
        double dmax = 0, viol = 0, fu = 0;
        bool ready = false;
    } ip;

    // V-cycles replayed from captured HIP graphs, keyed by the arguments that
    // vary between calls (r, z and the alpha diagonal); dropped whenever the
    // hierarchy is rebuilt.  Captured on a private stream, launched on s.
    struct VGraph {
        const double* r;
        double* z;
        double d;
        hipGraphExec_t exec;
    };
    std::vector<VGraph> vgraphs;
    hipStream_t cap_stream = nullptr;

    std::vector<void*> allocs;   // hipMalloc'd buffers (contexts without an arena)
    char* arena = nullptr;       // caller-owned device range (server slots), or null
    size_t arena_size = 0, arena_used = 0;
    size_t alloc_bytes = 0;      // device bytes taken, 256-byte granules

    // kernel-class profiling (vts_profile_start/stop): HIP events around
    // every launch of one class on this context's stream
    int prof_class = 0;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_n = 0;        // event pairs recorded
    int64_t prof_launches = 0;
    double prof_bytes = 0.0;
};

// every check vts_create makes before touching the device (no HIP call)
vts_status check_problem(const vts_problem* pr, std::string& err);

// vts_create with an optional caller-owned device arena of arena_bytes (the
// context then calls no hipMalloc; vts_destroy leaves the arena alone)
vts_status create_in(const vts_problem* pr, const vts_options* opt, void* stream, void* arena,
                     size_t arena_bytes, vts_ctx** out, std::string& err);

// profiling hooks (capi.cpp); prof_begin returns true if this launch is timed
// A kernel and its batched twin from one device body: NAME(ARGS a) runs
// BODY(a); NAME_b(const ARGS* tab) runs BODY(tab[blockIdx.y]), problem
// blockIdx.y of a group launch (its blockIdx.x, gridDim.x as alone).
#define VTS_KERNEL_PAIR(TPL, BOUNDS, NAME, ARGS, BODY)                                      \
    TPL __global__ void __launch_bounds__(BOUNDS) NAME(ARGS a) { BODY(a); }                 \
    TPL __global__ void __launch_bounds__(BOUNDS) NAME##_b(const ARGS* __restrict__ tab) {   \
        BODY(tab[blockIdx.y]);                                                              \
    }

// One kernel launch with its arguments in a struct: issued on c.s, or
// recorded (with the batched twin kb) while c.rec is set.
template <class A>
inline void vlaunch(Ctx& c, const void* k, const void* kb, dim3 g, dim3 b, const A& a) {
    if (c.rec) {
        c.rec->kernel(k, kb, g, b, &a, (uint32_t)sizeof(A));
        return;
    }
    void* args[] = {const_cast<A*>(&a)};
    (void)hipLaunchKernel(k, g, b, args, 0, c.s);
}

inline hipError_t vmemcpy(Ctx& c, void* dst, const void* src, size_t n, hipMemcpyKind kind) {
    if (c.rec) {
        c.rec->copy(dst, src, n, kind);
        return hipSuccess;
    }
    return hipMemcpyAsync(dst, src, n, kind, c.s);
}

// Preconditioned MINRES as steps between synchronizations (capi.cpp)
struct MrState {
    enum Phase { kStart, kIterate, kFinish, kDone };
    double eps = 0;
    int maxit = 0;
    bool stop_indef = false;
    int64_t n = 0;
    double *x = nullptr, *r1 = nullptr, *r2 = nullptr, *y = nullptr, *v = nullptr;
    double* wb[3] = {nullptr, nullptr, nullptr};
    int iw = 0, iw1 = 1, iw2 = 2;
    double beta1 = 0, beta = 0, beta_old = 0, cs = -1, sn = 0, dbar = 0, eps_l = 0, phibar = 0;
    double rel = 0;
    int it = 0;
    Phase phase = kStart;
    vts_status st = VTS_OK;
};
void mr_init(Ctx& c, MrState& m, double eps, int maxit, bool stop_indef);
void mr_issue_start(Ctx& c, MrState& m);
void mr_after_start(Ctx& c, MrState& m);
void mr_issue_iter(Ctx& c, MrState& m);
void mr_after_iter(Ctx& c, MrState& m);
void mr_finish(Ctx& c, MrState& m, vts_linstats* out);

// Group runner (group.cpp): a thread with its own stream that advances the
// MINRES solves handed to it one step at a time, all of them together; the
// device work of solves with the same launch sequence goes out as one launch
// per kernel over all of them.  Solves join and leave between steps.
struct GroupRunner;
struct GroupStats {
    int64_t cycles = 0;          // synchronized steps
    int64_t solves = 0;          // MINRES solves completed
    int64_t kernel_ops = 0;      // kernel launches the solves recorded
    int64_t launches = 0;        // launches issued for them
    int64_t max_batch = 0;       // largest number of solves in one launch
};
GroupRunner* group_runner_create(int device, std::string& err);
void group_runner_destroy(GroupRunner* g);
void group_runner_stats(GroupRunner* g, GroupStats* out);   // thread-safe
// MINRES of c's Newton system through c.group (blocks the calling thread)
vts_status group_minres(Ctx& c, double eps, vts_linstats* out, int maxit);

bool prof_begin(Ctx& c, int cls);
void prof_end(Ctx& c, double bytes, int launches = 1);

// algorithmic bytes of one colour pass: the colour's stencil rows and
// inverse diagonal blocks, r, acol, z (read and write), neighbour z values
template <typename T>
inline double gs_color_bytes(const Level<T>& L, int col, size_t ts) {
    const double cnt = (double)(L.coff[col + 1] - L.coff[col]);
    return cnt * (kStencilVals + 9 + 12) * ts + ((double)L.nn - cnt) * 3 * ts;
}

// compulsory bytes of one colour pass on the finest level without a stored
// stencil: per node of the colour r, acol, dinv, its 24 b values and z written;
// per element rho', w and b^T z read and written; z of every node read
template <typename T>
inline double gs_mf_color_bytes(const Level<T>& L, int col, size_t ts) {
    const double cnt = (double)(L.coff[col + 1] - L.coff[col]);
    return (cnt * (3 + 3 + 9 + 24 + 3) + (double)L.m * 4 + (double)L.nn * 3) * ts;
}

// host-side finite-element tables (host_fe.cpp)
void element_stiffness(double E, double nu, double h, double* Ke576);
void child_interp(double* Q512);                       // Q[c][a][A]
void galerkin_child_matrices(const double* Ke, const double* Q, double* Mc);

// launchers (kernels.hip); all asynchronous on ctx.s
void launch_apply_K_f64(Ctx& c, const double* rho, const double* x, double* y);
void launch_apply_K_case(Ctx& c, const double* rho, const double* x, double* y);  // one case
void launch_apply_K_f32(Ctx& c, const float* rho, const float* x, float* y);
void launch_energy(Ctx& c, const double* u, double* e);
void launch_eval(Ctx& c);                    // e, be, coefficients, sums -> red[0..]
void launch_grad(Ctx& c);                    // g1, rhs_u, ||g1||^2 -> red
void launch_apply_S(Ctx& c, const double* x, double* y);
void launch_dnu(Ctx& c);                     // c1, c2, dnl, dnh, slope parts -> red
void launch_linesearch(Ctx& c, double kappa, double dalpha); // elementwise Delta L -> red
void launch_update(Ctx& c, double kappa);    // u, nu
void launch_outer_eval(Ctx& c);              // gap, dual parts, stationarity -> red
// KKT terms of (rho, u, lam) -> red[STAT, SUM_RHO, WT (||Ku-f||^2), AUX (box), MRALPHA (max hi)];
// Ku: n_dof scratch; overwrites e
void launch_kkt(Ctx& c, double lam, double* Ku);
void launch_mult_update(Ctx& c, int rho_only);
void launch_penalty_update(Ctx& c);
void launch_init_state(Ctx& c);
void launch_dot(Ctx& c, const double* x, const double* y, int64_t n, int slot);
void launch_copy1(Ctx& c, const double* src, double* dst);
void launch_set(Ctx& c, double* dst, double v);
void launch_fill(Ctx& c, double* dst, double v, int64_t n);
void launch_scale(Ctx& c, double* dst, const double* src, double a, int64_t n);
void launch_axpy(Ctx& c, double* y, double a, const double* x, int64_t n);
// y -= (red[slot] / div) x, the scalar read on the device
void launch_axpy_red(Ctx& c, double* y, int slot, double div, const double* x, int64_t n);
// damped optimality criteria (Algorithm 4)
void launch_doc_setup(Ctx& c);                               // r1 = rho, w = 0, rhs = [f; 0]
void launch_doc_volume(Ctx& c, double q, double alpha);     // sum rho+(alpha) -> red[SL_SUM_RHO]
void launch_doc_candidate(Ctx& c, double q, double alpha, double* out); // max |drho| -> red[SL_STAT]
// primal-dual interior point method (Algorithm 3)
void launch_ip_eval(Ctx& c, double r, double s);     // e, be, W, z, res_3, X; sums -> red[6..16]
void launch_ip_dir(Ctx& c, double r, double s);      // drho (c1), dnl, dnh; step maxima -> red[0..2]
void launch_ip_update(Ctx& c, double ku, double kl, double kh);
void launch_minres_w(Ctx& c, double* w, const double* v, const double* w1, const double* w2,
                     double eps_old, double delta, double inv_gamma, double* x, double phi,
                     int64_t n);
void launch_round_rho(Ctx& c);

// operator.hip: tiled element operators (sum/difference form of K_e)
bool tile_ok(const Ctx& c);
int apply_S_tile_blocks(const Ctx& c);
void launch_apply_K_tile_f64(Ctx& c, const double* rho, const double* x, double* y);
void launch_apply_K_tile_f32(Ctx& c, const float* rho, const float* x, float* y);
void launch_apply_S_tile(Ctx& c, const double* x, double* y);
// the same with the per-workgroup partial sums in `partials`
void launch_apply_S_tile_ws(Ctx& c, const double* x, double* y, double* partials);
// matrix-free finest level of the V-cycle (operator.hip): residual with
// per-workgroup partials of acol . z, and the element products b_e^T z_e
template <typename T>
void launch_fine_resid(Ctx& c, const Level<T>& L, const T* u, const T* r1, const T* w,
                       double* parts);
template <typename T>
void launch_fine_tdot(Ctx& c, const Level<T>& L, const T* u, const T* r1, const T* w, T* te);
int fine_resid_blocks(const Ctx& c);
// allocation-free S-apply: the device address of the file-scope workspace of
// kScratchPartials doubles (looked up once per device)
constexpr int kScratchPartials = 1 << 16;
constexpr int kMaxScratchDevices = 64;
vts_status scratch_partials(int device, double** out, std::string& err);
bool walsh_form(const double* Ke, double* kh8);    // host_fe.cpp

// several load cases (multiload.hip): evaluation, gradient, batched K,
// S-apply, Delta nu, energies, update, and the multigrid with node blocks
// over all cases
void ml_launch_eval(Ctx& c);
void ml_launch_grad(Ctx& c);
void ml_apply_K(Ctx& c, const double* coef, const double* x, double* y);
void ml_apply_S(Ctx& c, const double* x, double* y);
void ml_launch_dnu(Ctx& c);
void ml_launch_energy(Ctx& c, const double* u, double* e);
void ml_launch_update(Ctx& c, double kappa);
vts_status ml_create(Ctx& c, const std::vector<uint8_t>& fine_mask);
void ml_destroy(Ctx& c);
int ml_mg_build(Ctx& c);
void ml_vcycle(Ctx& c, const double* r, double* z);
// capi.cpp: a device buffer of the context, and the coarse DOF mask by injection
vts_status ml_alloc(Ctx& c, void** ptr, size_t bytes);
std::vector<uint8_t> ml_coarsen(const std::vector<uint8_t>& fine_mask, int nx, int ny, int nz);

template <typename T> void mg_build(Ctx& c, Hierarchy<T>& H);
template <typename T> void mg_vcycle(Ctx& c, Hierarchy<T>& H, const double* r, double* z);
template <typename T> int mg_check_factor(Ctx& c, Hierarchy<T>& H);

// reduction slot names
enum Slot {
    SL_SUM_R1 = 0, SL_SUM_Z, SL_SUM_W, SL_G3SQ, SL_G4SQ, SL_G1SQ,
    SL_DOT = 6, SL_SLOPE_NU = 7, SL_LS = 8, SL_GAP = 9, SL_NLO = 10, SL_NHI = 11,
    SL_STAT = 12, SL_SUM_RHO = 13, SL_WT = 14, SL_AUX = 15, SL_MRALPHA = 16
};

// the interior point evaluation's reduction: kIpEvalQ quantities in slots
// kIpEvalSlot.. (sums of rho, z, W, res_3^2, the gap term, nu_lo dlo,
// nu_hi dhi, nu_lo^2, nu_hi^2; maxima of the complementarity products and of
// the bound violation)
constexpr int kIpEvalQ = 11;
constexpr int kIpEvalSlot = SL_DOT;
constexpr uint32_t kIpEvalMax = 0x600u;

}  // namespace vts

// the opaque handle of the C ABI is the context itself
struct vts_ctx : public vts::Ctx {};

