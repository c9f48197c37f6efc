// Host-side checks of libvts built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (sanitize/build.py): the
// option defaults, the finite-element tables, problem validation and
// footprints, the error returns of vts_create and the request loop for
// invalid input, and (where a device is present) one small solve, a
// checkpoint round trip and a served request.  Without a device the
// device-side calls must fail cleanly with a status, never crash.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/vts.h"
#include "../csrc/vts_internal.hpp"

static int failures = 0;
#define EXPECT(c)                                                                  \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "host_checks: %s failed (line %d)\n", #c, __LINE__); \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

struct Cant {
    int nx, ny, nz, levels;
    std::vector<uint8_t> fixed;
    std::vector<double> f;
    vts_problem p{};
    Cant(int nx_, int ny_, int nz_, int l) : nx(nx_), ny(ny_), nz(nz_), levels(l) {
        const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
        fixed.assign(3 * NX * NY * NZ, 0);
        f.assign(3 * NX * NY * NZ, 0.0);
        for (int k = 0; k < NZ; ++k)
            for (int j = 0; j < NY; ++j) {
                const int n0 = NX * (j + NY * k);
                fixed[3 * n0] = fixed[3 * n0 + 1] = fixed[3 * n0 + 2] = 1;   // x = 0 clamped
                f[3 * (n0 + nx) + 2] = (k == 0) ? -1.0 : 0.0;               // edge load
            }
        p.nx = nx;
        p.ny = ny;
        p.nz = nz;
        p.levels = l;
        p.E = 1.0;
        p.nu = 0.3;
        p.h = 1.0;
        p.fixed_host = fixed.data();
        p.f_host = f.data();
        p.V = 0.3 * nx * ny * nz;
        p.rho_lo_s = 1e-3;
        p.rho_hi_s = 1.0;
        p.precision = VTS_FP64;
    }
};

int main() {
    vts_options o;
    vts_default_options(&o);
    EXPECT(o.beta == 0.3 && o.gamma == 0.3 && o.log_path == nullptr && o.kkt_tol > 0);

    double Ke[576], Q[512], kh[8];
    vts::element_stiffness(1.0, 0.3, 1.0, Ke);
    double asym = 0.0;
    for (int a = 0; a < 24; ++a)
        for (int b = 0; b < 24; ++b) asym = std::fmax(asym, std::fabs(Ke[a * 24 + b] - Ke[b * 24 + a]));
    EXPECT(asym < 1e-14);
    EXPECT(vts::walsh_form(Ke, kh));
    vts::child_interp(Q);
    std::vector<double> Mc(8 * 576);
    vts::galerkin_child_matrices(Ke, Q, Mc.data());

    Cant good(8, 4, 4, 3);
    const size_t foot = vts_footprint_bytes(&good.p, &o);
    EXPECT(foot > 0);
    // invalid problems: rejected before any device work
    {
        Cant bad(8, 4, 4, 3);
        bad.f[3 * 10 + 1] = NAN;
        vts_ctx* c = nullptr;
        EXPECT(vts_create(&bad.p, &o, nullptr, &c) == VTS_EINVAL && c == nullptr);
        EXPECT(vts_footprint_bytes(&bad.p, &o) == foot);   // sizes only
    }
    {
        Cant bad(8, 4, 4, 3);
        bad.p.V = 10.0 * 8 * 4 * 4;   // more than rho_hi allows
        vts_ctx* c = nullptr;
        EXPECT(vts_create(&bad.p, &o, nullptr, &c) == VTS_EINVAL);
    }
    {
        Cant bad(8, 4, 4, 3);
        for (auto& v : bad.fixed) v = 0;   // no support: K(rho) singular
        vts_ctx* c = nullptr;
        EXPECT(vts_create(&bad.p, &o, nullptr, &c) == VTS_EINVAL);
    }
    {
        Cant bad(7, 4, 4, 3);   // 7 elements do not coarsen twice
        vts_ctx* c = nullptr;
        EXPECT(vts_create(&bad.p, &o, nullptr, &c) == VTS_EINVAL);
    }
    {
        // several load cases: f holds nload cases; a NaN in the second is
        // found, mixed precision and more than 4 cases are refused, and the
        // footprint (server admission) is for one case only
        Cant two(8, 4, 4, 3);
        std::vector<double> f2(two.f);
        f2.insert(f2.end(), two.f.begin(), two.f.end());
        two.p.f_host = f2.data();
        two.p.nload = 2;
        EXPECT(vts_footprint_bytes(&two.p, &o) == 0);
        vts_ctx* c = nullptr;
        f2[two.f.size() + 3 * 12 + 2] = NAN;
        EXPECT(vts_create(&two.p, &o, nullptr, &c) == VTS_EINVAL && c == nullptr);
        f2[two.f.size() + 3 * 12 + 2] = 0.0;
        two.p.precision = VTS_MIXED;
        EXPECT(vts_create(&two.p, &o, nullptr, &c) == VTS_EINVAL);
        two.p.precision = VTS_FP64;
        two.p.nload = 5;
        EXPECT(vts_create(&two.p, &o, nullptr, &c) == VTS_EINVAL);
    }
    // a valid problem: solved where a device exists, a clean device error otherwise
    int ndev = 0;
    const bool gpu = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
    vts_ctx* c = nullptr;
    const vts_status st = vts_create(&good.p, &o, nullptr, &c);
    if (gpu) {
        EXPECT(st == VTS_OK && c != nullptr);
        if (c) {
            EXPECT(vts_allocated_bytes(c) <= foot);
            vts_result r{};
            EXPECT(vts_pbm_solve(c, &r) == VTS_OK && r.kkt <= 1e-6);
            size_t bytes = 0;
            EXPECT(vts_get_state(c, nullptr, &bytes) == VTS_OK && bytes > 0);
            std::vector<char> buf(bytes);
            EXPECT(vts_get_state(c, buf.data(), &bytes) == VTS_OK);
            EXPECT(vts_set_state(c, buf.data(), bytes) == VTS_OK);
            EXPECT(vts_set_state(c, buf.data(), bytes - 8) == VTS_EINVAL);
            vts_destroy(c);
        }
    } else {
        EXPECT(st != VTS_OK && c == nullptr);
    }
    vts_server* S = nullptr;
    const vts_status ss = vts_server_create(2, size_t(1) << 28, &S);
    if (gpu) {
        EXPECT(ss == VTS_OK && S != nullptr);
        if (S) {
            Cant bad(8, 4, 4, 3);
            bad.p.V = -1.0;
            int64_t id = 0;
            EXPECT(vts_server_submit(S, &bad.p, nullptr, &id) == VTS_EINVAL);
            EXPECT(vts_server_submit(S, &good.p, &o, &id) == VTS_OK);
            vts_request_info info{};
            int got = 0;
            for (int t = 0; t < 600 && got == 0; ++t) got = vts_server_poll(S, &info, 1, 0.1);
            EXPECT(got == 1 && info.status == VTS_OK);
            int64_t gs[5];
            vts_server_group_stats(S, gs);
            vts_server_destroy(S);
        }
    } else {
        EXPECT(ss != VTS_OK && S == nullptr);
    }
    std::printf("host_checks: %s (%s)\n", failures ? "FAILED" : "ok", gpu ? "with device" : "no device");
    return failures ? 1 : 0;
}
