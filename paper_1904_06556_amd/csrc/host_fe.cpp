// Host-side constant tables: the Q1 element stiffness K_e and the nodal
// interpolation weights between a coarse element and its 8 children.
//
// K_e (Section 6.2: trilinear hexahedra): isotropic linear elasticity with
// Lame constants lam = E nu/((1+nu)(1-2nu)), mu = E/(2(1+nu)) on a cube of
// side h,
//   K[3a+c][3b+d] = int lam dN_a/dx_c dN_b/dx_d + mu dN_a/dx_d dN_b/dx_c
//                 + mu delta_cd grad N_a . grad N_b,
// evaluated exactly as a product of 1D integrals of the linear shape
// functions (the integrand is separable); the result scales with h in 3D.
#include <cmath>
#include <algorithm>
#include <cstring>

#include "vts_internal.hpp"

namespace vts {

namespace {

// int_0^1 of (shape or slope of side a) * (shape or slope of side b), unit interval
double line_integral(int a, int b, bool da, bool db) {
    const double sa = a ? 1.0 : -1.0, sb = b ? 1.0 : -1.0;
    if (da && db) return sa * sb;
    if (da) return 0.5 * sa;
    if (db) return 0.5 * sb;
    return a == b ? 1.0 / 3.0 : 1.0 / 6.0;
}

// int over the unit cube of d_p N_A * d_q N_B
double cube_integral(int A, int B, int p, int q) {
    double r = 1.0;
    for (int k = 0; k < 3; ++k) {
        const int ak = (A >> k) & 1, bk = (B >> k) & 1;
        r *= line_integral(ak, bk, p == k, q == k);
    }
    return r;
}

// weight of parent-local coordinate A (0 or 1, at fine positions 0 and 2)
// for fine position t in {0, 1, 2}
double line_interp(int t, int A) {
    if (t == 1) return 0.5;
    return t == 2 * A ? 1.0 : 0.0;
}

}  // namespace

void element_stiffness(double E, double nu, double h, double* K) {
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            double gg = 0.0;
            for (int k = 0; k < 3; ++k) gg += cube_integral(a, b, k, k);
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) {
                    double v = lam * cube_integral(a, b, c, d) + mu * cube_integral(a, b, d, c);
                    if (c == d) v += mu * gg;
                    // unit cube -> side h: gradients scale 1/h, volume h^3
                    K[(3 * a + c) * 24 + 3 * b + d] = v * h;
                }
        }
}

void child_interp(double* Q) {
    for (int c = 0; c < 8; ++c)
        for (int a = 0; a < 8; ++a)
            for (int A = 0; A < 8; ++A) {
                double w = 1.0;
                for (int k = 0; k < 3; ++k) {
                    const int t = ((c >> k) & 1) + ((a >> k) & 1);
                    w *= line_interp(t, (A >> k) & 1);
                }
                Q[(c * 8 + a) * 8 + A] = w;
            }
}

void galerkin_child_matrices(const double* Ke, const double* Q, double* Mc) {
    // M_c = (Q_c x I3)^T K_e (Q_c x I3)
    for (int c = 0; c < 8; ++c) {
        const double* q = Q + c * 64;
        double* M = Mc + c * 576;
        for (int A = 0; A < 8; ++A)
            for (int i = 0; i < 3; ++i)
                for (int B = 0; B < 8; ++B)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int a = 0; a < 8; ++a) {
                            const double qa = q[a * 8 + A];
                            if (qa == 0.0) continue;
                            for (int b = 0; b < 8; ++b) {
                                const double qb = q[b * 8 + B];
                                if (qb == 0.0) continue;
                                s += qa * Ke[(3 * a + i) * 24 + 3 * b + j] * qb;
                            }
                        }
                        M[(3 * A + i) * 24 + 3 * B + j] = s;
                    }
    }
}

// Kh = H K_e H / 64 with H = H8 x I3, H8[m][a] = (-1)^popcount(m & a).
// Returns true (and the coefficients A..H) if Kh has exactly the structure
// that the tiled kernels expand: 45 non-zeros in the classes below, every
// other entry zero (relative tolerance 1e-13).
bool walsh_form(const double* Ke, double* kh8) {
    auto h8 = [](int m, int a) { return (__builtin_popcount(m & a) & 1) ? -1.0 : 1.0; };
    double Kh[24][24];
    double mx = 0.0;
    for (int r = 0; r < 24; ++r)
        for (int c = 0; c < 24; ++c) {
            double sum = 0.0;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b)
                    sum += h8(r / 3, a) * Ke[(3 * a + r % 3) * 24 + 3 * b + c % 3] * h8(b, c / 3);
            Kh[r][c] = sum / 64.0;
            mx = std::max(mx, std::fabs(Kh[r][c]));
        }
    // class of each entry: 0..7 = A..H, -1 = zero
    int cls[24][24];
    for (int r = 0; r < 24; ++r)
        for (int c = 0; c < 24; ++c) cls[r][c] = -1;
    const int nrm[3] = {3, 7, 14};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) cls[nrm[p]][nrm[q]] = (p == q) ? 0 : 1;
    const int shear[3][2] = {{4, 6}, {5, 12}, {8, 13}};
    for (auto& sp : shear)
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) cls[sp[p]][sp[q]] = 2;
    const int pair[3][2] = {{9, 20}, {10, 17}, {15, 19}};
    for (auto& pp : pair)
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) cls[pp[p]][pp[q]] = (p == q) ? 3 : 4;
    const int tri[3] = {11, 16, 18};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) cls[tri[p]][tri[q]] = (p == q) ? 5 : 6;
    for (int q = 21; q < 24; ++q) cls[q][q] = 7;
    const int rep[8][2] = {{3, 3}, {3, 7}, {4, 4}, {9, 9}, {9, 20}, {11, 11}, {11, 16}, {21, 21}};
    for (int q = 0; q < 8; ++q) kh8[q] = Kh[rep[q][0]][rep[q][1]];
    for (int r = 0; r < 24; ++r)
        for (int c = 0; c < 24; ++c) {
            const double want = cls[r][c] < 0 ? 0.0 : kh8[cls[r][c]];
            if (std::fabs(Kh[r][c] - want) > 1e-13 * mx) return false;
        }
    return true;
}

}  // namespace vts
