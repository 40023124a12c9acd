// opcount.cpp -- operation-counting build of the oracle's C core.
//
// TEST INFRASTRUCTURE ONLY (a measurement of the oracle, not part of the HIP
// path).  oracle.c is compiled as C++ with `double` replaced by a type that
// counts every floating-point add/subtract, multiply, divide, square root,
// trigonometric call and comparison.  Its main program counts
//   - the pointwise functions once each (prim, flux pieces, MC slope, fast
//     speed, Rusanov flux, sources),
//   - the spatial operator L(U) on a spherical 16 x 12 x 12 patch, per
//     interior cell, and
//   - the CFL rate per cell,
// and prints them as `key value` lines.  The operator follows the method's
// definition literally (every face reconstructs both neighbouring cells from
// three primitive conversions each; metric factors from trigonometry per
// cell), so its count is an upper bound for what an implementation must
// execute; the GPU kernel reconstructs each cell once per direction and reads
// tabulated metrics.
//
// Build and run (tests/test_oracle_opcount.py does this):
//   g++ -O1 -std=c++17 oracle/opcount.cpp -o opcount && ./opcount
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <vector>

namespace opc {
struct Counts {
    long add = 0, mul = 0, div = 0, sqrt = 0, trig = 0, cmp = 0;
    long flops() const { return add + mul + div + sqrt; }
};
Counts c;
}  // namespace opc

struct cd {
    double v;
    cd() = default;
    cd(double x) : v(x) {}
};
inline cd operator+(cd a, cd b) { opc::c.add++; return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { opc::c.add++; return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { opc::c.mul++; return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { opc::c.div++; return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }                      // sign flip: not counted
inline cd &operator+=(cd &a, cd b) { a = a + b; return a; }
inline cd &operator-=(cd &a, cd b) { a = a - b; return a; }
inline cd &operator*=(cd &a, cd b) { a = a * b; return a; }
inline cd &operator/=(cd &a, cd b) { a = a / b; return a; }
inline bool operator<(cd a, cd b) { opc::c.cmp++; return a.v < b.v; }
inline bool operator<=(cd a, cd b) { opc::c.cmp++; return a.v <= b.v; }
inline bool operator>(cd a, cd b) { opc::c.cmp++; return a.v > b.v; }
inline bool operator>=(cd a, cd b) { opc::c.cmp++; return a.v >= b.v; }
inline bool operator==(cd a, cd b) { opc::c.cmp++; return a.v == b.v; }
inline bool operator!=(cd a, cd b) { opc::c.cmp++; return a.v != b.v; }
inline cd sqrt(cd a) { opc::c.sqrt++; return cd(std::sqrt(a.v)); }
inline cd fabs(cd a) { return cd(std::fabs(a.v)); }                 // sign bit: not counted
inline cd sin(cd a) { opc::c.trig++; return cd(std::sin(a.v)); }
inline cd cos(cd a) { opc::c.trig++; return cd(std::cos(a.v)); }
inline bool isfinite(cd a) { return std::isfinite(a.v); }

#define double cd
#include "oracle.c"
#undef double

namespace {
opc::Counts snap() { return opc::c; }
opc::Counts diff(const opc::Counts &a, const opc::Counts &b)
{
    opc::Counts d;
    d.add = b.add - a.add;
    d.mul = b.mul - a.mul;
    d.div = b.div - a.div;
    d.sqrt = b.sqrt - a.sqrt;
    d.trig = b.trig - a.trig;
    d.cmp = b.cmp - a.cmp;
    return d;
}
void put(const char *key, const opc::Counts &d, double per = 1.0)
{
    std::printf("%s add %.2f mul %.2f div %.2f sqrt %.2f trig %.2f cmp %.2f flops %.2f\n", key, d.add / per,
                d.mul / per, d.div / per, d.sqrt / per, d.trig / per, d.cmp / per, d.flops() / per);
}
// a smooth magnetised wind-like state at cell (r, theta, phi)
void state(double r, double t, double ph, double u[NV])
{
    const double gamma = 1.5;
    const double rho = 300.0 / (r * r * 100.0) * (1.0 + 0.1 * std::sin(3.0 * ph) * std::sin(t));
    const double vr = 0.45 + 0.05 * std::cos(2.0 * t), vt = 0.01 * std::sin(ph), vp = -0.02 * std::sin(t);
    const double p = 0.02 * std::pow(r / 0.1, -2.0 * gamma);
    const double br = 6.5e-3 / (r * r), bt = 1e-4 * std::cos(t), bp = -6.5e-3 * std::sin(t) / r;
    u[0] = rho;
    u[1] = rho * vr;
    u[2] = rho * vt;
    u[3] = rho * vp;
    u[4] = p / (gamma - 1.0) + 0.5 * rho * (vr * vr + vt * vt + vp * vp) + 0.5 * (br * br + bt * bt + bp * bp);
    u[5] = br;
    u[6] = bt;
    u[7] = bp;
}
}  // namespace

int main()
{
    const int ni = 16, nj = 12, nk = 12;
    std::vector<cd> f0(ni + 5), f1(nj + 5), f2(nk + 5);
    const double r0 = 0.3, q = std::pow(2.0 / 0.1, 1.0 / 512.0);
    const double t0 = 1.2, dt = 2.0 * M_PI / 180.0 * 2.0 / 3.0, p0 = 0.4, dp = 2.0 * M_PI / 180.0;
    for (int m = -2; m <= ni + 2; ++m) f0[m + 2] = cd(r0 * std::pow(q, m));
    for (int m = -2; m <= nj + 2; ++m) f1[m + 2] = cd(t0 + m * dt);
    for (int m = -2; m <= nk + 2; ++m) f2[m + 2] = cd(p0 + m * dp);
    ora_patch P{};
    P.ni = ni;
    P.nj = nj;
    P.nk = nk;
    P.cartesian = 0;
    P.f0 = f0.data();
    P.f1 = f1.data();
    P.f2 = f2.data();
    P.gamma = cd(1.5);
    P.omega = cd(0.01);
    P.gm = cd(0.0045);
    P.limiter = 0;
    P.nv = NV;
    const size_t ng = (size_t)NV * (nk + 4) * (nj + 4) * (ni + 4);
    std::vector<cd> U(ng), L((size_t)NV * ni * nj * nk);
    std::vector<cd> F0((size_t)NV * nk * nj * (ni + 1)), F1((size_t)NV * nk * (nj + 1) * ni),
        F2((size_t)NV * (nk + 1) * nj * ni);
    for (int k = -2; k < nk + 2; ++k)
        for (int j = -2; j < nj + 2; ++j)
            for (int i = -2; i < ni + 2; ++i) {
                double u[NV];
                state(0.5 * (f0[i + 2].v + f0[i + 3].v), 0.5 * (f1[j + 2].v + f1[j + 3].v),
                      0.5 * (f2[k + 2].v + f2[k + 3].v), u);
                for (int v = 0; v < NV; ++v) U[gix(&P, v, i, j, k)] = cd(u[v]);
            }
    const long cells = (long)ni * nj * nk;
    std::printf("cells %ld\n", cells);
    std::printf("faces %ld\n", (long)(ni + 1) * nj * nk + (long)ni * (nj + 1) * nk + (long)ni * nj * (nk + 1));

    // pointwise pieces, once each on a cell of the patch
    cd u[NV], w[NV], w2[NV], f[NV], S[NV];
    for (int v = 0; v < NV; ++v) u[v] = U[gix(&P, v, 3, 4, 5)];
    opc::Counts a = snap();
    ora_prim(u, w, P.gamma);
    put("prim", diff(a, snap()));
    for (int v = 0; v < NV; ++v) w2[v] = w[v] * cd(1.01);
    a = snap();
    ora_fast_speed(w, 0, P.gamma);
    put("fast_speed", diff(a, snap()));
    a = snap();
    ora_rusanov(w, w2, 0, P.gamma, f);
    put("rusanov", diff(a, snap()));
    a = snap();
    ora_mc_slope(w[0], w2[0], w[0] * cd(1.03), cd(0.0), cd(1.0), cd(2.1));
    put("mc_slope", diff(a, snap()));
    a = snap();
    ora_sources(w, cd(2.0), cd(0.3), cd(0.5), cd(0.9), cd(0.2), P.omega, P.gm, S);
    put("sources", diff(a, snap()));

    // the operator and the CFL rate, per interior cell
    a = snap();
    const int bad = ora_rhs(&P, U.data(), L.data(), F0.data(), F1.data(), F2.data());
    put("rhs_per_cell", diff(a, snap()), (double)cells);
    a = snap();
    ora_max_rate(&P, U.data());
    put("rate_per_cell", diff(a, snap()), (double)cells);
    std::printf("bad %d\n", bad);
    return 0;
}
