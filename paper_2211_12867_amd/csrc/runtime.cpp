// runtime.cpp -- host runtime and C ABI of the Icarus hot-path library.
//
// Owns the block forest of every member, the per-level metric tables, the
// device pools and the task lists the kernels walk; builds neighbour, ghost
// slab and reflux descriptors after every forest change; runs the two-stage
// step (eagerly or as a replayed HIP graph) and the regrid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <stdexcept>
#include <string>
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <unordered_map>
#include <thread>
#include <vector>

#include "../../include/icarus.h"
#include "devmem.h"
#include "kernels.h"
#include "mlp.h"

namespace {

// ---------------------------------------------------------------------------
// constants and code units (length 1 AU, speed 1000 km/s)
// ---------------------------------------------------------------------------
constexpr double kAU = 1.495978707e11;
constexpr double kV0 = 1.0e6;
constexpr double kT0 = kAU / kV0;
constexpr double kMP = 1.67262192e-27;
constexpr double kKB = 1.380649e-23;
constexpr double kRHO0 = kMP * 1.0e6;
constexpr double kP0 = kRHO0 * kV0 * kV0;
const double kMU0 = 4.0e-7 * M_PI;
const double kB0 = std::sqrt(kMU0 * kP0);

thread_local std::string g_err;

struct Error : std::runtime_error {
    ic_status code;
    Error(ic_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(x)                                                                                \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess)                                                                      \
            throw Error(IC_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));              \
    } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// device allocations: hipMalloc, or the caller's allocator
// ---------------------------------------------------------------------------
namespace {
struct DevAllocator {
    ic_alloc_fn alloc = nullptr;   // nullptr: hipMalloc / hipFree
    ic_free_fn release = nullptr;
    void *user = nullptr;
};
std::mutex g_dev_mutex;
DevAllocator g_dev_alloc;
std::unordered_map<void *, DevAllocator> g_dev_owner;   // pointers from a caller's allocator
}  // namespace

void *dev_malloc(size_t bytes)
{
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    const DevAllocator a = g_dev_alloc;
    if (!a.alloc) {
        void *p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void *p = a.alloc(bytes, a.user);
    if (p) g_dev_owner[p] = a;
    return p;
}

void dev_free(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    auto it = g_dev_owner.find(p);
    if (it == g_dev_owner.end()) {
        (void)hipFree(p);
        return;
    }
    const DevAllocator a = it->second;
    g_dev_owner.erase(it);
    a.release(p, a.user);
}

namespace {
template <class T>
struct DBuf {  // device buffer with a capacity in elements; released with its owner
    T *p = nullptr;
    size_t cap = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), cap(o.cap)
    {
        o.p = nullptr;
        o.cap = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            cap = o.cap;
            o.p = nullptr;
            o.cap = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t n)
    {
        if (n <= cap) return;
        dev_free(p);
        p = nullptr;
        cap = 0;
        p = (T *)dev_malloc(std::max<size_t>(n, 1) * sizeof(T));
        if (!p) throw Error(IC_E_NOMEM, "device allocation failed");
        cap = std::max<size_t>(n, 1);
    }
    void release()
    {
        dev_free(p);
        p = nullptr;
        cap = 0;
    }
};

// ---------------------------------------------------------------------------
// real spherical harmonics l = 1..3, orthonormal, no Condon-Shortley phase
// ---------------------------------------------------------------------------
double harmonic_sum(const double *alm, double th, double ph)
{
    const double x = std::cos(th), s = std::sin(th);
    auto P = [&](int l, int m) -> double {
        if (l == 1) return m == 0 ? x : s;
        if (l == 2) return m == 0 ? (3.0 * x * x - 1.0) / 2.0 : (m == 1 ? 3.0 * x * s : 3.0 * s * s);
        switch (m) {
        case 0: return (5.0 * x * x * x - 3.0 * x) / 2.0;
        case 1: return 1.5 * (5.0 * x * x - 1.0) * s;
        case 2: return 15.0 * x * s * s;
        default: return 15.0 * s * s * s;
        }
    };
    auto fact = [](int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; };
    double f = 0.0;
    int q = 0;
    for (int l = 1; l <= 3; ++l)
        for (int m = -l; m <= l; ++m, ++q) {
            const int a = std::abs(m);
            const double N = std::sqrt((2 * l + 1) / (4.0 * M_PI) * fact(l - a) / fact(l + a));
            double y;
            if (m == 0) y = N * P(l, 0);
            else if (m > 0) y = std::sqrt(2.0) * N * P(l, a) * std::cos(a * ph);
            else y = std::sqrt(2.0) * N * P(l, a) * std::sin(a * ph);
            f += alm[q] * y;
        }
    return f;
}

// ---------------------------------------------------------------------------
// forest keys
// ---------------------------------------------------------------------------
struct Key {
    int l, i, j, k;
    bool operator<(const Key &o) const
    {
        if (l != o.l) return l < o.l;
        if (k != o.k) return k < o.k;
        if (j != o.j) return j < o.j;
        return i < o.i;
    }
    bool operator==(const Key &o) const { return l == o.l && i == o.i && j == o.j && k == o.k; }
};

uint64_t morton(int i, int j, int k)
{
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b) {
        key |= (uint64_t)((i >> b) & 1) << (3 * b);
        key |= (uint64_t)((j >> b) & 1) << (3 * b + 1);
        key |= (uint64_t)((k >> b) & 1) << (3 * b + 2);
    }
    return key;
}

// leaves in ascending (level, Morton) order (the ABI's block order)
std::vector<Key> abi_sorted(const std::map<Key, int> &leaves)
{
    std::vector<std::pair<std::pair<int, uint64_t>, Key>> v;
    v.reserve(leaves.size());
    for (auto &kv : leaves)
        v.push_back({{kv.first.l, morton(kv.first.i, kv.first.j, kv.first.k)}, kv.first});
    std::sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    std::vector<Key> out;
    out.reserve(v.size());
    for (auto &e : v) out.push_back(e.second);
    return out;
}

// hash code of a block key (indices are below 2^20 on every level)
inline uint64_t kcode(const Key &k)
{
    return ((uint64_t)k.l << 60) | ((uint64_t)(k.i & 0xFFFFF) << 40) | ((uint64_t)(k.j & 0xFFFFF) << 20) |
           (uint64_t)(k.k & 0xFFFFF);
}

// Hash map from a nonzero 64-bit key (a kcode: level >= 1 sets the top bits)
// to an int: open addressing with linear probing, power-of-two capacity kept
// at most half full, multiplicative (Fibonacci) hashing.  Lookups only; the
// regrid never iterates over it, so its order does not matter.
struct FlatMap {
    std::vector<uint64_t> keys;
    std::vector<int> vals;
    size_t mask = 0, count = 0;
    int shift = 64;
    explicit FlatMap(size_t n = 0) { reserve(n); }
    size_t pos(uint64_t k) const { return (size_t)((k * 0x9E3779B97F4A7C15ull) >> shift); }
    void reserve(size_t n)
    {
        size_t cap = 16;
        int bits = 4;
        while (cap < 2 * n + 2) {
            cap *= 2;
            ++bits;
        }
        if (cap <= keys.size()) return;
        std::vector<uint64_t> ok(cap, 0);
        std::vector<int> ov(cap, 0);
        ok.swap(keys);
        ov.swap(vals);
        mask = cap - 1;
        shift = 64 - bits;
        for (size_t q = 0; q < ok.size(); ++q)
            if (ok[q]) {
                size_t r = pos(ok[q]);
                while (keys[r]) r = (r + 1) & mask;
                keys[r] = ok[q];
                vals[r] = ov[q];
            }
    }
    const int *find(uint64_t k) const
    {
        for (size_t q = pos(k);; q = (q + 1) & mask) {
            if (keys[q] == k) return &vals[q];
            if (!keys[q]) return nullptr;
        }
    }
    // the value of k, inserted as 0 if absent (the reference lasts until the next insertion)
    int &operator[](uint64_t k)
    {
        if (2 * (count + 1) > keys.size()) reserve(count + 1);
        for (size_t q = pos(k);; q = (q + 1) & mask) {
            if (keys[q] == k) return vals[q];
            if (!keys[q]) {
                keys[q] = k;
                vals[q] = 0;
                ++count;
                return vals[q];
            }
        }
    }
    bool insert(uint64_t k)    // true if k was absent (value 0)
    {
        const size_t before = count;
        (*this)[k];
        return count != before;
    }
    bool contains(uint64_t k) const { return find(k) != nullptr; }
};

// hashed view of a leaf map: key -> local slot
struct LeafIndex {
    FlatMap h;
    explicit LeafIndex(const std::map<Key, int> &leaves) : h(leaves.size())
    {
        for (auto &kv : leaves) h[kcode(kv.first)] = kv.second;
    }
    int find(const Key &k) const   // local slot, or -1
    {
        const int *v = h.find(kcode(k));
        return v ? *v : -1;
    }
};

struct Member {
    std::map<Key, int> leaves;     // leaf -> local slot
    std::vector<int> free_slots;
    ic_cme_cfg cme{};
};

struct HostLevel {
    int n[3];
    std::vector<RecR> r;
    std::vector<RecT> t;
    std::vector<RecP> p;
    std::vector<double> f[3];      // faces, index m + 2
    std::vector<double> wind;      // [6][nt][np]
    std::vector<double> cosd;      // [member][nt][np]
    DBuf<RecR> dr;
    DBuf<RecT> dt;
    DBuf<RecP> dp;
    DBuf<double> dwind, dcosd;
};

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// the sim
// ---------------------------------------------------------------------------
struct ic_sim {
    ic_grid_cfg grid{};
    ic_phys_cfg phys{};
    ic_wind_cfg wind{};
    ic_amr_cfg amr{};
    int nm = 1;
    int B[3] = {0, 0, 0};
    int NC = 0;
    int nv = 8;                     // conserved variables per cell: 8, or 9 with the tracer
    int nb[3] = {0, 0, 0};         // base blocks per direction
    int max_blocks = 0;
    int max_level = 1;
    bool periodic[3] = {false, false, false};
    bool cart = false;
    double r_in = 0.1;
    double omega_code = 0.0, gm_code = 0.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Launchers L{};
    bool poisoned = false;

    std::vector<HostLevel> lv;     // index = level, 1..max_level
    std::vector<Member> mem;

    // device state
    DBuf<double> U, Us, slabs, freg;
    DBuf<double> divb;              // parabolic cleaning: div B of the stage input (when C_d > 0)
    DBuf<BlockDesc> desc;
    DBuf<LevelGeo> geo;
    DBuf<MemberConst> mc;
    DBuf<int> items, nitems, mbeg, mend;
    DBuf<double> dt, t, tend, dt_last, rate;
    DBuf<int> bad;
    DBuf<unsigned long long> floors;   // per member: cells the density / pressure floor acted on
    DBuf<long> nsteps;
    DBuf<SlabTask> slab_tasks;
    DBuf<int> slab_ranges;        // [2 * (IC_MAX_LEVEL + 2)]
    DBuf<RefluxTask> rf_tasks;
    DBuf<int> rf_ranges, rf_ntasks;
    DBuf<int8_t> flags;
    DBuf<MoveTask> moves;
    DBuf<SampleDesc> sdesc;
    DBuf<double> sout, ring;
    DBuf<int> ring_count;
    int ring_cap = 1 << 16;
    long slab_stride = 0, reg_stride = 0;

    // host mirrors of the task lists
    int n_items = 0;
    int n_slabs = 0, n_regs = 0, n_rf_tasks = 0;
    int pass_lo[IC_MAX_LEVEL + 2] = {0}, pass_hi[IC_MAX_LEVEL + 2] = {0};
    bool any_prolong = false, any_reflux = false;
    std::vector<BlockDesc> hdesc;
    double zone_updates = 0.0;
    long host_steps = 0;
    long since_regrid = 0;          // steps since the last regrid (ic_advance regrids when it reaches regrid_every)
    double sample_point[3] = {1.0, 90.0, 0.0};

    // graph
    // graph: [0] one step, [1] GRAPH_STEPS steps in one replay
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<int> sig;       // launch sizes the graph was captured with
        double dt_fixed = -1.0;
    } graphs[2];
    bool graph_dirty = true;        // a buffer or the schedule changed: both graphs are stale
    bool use_graph = true;

    // learned flags
    MlpDevice mlp;
    long n_regrids = 0, n_learned = 0, n_judged = 0, n_fallbacks = 0;
    std::vector<int> fallback_left;
    double last_recall = -1.0;

    // timing
    bool timing = false;
    // stage-kernel schedule (ic_autotune / ic_set_tuning): waves per SIMD of
    // the register allocation, launch grid (0 = one work-group per work item),
    // XCD-contiguous work order
    int tune_waves = 2, tune_grid = 0, tune_xcd = 0, tune_ksplit = 1;
    // measured schedules by log2 bucket of the work-list size {waves, grid, xcd, ksplit};
    // pinned: ic_set_tuning's schedule holds whatever the work list
    std::map<int, std::array<int, 4>> tuned;
    bool tune_pinned = false;
    std::vector<hipEvent_t> ev;   // pairs
    long timed = 0;
    // pinned staging area of the table uploads (Upload) and its device copy
    char *hstage = nullptr;
    size_t hstage_cap = 0;
    DBuf<char> dstage;
    // pinned landing area of the per-step status (non-physical flags, step
    // count, t, dt), read back with one synchronisation per ic_step
    char *hstat = nullptr;
    bool tend_finite = false;       // an ic_advance end time is in tend (else "no end")
    int leaves_per_level0[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // member 0, kept by rebuild

    int slot_of(int m, int local) const { return m * max_blocks + local; }
};

namespace {

// ---------------------------------------------------------------------------
// geometry tables (host, fp64)
// ---------------------------------------------------------------------------
void build_level(ic_sim *s, int l)
{
    HostLevel &L = s->lv[l];
    const int fac = 1 << (l - 1);
    for (int d = 0; d < 3; ++d) L.n[d] = s->grid.n[d] * fac;
    const double deg = M_PI / 180.0;
    for (int d = 0; d < 3; ++d) {
        const int n = L.n[d];
        std::vector<double> &f = L.f[d];
        f.assign(n + 5, 0.0);
        double x0 = s->grid.x0[d], x1 = s->grid.x1[d];
        if (!s->cart && d > 0) {
            x0 = x0 * deg;
            x1 = x1 * deg;
        }
        if (!s->cart && d == 0 && s->grid.stretched_r) {
            const double lg = std::log(x1 / x0);
            for (int m = -2; m <= n + 2; ++m) f[m + 2] = x0 * std::exp(m * (lg / n));
        } else {
            const double h = (x1 - x0) / n;
            for (int m = -2; m <= n + 2; ++m) f[m + 2] = x0 + m * h;
        }
        f[2] = x0;
        f[n + 2] = x1;
    }
    auto xc = [&](int d, int m) { return 0.5 * (L.f[d][m + 2] + L.f[d][m + 3]); };
    auto fc = [&](int d, int m) { return L.f[d][m + 2]; };
    auto lim = [&](int d, int m, double &idm, double &idp, double &idc, double &hm, double &hp) {
        const int n = L.n[d];
        const double x = xc(d, m);
        idm = m - 1 >= -2 ? 1.0 / (x - xc(d, m - 1)) : 0.0;
        idp = m + 1 <= n + 1 ? 1.0 / (xc(d, m + 1) - x) : 0.0;
        idc = (m - 1 >= -2 && m + 1 <= n + 1) ? 1.0 / (xc(d, m + 1) - xc(d, m - 1)) : 0.0;
        hm = x - fc(d, m);
        hp = fc(d, m + 1) - x;
    };
    auto vw = [&](int d, int m) {
        const double a = fc(d, m), b = fc(d, m + 1);
        if (s->cart) return b - a;
        if (d == 0) return (b * b * b - a * a * a) / 3.0;
        if (d == 1) return std::cos(a) - std::cos(b);
        return b - a;
    };
    auto poff = [&](int d, int m) {
        const int c = floordiv(m, 2);
        const int c0 = 2 * c, c1 = 2 * c + 1;
        const double w0 = vw(d, c0), w1 = vw(d, c1);
        const double xbar = (w0 * xc(d, c0) + w1 * xc(d, c1)) / (w0 + w1);
        return xc(d, m) - xbar;
    };
    // radial
    L.r.assign(L.n[0] + 4, RecR{});
    for (int m = -2; m < L.n[0] + 2; ++m) {
        RecR &R = L.r[m + 2];
        lim(0, m, R.idm, R.idp, R.idc, R.hm, R.hp);
        const double a = fc(0, m), b = fc(0, m + 1);
        R.rc = xc(0, m);
        R.icfl = 1.0 / (b - a);
        R.vw = vw(0, m);
        R.poff = poff(0, m);
        if (s->cart) {
            R.am = R.ap = 1.0 / (b - a);
            R.rt = 1.0;
            R.irc = 1.0;
            R.r2f = 1.0;
            R.r2h = b - a;
        } else {
            const double dr3 = b * b * b - a * a * a;
            R.am = 3.0 * a * a / dr3;
            R.ap = 3.0 * b * b / dr3;
            R.rt = 1.5 * (b * b - a * a) / dr3;
            R.irc = 1.0 / R.rc;
            R.r2f = a * a;
            R.r2h = 0.5 * (b * b - a * a);
        }
    }
    // colatitude
    L.t.assign(L.n[1] + 4, RecT{});
    for (int m = -2; m < L.n[1] + 2; ++m) {
        RecT &T = L.t[m + 2];
        lim(1, m, T.idm, T.idp, T.idc, T.hm, T.hp);
        const double a = fc(1, m), b = fc(1, m + 1);
        T.tc = xc(1, m);
        T.icfl = 1.0 / (b - a);
        T.vw = vw(1, m);
        T.poff = poff(1, m);
        if (s->cart) {
            T.thm = T.thp = 1.0 / (b - a);
            T.ctil = 0.0;
            T.sinc = 1.0;
            T.cosc = 0.0;
            T.phf = 1.0;
            T.isinc = 1.0;
            T.sf = 1.0;
            T.dth = b - a;
        } else {
            const double dmu = std::cos(a) - std::cos(b);
            T.thm = std::sin(a) / dmu;
            T.thp = std::sin(b) / dmu;
            T.ctil = (std::sin(b) - std::sin(a)) / dmu;
            T.sinc = std::sin(T.tc);
            T.cosc = std::cos(T.tc);
            T.phf = (b - a) / dmu;
            T.isinc = 1.0 / T.sinc;
            T.sf = std::sin(a);
            T.dth = b - a;
        }
    }
    // longitude
    L.p.assign(L.n[2] + 4, RecP{});
    for (int m = -2; m < L.n[2] + 2; ++m) {
        RecP &P = L.p[m + 2];
        lim(2, m, P.idm, P.idp, P.idc, P.hm, P.hp);
        const double a = fc(2, m), b = fc(2, m + 1);
        P.iw = 1.0 / (b - a);
        P.vw = b - a;
        P.poff = poff(2, m);
        P.pc = xc(2, m);
    }
    // inner-boundary wind at this level's (theta, phi) centres
    const int nt = L.n[1], np = L.n[2];
    L.wind.assign((size_t)6 * nt * np, 0.0);
    L.cosd.assign((size_t)s->nm * nt * np, -2.0);
    if (!s->cart) {
        const ic_wind_cfg &w = s->wind;
        const double Bmag = w.B_nT * 1.0e-9 / kB0;
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                const double th = L.t[j + 2].tc, ph = L.p[k + 2].pc;
                double vk;
                if (w.f_max <= w.f_min) {
                    vk = w.v_min_kms;
                } else {
                    const double f = harmonic_sum(w.alm, th, ph);
                    vk = w.v_min_kms + (w.v_max_kms - w.v_min_kms) * (f - w.f_min) / (w.f_max - w.f_min);
                    vk = std::min(std::max(vk, w.v_min_kms), w.v_max_kms);
                }
                const double n = w.n_ref_cm3 * std::pow(vk / w.v_ref_kms, -2.0);
                const double vr = vk * 1.0e3 / kV0;
                const double vp = -s->omega_code * s->r_in * std::sin(th);
                const double br = Bmag / std::sqrt(1.0 + (vp / vr) * (vp / vr));
                const double bp = br * vp / vr;
                const size_t o = (size_t)j * np + k, pl = (size_t)nt * np;
                L.wind[0 * pl + o] = n * 1.0e6 * kMP / kRHO0;
                L.wind[1 * pl + o] = vr;
                L.wind[2 * pl + o] = vp;
                L.wind[3 * pl + o] = 2.0 * n * 1.0e6 * kKB * w.T_K / kP0;
                L.wind[4 * pl + o] = br;
                L.wind[5 * pl + o] = bp;
                for (int m = 0; m < s->nm; ++m) {
                    const ic_cme_cfg &c = s->mem[m].cme;
                    const double tc = c.colat_deg * deg, pc = c.lon_deg * deg;
                    L.cosd[(size_t)m * pl + o] =
                        std::sin(th) * std::sin(tc) * std::cos(ph - pc) + std::cos(th) * std::cos(tc);
                }
            }
    }
    L.dr.alloc(L.r.size());
    L.dt.alloc(L.t.size());
    L.dp.alloc(L.p.size());
    L.dwind.alloc(L.wind.size());
    L.dcosd.alloc(L.cosd.size());
    HIPCHECK(hipMemcpy(L.dr.p, L.r.data(), L.r.size() * sizeof(RecR), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.dt.p, L.t.data(), L.t.size() * sizeof(RecT), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.dp.p, L.p.data(), L.p.size() * sizeof(RecP), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.dwind.p, L.wind.data(), L.wind.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.dcosd.p, L.cosd.data(), L.cosd.size() * sizeof(double), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------------------
// descriptors and task lists after a forest change
// ---------------------------------------------------------------------------
int nblocks_at(const ic_sim *s, int l, int d) { return s->nb[d] << (l - 1); }

bool wrap_idx(const ic_sim *s, int l, int idx[3])
{
    for (int d = 0; d < 3; ++d) {
        const int n = nblocks_at(s, l, d);
        if (idx[d] < 0 || idx[d] >= n) {
            if (!s->periodic[d]) return false;
            idx[d] = ((idx[d] % n) + n) % n;
        }
    }
    return true;
}

int items_bucket(const ic_sim *s)         // log2 bucket of the work-list size
{
    int b = 0;
    while ((1 << (b + 1)) <= std::max(1, s->n_items)) ++b;
    return b;
}

void apply_tuning(ic_sim *s, int waves, int grid, int xcd, int ksplit);

// Stage-kernel schedule for the current work list: the one ic_autotune measured
// for its size bucket, else two waves per SIMD, one work-group per work item
// and a k-split until there are >= 512 work-groups (two per CU).  A schedule
// set by ic_set_tuning is kept.
void select_schedule(ic_sim *s)
{
    if (s->tune_pinned) return;
    int w = 2, g = 0, x = 0, ks = 1;
    auto it = s->tuned.find(items_bucket(s));
    if (it != s->tuned.end()) {
        w = it->second[0];
        g = it->second[1];
        x = it->second[2];
        ks = it->second[3];
    } else {
        while (ks < 4 && 2 * ks <= s->B[2] && s->n_items * ks < 512) ks *= 2;
    }
    if (w != s->tune_waves || g != s->tune_grid || x != s->tune_xcd || ks != s->tune_ksplit) apply_tuning(s, w, g, x, ks);
}

// Host worker threads kept for the life of the process (starting threads for
// every call cost ~0.1 ms each, several times per regrid).  run(n, f) calls
// f(0 .. n-1) on the workers and the calling thread; indices are handed out
// under the mutex, and run returns only when no worker holds f any more.
// One run at a time.  (A process that forks after the first run gets no
// workers in the child: runs there would wait forever; the library does not
// fork.)
class HostPool {
public:
    static HostPool &get()
    {
        static HostPool pool(std::min(16, (int)std::max(1u, std::thread::hardware_concurrency())) - 1);
        return pool;
    }
    int workers() const { return (int)th_.size(); }
    void run(int n, const std::function<void(int)> &f)
    {
        std::lock_guard<std::mutex> one(run_mu_);
        std::unique_lock<std::mutex> g(mu_);
        job_ = &f;
        n_ = n;
        next_ = 0;
        cv_work_.notify_all();
        while (next_ < n_) {
            const int i = next_++;
            ++active_;
            g.unlock();
            f(i);
            g.lock();
            --active_;
        }
        cv_done_.wait(g, [&] { return active_ == 0; });
        job_ = nullptr;
        n_ = 0;
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        for (auto &t : th_) t.join();
    }

private:
    explicit HostPool(int nw)
    {
        for (int t = 0; t < nw; ++t) th_.emplace_back([this] { loop(); });
    }
    void loop()
    {
        std::unique_lock<std::mutex> g(mu_);
        for (;;) {
            cv_work_.wait(g, [&] { return stop_ || (job_ && next_ < n_); });
            if (stop_) return;
            const int i = next_++;
            const std::function<void(int)> *f = job_;
            ++active_;
            g.unlock();
            (*f)(i);
            g.lock();
            if (--active_ == 0) cv_done_.notify_all();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_, run_mu_;
    std::condition_variable cv_work_, cv_done_;
    const std::function<void(int)> *job_ = nullptr;
    int n_ = 0, next_ = 0, active_ = 0;
    bool stop_ = false;
};

// f(m) for every member m, on the host pool when there are several members
// (members are independent); the first exception (in member order) is rethrown.
template <class F>
void for_members(int nm, F &&f)
{
    if (nm <= 1 || HostPool::get().workers() == 0) {
        for (int m = 0; m < nm; ++m) f(m);
        return;
    }
    std::vector<std::exception_ptr> err(nm);
    const std::function<void(int)> job = [&](int m) {
        try {
            f(m);
        } catch (...) {
            err[m] = std::current_exception();
        }
    };
    HostPool::get().run(nm, job);
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// Host-to-device uploads of small tables: queued, then staged in one pinned
// buffer and enqueued as asynchronous copies on the sim's stream, with one
// synchronisation at the end (a synchronous copy from pageable memory costs
// tens of microseconds each).  Sources must stay alive until flush().
// Table uploads.  The items are packed into the pinned staging area behind a
// table of where each goes, moved to the device in one copy, and placed there
// by one kernel (a copy per item cost ~10 us of launch latency each, about
// ten per regrid).
struct UpItem {
    unsigned long long dst, off, n;     // device address, offset in the staging area, bytes
};

__global__ void __launch_bounds__(256) k_scatter(const char *__restrict__ stage, int nitems)
{
    const UpItem *items = reinterpret_cast<const UpItem *>(stage);
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const UpItem e = items[i];
        if (((e.dst | e.n) & 15) == 0) {           // 16-byte pieces (staging offsets are 256-byte aligned)
            const uint4 *src = reinterpret_cast<const uint4 *>(stage + e.off);
            uint4 *dst = reinterpret_cast<uint4 *>(e.dst);
            for (unsigned long long w = threadIdx.x; w < e.n / 16; w += blockDim.x) dst[w] = src[w];
        } else {                                   // 4-byte pieces (every table holds 4-byte fields)
            const unsigned *src = reinterpret_cast<const unsigned *>(stage + e.off);
            unsigned *dst = reinterpret_cast<unsigned *>(e.dst);
            for (unsigned long long w = threadIdx.x; w < e.n / 4; w += blockDim.x) dst[w] = src[w];
        }
    }
}

struct Upload {
    ic_sim *s;
    struct Item { void *dst; const void *src; size_t n; };
    std::vector<Item> q;
    explicit Upload(ic_sim *sim) : s(sim) {}
    void add(void *dst, const void *src, size_t n)
    {
        if (n) q.push_back({dst, src, n});
    }
    void flush()
    {
        if (q.empty()) return;
        const size_t head = (q.size() * sizeof(UpItem) + 255) & ~(size_t)255;
        size_t tot = head;
        for (const Item &e : q) tot += (e.n + 255) & ~(size_t)255;
        if (tot > s->hstage_cap) {
            HIPCHECK(hipStreamSynchronize(s->stream));
            if (s->hstage) HIPCHECK(hipHostFree(s->hstage));
            s->hstage = nullptr;
            s->hstage_cap = 0;
            const size_t cap = std::max(tot + tot / 2, (size_t)1 << 16);
            if (hipHostMalloc((void **)&s->hstage, cap) != hipSuccess)
                throw Error(IC_E_NOMEM, "pinned host allocation failed");
            s->hstage_cap = cap;
            s->dstage.alloc(cap);
        }
        UpItem *tab = reinterpret_cast<UpItem *>(s->hstage);
        size_t off = head;
        int n = 0;
        for (const Item &e : q) {
            std::memcpy(s->hstage + off, e.src, e.n);
            if (e.n % 4 == 0)
                tab[n++] = UpItem{(unsigned long long)(uintptr_t)e.dst, off, e.n};
            else
                HIPCHECK(hipMemcpyAsync(e.dst, s->hstage + off, e.n, hipMemcpyHostToDevice, s->stream));
            off += (e.n + 255) & ~(size_t)255;
        }
        if (n > 0) {
            HIPCHECK(hipMemcpyAsync(s->dstage.p, s->hstage, off, hipMemcpyHostToDevice, s->stream));
            hipLaunchKernelGGL(k_scatter, dim3(std::min(n, 1024)), dim3(256), 0, s->stream, s->dstage.p, n);
            HIPCHECK(hipGetLastError());
        }
        HIPCHECK(hipStreamSynchronize(s->stream));   // the staging areas may be reused now
        q.clear();
    }
};

void rebuild(ic_sim *s)
{
    HIPCHECK(hipStreamSynchronize(s->stream));
    const int NS = s->nm * s->max_blocks;
    // descriptors are uploaded for the used slot range of each member only
    // (leaves take the lowest free slots); kernels read no other slot
    if ((int)s->hdesc.size() != NS) s->hdesc.assign(NS, BlockDesc{});
    // Per member in parallel (members share no block): slab and flux-register
    // numbers are member-local, then offset by the counts of the members
    // before it, which gives the same numbering as one pass over the members
    // in order (registers are keyed by slot, and slots belong to one member).
    struct Lists {
        std::vector<int> items;
        std::vector<SlabTask> pass1;
        std::vector<std::vector<SlabTask>> prol;
        std::vector<RefluxTask> rf;
        int nslab = 0, nreg = 0;
    };
    std::vector<Lists> ml(s->nm);
    std::vector<int> hi(s->nm, 0);
    for_members(s->nm, [&](int m) {
        Lists &L = ml[m];
        L.prol.resize(IC_MAX_LEVEL + 2);
        for (auto &kv : s->mem[m].leaves) hi[m] = std::max(hi[m], kv.second + 1);
        std::fill(s->hdesc.begin() + (size_t)m * s->max_blocks, s->hdesc.begin() + (size_t)m * s->max_blocks + hi[m],
                  BlockDesc{});
        FlatMap regs(64);                        // slot * 8 + face + 1 -> register + 1 (numbered in order of first use)
        auto get_reg = [&](int slot, int face) {
            int &v = regs[(uint64_t)slot * 8 + face + 1];
            if (v == 0) v = (int)regs.count;     // just inserted: the next number
            return v - 1;
        };
        Member &M = s->mem[m];
        const std::vector<Key> keys = abi_sorted(M.leaves);
        const LeafIndex idx(M.leaves);
        for (const Key &key : keys) {
            const int slot = s->slot_of(m, idx.find(key));
            L.items.push_back(slot);
            BlockDesc &bd = s->hdesc[slot];
            bd.level = key.l;
            bd.member = m;
            const int bi[3] = {key.i, key.j, key.k};
            for (int d = 0; d < 3; ++d) bd.org[d] = bi[d] * s->B[d];
            bd.reflux_mask = 0;
            for (int f = 0; f < 6; ++f) bd.freg[f] = -1;
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1, side = f & 1;
                int nbi[3] = {bi[0], bi[1], bi[2]};
                nbi[d] += side ? 1 : -1;
                int w[3] = {nbi[0], nbi[1], nbi[2]};
                if (!wrap_idx(s, key.l, w)) {
                    const int kind = s->grid.bc[d][side];
                    if (kind == IC_BC_INNER) {
                        SlabTask tk{};
                        tk.type = SLAB_INNER;
                        tk.slab = L.nslab++;
                        tk.slot = slot;
                        tk.face = f;
                        bd.nbr[f] = slab_code(tk.slab);
                        L.pass1.push_back(tk);
                    } else {
                        bd.nbr[f] = NBR_OUTFLOW;
                    }
                    continue;
                }
                const int same = idx.find(Key{key.l, w[0], w[1], w[2]});
                if (same >= 0) {
                    bd.nbr[f] = s->slot_of(m, same);
                    continue;
                }
                const Key ckey{key.l - 1, w[0] >> 1, w[1] >> 1, w[2] >> 1};
                const int coarse = key.l > 1 ? idx.find(ckey) : -1;
                if (coarse >= 0) {
                    const int cslot = s->slot_of(m, coarse);
                    SlabTask tk{};
                    tk.type = SLAB_PROLONG;
                    tk.slab = L.nslab++;
                    tk.slot = slot;
                    tk.face = f;
                    tk.src[0] = cslot;
                    const int corg[3] = {ckey.i * s->B[0], ckey.j * s->B[1], ckey.k * s->B[2]};
                    for (int e = 0; e < 3; ++e) {
                        int cw = 0;
                        if (e == d && nbi[d] != w[d]) {
                            const int nc = s->lv[key.l - 1].n[d];
                            cw = side ? -nc : nc;
                        }
                        tk.cwrap[e] = cw;
                        tk.shift[e] = cw - corg[e];
                    }
                    bd.nbr[f] = slab_code(tk.slab);
                    bd.freg[f] = get_reg(slot, f);
                    L.prol[key.l].push_back(tk);
                    continue;
                }
                // finer neighbours: the four children of the neighbour region on this face
                SlabTask tk{};
                tk.type = SLAB_RESTRICT;
                tk.slab = L.nslab++;
                tk.slot = slot;
                tk.face = f;
                const int e1 = tan1(d), e2 = tan2(d);
                RefluxTask rt{};
                rt.slot = slot;
                rt.face = f;
                for (int q = 0; q < 4; ++q) {
                    int c[3];
                    c[d] = 2 * w[d] + (side ? 0 : 1);
                    c[e1] = 2 * w[e1] + (q & 1);
                    c[e2] = 2 * w[e2] + (q >> 1);
                    const int fl = idx.find(Key{key.l + 1, c[0], c[1], c[2]});
                    if (fl < 0) throw Error(IC_E_INVALID, "forest violates 2:1 balance");
                    tk.src[q] = s->slot_of(m, fl);
                    rt.freg[q] = get_reg(tk.src[q], f ^ 1);
                }
                for (int e = 0; e < 3; ++e) {
                    tk.shift[e] = 0;
                    tk.fbase[e] = 2 * w[e];
                }
                tk.fbase[d] = 2 * w[d] + (side ? 0 : 1);
                if (nbi[d] != w[d]) {
                    const int n = s->lv[key.l].n[d];
                    tk.shift[d] = side ? -n : n;
                }
                bd.nbr[f] = slab_code(tk.slab);
                bd.freg[f] = get_reg(slot, f);
                bd.reflux_mask |= 1 << f;
                rt.creg = bd.freg[f];
                L.rf.push_back(rt);
                L.pass1.push_back(tk);
            }
        }
        L.nreg = (int)regs.count;
    });
    std::vector<int> slab_off(s->nm + 1, 0), reg_off(s->nm + 1, 0);
    for (int m = 0; m < s->nm; ++m) {
        slab_off[m + 1] = slab_off[m] + ml[m].nslab;
        reg_off[m + 1] = reg_off[m] + ml[m].nreg;
    }
    // offsets and concatenation in member order (serial: cheap next to the leaf loop)
    std::vector<int> items, mbeg(s->nm), mend(s->nm);
    std::vector<SlabTask> pass1;
    std::vector<std::vector<SlabTask>> prol(IC_MAX_LEVEL + 2);
    std::vector<RefluxTask> rf;
    for (int m = 0; m < s->nm; ++m) {
        Lists &L = ml[m];
        const int so = slab_off[m], ro = reg_off[m];
        if (so != 0 || ro != 0) {
            for (int slot : L.items) {
                BlockDesc &bd = s->hdesc[slot];
                for (int f = 0; f < 6; ++f) {
                    if (bd.nbr[f] <= slab_code(0)) bd.nbr[f] = slab_code(nbr_slab(bd.nbr[f]) + so);
                    if (bd.freg[f] >= 0) bd.freg[f] += ro;
                }
            }
            for (auto &tk : L.pass1) tk.slab += so;
            for (auto &v : L.prol)
                for (auto &tk : v) tk.slab += so;
            for (auto &rt : L.rf) {
                rt.creg += ro;
                for (int q = 0; q < 4; ++q) rt.freg[q] += ro;
            }
        }
        mbeg[m] = (int)items.size();
        items.insert(items.end(), L.items.begin(), L.items.end());
        mend[m] = (int)items.size();
        pass1.insert(pass1.end(), L.pass1.begin(), L.pass1.end());
        for (int l = 0; l < IC_MAX_LEVEL + 2; ++l) prol[l].insert(prol[l].end(), L.prol[l].begin(), L.prol[l].end());
        rf.insert(rf.end(), L.rf.begin(), L.rf.end());
    }
    const int nslab = slab_off[s->nm];
    // task lists: pass 1 (inner + restrict), then prolongation by owner level
    std::vector<SlabTask> all = pass1;
    s->pass_lo[0] = 0;
    s->pass_hi[0] = (int)pass1.size();
    s->any_prolong = false;
    for (int l = 2; l <= s->max_level; ++l) {
        s->pass_lo[l] = (int)all.size();
        all.insert(all.end(), prol[l].begin(), prol[l].end());
        s->pass_hi[l] = (int)all.size();
        if (!prol[l].empty()) s->any_prolong = true;
    }
    std::sort(rf.begin(), rf.end(), [](const RefluxTask &a, const RefluxTask &b) {
        return a.slot != b.slot ? a.slot < b.slot : a.face < b.face;
    });
    // per reflux task, the range of its coarse block's tasks (a work-group per
    // task; a cell on several of the block's faces is corrected by the last)
    std::vector<int> rfr(2 * rf.size());
    for (size_t q = 0; q < rf.size();) {
        size_t e = q;
        while (e < rf.size() && rf[e].slot == rf[q].slot) ++e;
        for (size_t p = q; p < e; ++p) {
            rfr[2 * p] = (int)q;
            rfr[2 * p + 1] = (int)e;
        }
        q = e;
    }
    s->n_items = (int)items.size();
    s->n_slabs = nslab;
    s->n_regs = reg_off[s->nm];
    s->n_rf_tasks = (int)rf.size();
    s->any_reflux = !rf.empty();

    // capacities (growing a buffer invalidates a captured graph)
    auto grow = [&](auto &buf, size_t need) {
        if (need > buf.cap) {
            buf.alloc(std::max(need + need / 2, (size_t)64));
            s->graph_dirty = true;
        }
    };
    grow(s->slabs, (size_t)std::max(nslab, 1) * s->slab_stride);
    grow(s->freg, (size_t)std::max(s->n_regs, 1) * s->reg_stride);
    grow(s->slab_tasks, all.size() + 1);
    grow(s->rf_tasks, rf.size() + 1);
    grow(s->rf_ranges, rfr.size() + 2);

    Upload up(s);
    for (int m = 0; m < s->nm; ++m)
        up.add(s->desc.p + (size_t)m * s->max_blocks, s->hdesc.data() + (size_t)m * s->max_blocks,
               hi[m] * sizeof(BlockDesc));
    up.add(s->items.p, items.data(), items.size() * sizeof(int));
    up.add(s->nitems.p, &s->n_items, sizeof(int));
    up.add(s->mbeg.p, mbeg.data(), s->nm * sizeof(int));
    up.add(s->mend.p, mend.data(), s->nm * sizeof(int));
    up.add(s->slab_tasks.p, all.data(), all.size() * sizeof(SlabTask));
    std::vector<int> ranges(2 * (IC_MAX_LEVEL + 2), 0);
    for (int l = 0; l <= IC_MAX_LEVEL + 1; ++l) {
        if (l == 0 || (l >= 2 && l <= s->max_level)) {
            ranges[2 * l] = s->pass_lo[l];
            ranges[2 * l + 1] = s->pass_hi[l];
        }
    }
    // entry 1 (no level 1 prolongation exists): every prolongation task of every
    // level in one pass.  A prolongation stencil reads its coarse parent and
    // the parent's axis neighbours: interior cells, restriction or inner
    // slabs (pass 1), never another prolongation slab -- that would need a
    // level-(l-2) block touching a level-l block along an edge, which the
    // 2:1 balance over all 26 neighbours rules out.
    ranges[2] = s->pass_lo[2];
    ranges[3] = s->pass_hi[s->max_level];
    up.add(s->slab_ranges.p, ranges.data(), ranges.size() * sizeof(int));
    up.add(s->rf_tasks.p, rf.data(), rf.size() * sizeof(RefluxTask));
    up.add(s->rf_ranges.p, rfr.data(), rfr.size() * sizeof(int));
    up.add(s->rf_ntasks.p, &s->n_rf_tasks, sizeof(int));
    up.flush();
    for (int l = 0; l < 8; ++l) s->leaves_per_level0[l] = 0;
    for (auto &kv : s->mem[0].leaves)
        if (kv.first.l <= 8) s->leaves_per_level0[kv.first.l - 1]++;
    select_schedule(s);
}

// ---------------------------------------------------------------------------
// kernel arguments and the step
// ---------------------------------------------------------------------------
KArgs base_args(ic_sim *s)
{
    KArgs a{};
    a.desc = s->desc.p;
    a.slabs = s->slabs.p;
    a.freg = s->freg.p;
    a.geo = s->geo.p;
    a.mc = s->mc.p;
    a.items = s->items.p;
    a.nitems = s->nitems.p;
    a.dt = s->dt.p;
    a.t = s->t.p;
    a.rate = s->rate.p;
    a.bad = s->bad.p;
    a.floors = s->floors.p;
    a.slab_stride = s->slab_stride;
    a.reg_stride = s->reg_stride;
    a.gas.g = s->phys.gamma;
    a.gas.gm1 = s->phys.gamma - 1.0;
    a.gas.igm1 = 1.0 / (s->phys.gamma - 1.0);
    a.omega = s->omega_code;
    a.gm = s->gm_code;
    a.rho_floor = s->phys.rho_floor;
    a.p_floor = s->phys.p_floor;
    a.cart = s->cart ? 1 : 0;
    a.xcd_order = s->tune_xcd;
    a.ksplit = s->tune_ksplit;
    a.divb = s->divb.p;
    a.divb_cd = s->phys.divb_cd;
    a.nv = s->nv;
    return a;
}

int grid_for(int n, int cap) { return std::max(1, std::min(n, cap)); }

// Launch size for n work items, rounded up to one of 8 steps per power of two
// (1400 -> 1408, 1433 -> 1536): the kernels stride over device-side counts and
// let surplus work-groups exit, so a size that covers n is enough, and a
// captured step graph survives regrids that move n within one step.
int quant_grid(int n, int cap)
{
    n = std::max(1, n);
    int b = 1;
    while (b * 2 <= n) b *= 2;
    const int step = std::max(1, b / 8);
    return std::max(1, std::min((n + step - 1) / step * step, cap));
}

// stage launch: one work-group per work item, or a persistent grid of
// tune_grid work-groups striding over the work list
int stage_grid(const ic_sim *s)
{
    const int n = quant_grid(s->n_items * s->tune_ksplit, 1 << 30);
    return s->tune_grid > 0 ? std::min(n, s->tune_grid) : n;
}

// ghost-slab launches: one work-group per task of the pass (the kernels
// stride over the device-side task ranges, so any size is correct)
int slab_grid(const ic_sim *s, int pass)
{
    const int n = pass == 0 ? s->pass_hi[0] - s->pass_lo[0]
                            : (s->max_level > 1 ? s->pass_hi[s->max_level] - s->pass_lo[2] : 0);
    return quant_grid(n, 8192);
}

int reflux_grid(const ic_sim *s) { return s->any_reflux ? quant_grid(s->n_rf_tasks, 8192) : 0; }

// launch sizes of a step; a captured step graph is re-made when they change
std::vector<int> launch_sig(const ic_sim *s)
{
    return {stage_grid(s), slab_grid(s, 0), slab_grid(s, 1), reflux_grid(s)};
}

void fill_ghosts(ic_sim *s, double *Uin, double tfrac)
{
    KArgs a = base_args(s);
    a.U = Uin;
    a.tfrac = tfrac;
    s->L.slabs(dim3(slab_grid(s, 0)), s->stream, a, s->slab_tasks.p, s->slab_ranges.p, 0);
    if (s->max_level > 1) s->L.slabs(dim3(slab_grid(s, 1)), s->stream, a, s->slab_tasks.p, s->slab_ranges.p + 2, 1);
}

void stage(ic_sim *s, double *Uin, double *Ubase, double *Uout, double alpha, int want_rate)
{
    // with the cleaning, the CFL maxima and the output check follow it (clean)
    if (s->phys.divb_cd > 0.0) want_rate = 0;
    KArgs a = base_args(s);
    a.U = Uin;
    a.Ubase = Ubase;
    a.Uout = Uout;
    a.alpha = alpha;
    a.want_rate = want_rate;
    const int g = stage_grid(s);
    if (s->timing) {
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, s->stream));
        s->L.stage(dim3(g), s->stream, a, s->tune_waves, s->phys.limiter);
        HIPCHECK(hipEventRecord(e1, s->stream));
        s->ev.push_back(e0);
        s->ev.push_back(e1);
    } else {
        s->L.stage(dim3(g), s->stream, a, s->tune_waves, s->phys.limiter);
    }
    if (s->any_reflux) s->L.reflux(dim3(reflux_grid(s)), s->stream, a, s->rf_tasks.p, s->rf_ranges.p, s->rf_ntasks.p);
}

// div B of the stage input Uin (ghosts filled) into s->divb
void divb(ic_sim *s, double *Uin)
{
    KArgs a = base_args(s);
    a.U = Uin;
    s->L.divb(dim3(quant_grid(s->n_items, 1 << 30)), s->stream, a);
}

// parabolic cleaning of the stage result Uout from the stage input Uin (its
// div B in s->divb); want_rate: the stage's output check and CFL maxima here
void clean(ic_sim *s, double *Uin, double *Uout, double alpha, int want_rate)
{
    KArgs a = base_args(s);
    a.U = Uin;
    a.Uout = Uout;
    a.alpha = alpha;
    a.want_rate = want_rate;
    s->L.clean(dim3(quant_grid(s->n_items, 1 << 30)), s->stream, a);
}

// Hancock predictor into Uout (the first stage of the one-step form): one
// work-group per work item
void predictor(ic_sim *s, double *Uin, double *Uout)
{
    KArgs a = base_args(s);
    a.U = Uin;
    a.Ubase = Uin;
    a.Uout = Uout;
    a.alpha = 0.5;
    a.want_rate = 0;
    s->L.hancock(dim3(quant_grid(s->n_items, 1 << 30)), s->stream, a, s->phys.limiter);
}

void enqueue_rate(ic_sim *s)
{
    KArgs a = base_args(s);
    a.U = s->U.p;
    s->L.rate(dim3(grid_for(s->n_items, 16384)), s->stream, a);
}

// sample at the point; end_step: the same launch first ends the step (t += dt)
void enqueue_sample(ic_sim *s, int record, bool end_step = false)
{
    KArgs a = base_args(s);
    a.U = s->U.p;
    s->L.sample(dim3(s->nm), s->stream, a, s->sdesc.p, s->nm, s->sout.p, s->ring.p, s->ring_count.p,
                s->ring_cap, record, end_step ? s->t.p : nullptr, end_step ? s->nsteps.p : nullptr);
}

void enqueue_step(ic_sim *s, double dt_fixed_code, bool record)
{
    KArgs a = base_args(s);
    launch_dt(s->stream, a, s->mbeg.p, s->mend.p, s->nm, s->phys.cfl, dt_fixed_code, s->tend.p, s->dt_last.p);
    const bool cleaning = s->phys.divb_cd > 0.0;
    fill_ghosts(s, s->U.p, 0.0);
    if (cleaning) divb(s, s->U.p);
    if (s->phys.scheme == IC_SCHEME_HANCOCK) predictor(s, s->U.p, s->Us.p);
    else stage(s, s->U.p, s->U.p, s->Us.p, 0.5, 0);
    if (cleaning) clean(s, s->U.p, s->Us.p, 0.5, 0);
    fill_ghosts(s, s->Us.p, 0.5);
    if (cleaning) divb(s, s->Us.p);
    stage(s, s->Us.p, s->U.p, s->U.p, 1.0, 1);
    if (cleaning) clean(s, s->Us.p, s->U.p, 1.0, 1);
    if (record) enqueue_sample(s, 1, true);       // ends the step and records the sample
    else launch_time(s->stream, s->t.p, s->dt.p, s->nsteps.p, s->nm);
}

// Steps per replay of the multi-step graph: one graph launch per step leaves
// a gap of ~8 us before each step's first kernel, as long as a short step on
// a small grid.  Within a replay the steps follow each other on the device
// (dt, clipped to the end time, is reduced on the device; a member past its
// end time takes dt = 0 and its kernels do nothing).
constexpr int GRAPH_STEPS = 5;

void release_graphs(ic_sim *s)
{
    for (auto &g : s->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
    }
}

// nsteps (1 or GRAPH_STEPS) steps, each recording the sample, in one replay of
// a captured graph (re-captured when a buffer, the schedule or a launch size
// changed), or enqueued directly while kernel timing is on
void run_steps(ic_sim *s, double dt_fixed_code, int nsteps)
{
    if (s->timing || !s->use_graph) {
        for (int q = 0; q < nsteps; ++q) enqueue_step(s, dt_fixed_code, true);
        return;
    }
    if (s->graph_dirty) {
        release_graphs(s);
        s->graph_dirty = false;
    }
    auto &G = s->graphs[nsteps > 1 ? 1 : 0];
    if (G.exec == nullptr || G.dt_fixed != dt_fixed_code || G.sig != launch_sig(s)) {
        if (G.exec) HIPCHECK(hipGraphExecDestroy(G.exec));
        G.exec = nullptr;
        hipGraph_t g;
        HIPCHECK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        for (int q = 0; q < nsteps; ++q) enqueue_step(s, dt_fixed_code, true);
        HIPCHECK(hipStreamEndCapture(s->stream, &g));
        HIPCHECK(hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0));
        HIPCHECK(hipGraphDestroy(g));
        G.dt_fixed = dt_fixed_code;
        G.sig = launch_sig(s);
    }
    HIPCHECK(hipGraphLaunch(G.exec, s->stream));
}

std::string describe_bad(ic_sim *s, int m, int slot, int cell);

void check_bad(ic_sim *s)
{
    std::vector<int> bad(2 * s->nm);
    HIPCHECK(hipMemcpyAsync(bad.data(), s->bad.p, 2 * s->nm * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
    for (int m = 0; m < s->nm; ++m)
        if (bad[2 * m]) {
            s->poisoned = true;
            throw Error(IC_E_UNPHYSICAL, "member " + std::to_string(m) +
                                             ": a leaf cell has rho <= 0, p <= 0 or a non-finite value" +
                                             describe_bad(s, m, bad[2 * m] - 1, bad[2 * m + 1]));
        }
}

void fill_info(ic_sim *s, ic_info *out)
{
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    long st = 0;
    double t = 0, dtl = 0;
    HIPCHECK(hipMemcpyAsync(&st, s->nsteps.p, sizeof(long), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipMemcpyAsync(&t, s->t.p, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipMemcpyAsync(&dtl, s->dt_last.p, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
    out->steps = st;
    out->t_s = t * kT0;
    out->dt_s = dtl * kT0;
    out->zone_updates = s->zone_updates;
    out->leaves = (int)s->mem[0].leaves.size();
    for (int l = 0; l < 8; ++l) out->leaves_per_level[l] = s->leaves_per_level0[l];
}

long total_cells(const ic_sim *s)
{
    long n = 0;
    for (auto &M : s->mem) n += (long)M.leaves.size() * s->NC;
    return n;
}

// ---------------------------------------------------------------------------
// sampling descriptor (host side: which cells, which weights)
// ---------------------------------------------------------------------------
const Key *covering_leaf(const Member &M, int l, int bi, int bj, int bk, Key *out)
{
    int i = bi, j = bj, k = bk;
    for (int q = l; q >= 1; --q) {
        auto it = M.leaves.find(Key{q, i, j, k});
        if (it != M.leaves.end()) {
            *out = it->first;
            return out;
        }
        i >>= 1; j >>= 1; k >>= 1;
    }
    return nullptr;
}

bool build_sample(ic_sim *s, int m, double r, double th_deg, double ph_deg, SampleDesc *sd)
{
    const Member &M = s->mem[m];
    double x[3] = {r, th_deg, ph_deg};
    if (!s->cart) {
        x[1] = th_deg * (M_PI / 180.0);
        x[2] = ph_deg * (M_PI / 180.0);
    }
    // finest leaf containing the point
    int lvl = -1;
    for (int l = s->max_level; l >= 1 && lvl < 0; --l) {
        const HostLevel &L = s->lv[l];
        int idx[3];
        for (int d = 0; d < 3; ++d) {
            const std::vector<double> &f = L.f[d];
            const int n = L.n[d];
            double xx = x[d];
            if (s->periodic[d]) {
                const double P = f[n + 2] - f[2];
                xx = std::fmod(xx - f[2], P);
                if (xx < 0) xx += P;
                xx += f[2];
            }
            if (xx < f[2] || xx > f[n + 2]) return false;
            int c = (int)(std::upper_bound(f.begin() + 2, f.begin() + n + 3, xx) - (f.begin() + 2)) - 1;
            idx[d] = std::min(std::max(c, 0), n - 1);
        }
        if (M.leaves.count(Key{l, idx[0] / s->B[0], idx[1] / s->B[1], idx[2] / s->B[2]})) lvl = l;
    }
    if (lvl < 0) return false;
    const HostLevel &L = s->lv[lvl];
    int lo[3];
    double wt[3];
    for (int d = 0; d < 3; ++d) {
        const int n = L.n[d];
        std::vector<double> c(n);
        for (int q = 0; q < n; ++q) c[q] = 0.5 * (L.f[d][q + 2] + L.f[d][q + 3]);
        if (s->periodic[d]) {
            const double P = L.f[d][n + 2] - L.f[d][2];
            double xx = std::fmod(x[d] - c[0], P);
            if (xx < 0) xx += P;
            xx += c[0];
            int q = (int)(std::upper_bound(c.begin(), c.end(), xx) - c.begin()) - 1;
            lo[d] = q;
            const double chi = q >= n - 1 ? c[0] + P : c[q + 1];
            wt[d] = (xx - c[q]) / (chi - c[q]);
        } else {
            int q = (int)(std::upper_bound(c.begin(), c.end(), x[d]) - c.begin()) - 1;
            if (q < 0) { lo[d] = 0; wt[d] = 0.0; }
            else if (q >= n - 1) { lo[d] = n - 2; wt[d] = 1.0; }
            else { lo[d] = q; wt[d] = (x[d] - c[q]) / (c[q + 1] - c[q]); }
        }
    }
    for (int o = 0; o < 8; ++o) {
        const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
        int g[3];
        double w = 1.0;
        for (int d = 0; d < 3; ++d) {
            g[d] = lo[d] + off[d];
            if (s->periodic[d]) g[d] = ((g[d] % L.n[d]) + L.n[d]) % L.n[d];
            w *= off[d] ? wt[d] : 1.0 - wt[d];
        }
        SampleEntry &e = sd->e[o];
        e.w = w;
        Key c;
        if (covering_leaf(M, lvl, g[0] / s->B[0], g[1] / s->B[1], g[2] / s->B[2], &c)) {
            const int sh = lvl - c.l;
            e.kind = 0;
            e.slot = s->slot_of(m, M.leaves.at(c));
            e.level = c.l;
            const int cg[3] = {g[0] >> sh, g[1] >> sh, g[2] >> sh};
            e.cell[0] = cg[0] - c.i * s->B[0];
            e.cell[1] = cg[1] - c.j * s->B[1];
            e.cell[2] = cg[2] - c.k * s->B[2];
        } else {
            // covered by finer leaves: mean of the 8 children (one level finer)
            const int fg[3] = {2 * g[0], 2 * g[1], 2 * g[2]};
            Key f{lvl + 1, fg[0] / s->B[0], fg[1] / s->B[1], fg[2] / s->B[2]};
            auto it = M.leaves.find(f);
            if (it == M.leaves.end()) return false;
            e.kind = 1;
            e.slot = s->slot_of(m, it->second);
            e.level = lvl + 1;
            for (int d = 0; d < 3; ++d) e.g[d] = fg[d];
            e.cell[0] = fg[0] - f.i * s->B[0];
            e.cell[1] = fg[1] - f.j * s->B[1];
            e.cell[2] = fg[2] - f.k * s->B[2];
        }
    }
    sd->valid = 1;
    return true;
}

void update_sample_desc(ic_sim *s)
{
    std::vector<SampleDesc> sd(s->nm);
    for (int m = 0; m < s->nm; ++m) {
        std::memset(&sd[m], 0, sizeof(SampleDesc));
        if (!build_sample(s, m, s->sample_point[0], s->sample_point[1], s->sample_point[2], &sd[m]))
            sd[m].valid = 0;
    }
    Upload up(s);
    up.add(s->sdesc.p, sd.data(), s->nm * sizeof(SampleDesc));
    up.flush();
}

// ---------------------------------------------------------------------------
// regrid (host forest logic, device data movement)
// ---------------------------------------------------------------------------
struct Forest {
    const ic_sim *s;
    const std::map<Key, int> &leaves;
    int maxl;
    LeafIndex index;
    Forest(const ic_sim *s_, const std::map<Key, int> &l, int m) : s(s_), leaves(l), maxl(m), index(l) {}
    int nblk(int l, int d) const { return s->nb[d] << (l - 1); }
    bool has(const Key &k) const { return index.find(k) >= 0; }
    bool wrap(int l, int idx[3]) const { return wrap_idx(s, l, idx); }
    // closures of a and b touch (face, edge or corner), through periodic directions
    bool touch(const Key &a, const Key &b) const
    {
        const int L = std::max(std::max(a.l, b.l), maxl);
        const int sa = 1 << (L - a.l), sb = 1 << (L - b.l);
        const int ai[3] = {a.i, a.j, a.k}, bi[3] = {b.i, b.j, b.k};
        for (int d = 0; d < 3; ++d) {
            const int n = nblk(L, d);
            const int a0 = ai[d] * sa, a1 = (ai[d] + 1) * sa, b0 = bi[d] * sb, b1 = (bi[d] + 1) * sb;
            bool ok = false;
            const int shifts[3] = {-n, 0, n};
            for (int q = 0; q < 3; ++q) {
                if (!s->periodic[d] && q != 1) continue;
                if (a0 <= b1 + shifts[q] && b0 + shifts[q] <= a1) ok = true;
            }
            if (!ok) return false;
        }
        return true;
    }
    // leaves at exactly `level` whose closure touches `leaf`
    std::vector<Key> touching(const Key &leaf, int level) const
    {
        std::vector<Key> out;
        int lo[3], hi[3];
        const int li[3] = {leaf.i, leaf.j, leaf.k};
        if (level <= leaf.l) {
            const int sh = leaf.l - level;
            for (int d = 0; d < 3; ++d) { lo[d] = (li[d] >> sh) - 1; hi[d] = (li[d] >> sh) + 1; }
        } else {
            const int sh = level - leaf.l;
            for (int d = 0; d < 3; ++d) { lo[d] = (li[d] << sh) - 1; hi[d] = ((li[d] + 1) << sh); }
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    int w[3] = {i, j, k};
                    if (!wrap(level, w)) continue;
                    Key c{level, w[0], w[1], w[2]};
                    if (!has(c) || c == leaf) continue;
                    if (std::find(out.begin(), out.end(), c) != out.end()) continue;
                    if (touch(leaf, c)) out.push_back(c);
                }
        return out;
    }
    std::vector<Key> face_neighbours(const Key &leaf, int d, int side) const
    {
        int idx[3] = {leaf.i, leaf.j, leaf.k};
        idx[d] += side ? 1 : -1;
        if (!wrap(leaf.l, idx)) return {};
        for (int l = leaf.l, i = idx[0], j = idx[1], k = idx[2]; l >= 1; --l, i >>= 1, j >>= 1, k >>= 1)
            if (has(Key{l, i, j, k})) return {Key{l, i, j, k}};
        std::vector<Key> out;
        std::vector<Key> stack{Key{leaf.l, idx[0], idx[1], idx[2]}};
        while (!stack.empty()) {
            Key c = stack.back();
            stack.pop_back();
            for (int o = 0; o < 8; ++o) {
                const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
                if (off[d] != (side ? 0 : 1)) continue;
                Key ch{c.l + 1, 2 * c.i + off[0], 2 * c.j + off[1], 2 * c.k + off[2]};
                if (ch.l > maxl + 1) continue;
                if (has(ch)) out.push_back(ch);
                else stack.push_back(ch);
            }
        }
        return out;
    }
};

// where the first non-physical cell of member m sits: leaf, cell, its current
// conserved values and the levels of the leaf's face neighbours
std::string describe_bad(ic_sim *s, int m, int slot, int cell)
{
    std::string out;
    const Member &M = s->mem[m];
    const Key *key = nullptr;
    for (auto &kv : M.leaves)
        if (s->slot_of(m, kv.second) == slot) key = &kv.first;
    char buf[512];
    if (!key) return " (slot " + std::to_string(slot) + " is no current leaf)";
    const int ci = cell % s->B[0], cj = (cell / s->B[0]) % s->B[1], ck = cell / (s->B[0] * s->B[1]);
    std::snprintf(buf, sizeof buf, " at leaf (level %d, %d, %d, %d) cell (%d, %d, %d)", key->l, key->i, key->j, key->k,
                  ci, cj, ck);
    out += buf;
    const size_t nc = (size_t)s->B[0] * s->B[1] * s->B[2];
    double u[8];
    for (int v = 0; v < 8; ++v)
        if (hipMemcpy(&u[v], s->U.p + ((size_t)slot * s->nv + v) * nc + cell, sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return out;
    std::snprintf(buf, sizeof buf, "; U = (%.4g, %.4g, %.4g, %.4g, %.4g, %.4g, %.4g, %.4g)", u[0], u[1], u[2], u[3],
                  u[4], u[5], u[6], u[7]);
    out += buf;
    Forest F{s, M.leaves, s->max_level};
    out += "; face-neighbour levels";
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) {
            out += d == 0 && side == 0 ? " " : "/";
            std::string lv;
            for (const Key &n : F.face_neighbours(*key, d, side)) lv += (lv.empty() ? "" : ",") + std::to_string(n.l);
            out += lv.empty() ? "-" : lv;
        }
    return out;
}


void regrid_member(ic_sim *s, int m, const FlatMap &flags_in, int buffer_blocks,
                   std::vector<MoveTask> &moves, std::vector<int> &to_free)
{
    Member &M = s->mem[m];
    Forest F{s, M.leaves, s->max_level};
    // flags per leaf (hashed); every pass below walks the leaves in key order
    FlatMap f(2 * M.leaves.size() + 1);
    for (auto &kv : M.leaves) {
        const int *fi = flags_in.find(kcode(kv.first));
        int v = fi ? *fi : 0;
        if (v == 1 && kv.first.l >= s->max_level) v = 0;
        if (v == -1 && kv.first.l <= 1) v = 0;
        f[kcode(kv.first)] = v;
    }
    // buffer
    std::vector<Key> orig;
    for (auto &kv : M.leaves) if (f[kcode(kv.first)] == 1) orig.push_back(kv.first);
    for (const Key &b : orig)
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side)
                for (const Key &n : F.face_neighbours(b, d, side)) {
                    int &fn = f[kcode(n)];
                    if (buffer_blocks && n.l < s->max_level && n.l <= b.l) fn = 1;
                    else if (fn == -1) fn = 0;
                }
    // 2:1 closure
    bool changed = true;
    while (changed) {
        changed = false;
        for (auto &kv : M.leaves) {
            const Key &b = kv.first;
            if (b.l < 2 || f[kcode(b)] != 1) continue;
            for (const Key &n : F.touching(b, b.l - 1)) {
                int &fn = f[kcode(n)];
                if (fn != 1) {
                    fn = 1;
                    changed = true;
                }
            }
        }
    }
    std::vector<Key> refined;
    for (auto &kv : M.leaves) if (f[kcode(kv.first)] == 1) refined.push_back(kv.first);
    // internal nodes (strict ancestors of leaves) of the forest after the refinements
    FlatMap internal(2 * M.leaves.size() + 8 * refined.size() + 1);
    auto add_ancestors = [&](Key a) {
        while (a.l > 1) {
            a = Key{a.l - 1, a.i >> 1, a.j >> 1, a.k >> 1};
            if (!internal.insert(kcode(a))) break;      // its ancestors are in already
        }
    };
    for (auto &kv : M.leaves)
        if (f[kcode(kv.first)] != 1) add_ancestors(kv.first);
    for (const Key &b : refined) {
        internal.insert(kcode(b));
        add_ancestors(b);
    }
    // coarsening: complete sibling octets of COARSEN leaves, if the parent touches
    // no leaf two or more levels finer in the refined forest.  Such a leaf exists
    // exactly when a child-level cell touching the parent (indices 2p-1 .. 2p+2
    // per direction) is an internal node: its leaves tile it, so one of them
    // meets the shared boundary, and every such leaf lies in such a cell.
    std::map<Key, int> parents;                   // parent -> COARSEN children
    for (auto &kv : M.leaves)
        if (f[kcode(kv.first)] == -1) {
            const Key &b = kv.first;
            parents[Key{b.l - 1, b.i >> 1, b.j >> 1, b.k >> 1}]++;
        }
    std::vector<Key> coarsened;
    for (auto &kv : parents) {
        if (kv.second != 8) continue;
        const Key &p = kv.first;
        bool ok = true;
        if (p.l + 2 <= s->max_level) {
            const int cl = p.l + 1;
            for (int dk = -1; dk <= 2 && ok; ++dk)
                for (int dj = -1; dj <= 2 && ok; ++dj)
                    for (int di = -1; di <= 2 && ok; ++di) {
                        int w[3] = {2 * p.i + di, 2 * p.j + dj, 2 * p.k + dk};
                        if (!wrap_idx(s, cl, w)) continue;
                        if (internal.contains(kcode(Key{cl, w[0], w[1], w[2]}))) ok = false;
                    }
        }
        if (ok) coarsened.push_back(p);
    }
    // capacity check
    long nnew = (long)M.leaves.size() + 7 * (long)refined.size() - 7 * (long)coarsened.size();
    long transient = (long)M.leaves.size() + 8 * (long)refined.size() + (long)coarsened.size();
    if (nnew > s->max_blocks || transient > s->max_blocks)
        throw Error(IC_E_CAPACITY, "member " + std::to_string(m) + ": regrid needs " +
                                       std::to_string(std::max(nnew, transient)) + " block slots, pool has " +
                                       std::to_string(s->max_blocks));
    auto alloc_slot = [&]() {
        const int q = M.free_slots.back();
        M.free_slots.pop_back();
        return q;
    };
    // applied to the leaf map in place: refined leaves and the children of
    // coarsened parents are disjoint, so every lookup below sees the old leaf
    for (const Key &p : refined) {
        const int ps = M.leaves.at(p);
        for (int o = 0; o < 8; ++o) {
            Key ch{p.l + 1, 2 * p.i + (o & 1), 2 * p.j + ((o >> 1) & 1), 2 * p.k + ((o >> 2) & 1)};
            const int cs = alloc_slot();
            M.leaves[ch] = cs;
            MoveTask t{};
            t.type = MOVE_PROLONG;
            t.dst = s->slot_of(m, cs);
            t.src[0] = s->slot_of(m, ps);
            t.src[1] = o;
            t.level = ch.l;
            t.org[0] = ch.i * s->B[0];
            t.org[1] = ch.j * s->B[1];
            t.org[2] = ch.k * s->B[2];
            moves.push_back(t);
        }
        M.leaves.erase(p);
        to_free.push_back(s->slot_of(m, ps));
    }
    for (const Key &p : coarsened) {
        const int pslot = alloc_slot();
        MoveTask t{};
        t.type = MOVE_RESTRICT;
        t.dst = s->slot_of(m, pslot);
        t.level = p.l;
        t.org[0] = p.i * s->B[0];
        t.org[1] = p.j * s->B[1];
        t.org[2] = p.k * s->B[2];
        for (int o = 0; o < 8; ++o) {
            Key ch{p.l + 1, 2 * p.i + (o & 1), 2 * p.j + ((o >> 1) & 1), 2 * p.k + ((o >> 2) & 1)};
            const int cs = M.leaves.at(ch);
            t.src[o] = s->slot_of(m, cs);
            M.leaves.erase(ch);
            to_free.push_back(s->slot_of(m, cs));
        }
        M.leaves[p] = pslot;
        moves.push_back(t);
    }
}

// plain criterion on the current state (ghosts must be filled) into fl, per
// pool slot; level_cap = s->max_level gives the block flags, a huge cap gives
// REFINE wherever a cell meets the refinement condition whatever the level
void run_indicator(ic_sim *s, std::vector<int8_t> &fl, int level_cap, int criterion)
{
    KArgs a = base_args(s);
    a.U = s->U.p;
    IndicatorParams p{};
    const double deg = M_PI / 180.0;
    p.max_level = level_cap;
    p.eps = s->amr.eps_lohner;
    p.tol_r = s->amr.tol_refine;
    p.tol_c = s->amr.tol_coarsen;
    p.w_rho = s->amr.w_rho;
    p.w_v = s->amr.w_v;
    p.use_windows = s->amr.use_windows;
    p.lon_e = s->amr.lon_earth_deg * deg;
    p.clt_e = s->amr.clt_earth_deg * deg;
    p.dlon_e = s->amr.dlon_earth_deg * deg;
    p.dclt_e = s->amr.dclt_earth_deg * deg;
    p.dlon_c = s->amr.dlon_cme_deg * deg;
    p.criterion = criterion;
    p.tr_r = s->amr.tracer_refine;
    p.tr_c = s->amr.tracer_coarsen;
    s->L.indicator(dim3(grid_for(s->n_items, 16384)), s->stream, a, s->flags.p, p);
    HIPCHECK(hipMemcpyAsync(fl.data(), s->flags.p, fl.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
}

void plain_flags(ic_sim *s, std::vector<int8_t> &fl) { run_indicator(s, fl, s->max_level, s->amr.criterion); }

// network probabilities of every leaf in work-list order into s->mlp.prob
void learned_prob(ic_sim *s)
{
    if (!s->mlp.ready) throw Error(IC_E_INVALID, "no network installed (ic_mlp_set)");
    for (int d = 0; d < 3; ++d)
        if (s->B[d] % 4) throw Error(IC_E_INVALID, "learned flags need block dims divisible by 4");
    s->mlp.reserve(s->n_items);
    KArgs a = base_args(s);
    a.U = s->U.p;
    mlp_features(s->stream, a, s->B[0], s->B[1], s->B[2], s->items.p, s->nitems.p, s->n_items, nullptr,
                 s->mlp.mean, s->mlp.istd, s->mlp.xb);
    s->mlp.forward(s->stream, s->n_items);
}

// 1 if some cell centre of the leaf lies in the refinement windows of member m
// (the cell test of the indicator: |lon - lon_E| <= dlon_E, |colat - colat_E|
// <= dclt_E and, with a CME, |lon - lon_CME| <= dlon_CME); always 1 without
// windows.  The windows separate in colatitude and longitude.
bool leaf_in_windows(const ic_sim *s, int m, const Key &key)
{
    if (!s->amr.use_windows || s->cart) return true;
    const double deg = M_PI / 180.0, PI = 3.14159265358979323846;
    const HostLevel &L = s->lv[key.l];
    auto wrap = [&](double x) {
        const double y = x - 2.0 * PI * std::floor((x + PI) / (2.0 * PI));
        return y == -PI ? PI : y;
    };
    bool th = false;
    for (int j = 0; j < s->B[1] && !th; ++j)
        th = std::fabs(L.t[key.j * s->B[1] + j + 2].tc - s->amr.clt_earth_deg * deg) <= s->amr.dclt_earth_deg * deg;
    if (!th) return false;
    const bool cme_on = s->mem[m].cme.enabled != 0;
    for (int k = 0; k < s->B[2]; ++k) {
        const double pc = L.p[key.k * s->B[2] + k + 2].pc;
        if (std::fabs(wrap(pc - s->amr.lon_earth_deg * deg)) <= s->amr.dlon_earth_deg * deg &&
            (!cme_on || std::fabs(wrap(pc - s->mem[m].cme.lon_deg * deg)) <= s->amr.dlon_cme_deg * deg))
            return true;
    }
    return false;
}

float learned_threshold(const ic_sim *s)
{
    return s->amr.learned_threshold > 0.0 ? (float)s->amr.learned_threshold : 0.5f;
}

// learned flags per pool slot: REFINE where the network gives p >= threshold and
// the leaf touches the windows, else COARSEN
void learned_flags(ic_sim *s, std::vector<int8_t> &fl)
{
    learned_prob(s);
    mlp_prob_flags(s->stream, s->mlp.prob, s->items.p, s->n_items, learned_threshold(s), s->flags.p);
    HIPCHECK(hipMemcpyAsync(fl.data(), s->flags.p, fl.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
    for (int m = 0; m < s->nm; ++m)
        for (auto &kv : s->mem[m].leaves) {
            const int slot = s->slot_of(m, kv.second);
            if (fl[slot] == IC_FLAG_REFINE && !leaf_in_windows(s, m, kv.first)) fl[slot] = IC_FLAG_COARSEN;
        }
}

void do_regrid(ic_sim *s, const int8_t *user_flags)
{
    // ghosts of the current state (prolongation of new children reads them)
    fill_ghosts(s, s->U.p, 0.0);
    std::vector<int8_t> fl((size_t)s->nm * s->max_blocks, 0);
    const int src = s->amr.source;
    if (!user_flags && src != IC_SOURCE_PLAIN && s->max_level > 1) {
        // learned flags, judged by the plain criterion every judge_every-th regrid
        if ((int)s->fallback_left.size() != s->nm) s->fallback_left.assign(s->nm, 0);
        learned_flags(s, fl);
        s->n_learned++;
        const bool judge = src == IC_SOURCE_LEARNED_JUDGED && s->amr.judge_every > 0 &&
                           s->n_regrids % s->amr.judge_every == 0;
        bool any_fb = false;
        for (int m = 0; m < s->nm; ++m) any_fb = any_fb || s->fallback_left[m] > 0;
        if (judge || any_fb) {
            std::vector<int8_t> pl(fl.size(), 0);
            plain_flags(s, pl);
            if (judge) s->n_judged++;
            for (int m = 0; m < s->nm; ++m) {
                bool use_plain = s->fallback_left[m] > 0;
                if (use_plain) s->fallback_left[m]--;
                if (judge) {
                    long hit = 0, tot = 0;
                    for (auto &kv : s->mem[m].leaves) {
                        const int slot = s->slot_of(m, kv.second);
                        if (pl[slot] == 1) {
                            ++tot;
                            if (fl[slot] == 1) ++hit;
                        }
                    }
                    const double recall = tot ? (double)hit / tot : 1.0;
                    if (m == 0) s->last_recall = recall;
                    if (recall < s->amr.judge_recall) {
                        s->n_fallbacks++;
                        s->fallback_left[m] = 10;
                        use_plain = true;
                    }
                }
                if (use_plain)
                    for (auto &kv : s->mem[m].leaves) {
                        const int slot = s->slot_of(m, kv.second);
                        fl[slot] = pl[slot];
                    }
            }
        }
    } else if (!user_flags) {
        plain_flags(s, fl);
    }
    // members in parallel; moves and freed slots concatenated in member order
    std::vector<std::vector<MoveTask>> mv(s->nm);
    std::vector<std::vector<int>> fr(s->nm);
    for_members(s->nm, [&](int m) {
        Member &M = s->mem[m];
        FlatMap f(M.leaves.size());
        if (user_flags) {                             // given in the ABI block order
            const std::vector<Key> keys = abi_sorted(M.leaves);
            for (size_t q = 0; q < keys.size(); ++q) f[kcode(keys[q])] = user_flags[(size_t)m * s->max_blocks + q];
        } else {
            for (auto &kv : M.leaves) f[kcode(kv.first)] = fl[s->slot_of(m, kv.second)];
        }
        regrid_member(s, m, f, s->amr.buffer_blocks, mv[m], fr[m]);
    });
    std::vector<MoveTask> moves;
    std::vector<int> to_free;
    for (int m = 0; m < s->nm; ++m) {
        moves.insert(moves.end(), mv[m].begin(), mv[m].end());
        to_free.insert(to_free.end(), fr[m].begin(), fr[m].end());
    }
    if (!moves.empty()) {
        s->moves.alloc(moves.size());
        Upload up(s);
        up.add(s->moves.p, moves.data(), moves.size() * sizeof(MoveTask));
        up.flush();
        KArgs a = base_args(s);
        a.U = s->U.p;
        s->L.move(dim3(grid_for((int)moves.size(), 16384)), s->stream, a, s->U.p, s->moves.p, (int)moves.size());
        HIPCHECK(hipStreamSynchronize(s->stream));
    }
    for (int slot : to_free) s->mem[slot / s->max_blocks].free_slots.push_back(slot % s->max_blocks);
    s->n_regrids++;
    s->since_regrid = 0;
    rebuild(s);
    update_sample_desc(s);
    enqueue_rate(s);
}

void check_sim(ic_sim *s)
{
    if (!s) throw Error(IC_E_INVALID, "null sim");
    if (s->poisoned) throw Error(IC_E_STATE, "sim is poisoned by an earlier error");
}

template <class F>
ic_status guard(ic_sim *s, F &&f)
{
    try {
        f();
        return IC_OK;
    } catch (const Error &e) {
        g_err = e.what();
        if (s && (e.code == IC_E_UNPHYSICAL || e.code == IC_E_DEVICE || e.code == IC_E_CAPACITY))
            s->poisoned = true;
        return e.code;
    } catch (const std::exception &e) {
        g_err = e.what();
        return IC_E_INVALID;
    }
}

void set_initial_state(ic_sim *s)
{
    // relaxation start: rho ~ r^-2, v_r const, p ~ r^-2g, B_r ~ r^-2, v_phi = -omega r sin(theta)
    std::vector<double> h((size_t)s->NC * s->nv);    // a tracer starts at 0 (no CME material)
    for (int m = 0; m < s->nm; ++m) {
        for (auto &kv : s->mem[m].leaves) {
            const Key &key = kv.first;
            const HostLevel &L = s->lv[key.l];
            const HostLevel &L1 = s->lv[1];
            (void)L1;
            const int nt = L.n[1], np = L.n[2];
            const size_t pl = (size_t)nt * np;
            for (int k = 0; k < s->B[2]; ++k)
                for (int j = 0; j < s->B[1]; ++j)
                    for (int i = 0; i < s->B[0]; ++i) {
                        const int gi = key.i * s->B[0] + i, gj = key.j * s->B[1] + j, gk = key.k * s->B[2] + k;
                        double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                        if (!s->cart) {
                            const size_t o = (size_t)gj * np + gk;
                            const double r = L.r[gi + 2].rc, th = L.t[gj + 2].tc;
                            const double x = s->r_in / r;
                            w[0] = L.wind[0 * pl + o] * x * x;
                            w[1] = L.wind[1 * pl + o];
                            w[3] = -s->omega_code * r * std::sin(th);
                            w[4] = L.wind[3 * pl + o] * std::pow(x, 2.0 * s->phys.gamma);
                            w[5] = L.wind[4 * pl + o] * x * x;
                            w[7] = w[5] != 0.0 ? w[5] * w[3] / w[1] : 0.0;
                        } else {
                            w[0] = 1.0;
                            w[4] = 1.0;
                        }
                        const double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
                        const double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
                        double u[8] = {w[0], w[0] * w[1], w[0] * w[2], w[0] * w[3],
                                       w[4] / (s->phys.gamma - 1.0) + 0.5 * w[0] * v2 + 0.5 * b2, w[5], w[6], w[7]};
                        for (int v = 0; v < 8; ++v)
                            h[(size_t)v * s->NC + i + s->B[0] * (j + s->B[1] * k)] = u[v];
                    }
            const int slot = s->slot_of(m, kv.second);
            HIPCHECK(hipMemcpy(s->U.p + (size_t)slot * s->nv * s->NC, h.data(), h.size() * sizeof(double),
                               hipMemcpyHostToDevice));
        }
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
namespace {
// cache key of a schedule: device, block shape, variables; then "/items2^<bucket>"
std::string tune_prefix(const ic_sim *s)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        throw Error(IC_E_DEVICE, "hipGetDeviceProperties failed");
    std::string arch = prop.gcnArchName;
    for (auto &c : arch)
        if (c == ' ') c = '_';
    return arch + "/cu" + std::to_string(prop.multiProcessorCount) + "/b" + std::to_string(s->B[0]) + "x" +
           std::to_string(s->B[1]) + "x" + std::to_string(s->B[2]) + "/nvar" + std::to_string(s->nv) + "/items2^";
}

void apply_tuning(ic_sim *s, int waves, int grid, int xcd, int ksplit)
{
    if ((waves != 1 && waves != 2) || grid < 0 || (xcd != 0 && xcd != 1) || ksplit < 1 || ksplit > KSPLIT_MAX ||
        ksplit > s->B[2])
        throw Error(IC_E_INVALID, "tuning: waves_per_simd 1 or 2, grid >= 0, xcd_order 0 or 1, "
                                  "ksplit 1 .. " + std::to_string(KSPLIT_MAX) + " (at most the block's phi size)");
    s->tune_waves = waves;
    s->tune_grid = grid;
    s->tune_xcd = xcd;
    s->tune_ksplit = ksplit;
    s->graph_dirty = true;
}

// mean stage-1 kernel time [ms] of the current schedule on the current state
double time_stage(ic_sim *s, int reps)
{
    KArgs a = base_args(s);
    a.U = s->U.p;
    a.Ubase = s->U.p;
    a.Uout = s->Us.p;
    a.alpha = 0.5;
    a.want_rate = 0;
    const int g = stage_grid(s);
    s->L.stage(dim3(g), s->stream, a, s->tune_waves, s->phys.limiter);      // warm-up
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipEventRecord(e0, s->stream));
    for (int r = 0; r < reps; ++r) s->L.stage(dim3(g), s->stream, a, s->tune_waves, s->phys.limiter);
    HIPCHECK(hipEventRecord(e1, s->stream));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}
}  // namespace

extern "C" {

const char *ic_last_error(void) { return g_err.c_str(); }

void ic_units(double out[6])
{
    out[0] = kAU;
    out[1] = kV0;
    out[2] = kT0;
    out[3] = kRHO0;
    out[4] = kP0;
    out[5] = kB0;
}

int ic_pool_capacity(const ic_sim *s) { return s ? s->max_blocks : 0; }

ic_status ic_set_device_allocator(ic_alloc_fn alloc, ic_free_fn release, void *user)
{
    if (!alloc != !release) {
        g_err = "ic_set_device_allocator: give both alloc and release, or neither";
        return IC_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    g_dev_alloc = DevAllocator{alloc, release, user};
    return IC_OK;
}

int ic_block_supported(int bi, int bj, int bk)
{
    Launchers L;
    return get_launchers(bi, bj, bk, 8, &L) ? 1 : 0;
}

ic_status ic_create(const ic_grid_cfg *grid, const ic_phys_cfg *phys, const ic_wind_cfg *wind,
                    const ic_cme_cfg *cmes, int n_members, const ic_amr_cfg *amr, void *hip_stream,
                    ic_sim **out)
{
    ic_sim *s = nullptr;
    ic_status st = guard(nullptr, [&]() {
        if (!grid || !phys || !out || n_members < 1) throw Error(IC_E_INVALID, "null argument or n_members < 1");
        if (grid->geometry == IC_GEOM_SPHERICAL && !wind) throw Error(IC_E_INVALID, "spherical geometry needs a wind");
        if (grid->max_level < 1 || grid->max_level > IC_MAX_LEVEL)
            throw Error(IC_E_INVALID, "max_level must be in 1.." + std::to_string(IC_MAX_LEVEL));
        if (grid->max_level > 1 && !amr) throw Error(IC_E_INVALID, "max_level > 1 needs an amr config");
        if (!(phys->gamma > 1.0) || !(phys->cfl > 0.0)) throw Error(IC_E_INVALID, "gamma must exceed 1 and cfl be positive");
        if (phys->limiter < IC_LIM_MC || phys->limiter > IC_LIM_VANLEER) throw Error(IC_E_INVALID, "unknown limiter");
        if (phys->scheme != IC_SCHEME_TWO_STAGE && phys->scheme != IC_SCHEME_HANCOCK)
            throw Error(IC_E_INVALID, "unknown time scheme");
        if (!(phys->divb_cd >= 0.0 && phys->divb_cd <= 1.0))
            throw Error(IC_E_INVALID, "the cleaning coefficient divb_cd must lie in [0, 1]");
        if (phys->tracer != 0 && phys->tracer != 1) throw Error(IC_E_INVALID, "tracer must be 0 or 1");
        if (amr) {
            if (amr->criterion < IC_CRIT_SHOCK || amr->criterion > IC_CRIT_COMBINED)
                throw Error(IC_E_INVALID, "unknown refinement criterion");
            if (amr->criterion != IC_CRIT_SHOCK && !phys->tracer)
                throw Error(IC_E_INVALID, "the tracer and combined criteria need phys->tracer = 1");
            if (amr->criterion != IC_CRIT_SHOCK &&
                !(amr->tracer_refine >= amr->tracer_coarsen && amr->tracer_coarsen >= 0.0))
                throw Error(IC_E_INVALID, "tracer thresholds need tracer_refine >= tracer_coarsen >= 0");
            if (amr->criterion != IC_CRIT_SHOCK && amr->source != IC_SOURCE_PLAIN)
                throw Error(IC_E_INVALID, "learned flags predict the shock criterion only");
        }
        s = new ic_sim();
        s->grid = *grid;
        s->phys = *phys;
        if (wind) s->wind = *wind;
        if (amr) s->amr = *amr;
        s->nm = n_members;
        s->cart = grid->geometry == IC_GEOM_CARTESIAN;
        s->max_level = grid->max_level;
        s->stream = (hipStream_t)hip_stream;
        if (!s->stream) {
            HIPCHECK(hipStreamCreate(&s->stream));   // graph capture needs a stream of its own
            s->own_stream = true;
        }
        for (int d = 0; d < 3; ++d) {
            s->B[d] = grid->block[d];
            if (s->B[d] < 4 || s->B[d] % 2) throw Error(IC_E_INVALID, "block dims must be even and >= 4");
            if (grid->n[d] <= 0 || grid->n[d] % s->B[d]) throw Error(IC_E_INVALID, "cells must be a multiple of the block size");
            s->nb[d] = grid->n[d] / s->B[d];
            const bool p0 = grid->bc[d][0] == IC_BC_PERIODIC, p1 = grid->bc[d][1] == IC_BC_PERIODIC;
            if (p0 != p1) throw Error(IC_E_INVALID, "periodic boundaries must be periodic on both sides");
            s->periodic[d] = p0;
            for (int side = 0; side < 2; ++side) {
                const int b = grid->bc[d][side];
                if (b != IC_BC_OUTFLOW && b != IC_BC_PERIODIC && b != IC_BC_INNER)
                    throw Error(IC_E_INVALID, "unknown boundary kind");
                if (b == IC_BC_INNER && (s->cart || d != 0 || side != 0))
                    throw Error(IC_E_INVALID, "the inner boundary is the lower r boundary of a spherical grid");
            }
            if (!(grid->x1[d] > grid->x0[d])) throw Error(IC_E_INVALID, "empty domain");
        }
        if (!s->cart && grid->x0[0] <= 0.0) throw Error(IC_E_INVALID, "r_in must be positive");
        s->nv = phys->tracer ? 9 : 8;
        if (!get_launchers(s->B[0], s->B[1], s->B[2], s->nv, &s->L))
            throw Error(IC_E_INVALID, "block shape not built into the library");
        s->NC = s->B[0] * s->B[1] * s->B[2];
        s->r_in = s->cart ? 0.0 : grid->x0[0];
        s->omega_code = s->cart ? 0.0 : phys->omega * kT0;
        s->gm_code = s->cart ? 0.0 : phys->gm / (kAU * kV0 * kV0);
        const long nbase = (long)s->nb[0] * s->nb[1] * s->nb[2];
        long cap = grid->max_blocks > 0 ? grid->max_blocks : nbase;
        if (grid->max_blocks <= 0)
            for (int l = 2; l <= s->max_level && cap < 32768; ++l) cap *= 8;
        if (grid->max_blocks <= 0) cap = std::min(cap, std::max(nbase, 32768L));
        if (cap < nbase) throw Error(IC_E_CAPACITY, "max_blocks below the base block count");
        s->max_blocks = (int)cap;
        s->mem.resize(s->nm);
        for (int m = 0; m < s->nm; ++m) {
            if (cmes) s->mem[m].cme = cmes[m];
            else s->mem[m].cme.enabled = 0;
        }
        int dev = 0;
        HIPCHECK(hipGetDevice(&dev));
        // levels
        s->lv.resize(s->max_level + 2);
        for (int l = 1; l <= s->max_level; ++l) build_level(s, l);
        std::vector<LevelGeo> lg(IC_MAX_LEVEL + 2);
        for (int l = 1; l <= s->max_level; ++l) {
            HostLevel &L = s->lv[l];
            lg[l].r = L.dr.p;
            lg[l].t = L.dt.p;
            lg[l].p = L.dp.p;
            for (int d = 0; d < 3; ++d) lg[l].n[d] = L.n[d];
            lg[l].wind = L.dwind.p;
            lg[l].cosd = L.dcosd.p;
        }
        s->geo.alloc(lg.size());
        HIPCHECK(hipMemcpy(s->geo.p, lg.data(), lg.size() * sizeof(LevelGeo), hipMemcpyHostToDevice));
        // member constants
        std::vector<MemberConst> mc(s->nm);
        for (int m = 0; m < s->nm; ++m) {
            const ic_cme_cfg &c = s->mem[m].cme;
            MemberConst &q = mc[m];
            q.enabled = (cmes && c.enabled && !s->cart) ? 1 : 0;
            q.r_in = s->r_in;
            q.lon_cme = c.lon_deg * (M_PI / 180.0);
            if (q.enabled) {
                q.t0 = c.t_start_s / kT0;
                q.v = c.v_kms * 1.0e3 / kV0;
                q.r_half = s->r_in * std::sin(c.half_width_deg * (M_PI / 180.0));
                q.tact = std::min(c.duration_s / kT0, 2.0 * q.r_half / q.v);
                q.rho = c.n_cm3 * 1.0e6 * kMP / kRHO0;
                q.p = 2.0 * c.n_cm3 * 1.0e6 * kKB * c.T_K / kP0;
            }
        }
        s->mc.alloc(s->nm);
        HIPCHECK(hipMemcpy(s->mc.p, mc.data(), s->nm * sizeof(MemberConst), hipMemcpyHostToDevice));
        // pools
        const size_t NS = (size_t)s->nm * s->max_blocks;
        s->U.alloc(NS * s->nv * s->NC);
        s->Us.alloc(NS * s->nv * s->NC);
        if (s->phys.divb_cd > 0.0) s->divb.alloc(NS * s->NC);
        s->desc.alloc(NS);
        s->items.alloc(NS);
        s->nitems.alloc(1);
        s->mbeg.alloc(s->nm);
        s->mend.alloc(s->nm);
        s->dt.alloc(s->nm);
        s->t.alloc(s->nm);
        s->tend.alloc(s->nm);
        s->dt_last.alloc(s->nm);
        s->rate.alloc(NS * KSPLIT_MAX);
        s->bad.alloc(2 * s->nm);
        s->floors.alloc(2 * s->nm);
        s->nsteps.alloc(s->nm);
        s->slab_ranges.alloc(2 * (IC_MAX_LEVEL + 2));
        s->rf_ntasks.alloc(1);
        s->flags.alloc(NS);
        s->sdesc.alloc(s->nm);
        s->sout.alloc((size_t)s->nm * 8);
        s->ring.alloc((size_t)s->nm * s->ring_cap * 9);
        s->ring_count.alloc(s->nm);
        int maxface = std::max(s->B[0] * s->B[1], std::max(s->B[0] * s->B[2], s->B[1] * s->B[2]));
        s->slab_stride = 2L * s->nv * maxface;
        s->reg_stride = (long)s->nv * maxface;
        std::vector<double> zeros(s->nm, 0.0), big(s->nm, 1e300);
        HIPCHECK(hipMemcpy(s->t.p, zeros.data(), s->nm * sizeof(double), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s->dt.p, zeros.data(), s->nm * sizeof(double), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s->dt_last.p, zeros.data(), s->nm * sizeof(double), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s->tend.p, big.data(), s->nm * sizeof(double), hipMemcpyHostToDevice));
        HIPCHECK(hipMemset(s->bad.p, 0, 2 * s->nm * sizeof(int)));
        HIPCHECK(hipMemset(s->floors.p, 0, 2 * s->nm * sizeof(unsigned long long)));
        HIPCHECK(hipMemset(s->nsteps.p, 0, s->nm * sizeof(long)));
        HIPCHECK(hipMemset(s->ring_count.p, 0, s->nm * sizeof(int)));
        HIPCHECK(hipMemset(s->rate.p, 0, NS * KSPLIT_MAX * sizeof(double)));
        // base forest
        for (int m = 0; m < s->nm; ++m) {
            Member &M = s->mem[m];
            for (int q = s->max_blocks - 1; q >= 0; --q) M.free_slots.push_back(q);
            for (int k = 0; k < s->nb[2]; ++k)
                for (int j = 0; j < s->nb[1]; ++j)
                    for (int i = 0; i < s->nb[0]; ++i) {
                        const int q = M.free_slots.back();
                        M.free_slots.pop_back();
                        M.leaves[Key{1, i, j, k}] = q;
                    }
        }
        rebuild(s);
        set_initial_state(s);
        update_sample_desc(s);
        enqueue_rate(s);
        HIPCHECK(hipStreamSynchronize(s->stream));
        *out = s;
    });
    if (st != IC_OK && s) {
        ic_destroy(s);
    }
    return st;
}

void ic_destroy(ic_sim *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    release_graphs(s);
    for (auto e : s->ev) (void)hipEventDestroy(e);
    for (auto &L : s->lv) {
        L.dr.release(); L.dt.release(); L.dp.release(); L.dwind.release(); L.dcosd.release();
    }
    s->U.release(); s->Us.release(); s->divb.release(); s->slabs.release(); s->freg.release(); s->desc.release();
    s->geo.release(); s->mc.release(); s->items.release(); s->nitems.release(); s->mbeg.release();
    s->mend.release(); s->dt.release(); s->t.release(); s->tend.release(); s->dt_last.release();
    s->rate.release(); s->bad.release(); s->floors.release(); s->nsteps.release(); s->slab_tasks.release();
    s->slab_ranges.release(); s->rf_tasks.release(); s->rf_ranges.release(); s->rf_ntasks.release();
    s->flags.release(); s->moves.release(); s->sdesc.release(); s->sout.release(); s->ring.release();
    s->ring_count.release(); s->dstage.release();
    if (s->hstage) (void)hipHostFree(s->hstage);
    if (s->hstat) (void)hipHostFree(s->hstat);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Pinned host landing area of the per-step status: per member the
// non-physical flags, t and the step count, then dt_last of member 0, and a
// host-to-device area for the end times.  Reads go through one async copy per
// array and one synchronisation.
struct Status {
    int *bad;       // [2 nm]
    double *t;      // [nm]
    long *ns;       // [nm]
    double *dtl;    // [1]
    double *tend;   // [nm], host-to-device
};

Status status_buffer(ic_sim *s)
{
    const size_t nm = (size_t)s->nm, a = ((8 * nm + 63) / 64) * 64;
    if (!s->hstat) {
        if (hipHostMalloc((void **)&s->hstat, 4 * a + 64) != hipSuccess) {
            s->hstat = nullptr;
            throw Error(IC_E_NOMEM, "pinned host status buffer");
        }
    }
    Status st;
    st.bad = (int *)s->hstat;
    st.t = (double *)(s->hstat + a);
    st.ns = (long *)(s->hstat + 2 * a);
    st.tend = (double *)(s->hstat + 3 * a);
    st.dtl = (double *)(s->hstat + 4 * a);
    return st;
}

// enqueue the status copies (device to pinned host), synchronise, and fail on
// a non-physical cell
Status read_status(ic_sim *s)
{
    Status st = status_buffer(s);
    HIPCHECK(hipMemcpyAsync(st.bad, s->bad.p, 2 * s->nm * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipMemcpyAsync(st.t, s->t.p, s->nm * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipMemcpyAsync(st.ns, s->nsteps.p, s->nm * sizeof(long), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipMemcpyAsync(st.dtl, s->dt_last.p, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
    for (int m = 0; m < s->nm; ++m)
        if (st.bad[2 * m]) {
            s->poisoned = true;
            throw Error(IC_E_UNPHYSICAL, "member " + std::to_string(m) +
                                             ": a leaf cell has rho <= 0, p <= 0 or a non-finite value" +
                                             describe_bad(s, m, st.bad[2 * m] - 1, st.bad[2 * m + 1]));
        }
    return st;
}

void info_from_status(const ic_sim *s, const Status &st, ic_info *out)
{
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->steps = st.ns[0];
    out->t_s = st.t[0] * kT0;
    out->dt_s = *st.dtl * kT0;
    out->zone_updates = s->zone_updates;
    out->leaves = (int)s->mem[0].leaves.size();
    for (int l = 0; l < 8; ++l) out->leaves_per_level[l] = s->leaves_per_level0[l];
}

// end times back to "none" (asynchronous from the pinned area)
void clear_tend(ic_sim *s)
{
    Status st = status_buffer(s);
    for (int m = 0; m < s->nm; ++m) st.tend[m] = 1e300;
    HIPCHECK(hipMemcpyAsync(s->tend.p, st.tend, s->nm * sizeof(double), hipMemcpyHostToDevice, s->stream));
    s->tend_finite = false;
}

ic_status ic_step(ic_sim *s, double dt_fixed_s, ic_info *out)
{
    return guard(s, [&]() {
        check_sim(s);
        if (dt_fixed_s < 0.0) throw Error(IC_E_INVALID, "negative dt");
        if (s->tend_finite) clear_tend(s);
        run_steps(s, dt_fixed_s / kT0, 1);
        s->zone_updates += (double)total_cells(s);
        s->host_steps++;
        s->since_regrid++;
        const Status st = read_status(s);          // one round trip
        info_from_status(s, st, out);
    });
}

ic_status ic_advance(ic_sim *s, double dt_s, long max_steps, ic_info *out)
{
    return guard(s, [&]() {
        check_sim(s);
        if (!(dt_s >= 0.0) || max_steps < 0) throw Error(IC_E_INVALID, "negative duration or step limit");
        Status st = read_status(s);
        std::vector<double> tend(s->nm);
        std::vector<long> ns(st.ns, st.ns + s->nm);
        for (int m = 0; m < s->nm; ++m) tend[m] = st.t[m] + dt_s / kT0;
        // the pinned end-time area is not written again before the next synchronisation
        for (int m = 0; m < s->nm; ++m) st.tend[m] = tend[m];
        HIPCHECK(hipMemcpyAsync(s->tend.p, st.tend, s->nm * sizeof(double), hipMemcpyHostToDevice, s->stream));
        s->tend_finite = true;
        const int every = (s->max_level > 1 && s->amr.regrid_every > 0) ? s->amr.regrid_every : 0;
        long done = 0;
        // The regrid cadence counts steps across calls (since_regrid): a batch
        // runs the steps still due before the next regrid, and the regrid
        // follows the step that completes the count, so advancing in pieces
        // gives the forests of one advance over the whole span.  Zone updates:
        // per member, the steps it took (a member past its end time takes dt = 0
        // and does no work) times its leaf cells (fixed within a batch).
        if (every > 0 && s->since_regrid >= every) do_regrid(s, nullptr);
        while (done < max_steps) {
            const long due = every > 0 ? every - s->since_regrid : 20;
            const long batch = std::min<long>(max_steps - done, due);
            long q = 0;
            for (; q + GRAPH_STEPS <= batch; q += GRAPH_STEPS) run_steps(s, 0.0, GRAPH_STEPS);
            for (; q < batch; ++q) run_steps(s, 0.0, 1);
            done += batch;
            st = read_status(s);
            long taken = 0;
            for (int m = 0; m < s->nm; ++m) {
                s->zone_updates += (double)(st.ns[m] - ns[m]) * (double)s->mem[m].leaves.size() * s->NC;
                taken = std::max(taken, st.ns[m] - ns[m]);
                ns[m] = st.ns[m];
            }
            s->since_regrid += taken;
            if (every > 0 && s->since_regrid >= every) do_regrid(s, nullptr);
            bool all = true;
            for (int m = 0; m < s->nm; ++m) all = all && st.t[m] >= tend[m];
            if (all) break;
        }
        clear_tend(s);
        st = read_status(s);
        info_from_status(s, st, out);
    });
}

ic_status ic_regrid(ic_sim *s, const int8_t *flags, ic_info *out)
{
    return guard(s, [&]() {
        check_sim(s);
        if (s->max_level > 1 || flags) do_regrid(s, flags);
        HIPCHECK(hipStreamSynchronize(s->stream));
        fill_info(s, out);
    });
}

namespace {
// per-leaf indicator output of one member in ic_get_blocks order
void leaf_indicator(ic_sim *s, int member, int8_t *out, int n, int level_cap, bool hot)
{
    check_sim(s);
    if (member < 0 || member >= s->nm || !out) throw Error(IC_E_INVALID, "bad member or buffer");
    Member &M = s->mem[member];
    if (n < (int)M.leaves.size()) throw Error(IC_E_INVALID, "flag buffer too small");
    fill_ghosts(s, s->U.p, 0.0);
    std::vector<int8_t> fl((size_t)s->nm * s->max_blocks);
    // the look-ahead labels (hot) are the shock criterion's refinement condition
    run_indicator(s, fl, level_cap, hot ? CRIT_SHOCK : s->amr.criterion);
    const std::vector<Key> keys = abi_sorted(M.leaves);
    for (size_t q = 0; q < keys.size(); ++q) {
        const int8_t f = fl[s->slot_of(member, M.leaves[keys[q]])];
        out[q] = hot ? (int8_t)(f == IC_FLAG_REFINE) : f;
    }
}
}  // namespace

ic_status ic_eval_flags(ic_sim *s, int member, int8_t *flags, int n)
{
    return guard(s, [&]() { leaf_indicator(s, member, flags, n, s->max_level, false); });
}

ic_status ic_eval_hot(ic_sim *s, int member, int8_t *hot, int n)
{
    return guard(s, [&]() { leaf_indicator(s, member, hot, n, 1 << 20, true); });
}

ic_status ic_eval_window(ic_sim *s, int member, int8_t *in, int n)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !in) throw Error(IC_E_INVALID, "bad member or buffer");
        Member &M = s->mem[member];
        if (n < (int)M.leaves.size()) throw Error(IC_E_INVALID, "buffer too small");
        const std::vector<Key> keys = abi_sorted(M.leaves);
        for (size_t q = 0; q < keys.size(); ++q) in[q] = leaf_in_windows(s, member, keys[q]) ? 1 : 0;
    });
}

ic_status ic_sample(ic_sim *s, int member, double r_au, double colat_deg, double lon_deg, double prim_out[8])
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !prim_out) throw Error(IC_E_INVALID, "bad member or buffer");
        SampleDesc sd{};
        if (!build_sample(s, member, r_au, colat_deg, lon_deg, &sd)) throw Error(IC_E_OUTSIDE, "point outside the domain");
        std::vector<SampleDesc> all(s->nm);
        std::memset(all.data(), 0, all.size() * sizeof(SampleDesc));
        all[member] = sd;
        DBuf<SampleDesc> tmp;
        tmp.alloc(s->nm);
        HIPCHECK(hipMemcpy(tmp.p, all.data(), s->nm * sizeof(SampleDesc), hipMemcpyHostToDevice));
        KArgs a = base_args(s);
        a.U = s->U.p;
        s->L.sample(dim3(s->nm), s->stream, a, tmp.p, s->nm, s->sout.p, s->ring.p, s->ring_count.p, s->ring_cap, 0,
                    nullptr, nullptr);
        HIPCHECK(hipMemcpyAsync(prim_out, s->sout.p + member * 8, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        tmp.release();
    });
}

ic_status ic_set_sample_point(ic_sim *s, double r_au, double colat_deg, double lon_deg)
{
    return guard(s, [&]() {
        check_sim(s);
        s->sample_point[0] = r_au;
        s->sample_point[1] = colat_deg;
        s->sample_point[2] = lon_deg;
        update_sample_desc(s);
    });
}

ic_status ic_timeseries(ic_sim *s, int member, double *out, int *n_inout)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !out || !n_inout) throw Error(IC_E_INVALID, "bad argument");
        int cnt = 0;
        HIPCHECK(hipMemcpyAsync(&cnt, s->ring_count.p + member, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        const int have = std::min(cnt, s->ring_cap);
        const int n = std::min(have, *n_inout);
        std::vector<double> buf((size_t)s->ring_cap * 9);
        HIPCHECK(hipMemcpy(buf.data(), s->ring.p + (size_t)member * s->ring_cap * 9, buf.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
        for (int q = 0; q < n; ++q) {
            const int idx = (cnt - n + q) % s->ring_cap;
            std::memcpy(out + (size_t)q * 9, buf.data() + (size_t)idx * 9, 9 * sizeof(double));
            out[(size_t)q * 9] *= kT0;
        }
        *n_inout = n;
    });
}

ic_status ic_timeseries_clear(ic_sim *s)
{
    return guard(s, [&]() {
        check_sim(s);
        HIPCHECK(hipMemsetAsync(s->ring_count.p, 0, s->nm * sizeof(int), s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
    });
}

ic_status ic_get_blocks(ic_sim *s, int member, int32_t *lvl_ijk, int *n_inout)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !n_inout) throw Error(IC_E_INVALID, "bad argument");
        Member &M = s->mem[member];
        const std::vector<Key> keys = abi_sorted(M.leaves);
        if (!lvl_ijk || *n_inout < (int)keys.size()) {
            *n_inout = (int)keys.size();
            throw Error(IC_E_INVALID, "block buffer too small");
        }
        for (size_t q = 0; q < keys.size(); ++q) {
            lvl_ijk[4 * q + 0] = keys[q].l;
            lvl_ijk[4 * q + 1] = keys[q].i;
            lvl_ijk[4 * q + 2] = keys[q].j;
            lvl_ijk[4 * q + 3] = keys[q].k;
        }
        *n_inout = (int)keys.size();
    });
}

ic_status ic_get_state(ic_sim *s, int member, double *host_U, size_t n_doubles)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !host_U) throw Error(IC_E_INVALID, "bad argument");
        Member &M = s->mem[member];
        const std::vector<Key> keys = abi_sorted(M.leaves);
        const size_t per = (size_t)s->nv * s->NC;
        if (n_doubles < keys.size() * per) throw Error(IC_E_INVALID, "state buffer too small");
        HIPCHECK(hipStreamSynchronize(s->stream));
        for (size_t q = 0; q < keys.size(); ++q) {
            const int slot = s->slot_of(member, M.leaves[keys[q]]);
            HIPCHECK(hipMemcpy(host_U + q * per, s->U.p + (size_t)slot * per, per * sizeof(double), hipMemcpyDeviceToHost));
        }
    });
}

ic_status ic_set_state(ic_sim *s, int member, const int32_t *lvl_ijk, int n_blocks, const double *host_U, double t_s)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !lvl_ijk || !host_U || n_blocks < 1)
            throw Error(IC_E_INVALID, "bad argument");
        if (n_blocks > s->max_blocks) throw Error(IC_E_CAPACITY, "more blocks than the pool holds");
        // validate: levels, ranges, tiling, 2:1
        std::map<Key, int> leaves;
        long vol = 0;
        const int L = s->max_level;
        for (int q = 0; q < n_blocks; ++q) {
            Key k{lvl_ijk[4 * q], lvl_ijk[4 * q + 1], lvl_ijk[4 * q + 2], lvl_ijk[4 * q + 3]};
            if (k.l < 1 || k.l > L) throw Error(IC_E_INVALID, "block level out of range");
            const int idx[3] = {k.i, k.j, k.k};
            for (int d = 0; d < 3; ++d)
                if (idx[d] < 0 || idx[d] >= nblocks_at(s, k.l, d)) throw Error(IC_E_INVALID, "block index out of range");
            if (leaves.count(k)) throw Error(IC_E_INVALID, "duplicate block");
            leaves[k] = q;
            vol += 1L << (3 * (L - k.l));
        }
        if (vol != (long)s->nb[0] * s->nb[1] * s->nb[2] << (3 * (L - 1)))
            throw Error(IC_E_INVALID, "blocks do not tile the domain");
        Forest F{s, leaves, s->max_level};
        for (auto &kv : leaves) {
            int l = kv.first.l - 1, i = kv.first.i >> 1, j = kv.first.j >> 1, k = kv.first.k >> 1;
            for (; l >= 1; --l, i >>= 1, j >>= 1, k >>= 1)
                if (leaves.count(Key{l, i, j, k})) throw Error(IC_E_INVALID, "overlapping blocks");
            for (int lv = kv.first.l + 2; lv <= s->max_level; ++lv)
                if (!F.touching(kv.first, lv).empty()) throw Error(IC_E_INVALID, "blocks violate 2:1 balance");
        }
        Member &M = s->mem[member];
        M.leaves.clear();
        M.free_slots.clear();
        for (int q = s->max_blocks - 1; q >= 0; --q) M.free_slots.push_back(q);
        const size_t per = (size_t)s->nv * s->NC;
        HIPCHECK(hipStreamSynchronize(s->stream));
        for (int q = 0; q < n_blocks; ++q) {
            Key k{lvl_ijk[4 * q], lvl_ijk[4 * q + 1], lvl_ijk[4 * q + 2], lvl_ijk[4 * q + 3]};
            const int ls = M.free_slots.back();
            M.free_slots.pop_back();
            M.leaves[k] = ls;
            HIPCHECK(hipMemcpy(s->U.p + (size_t)s->slot_of(member, ls) * per, host_U + (size_t)q * per,
                               per * sizeof(double), hipMemcpyHostToDevice));
        }
        const double tc = t_s / kT0;
        HIPCHECK(hipMemcpy(s->t.p + member, &tc, sizeof(double), hipMemcpyHostToDevice));
        const int zero[2] = {0, 0};
        HIPCHECK(hipMemcpy(s->bad.p + 2 * member, zero, 2 * sizeof(int), hipMemcpyHostToDevice));
        s->since_regrid = 0;
        rebuild(s);
        update_sample_desc(s);
        enqueue_rate(s);
        HIPCHECK(hipStreamSynchronize(s->stream));
    });
}

ic_status ic_get_time(ic_sim *s, int member, double *t_s, double *dt_s)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm) throw Error(IC_E_INVALID, "bad member");
        double t = 0, d = 0;
        HIPCHECK(hipMemcpyAsync(&t, s->t.p + member, sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipMemcpyAsync(&d, s->dt_last.p + member, sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        if (t_s) *t_s = t * kT0;
        if (dt_s) *dt_s = d * kT0;
    });
}

ic_status ic_get_clock(ic_sim *s, int member, double *t_code, long *since_regrid)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm) throw Error(IC_E_INVALID, "bad member");
        double t = 0;
        HIPCHECK(hipMemcpyAsync(&t, s->t.p + member, sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        if (t_code) *t_code = t;
        if (since_regrid) *since_regrid = s->since_regrid;
    });
}

ic_status ic_set_clock(ic_sim *s, int member, double t_code, long since_regrid)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm) throw Error(IC_E_INVALID, "bad member");
        if (!std::isfinite(t_code) || since_regrid < 0) throw Error(IC_E_INVALID, "bad clock");
        HIPCHECK(hipMemcpyAsync(s->t.p + member, &t_code, sizeof(double), hipMemcpyHostToDevice, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        s->since_regrid = since_regrid;
    });
}

ic_status ic_floor_counts(ic_sim *s, int member, long *rho_floors, long *p_floors)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm) throw Error(IC_E_INVALID, "bad member");
        unsigned long long c[2] = {0, 0};
        HIPCHECK(hipMemcpyAsync(c, s->floors.p + 2 * member, sizeof(c), hipMemcpyDeviceToHost, s->stream));
        HIPCHECK(hipStreamSynchronize(s->stream));
        if (rho_floors) *rho_floors = (long)c[0];
        if (p_floors) *p_floors = (long)c[1];
    });
}

ic_status ic_shock_diagnostics(const double *t_s, const double *v, int n, double t_cme_s, double window_s,
                               double min_jump, double out[8])
{
    return guard(nullptr, [&]() {
        if (!t_s || !v || !out || n < 0 || !(window_s >= 0.0)) throw Error(IC_E_INVALID, "bad argument");
        const double nan = std::numeric_limits<double>::quiet_NaN();
        for (int q = 0; q < 8; ++q) out[q] = nan;
        if (n == 0) return;
        for (int q = 1; q < n; ++q)
            if (!(t_s[q] >= t_s[q - 1])) throw Error(IC_E_INVALID, "sample times must ascend");
        // speed before the shock: v at the CME start, linear between the samples
        // around it (the first or last sample outside the recorded span)
        double v_pre;
        if (t_cme_s <= t_s[0]) v_pre = v[0];
        else if (t_cme_s >= t_s[n - 1]) v_pre = v[n - 1];
        else {
            int q = 1;
            while (t_s[q] < t_cme_s) ++q;
            const double h = t_s[q] - t_s[q - 1];
            v_pre = (t_s[q] == t_cme_s || !(h > 0.0)) ? v[q]
                                                       : v[q - 1] + (t_cme_s - t_s[q - 1]) * (v[q] - v[q - 1]) / h;
        }
        out[2] = v_pre;
        // peak speed inside [t_cme, t_cme + window] (first sample of the maximum)
        int qmax = -1, qlast = -1;
        for (int q = 0; q < n; ++q)
            if (t_s[q] >= t_cme_s && t_s[q] <= t_cme_s + window_s) {
                if (qmax < 0 || v[q] > v[qmax]) qmax = q;
                qlast = q;
            }
        if (qmax < 0) {
            out[3] = v_pre;
            return;
        }
        const double v_max = v[qmax];
        out[3] = v_max;
        out[7] = t_s[qmax];
        if (v_max - v_pre < min_jump) return;
        // arrival: the first upward crossing of the half-rise level inside the
        // window by a segment that starts at or after the CME start; the top of
        // the jump: the first sample from the segment's end on after which the
        // speed no longer rises (or the window's last sample)
        const double thr = v_pre + 0.5 * (v_max - v_pre);
        const double tol = 1e-12 * std::max(1.0, std::fabs(t_cme_s));
        for (int q = 1; q < n; ++q) {
            if (!(t_s[q] >= t_cme_s && t_s[q] <= t_cme_s + window_s)) continue;
            if (v[q - 1] < thr && thr <= v[q] && t_s[q - 1] >= t_cme_s - tol) {
                const double ta = t_s[q - 1] + (thr - v[q - 1]) * (t_s[q] - t_s[q - 1]) / (v[q] - v[q - 1]);
                int top = q;
                while (top < qlast && v[top + 1] > v[top]) ++top;
                out[0] = ta - t_cme_s;
                out[1] = t_s[top] - ta;
                out[5] = t_s[top];
                out[6] = v[top];
                // mean slope of v from the arrival (v = thr) to the top of the jump
                out[4] = out[1] > 0.0 ? (v[top] - thr) / out[1] : nan;
                return;
            }
        }
    });
}

ic_status ic_features(ic_sim *s, int member, float *raw, int n)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm || !raw) throw Error(IC_E_INVALID, "bad argument");
        for (int d = 0; d < 3; ++d)
            if (s->B[d] % 4) throw Error(IC_E_INVALID, "features need block dims divisible by 4");
        const int nl = (int)s->mem[member].leaves.size();
        if (n < nl) throw Error(IC_E_INVALID, "feature buffer too small");
        std::vector<int> mb(s->nm);
        HIPCHECK(hipMemcpy(mb.data(), s->mbeg.p, s->nm * sizeof(int), hipMemcpyDeviceToHost));
        DBuf<float> out;
        out.alloc((size_t)nl * IC_MLP_IN);
        DBuf<int> cnt;
        cnt.alloc(1);
        HIPCHECK(hipMemcpy(cnt.p, &nl, sizeof(int), hipMemcpyHostToDevice));
        KArgs a = base_args(s);
        a.U = s->U.p;
        mlp_features(s->stream, a, s->B[0], s->B[1], s->B[2], s->items.p + mb[member], cnt.p, nl, out.p, nullptr,
                     nullptr, nullptr);
        HIPCHECK(hipStreamSynchronize(s->stream));
        HIPCHECK(hipMemcpy(raw, out.p, (size_t)nl * IC_MLP_IN * sizeof(float), hipMemcpyDeviceToHost));
        out.release();
        cnt.release();
    });
}

ic_status ic_mlp_set(ic_sim *s, const float *params, const float *mean, const float *std)
{
    return guard(s, [&]() {
        check_sim(s);
        if (!params || !mean || !std) throw Error(IC_E_INVALID, "null argument");
        for (int f = 0; f < IC_MLP_IN; ++f)
            if (!(std[f] > 0.0f)) throw Error(IC_E_INVALID, "std must be positive");
        HIPCHECK(hipStreamSynchronize(s->stream));
        s->mlp.set(params, mean, std);
    });
}

ic_status ic_eval_learned(ic_sim *s, int member, float *prob, int8_t *flags, int n)
{
    return guard(s, [&]() {
        check_sim(s);
        if (member < 0 || member >= s->nm) throw Error(IC_E_INVALID, "bad member");
        const int nl = (int)s->mem[member].leaves.size();
        if (n < nl) throw Error(IC_E_INVALID, "buffer too small");
        learned_prob(s);
        std::vector<int> mb(s->nm);
        HIPCHECK(hipMemcpy(mb.data(), s->mbeg.p, s->nm * sizeof(int), hipMemcpyDeviceToHost));
        std::vector<float> p(nl);
        HIPCHECK(hipStreamSynchronize(s->stream));
        HIPCHECK(hipMemcpy(p.data(), s->mlp.prob + mb[member], nl * sizeof(float), hipMemcpyDeviceToHost));
        const std::vector<Key> keys = abi_sorted(s->mem[member].leaves);
        for (int q = 0; q < nl; ++q) {
            if (prob) prob[q] = p[q];
            if (flags)
                flags[q] = p[q] >= learned_threshold(s) && leaf_in_windows(s, member, keys[q]) ? IC_FLAG_REFINE
                                                                                              : IC_FLAG_COARSEN;
        }
    });
}

ic_status ic_regrid_stats(ic_sim *s, long *learned, long *judged, long *fallbacks, double *last_recall)
{
    return guard(s, [&]() {
        check_sim(s);
        if (learned) *learned = s->n_learned;
        if (judged) *judged = s->n_judged;
        if (fallbacks) *fallbacks = s->n_fallbacks;
        if (last_recall) *last_recall = s->last_recall;
    });
}

ic_status ic_mlp_train(const float *raw, const uint8_t *y, long n, const ic_mlp_hparams *hp, float *params,
                       float *mean, float *std, float *loss_per_epoch)
{
    return guard(nullptr, [&]() {
        if (!raw || !y || !hp || !params || !mean || !std || n < 1) throw Error(IC_E_INVALID, "bad argument");
        if (hp->batch < 1 || hp->batch > n || hp->epochs < 0) throw Error(IC_E_INVALID, "bad hyper-parameters");
        MlpHparams h{hp->epochs, hp->batch, hp->lr, hp->beta1, hp->beta2, hp->eps, hp->seed, hp->pos_weight};
        try {
            mlp_train(raw, y, n, h, params, mean, std, loss_per_epoch);
        } catch (const std::runtime_error &e) {
            throw Error(IC_E_DEVICE, e.what());
        }
    });
}

ic_status ic_mlp_grad(const float *xnorm, const uint8_t *y, int n, float pos_weight, const float *params,
                      float *grad, float *loss)
{
    return guard(nullptr, [&]() {
        if (!xnorm || !y || !params || !grad || !loss || n < 1) throw Error(IC_E_INVALID, "bad argument");
        try {
            mlp_grad(xnorm, y, n, pos_weight, params, grad, loss);
        } catch (const std::runtime_error &e) {
            throw Error(IC_E_DEVICE, e.what());
        }
    });
}

ic_status ic_mlp_infer(const float *raw, long n, const float *params, const float *mean, const float *std, float *prob)
{
    return guard(nullptr, [&]() {
        if (!raw || !params || !mean || !std || !prob || n < 1) throw Error(IC_E_INVALID, "bad argument");
        for (int f = 0; f < IC_MLP_IN; ++f)
            if (!(std[f] > 0.0f)) throw Error(IC_E_INVALID, "std must be positive");
        try {
            mlp_infer(raw, n, params, mean, std, prob);
        } catch (const std::runtime_error &e) {
            throw Error(IC_E_DEVICE, e.what());
        }
    });
}

ic_status ic_mlp_infer_noalloc(const float *raw_dev, long n, const float *params_dev, const float *mean_dev,
                               const float *std_dev, float *prob_dev, void *hip_stream)
{
    static_assert(IC_MLP_NOALLOC_ROWS == 4096, "the header's row limit");
    static_assert(CRIT_SHOCK == IC_CRIT_SHOCK && CRIT_TRACER == IC_CRIT_TRACER && CRIT_COMBINED == IC_CRIT_COMBINED,
                  "criterion codes of the header and the kernels");
    return guard(nullptr, [&]() {
        if (!raw_dev || !params_dev || !mean_dev || !std_dev || !prob_dev || n < 0)
            throw Error(IC_E_INVALID, "bad argument");
        if (n > IC_MLP_NOALLOC_ROWS)
            throw Error(IC_E_INVALID, "ic_mlp_infer_noalloc: " + std::to_string(n) + " rows exceed the limit of " +
                                          std::to_string(IC_MLP_NOALLOC_ROWS) + " (the fixed scratch)");
        try {
            mlp_infer_noalloc(raw_dev, n, params_dev, mean_dev, std_dev, prob_dev, (hipStream_t)hip_stream);
        } catch (const std::invalid_argument &e) {
            throw Error(IC_E_INVALID, e.what());
        } catch (const std::runtime_error &e) {
            throw Error(IC_E_DEVICE, e.what());
        }
    });
}

ic_status ic_set_tuning(ic_sim *s, const ic_tune_info *t)
{
    return guard(s, [&]() {
        check_sim(s);
        if (!t) throw Error(IC_E_INVALID, "null tuning");
        HIPCHECK(hipStreamSynchronize(s->stream));
        apply_tuning(s, t->waves_per_simd, t->grid, t->xcd_order, t->ksplit);
        s->tune_pinned = true;
    });
}

ic_status ic_get_tuning(ic_sim *s, ic_tune_info *t)
{
    return guard(s, [&]() {
        check_sim(s);
        if (!t) throw Error(IC_E_INVALID, "null tuning");
        *t = ic_tune_info{};
        t->waves_per_simd = s->tune_waves;
        t->grid = s->tune_grid;
        t->xcd_order = s->tune_xcd;
        t->ksplit = s->tune_ksplit;
    });
}

ic_status ic_autotune(ic_sim *s, const char *cache_path, int reps, ic_tune_info *out)
{
    return guard(s, [&]() {
        check_sim(s);
        if (reps < 1) throw Error(IC_E_INVALID, "reps must be >= 1");
        HIPCHECK(hipStreamSynchronize(s->stream));
        const std::string prefix = tune_prefix(s);
        const int bucket = items_bucket(s);
        const std::string key = prefix + std::to_string(bucket);
        ic_tune_info res{};
        // cache: one line per result, "key waves grid xcd ksplit ms default_ms"; the last match
        // wins.  Entries of other work-list sizes on this device and block shape are kept
        // for the schedule choice after regrids.
        if (cache_path) {
            std::FILE *f = std::fopen(cache_path, "r");
            if (f) {
                char k[512];
                int w, g, x, ks;
                double ms, dms;
                while (std::fscanf(f, "%511s %d %d %d %d %lf %lf", k, &w, &g, &x, &ks, &ms, &dms) == 7) {
                    const std::string ks_(k);
                    if (ks_.compare(0, prefix.size(), prefix) == 0 && ks_.size() > prefix.size() &&
                        (w == 1 || w == 2) && g >= 0 && (x == 0 || x == 1) && (ks == 1 || ks == 2 || ks == 4) &&
                        ks <= s->B[2])
                        s->tuned[std::atoi(ks_.c_str() + prefix.size())] = {w, g, x, ks};
                    if (key == k) {
                        res.waves_per_simd = w;
                        res.grid = g;
                        res.xcd_order = x;
                        res.ksplit = ks;
                        res.stage_ms = ms;
                        res.default_ms = dms;
                        res.from_cache = 1;
                    }
                }
                std::fclose(f);
            }
        }
        if (!res.from_cache) {
            // stage 1 reads U, writes the scratch stage state: the sim's state is untouched
            KArgs a = base_args(s);
            launch_dt(s->stream, a, s->mbeg.p, s->mend.p, s->nm, s->phys.cfl, 0.0, s->tend.p, s->dt_last.p);
            fill_ghosts(s, s->U.p, 0.0);
            double best = 1e300;
            int dev = 0, cus = 256;
            hipDeviceProp_t prop{};
            if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
                cus = prop.multiProcessorCount;
            for (int ks : {1, 2, 4, 6, 12}) {
                if (ks > s->B[2]) continue;
                // more than four parts (down to one plane per work-group) only
                // for lists that four parts leave below two work-groups per CU
                if (ks > 4 && s->n_items * 4 >= 2 * cus) continue;
                const int n = std::max(1, s->n_items * ks);
                std::vector<int> grids{0};
                for (int g : {1024, 2048})
                    if (g < n) grids.push_back(g);
                for (int w : {2, 1}) {
                    // one wave per SIMD only pays while the work-groups do not fill
                    // every CU twice (measured 1.3-1.6x slower beyond)
                    if (w == 1 && n >= 2 * cus) continue;
                    for (int g : grids)
                        for (int x : {1, 0}) {
                            apply_tuning(s, w, g, x, ks);
                            const double ms = time_stage(s, reps);
                            res.candidates++;
                            if (w == 2 && g == 0 && x == 0 && ks == 1) res.default_ms = ms;
                            // a later candidate must be 1 % faster: near-ties keep the first in
                            // this order (XCD-contiguous order first, for its lower HBM traffic)
                            if (ms < 0.99 * best) {
                                best = ms;
                                res.waves_per_simd = w;
                                res.grid = g;
                                res.xcd_order = x;
                                res.ksplit = ks;
                                res.stage_ms = ms;
                            }
                        }
                }
            }
            if (cache_path) {
                std::FILE *f = std::fopen(cache_path, "a");
                if (f) {
                    std::fprintf(f, "%s %d %d %d %d %.6f %.6f\n", key.c_str(), res.waves_per_simd, res.grid,
                                 res.xcd_order, res.ksplit, res.stage_ms, res.default_ms);
                    std::fclose(f);
                }
            }
        }
        apply_tuning(s, res.waves_per_simd, res.grid, res.xcd_order, res.ksplit);
        s->tuned[bucket] = {res.waves_per_simd, res.grid, res.xcd_order, res.ksplit};
        s->tune_pinned = false;
        if (out) *out = res;
    });
}

ic_status ic_set_kernel_timing(ic_sim *s, int enable)
{
    return guard(s, [&]() {
        check_sim(s);
        HIPCHECK(hipStreamSynchronize(s->stream));
        for (auto e : s->ev) HIPCHECK(hipEventDestroy(e));
        s->ev.clear();
        s->timing = enable != 0;
    });
}

ic_status ic_stage_timing(ic_sim *s, long *launches, double *mean_ms)
{
    return guard(s, [&]() {
        check_sim(s);
        HIPCHECK(hipStreamSynchronize(s->stream));
        double tot = 0.0;
        const long n = (long)s->ev.size() / 2;
        for (long q = 0; q < n; ++q) {
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, s->ev[2 * q], s->ev[2 * q + 1]));
            tot += ms;
        }
        if (launches) *launches = n;
        if (mean_ms) *mean_ms = n ? tot / n : 0.0;
    });
}

}  // extern "C"
