// sanitize_driver.cpp -- drives every C-ABI entry point of the library through
// a short cone-CME run with refinement, learned flags, checkpoint and error
// paths, for a build whose host code is instrumented by AddressSanitizer and
// UndefinedBehaviorSanitizer (the device code is built as usual).  The host
// runtime -- forest updates, task lists, regrid bookkeeping, schedule cache,
// shock diagnostics -- then runs under the sanitizers on a real device.
// Prints "ok" and exits 0 when every call returns the expected status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/icarus.h"

namespace {
int failures = 0;

void expect(ic_status got, ic_status want, const char *what)
{
    if (got != want) {
        std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, ic_last_error());
        ++failures;
    }
}

ic_grid_cfg wedge_grid(int max_level)
{
    ic_grid_cfg g;
    std::memset(&g, 0, sizeof g);
    g.geometry = IC_GEOM_SPHERICAL;
    const double x0[3] = {0.1, 60.0, 0.0}, x1[3] = {1.1, 120.0, 90.0};
    for (int d = 0; d < 3; ++d) {
        g.x0[d] = x0[d];
        g.x1[d] = x1[d];
        g.block[d] = 12;
        g.bc[d][0] = g.bc[d][1] = IC_BC_OUTFLOW;
    }
    g.n[0] = 48, g.n[1] = 12, g.n[2] = 24;
    g.bc[0][0] = IC_BC_INNER;
    g.stretched_r = 1;
    g.max_level = max_level;
    return g;
}

ic_phys_cfg phys(int tracer)
{
    ic_phys_cfg p;
    std::memset(&p, 0, sizeof p);
    p.gamma = 1.5;
    p.cfl = 0.4;
    p.omega = 2.0 * M_PI / (25.38 * 86400.0);
    p.gm = 1.32712440018e20;
    p.rho_floor = 1e-6;
    p.p_floor = 1e-9;
    p.limiter = IC_LIM_MC;
    p.scheme = IC_SCHEME_TWO_STAGE;
    p.tracer = tracer;
    return p;
}

ic_wind_cfg wind()
{
    ic_wind_cfg w;
    std::memset(&w, 0, sizeof w);
    w.alm[1] = 0.8, w.alm[4] = -0.5, w.alm[9] = 0.3;
    w.f_min = -1.5, w.f_max = 1.5;
    w.v_min_kms = 350, w.v_max_kms = 700, w.n_ref_cm3 = 300, w.v_ref_kms = 450, w.T_K = 1e6, w.B_nT = 300;
    return w;
}

ic_cme_cfg cme()
{
    ic_cme_cfg c;
    std::memset(&c, 0, sizeof c);
    c.t_start_s = 0, c.duration_s = 6 * 3600.0, c.v_kms = 1400, c.half_width_deg = 35, c.colat_deg = 90;
    c.lon_deg = 30, c.n_cm3 = 1500, c.T_K = 0.8e6, c.enabled = 1;
    return c;
}

ic_amr_cfg amr(int source, int criterion)
{
    ic_amr_cfg a;
    std::memset(&a, 0, sizeof a);
    a.eps_lohner = 0.01, a.tol_refine = 0.1, a.tol_coarsen = 0.0125, a.w_rho = 0.5, a.w_v = 0.5;
    a.lon_earth_deg = 0, a.clt_earth_deg = 90, a.dlon_earth_deg = 60, a.dclt_earth_deg = 30, a.dlon_cme_deg = 90;
    a.use_windows = 1, a.regrid_every = 5, a.buffer_blocks = 1, a.source = source;
    a.judge_every = 3, a.judge_recall = 0.9, a.learned_threshold = 0.5;
    a.criterion = criterion, a.tracer_refine = 0.01, a.tracer_coarsen = 0.00125;
    return a;
}

void run_member_calls(ic_sim *s, int nv)
{
    ic_info info;
    expect(ic_step(s, 0.0, &info), IC_OK, "ic_step");
    expect(ic_advance(s, 1e12, 12, &info), IC_OK, "ic_advance");
    int n = ic_pool_capacity(s);
    std::vector<int32_t> blocks(4 * (size_t)n);
    expect(ic_get_blocks(s, 0, blocks.data(), &n), IC_OK, "ic_get_blocks");
    std::vector<int8_t> fl(n), hot(n), win(n);
    expect(ic_eval_flags(s, 0, fl.data(), n), IC_OK, "ic_eval_flags");
    expect(ic_eval_hot(s, 0, hot.data(), n), IC_OK, "ic_eval_hot");
    expect(ic_eval_window(s, 0, win.data(), n), IC_OK, "ic_eval_window");
    expect(ic_eval_flags(s, 0, fl.data(), n - 1), IC_E_INVALID, "ic_eval_flags short buffer");
    // a user-flag regrid (flags of member m at m * capacity): member 0 refines
    // every leaf that may refine, member 1 keeps its forest
    std::vector<int8_t> user(2 * (size_t)ic_pool_capacity(s), IC_FLAG_KEEP);
    for (int q = 0; q < n; ++q) user[q] = blocks[4 * q] < 3 ? IC_FLAG_REFINE : IC_FLAG_KEEP;
    expect(ic_regrid(s, user.data(), &info), IC_OK, "ic_regrid user flags");
    expect(ic_regrid(s, nullptr, &info), IC_OK, "ic_regrid plain");
    double prim[8];
    expect(ic_sample(s, 0, 1.0, 90.0, 10.0, prim), IC_OK, "ic_sample");
    expect(ic_sample(s, 0, 5.0, 90.0, 10.0, prim), IC_E_OUTSIDE, "ic_sample outside");
    int ns = 64;
    std::vector<double> ts(9 * (size_t)ns);
    expect(ic_timeseries(s, 0, ts.data(), &ns), IC_OK, "ic_timeseries");
    // checkpoint and restore
    n = ic_pool_capacity(s);
    expect(ic_get_blocks(s, 0, blocks.data(), &n), IC_OK, "ic_get_blocks 2");
    const size_t per = (size_t)nv * 12 * 12 * 12;
    std::vector<double> U(per * n);
    expect(ic_get_state(s, 0, U.data(), U.size()), IC_OK, "ic_get_state");
    expect(ic_get_state(s, 0, U.data(), U.size() - 1), IC_E_INVALID, "ic_get_state short buffer");
    double t_code = 0, t_s = 0, dt_s = 0;
    long since = 0;
    expect(ic_get_clock(s, 0, &t_code, &since), IC_OK, "ic_get_clock");
    expect(ic_get_time(s, 0, &t_s, &dt_s), IC_OK, "ic_get_time");
    expect(ic_set_state(s, 0, blocks.data(), n, U.data(), t_s), IC_OK, "ic_set_state");
    expect(ic_set_clock(s, 0, t_code, since), IC_OK, "ic_set_clock");
    expect(ic_set_clock(s, 0, NAN, 0), IC_E_INVALID, "ic_set_clock nan");
    std::vector<int32_t> bad_blocks(blocks.begin(), blocks.begin() + 4);
    expect(ic_set_state(s, 0, bad_blocks.data(), 1, U.data(), t_s), IC_E_INVALID, "ic_set_state no tiling");
    long rf = 0, pf = 0;
    expect(ic_floor_counts(s, 0, &rf, &pf), IC_OK, "ic_floor_counts");
    expect(ic_advance(s, 1e12, 6, &info), IC_OK, "ic_advance after restore");
}
}  // namespace

int main()
{
    char tmpl[] = "/tmp/icarus_san_XXXXXX";
    const int fd = mkstemp(tmpl);
    if (fd < 0) return 2;
    close(fd);
    const std::string cache = tmpl;

    // invalid configurations
    {
        ic_grid_cfg g = wedge_grid(3);
        ic_phys_cfg p = phys(0);
        ic_wind_cfg w = wind();
        ic_cme_cfg c = cme();
        ic_amr_cfg a = amr(IC_SOURCE_PLAIN, IC_CRIT_TRACER);
        ic_sim *s = nullptr;
        expect(ic_create(&g, &p, &w, &c, 1, &a, nullptr, &s), IC_E_INVALID, "tracer criterion without tracer");
        g.block[0] = 15;
        a = amr(IC_SOURCE_PLAIN, IC_CRIT_SHOCK);
        expect(ic_create(&g, &p, &w, &c, 1, &a, nullptr, &s), IC_E_INVALID, "block shape");
    }
    // plain and tracer runs with refinement, two members
    for (int tracer = 0; tracer < 2; ++tracer) {
        ic_grid_cfg g = wedge_grid(3);
        ic_phys_cfg p = phys(tracer);
        ic_wind_cfg w = wind();
        ic_cme_cfg c[2] = {cme(), cme()};
        c[1].lon_deg = 50;
        ic_amr_cfg a = amr(IC_SOURCE_PLAIN, tracer ? IC_CRIT_COMBINED : IC_CRIT_SHOCK);
        ic_sim *s = nullptr;
        expect(ic_create(&g, &p, &w, c, 2, &a, nullptr, &s), IC_OK, "ic_create");
        if (!s) break;
        ic_tune_info tune;
        expect(ic_autotune(s, cache.c_str(), 1, &tune), IC_OK, "ic_autotune");
        expect(ic_autotune(s, cache.c_str(), 1, &tune), IC_OK, "ic_autotune cached");
        expect(ic_get_tuning(s, &tune), IC_OK, "ic_get_tuning");
        expect(ic_set_tuning(s, &tune), IC_OK, "ic_set_tuning");
        expect(ic_set_sample_point(s, 1.0, 90.0, 20.0), IC_OK, "ic_set_sample_point");
        expect(ic_set_kernel_timing(s, 1), IC_OK, "ic_set_kernel_timing");
        run_member_calls(s, tracer ? 9 : 8);
        long launches = 0;
        double ms = 0;
        expect(ic_stage_timing(s, &launches, &ms), IC_OK, "ic_stage_timing");
        expect(ic_timeseries_clear(s), IC_OK, "ic_timeseries_clear");
        ic_destroy(s);
    }
    // learned flags: a random network, learned and judged regrids, training and inference
    {
        ic_grid_cfg g = wedge_grid(3);
        ic_phys_cfg p = phys(0);
        ic_wind_cfg w = wind();
        ic_cme_cfg c = cme();
        ic_amr_cfg a = amr(IC_SOURCE_LEARNED_JUDGED, IC_CRIT_SHOCK);
        ic_sim *s = nullptr;
        expect(ic_create(&g, &p, &w, &c, 1, &a, nullptr, &s), IC_OK, "ic_create learned");
        if (s) {
            std::mt19937 rng(7);
            std::normal_distribution<float> nd(0.0f, 0.05f);
            std::vector<float> params(IC_MLP_NPARAM), mean(IC_MLP_IN, 0.0f), sd(IC_MLP_IN, 1.0f);
            for (auto &x : params) x = nd(rng);
            expect(ic_mlp_set(s, params.data(), mean.data(), sd.data()), IC_OK, "ic_mlp_set");
            ic_info info;
            expect(ic_advance(s, 1e12, 16, &info), IC_OK, "ic_advance learned");
            int n = ic_pool_capacity(s);
            std::vector<int32_t> blocks(4 * (size_t)n);
            expect(ic_get_blocks(s, 0, blocks.data(), &n), IC_OK, "ic_get_blocks learned");
            std::vector<float> raw((size_t)n * IC_MLP_IN), prob(n);
            std::vector<int8_t> fl(n);
            expect(ic_features(s, 0, raw.data(), n), IC_OK, "ic_features");
            expect(ic_eval_learned(s, 0, prob.data(), fl.data(), n), IC_OK, "ic_eval_learned");
            long learned = 0, judged = 0, fallbacks = 0;
            double recall = 0;
            expect(ic_regrid_stats(s, &learned, &judged, &fallbacks, &recall), IC_OK, "ic_regrid_stats");
            std::vector<uint8_t> y(n);
            for (int q = 0; q < n; ++q) y[q] = (uint8_t)(q % 3 == 0);
            ic_mlp_hparams hp = {2, 16, 1e-3f, 0.9f, 0.999f, 1e-8f, 1u, 0.0f};
            std::vector<float> tp(IC_MLP_NPARAM), tm(IC_MLP_IN), tsd(IC_MLP_IN), loss(2), grad(IC_MLP_NPARAM);
            expect(ic_mlp_train(raw.data(), y.data(), n, &hp, tp.data(), tm.data(), tsd.data(), loss.data()), IC_OK,
                   "ic_mlp_train");
            expect(ic_mlp_infer(raw.data(), n, tp.data(), tm.data(), tsd.data(), prob.data()), IC_OK,
                   "ic_mlp_infer");
            float l = 0;
            expect(ic_mlp_grad(raw.data(), y.data(), n, 1.0f, tp.data(), grad.data(), &l), IC_OK, "ic_mlp_grad");
            ic_destroy(s);
        }
    }
    // shock diagnostics (host only)
    {
        std::vector<double> t(200), v(200);
        for (int q = 0; q < 200; ++q) {
            t[q] = 1800.0 * q;
            v[q] = 400.0 + 300.0 / (1.0 + std::exp(-(t[q] - 1.5e5) / 3000.0));
        }
        double out[8];
        expect(ic_shock_diagnostics(t.data(), v.data(), 200, 0.0, 4 * 86400.0, 100.0, out), IC_OK,
               "ic_shock_diagnostics");
        t[5] = t[4] - 1.0;
        expect(ic_shock_diagnostics(t.data(), v.data(), 200, 0.0, 4 * 86400.0, 100.0, out), IC_E_INVALID,
               "ic_shock_diagnostics unordered");
    }
    std::remove(cache.c_str());
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
