// C ABI of libxsec: plan object, argument validation, workspace, launch sequencing.
#include "../../include/xsec.h"
#include "xs_internal.hpp"
#include "xs_lineprep.hpp"
#include "xs_forward.hpp"
#include "xs_adjoint.hpp"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <utility>
#include <vector>

namespace {

thread_local std::string g_err;

xs_status fail(xs_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

xs_status hip_fail(hipError_t e, const char* where) {
    return fail(XS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define XS_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct TimedRange {
    hipEvent_t a, b;
    int kind;   // 0 forward, 1 core, 2 prep
};

struct xs_plan {
    xs_opts o{};
    bool timing = false;
    std::vector<TimedRange> timed;
    double acc_ms[3] = {0, 0, 0};
    int64_t acc_n[3] = {0, 0, 0};
    xs::Geometry geo{};
    int P = 2;
    int waves = 4;
    size_t total_bytes = 0;

    // states
    int64_t n_states = 0;
    DevBuf E, g, J;
    // a0 table
    int n_j = 0;
    DevBuf tab_g, tab_n;
    // lines
    int64_t cap = 0, n_lines = 0, n_kept = 0;
    bool have_lines = false;
    DevBuf p_nu, p_elow, p_cA, p_gref, p_nexp, p_kc, p_klo, p_khi;
    DevBuf s_nu, s_elow, s_cA, s_gref, s_nexp, s_kc, s_klo, s_khi, s_orig;
    DevBuf k1, v1, k2, v2, hist, hoff, tsum;
    DevBuf off, flag;
    // FP32 Voigt core pre-pass
    DevBuf core_rc, core_cnt, core_bsum, core_off, core_val, core_tmp;
    DevBuf adj_pT, adj_pP, adj_part;
    int xcd_contiguous = 0;
    int lpt_order = 1;
    DevBuf tile_order;
    int n_order = 0;
    uint32_t* sorted_keys = nullptr;
    // partition function
    int q_cap = 0;
    DevBuf T_dev, Q, dQ, qpart;
    static constexpr int kQBlocks = 256;
    // tables
    xs::Tables tabs{};
    DevBuf tab_dev;

    void release(DevBuf& b) {
        if (b.p) { (void)hipFree(b.p); total_bytes -= b.bytes; }
        b.p = nullptr;
        b.bytes = 0;
    }
    xs_status ensure(DevBuf& b, size_t bytes, const char* what) {
        if (bytes == 0) bytes = 16;
        if (b.p && b.bytes >= bytes) return XS_OK;
        release(b);
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            b.p = nullptr;
            (void)hipGetLastError();
            return fail(XS_ERR_OOM, std::string("device allocation failed for ") + what + " (" +
                                        std::to_string(bytes) + " bytes)");
        }
        b.bytes = bytes;
        total_bytes += bytes;
        return XS_OK;
    }
    void drop_timed() {
        for (auto& t : timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
        timed.clear();
    }
    void release_all() {
        drop_timed();
        DevBuf* all[] = {&E, &g, &J, &tab_g, &tab_n, &p_nu, &p_elow, &p_cA, &p_gref, &p_nexp, &p_kc,
                         &p_klo, &p_khi, &s_nu, &s_elow, &s_cA, &s_gref, &s_nexp, &s_kc, &s_klo,
                         &s_khi, &s_orig, &k1, &v1, &k2, &v2, &hist, &hoff, &tsum, &off, &flag,
                         &T_dev, &Q, &dQ, &qpart, &tab_dev, &core_rc, &core_cnt, &core_bsum,
                         &core_off, &core_val, &core_tmp, &tile_order, &adj_pT, &adj_pP, &adj_part};
        for (DevBuf* b : all) release(*b);
    }
};

namespace {

template <class T>
T* as(DevBuf& b) { return static_cast<T*>(b.p); }

// Event pair around a launch sequence when timing is on.
struct Timer {
    xs_plan* p;
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(xs_plan* p_, hipStream_t s_, int k) : p(p_), s(s_), kind(k) {
        if (p->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else a = b = nullptr;
    }
    void stop() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            p->timed.push_back({a, b, kind});
            a = b = nullptr;
        }
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

xs_status validate_opts(const xs_opts* o) {
    if (!o) return fail(XS_ERR_ARG, "opts is NULL");
    if (!(std::isfinite(o->nu_a) && std::isfinite(o->nu_b) && o->nu_b > o->nu_a))
        return fail(XS_ERR_ARG, "grid needs finite nu_b > nu_a");
    if (o->n_points < 2 || o->n_points > (int64_t)1 << 30)
        return fail(XS_ERR_ARG, "n_points must be in [2, 2^30]");
    if (!(o->cutoff > 0.0) || !std::isfinite(o->cutoff)) return fail(XS_ERR_ARG, "cutoff must be > 0");
    if (!(o->mass_da > 0.0)) return fail(XS_ERR_ARG, "mass_da must be > 0");
    if (!(o->T0 > 0.0) || !(o->P0 > 0.0)) return fail(XS_ERR_ARG, "T0 and P0 must be > 0");
    if (o->profile < XS_DOPPLER || o->profile > XS_GH_BINNED) return fail(XS_ERR_UNSUPPORTED, "unknown profile");
    if (o->precision != XS_FP64 && o->precision != XS_FP32) return fail(XS_ERR_ARG, "unknown precision");
    if (o->broadening < XS_BROAD_CONST || o->broadening > XS_BROAD_A0_JLOWER)
        return fail(XS_ERR_ARG, "unknown broadening scheme");
    if (o->index_base != 0 && o->index_base != 1) return fail(XS_ERR_ARG, "index_base must be 0 or 1");
    if (o->profile == XS_GAUSS_FIXED && !(o->alpha_fixed > 0.0))
        return fail(XS_ERR_ARG, "alpha_fixed must be > 0 for XS_GAUSS_FIXED");
    if (o->broadening == XS_BROAD_CONST && !(o->gamma_const >= 0.0 && std::isfinite(o->n_const)))
        return fail(XS_ERR_ARG, "gamma_const must be >= 0 and n_const finite");
    if (o->slices_per_wave != 0 && o->slices_per_wave != 1 && o->slices_per_wave != 2 && o->slices_per_wave != 4)
        return fail(XS_ERR_ARG, "slices_per_wave must be 0, 1, 2 or 4");
    if (o->a_is_log != 0 && o->a_is_log != 1) return fail(XS_ERR_ARG, "a_is_log must be 0 or 1");
    if (o->waves_per_block != 0 && o->waves_per_block != 4 && o->waves_per_block != 8)
        return fail(XS_ERR_ARG, "waves_per_block must be 0, 4 or 8");
    const double dnu = (o->nu_b - o->nu_a) / (double)(o->n_points - 1);
    if (!(dnu > 0.0)) return fail(XS_ERR_ARG, "grid step underflows");
    const double hw = o->cutoff / dnu;
    if (hw > 4.0e8) return fail(XS_ERR_ARG, "cutoff spans more than 4e8 grid steps");
    if ((double)o->n_points + 2.0 * (hw + 3.0) > 2.0e9) return fail(XS_ERR_ARG, "grid plus cut-off halo too large");
    return XS_OK;
}

}  // namespace

extern "C" {

xs_status xs_opts_default(xs_opts* o) {
    if (!o) return fail(XS_ERR_ARG, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->cutoff = 25.0;
    o->T0 = 296.0;
    o->P0 = 1.0;
    o->profile = XS_VOIGT;
    o->precision = XS_FP32;
    o->broadening = XS_BROAD_PER_LINE;
    o->index_base = 0;
    return XS_OK;
}

xs_status xs_plan_create(const xs_opts* opts, xs_plan** out) {
    if (!out) return fail(XS_ERR_ARG, "out is NULL");
    *out = nullptr;
    xs_status st = validate_opts(opts);
    if (st != XS_OK) return st;
    xs_plan* p = new (std::nothrow) xs_plan();
    if (!p) return fail(XS_ERR_OOM, "host allocation failed");
    p->o = *opts;
    p->P = opts->slices_per_wave ? opts->slices_per_wave : 2;
    p->waves = opts->precision == XS_FP64 ? 4 : (opts->waves_per_block ? opts->waves_per_block : 4);
    if (const char* env = std::getenv("XSEC_XCD_CONTIGUOUS")) p->xcd_contiguous = std::atoi(env) ? 1 : 0;
    if (const char* env = std::getenv("XSEC_TILE_ORDER")) p->lpt_order = std::atoi(env) ? 1 : 0;
    xs::Geometry& G = p->geo;
    G.nu_a = opts->nu_a;
    G.dnu = (opts->nu_b - opts->nu_a) / (double)(opts->n_points - 1);
    G.cutoff = opts->cutoff;
    G.n_points = (int)opts->n_points;
    const double hw = opts->cutoff / G.dnu;
    G.hmax = (int)std::ceil(hw) + 2;
    G.hmin = (int)std::floor(hw) - 2;
    G.nkeys = G.n_points + 2 * G.hmax;
    xs::weideman_coefficients(24, &p->tabs.w24);
    xs::weideman_coefficients(40, &p->tabs.w40);
    xs::make_gh_pairs(2, &p->tabs.gh2);
    xs::make_gh_pairs(4, &p->tabs.gh4);
    xs::make_gh_pairs(6, &p->tabs.gh6);
    xs::make_gh_pairs(12, &p->tabs.gh12);
    xs::gauss_hermite_rule(xs::kGHConv, p->tabs.tconv, p->tabs.wconv);
    for (int j = 0; j < xs::kGHConv; ++j) {
        p->tabs.tconvf[j] = (float)p->tabs.tconv[j];
        p->tabs.wconvf[j] = (float)p->tabs.wconv[j];
    }
    if ((st = p->ensure(p->tab_dev, sizeof(xs::Tables), "quadrature tables")) != XS_OK) { delete p; return st; }
    {
        hipError_t e = hipMemcpy(p->tab_dev.p, &p->tabs, sizeof(xs::Tables), hipMemcpyHostToDevice);
        if (e != hipSuccess) { p->release_all(); delete p; return hip_fail(e, "hipMemcpy(tables)"); }
    }
    *out = p;
    g_err.clear();
    return XS_OK;
}

xs_status xs_plan_destroy(xs_plan* p) {
    if (!p) return XS_OK;
    (void)hipDeviceSynchronize();
    p->release_all();
    delete p;
    return XS_OK;
}

xs_status xs_set_states(xs_plan* p, int64_t n, const double* E, const int32_t* g, const int32_t* J,
                        void* stream) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (n <= 0 || n > ((int64_t)1 << 31) - 1) return fail(XS_ERR_ARG, "n_states must be in [1, 2^31-1]");
    if (!E || !g) return fail(XS_ERR_ARG, "E and g must be non-NULL");
    if (p->o.broadening == XS_BROAD_A0_JLOWER && !J) return fail(XS_ERR_ARG, "J is required for a0 broadening");
    hipStream_t s = static_cast<hipStream_t>(stream);
    p->have_lines = false;
    xs_status st;
    if ((st = p->ensure(p->E, n * sizeof(double), "states E")) != XS_OK) return st;
    if ((st = p->ensure(p->g, n * sizeof(int), "states g")) != XS_OK) return st;
    XS_HIP(hipMemcpyAsync(p->E.p, E, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    XS_HIP(hipMemcpyAsync(p->g.p, g, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (J) {
        if ((st = p->ensure(p->J, n * sizeof(int), "states J")) != XS_OK) return st;
        XS_HIP(hipMemcpyAsync(p->J.p, J, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    p->n_states = n;
    return XS_OK;
}

xs_status xs_set_broadening_table(xs_plan* p, int32_t n_j, const float* gref, const float* nexp) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (n_j <= 0 || !gref || !nexp) return fail(XS_ERR_ARG, "table needs n_j > 0 and both arrays");
    for (int i = 0; i < n_j; ++i)
        if (!(gref[i] >= 0.0f) || !std::isfinite(nexp[i])) return fail(XS_ERR_ARG, "table entries must be finite, gamma >= 0");
    xs_status st;
    if ((st = p->ensure(p->tab_g, n_j * sizeof(float), "a0 table")) != XS_OK) return st;
    if ((st = p->ensure(p->tab_n, n_j * sizeof(float), "a0 table")) != XS_OK) return st;
    XS_HIP(hipMemcpy(p->tab_g.p, gref, n_j * sizeof(float), hipMemcpyHostToDevice));
    XS_HIP(hipMemcpy(p->tab_n.p, nexp, n_j * sizeof(float), hipMemcpyHostToDevice));
    p->n_j = n_j;
    p->have_lines = false;
    return XS_OK;
}

xs_status xs_set_lines(xs_plan* p, int64_t n, const int32_t* upper, const int32_t* lower, const float* A,
                       const float* gref, const float* nexp, void* stream) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(XS_ERR_ARG, "n_lines must be in [0, 2^31-1]");
    if (n > 0 && (!upper || !lower || !A)) return fail(XS_ERR_ARG, "upper, lower and A must be non-NULL");
    const int broad = p->o.broadening;
    if (broad == XS_BROAD_PER_LINE && n > 0 && (!gref || !nexp))
        return fail(XS_ERR_ARG, "per-line broadening needs gamma_ref and n_exp");
    if (broad == XS_BROAD_A0_JLOWER && (p->n_j <= 0 || !p->J.p))
        return fail(XS_ERR_STATE, "a0 broadening needs xs_set_broadening_table and states J");
    hipStream_t s = static_cast<hipStream_t>(stream);
    p->have_lines = false;
    xs_status st;
    if (n > p->cap) {
        const size_t d = n * sizeof(double), f = n * sizeof(float), i4 = n * sizeof(int);
        struct { DevBuf* b; size_t sz; } req[] = {
            {&p->p_nu, d}, {&p->p_elow, d}, {&p->p_cA, d}, {&p->p_gref, f}, {&p->p_nexp, f},
            {&p->p_kc, i4}, {&p->p_klo, i4}, {&p->p_khi, i4},
            {&p->s_nu, d}, {&p->s_elow, d}, {&p->s_cA, d}, {&p->s_gref, f}, {&p->s_nexp, f},
            {&p->s_kc, i4}, {&p->s_klo, i4}, {&p->s_khi, i4}, {&p->s_orig, i4},
            {&p->k1, i4}, {&p->v1, i4}, {&p->k2, i4}, {&p->v2, i4},
            {&p->hist, (size_t)xs::radix_hist_len(n) * 4}, {&p->hoff, (size_t)xs::radix_hist_len(n) * 4},
            {&p->tsum, 4096 * 4}};
        for (auto& r : req) {
            p->release(*r.b);
        }
        p->cap = 0;
        for (auto& r : req)
            if ((st = p->ensure(*r.b, r.sz, "line workspace")) != XS_OK) return st;
        p->cap = n;
    }
    if ((st = p->ensure(p->off, (size_t)(p->geo.nkeys + 1) * sizeof(int), "offsets")) != XS_OK) return st;
    if ((st = p->ensure(p->flag, sizeof(int) * 4, "flags")) != XS_OK) return st;
    XS_HIP(hipMemsetAsync(p->flag.p, 0, sizeof(int), s));
    Timer tprep(p, s, 2);

    xs::PrepArgs a{};
    a.n = n;
    a.upper = upper; a.lower = lower; a.A = A;
    a.gref_line = gref; a.nexp_line = nexp;
    a.gref_tab = as<float>(p->tab_g); a.nexp_tab = as<float>(p->tab_n); a.n_j = p->n_j;
    a.gamma_const = (float)p->o.gamma_const; a.n_const = (float)p->o.n_const;
    a.broad = broad;
    a.index_base = p->o.index_base;
    a.a_is_log = p->o.a_is_log;
    a.E = as<double>(p->E); a.g = as<int>(p->g); a.J = as<int>(p->J);
    a.n_states = p->n_states;
    a.geo = p->geo;
    a.flag = as<int>(p->flag);
    a.p_nu = as<double>(p->p_nu); a.p_elow = as<double>(p->p_elow); a.p_cA = as<double>(p->p_cA);
    a.p_gref = as<float>(p->p_gref); a.p_nexp = as<float>(p->p_nexp);
    a.p_kc = as<int>(p->p_kc); a.p_klo = as<int>(p->p_klo); a.p_khi = as<int>(p->p_khi);
    a.keys = as<uint32_t>(p->k1); a.vals = as<uint32_t>(p->v1);
    XS_HIP(xs::launch_prep(a, s));

    uint32_t *sk = as<uint32_t>(p->k1), *sv = as<uint32_t>(p->v1);
    if (n > 0)
        XS_HIP(xs::launch_radix_sort(as<uint32_t>(p->k1), as<uint32_t>(p->v1), as<uint32_t>(p->k2),
                                     as<uint32_t>(p->v2), n, (uint32_t)p->geo.nkeys, as<uint32_t>(p->hist),
                                     as<uint32_t>(p->hoff), as<uint32_t>(p->tsum), &sk, &sv, s));
    p->sorted_keys = sk;
    xs::GatherArgs ga{};
    ga.n = n; ga.nkeys = p->geo.nkeys; ga.keys = sk; ga.vals = sv;
    ga.p_nu = a.p_nu; ga.p_elow = a.p_elow; ga.p_cA = a.p_cA; ga.p_gref = a.p_gref; ga.p_nexp = a.p_nexp;
    ga.p_kc = a.p_kc; ga.p_klo = a.p_klo; ga.p_khi = a.p_khi;
    ga.nu = as<double>(p->s_nu); ga.elow = as<double>(p->s_elow); ga.cA = as<double>(p->s_cA);
    ga.gref = as<float>(p->s_gref); ga.nexp = as<float>(p->s_nexp); ga.kc = as<int>(p->s_kc);
    ga.klo = as<int>(p->s_klo); ga.khi = as<int>(p->s_khi); ga.orig = as<int>(p->s_orig);
    XS_HIP(xs::launch_gather(ga, s));
    XS_HIP(xs::launch_offsets(sk, n, p->geo.nkeys, as<int>(p->off), s));
    tprep.stop();

    int flag = 0, kept = 0;
    XS_HIP(hipMemcpyAsync(&flag, p->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    XS_HIP(hipMemcpyAsync(&kept, as<int>(p->off) + p->geo.nkeys, sizeof(int), hipMemcpyDeviceToHost, s));
    XS_HIP(hipStreamSynchronize(s));
    if (flag & xs::kFlagIndex) return fail(XS_ERR_INDEX, "a transition's state index is out of range");
    if (flag & xs::kFlagNu) return fail(XS_ERR_NU_NONPOS, "a transition has E[upper] - E[lower] <= 0");
    if (flag & xs::kFlagKey) return fail(XS_ERR_ARG, "internal: window key out of range");
    p->n_lines = n;
    p->n_kept = kept;
    p->n_order = 0;
    if (p->lpt_order && kept > 0) {
        // tiles by decreasing number of overlapping lines (host sort of the tile costs)
        const xs::Geometry& G = p->geo;
        const int W = xs::tile_points(p->P, p->waves);
        const int nt = (G.n_points + W - 1) / W;
        std::vector<int> off(G.nkeys + 1);
        XS_HIP(hipMemcpy(off.data(), p->off.p, off.size() * sizeof(int), hipMemcpyDeviceToHost));
        std::vector<std::pair<int, int>> cost(nt);
        for (int t = 0; t < nt; ++t) {
            const int64_t k0 = (int64_t)t * W;                       // key of kc = t0 - hmax
            const int64_t k1 = std::min<int64_t>((int64_t)t * W + W + 2 * G.hmax, G.nkeys);
            cost[t] = {off[k1] - off[std::min<int64_t>(k0, G.nkeys)], t};
        }
        std::stable_sort(cost.begin(), cost.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first > b.first; });
        std::vector<int> order(nt);
        for (int t = 0; t < nt; ++t) order[t] = cost[t].second;
        if ((st = p->ensure(p->tile_order, nt * sizeof(int), "tile order")) != XS_OK) return st;
        XS_HIP(hipMemcpy(p->tile_order.p, order.data(), nt * sizeof(int), hipMemcpyHostToDevice));
        p->n_order = nt;
    }
    p->have_lines = true;
    return XS_OK;
}

xs_status xs_lines_kept(const xs_plan* p, int64_t* n_kept) {
    if (!p || !n_kept) return fail(XS_ERR_ARG, "NULL argument");
    if (!p->have_lines) return fail(XS_ERR_STATE, "no line set");
    *n_kept = p->n_kept;
    return XS_OK;
}

static xs_status run_partition(xs_plan* p, int nT, const double* T, hipStream_t s) {
    xs_status st;
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0) || !std::isfinite(T[i])) return fail(XS_ERR_ARG, "temperatures must be finite and > 0");
    if (nT > p->q_cap) {
        if ((st = p->ensure(p->T_dev, nT * sizeof(double), "T")) != XS_OK) return st;
        if ((st = p->ensure(p->Q, nT * sizeof(double), "Q")) != XS_OK) return st;
        if ((st = p->ensure(p->dQ, nT * sizeof(double), "dQ")) != XS_OK) return st;
        if ((st = p->ensure(p->qpart, (size_t)2 * nT * xs_plan::kQBlocks * sizeof(double), "Q partials")) != XS_OK)
            return st;
        p->q_cap = nT;
    }
    XS_HIP(hipMemcpyAsync(p->T_dev.p, T, nT * sizeof(double), hipMemcpyHostToDevice, s));
    XS_HIP(xs::launch_partition(as<double>(p->E), as<int>(p->g), p->n_states, as<double>(p->T_dev), nT,
                                as<double>(p->qpart), xs_plan::kQBlocks, as<double>(p->Q), as<double>(p->dQ), s));
    return XS_OK;
}

xs_status xs_partition_function(xs_plan* p, int32_t nT, const double* T, double* Q, double* dQdT, void* stream) {
    if (!p || !T) return fail(XS_ERR_ARG, "NULL argument");
    if (nT <= 0) return fail(XS_ERR_ARG, "n_T must be > 0");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    xs_status st = run_partition(p, nT, T, s);
    if (st != XS_OK) return st;
    if (Q) XS_HIP(hipMemcpyAsync(Q, p->Q.p, nT * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (dQdT) XS_HIP(hipMemcpyAsync(dQdT, p->dQ.p, nT * sizeof(double), hipMemcpyDeviceToDevice, s));
    return XS_OK;
}

xs_status xs_cross_section(xs_plan* p, int32_t n_tp, const double* T, const double* P, void* sigma,
                           void* stream) {
    if (!p || !T || !P || !sigma) return fail(XS_ERR_ARG, "NULL argument");
    if (n_tp <= 0) return fail(XS_ERR_ARG, "n_tp must be > 0");
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    for (int i = 0; i < n_tp; ++i)
        if (!(P[i] >= 0.0) || !std::isfinite(P[i])) return fail(XS_ERR_ARG, "pressures must be finite and >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    xs_status st = run_partition(p, n_tp, T, s);
    if (st != XS_OK) return st;
    const xs_opts& o = p->o;
    // (the FP32 Voigt path waits on the stream once per (T, P) to size its core buffer)
    const bool fp64 = o.precision == XS_FP64;
    const size_t elem = fp64 ? sizeof(double) : sizeof(float);
    const int W = xs::tile_points(p->P, p->waves);
    xs::FwdArgs a{};
    a.L.nu = as<double>(p->s_nu); a.L.elow = as<double>(p->s_elow); a.L.cA = as<double>(p->s_cA);
    a.L.gref = as<float>(p->s_gref); a.L.nexp = as<float>(p->s_nexp); a.L.kc = as<int>(p->s_kc);
    a.L.klo = as<int>(p->s_klo); a.L.khi = as<int>(p->s_khi); a.L.orig = as<int>(p->s_orig);
    a.G = p->geo;
    a.Q = as<double>(p->Q);
    a.off = as<int>(p->off);
    a.n_lines = (int)p->n_kept;
    a.n_tiles = (p->geo.n_points + W - 1) / W;
    a.xcd_contiguous = p->xcd_contiguous;
    a.tile_order = (p->n_order == a.n_tiles) ? as<int>(p->tile_order) : nullptr;
    a.alpha_fixed = o.alpha_fixed;
    a.tab = as<xs::Tables>(p->tab_dev);
    const bool core = !fp64 && o.profile == XS_VOIGT;
    if (core) {
        const size_t n = (size_t)std::max<int64_t>(p->n_kept, 1);
        const size_t nb = (size_t)xs::core_blocks((int64_t)n);
        if ((st = p->ensure(p->core_rc, n * sizeof(int), "core radii")) != XS_OK) return st;
        if ((st = p->ensure(p->core_cnt, n * sizeof(int), "core counts")) != XS_OK) return st;
        if ((st = p->ensure(p->core_off, n * sizeof(long long), "core offsets")) != XS_OK) return st;
        if ((st = p->ensure(p->core_bsum, nb * sizeof(unsigned long long), "core block sums")) != XS_OK) return st;
        if ((st = p->ensure(p->core_tmp, (4096 + 16) * sizeof(unsigned long long), "core scan")) != XS_OK) return st;
        a.core_rc = as<int>(p->core_rc);
        a.core_off = as<long long>(p->core_off);
    }
    const double numax = std::max(std::fabs(o.nu_b), std::fabs(o.nu_a)) + o.cutoff;
    for (int i = 0; i < n_tp; ++i) {
        xs::TPParam& tp = a.tp;
        tp.T = T[i];
        tp.P = P[i];
        tp.c2_over_T = xs::kC2 / T[i];
        tp.beta = std::sqrt(2.0 * xs::kKB * T[i] * xs::kLN2 / (o.mass_da * xs::kAMU)) / xs::kC_SI;
        tp.ln_T0_T = std::log(o.T0 / T[i]);
        tp.p_over_p0 = P[i] / o.P0;
        tp.iq = i;
        // radius (grid steps) beyond which the wing formula holds (Voigt, |x| >= 40) or a
        // Gaussian has underflowed (x^2 >= 110); Lorentz lines need no radius
        double xr = 0.0, alpha = 0.0;
        if (o.profile == XS_VOIGT) { xr = 40.0; alpha = numax * tp.beta; }
        else if (o.profile == XS_DOPPLER) { xr = 10.5; alpha = numax * tp.beta; }
        else if (o.profile == XS_GAUSS_FIXED) { xr = 10.5; alpha = o.alpha_fixed; }
        const double rmd = xr * alpha / (xs::kSQRT_LN2 * p->geo.dnu) + 2.0;
        tp.rm = rmd > 1.0e9 ? 1000000000 : (int)std::ceil(rmd);
        a.seg = (!fp64 && o.profile <= XS_VOIGT && 64.0 * p->P + rmd + 1.0 <= (double)p->geo.hmin) ? 1 : 0;
        a.sigma = static_cast<char*>(sigma) + (size_t)i * (size_t)p->geo.n_points * elem;
        if (core && p->n_kept > 0) {
            xs::CoreArgs c{};
            c.L = a.L; c.G = a.G; c.tp = tp; c.Q = a.Q; c.n_lines = a.n_lines; c.tab = a.tab;
            c.rc = as<int>(p->core_rc); c.cnt = as<int>(p->core_cnt);
            c.bsum = as<unsigned long long>(p->core_bsum); c.coff = as<long long>(p->core_off);
            c.scan_tmp = as<unsigned long long>(p->core_tmp);
            Timer tc(p, s, 1);
            XS_HIP(xs::launch_core_count(c, s));
            tc.stop();
            unsigned long long total = 0;
            XS_HIP(hipMemcpyAsync(&total, as<unsigned long long>(p->core_tmp) + 4096, sizeof(total),
                                  hipMemcpyDeviceToHost, s));
            XS_HIP(hipStreamSynchronize(s));
            if ((st = p->ensure(p->core_val, (size_t)std::max<unsigned long long>(total, 1) * sizeof(float),
                                "core values")) != XS_OK)
                return st;
            c.val = as<float>(p->core_val);
            Timer te(p, s, 1);
            XS_HIP(xs::launch_core_eval(c, s));
            te.stop();
            a.core_val = c.val;
        }
        Timer tf(p, s, 0);
        XS_HIP(xs::launch_forward(o.profile, fp64 ? 1 : 0, p->waves, p->P, a, s));
        tf.stop();
    }
    return XS_OK;
}

xs_status xs_cross_section_adjoint(xs_plan* p, double T, double P, const void* gbar, double* dT, double* dP,
                                   void* dlnA, void* dgref, void* dn, void* stream) {
    if (!p || !gbar) return fail(XS_ERR_ARG, "NULL argument");
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    if (p->o.profile != XS_VOIGT) return fail(XS_ERR_UNSUPPORTED, "the adjoint is implemented for XS_VOIGT");
    if ((dgref || dn) && p->o.broadening != XS_BROAD_PER_LINE)
        return fail(XS_ERR_UNSUPPORTED, "gamma_ref / n gradients need per-line broadening");
    if (!(P >= 0.0) || !std::isfinite(P)) return fail(XS_ERR_ARG, "pressure must be finite and >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    xs_status st = run_partition(p, 1, &T, s);
    if (st != XS_OK) return st;
    const size_t n = (size_t)std::max<int64_t>(p->n_kept, 1);
    if ((st = p->ensure(p->adj_pT, n * sizeof(double), "adjoint partials")) != XS_OK) return st;
    if ((st = p->ensure(p->adj_pP, n * sizeof(double), "adjoint partials")) != XS_OK) return st;
    if ((st = p->ensure(p->adj_part, 512 * sizeof(double), "adjoint reduction")) != XS_OK) return st;
    const xs_opts& o = p->o;
    xs::AdjArgs a{};
    a.L.nu = as<double>(p->s_nu); a.L.elow = as<double>(p->s_elow); a.L.cA = as<double>(p->s_cA);
    a.L.gref = as<float>(p->s_gref); a.L.nexp = as<float>(p->s_nexp); a.L.kc = as<int>(p->s_kc);
    a.L.klo = as<int>(p->s_klo); a.L.khi = as<int>(p->s_khi); a.L.orig = as<int>(p->s_orig);
    a.G = p->geo;
    a.tp.T = T;
    a.tp.P = P;
    a.tp.c2_over_T = xs::kC2 / T;
    a.tp.beta = std::sqrt(2.0 * xs::kKB * T * xs::kLN2 / (o.mass_da * xs::kAMU)) / xs::kC_SI;
    a.tp.ln_T0_T = std::log(o.T0 / T);
    a.tp.p_over_p0 = P / o.P0;
    a.P0 = o.P0;
    a.Q = as<double>(p->Q);
    a.dQ = as<double>(p->dQ);
    a.gbar = gbar;
    a.n_lines = (int)p->n_kept;
    a.tab = as<xs::Tables>(p->tab_dev);
    a.dlnA = dlnA; a.dgref = dgref; a.dn = dn;
    a.pT = as<double>(p->adj_pT);
    a.pP = as<double>(p->adj_pP);
    Timer tf(p, s, 0);
    XS_HIP(xs::launch_adjoint(a, o.precision == XS_FP64 ? 1 : 0, p->n_lines, as<double>(p->adj_part), dT, dP, s));
    tf.stop();
    return XS_OK;
}

xs_status xs_set_timing(xs_plan* p, int enable) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (enable) {
        p->drop_timed();
        for (int k = 0; k < 3; ++k) { p->acc_ms[k] = 0; p->acc_n[k] = 0; }
    }
    p->timing = enable != 0;
    return XS_OK;
}

xs_status xs_kernel_times(xs_plan* p, xs_timings* out) {
    if (!p || !out) return fail(XS_ERR_ARG, "NULL argument");
    for (auto& t : p->timed) {
        XS_HIP(hipEventSynchronize(t.b));
        float ms = 0.0f;
        XS_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        p->acc_ms[t.kind] += ms;
        p->acc_n[t.kind] += 1;
    }
    p->drop_timed();
    out->forward_ms = p->acc_ms[0];
    out->core_ms = p->acc_ms[1];
    out->prep_ms = p->acc_ms[2];
    out->forward_launches = p->acc_n[0];
    out->core_launches = p->acc_n[1];
    out->prep_launches = p->acc_n[2];
    return XS_OK;
}

size_t xs_workspace_bytes(const xs_plan* p) { return p ? p->total_bytes : 0; }

const char* xs_last_error(void) { return g_err.c_str(); }

int xs_version(void) { return XS_ABI_VERSION; }

}  // extern "C"
