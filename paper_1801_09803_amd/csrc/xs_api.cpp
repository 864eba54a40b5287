// C ABI of libxsec: plan object, argument validation, workspace, launch sequencing of
// the batched cross-section pipeline, its graph capture, and the tile-shape autotuner.
#include "../../include/xsec.h"
#include "xs_internal.hpp"
#include "xs_lineprep.hpp"
#include "xs_forward.hpp"
#include "xs_adjoint.hpp"
#include "xs_states.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
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

#define XS_TRY(call)                                          \
    do {                                                      \
        xs_status s_ = (call);                                \
        if (s_ != XS_OK) return s_;                           \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

void dev_release(DevBuf& b, size_t* total) {
    if (b.p) { (void)hipFree(b.p); *total -= b.bytes; }
    b.p = nullptr;
    b.bytes = 0;
}

// Device allocation with accounting; a buffer is only replaced when it must grow.
xs_status dev_ensure(DevBuf& b, size_t bytes, const char* what, size_t* total) {
    if (bytes == 0) bytes = 16;
    if (b.p && b.bytes >= bytes) return XS_OK;
    dev_release(b, total);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(XS_ERR_OOM, std::string("device allocation failed for ") + what + " (" +
                                    std::to_string(bytes) + " bytes)");
    }
    b.bytes = bytes;
    *total += bytes;
    return XS_OK;
}

// Pinned host staging buffer for the small per-call copies (temperatures, per-(T, P)
// parameters, count read-back).  Copies from it are asynchronous, so it is rewritten
// only after the event recorded behind the last copy has completed.
struct Stage {
    void* h = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;

    xs_status get(size_t bytes, void** out) {
        if (pending) {
            XS_HIP(hipEventSynchronize(ev));
            pending = false;
        }
        if (bytes > cap) {
            if (h) (void)hipHostFree(h);
            h = nullptr;
            cap = 0;
            XS_HIP(hipHostMalloc(&h, bytes, hipHostMallocDefault));
            cap = bytes;
        }
        if (!ev) XS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        *out = h;
        return XS_OK;
    }
    xs_status record(hipStream_t s) {
        XS_HIP(hipEventRecord(ev, s));
        pending = true;
        return XS_OK;
    }
    void release() {
        if (pending) (void)hipEventSynchronize(ev);
        pending = false;
        if (h) (void)hipHostFree(h);
        if (ev) (void)hipEventDestroy(ev);
        h = nullptr;
        ev = nullptr;
        cap = 0;
    }
};

// Device buffers of the batched cross-section pipeline: one set per plan for direct
// calls and one per captured graph (a graph replays against its own buffers).
struct Workset {
    DevBuf T, Q, dQ, qpart;   // temperatures of the call, Q(T), dQ/dT, partial sums
    DevBuf tps;               // xs::TPParam per (T, P) of the call
    DevBuf rc, cnt, coff;     // core pre-pass rows [tp_block][n_kept]
    DevBuf bsum, tmp;         // per row: core count block sums, scan scratch
    DevBuf val;               // core values of one block of (T, P)
    DevBuf hot, cold, xscale; // FP32 line records [tp_block][n_kept] (32 or 48 + 64 + 8 B per line)
    DevBuf vv;                // Vectorized Voigt {beta, intensity factor} [tp_block][n_kept]
    DevBuf sl;                // super-lines: per-line intensities [tp_block][n_kept]
    DevBuf th_bsum, th_tmp;   // intensity threshold: block counts, scan scratch per row
    DevBuf th_pos, th_map, th_offs;   // per row: positions [n+1], kept lines [n], offsets [nkeys+1]
    DevBuf part;              // per-part sums [tp_block][n_split][n_points] when n_split > 1
    DevBuf far;               // FP32 Voigt: node-sampled far-wing sums [tp_block][2][n_points]
    DevBuf far_nodes;         // FP32 Voigt: far kernel node totals [tp_block][waves][16][kFarShares]
    DevBuf out;               // autotuner output scratch
    size_t bytes = 0;
    Stage stage;
    int rows = 0;             // core rows allocated
    int64_t row_stride = 0;

    xs_status ensure(DevBuf& b, size_t n, const char* what) { return dev_ensure(b, n, what, &bytes); }
    void release() {
        DevBuf* all[] = {&T, &Q, &dQ, &qpart, &tps, &rc, &cnt, &coff, &bsum, &tmp, &val, &hot, &cold, &xscale,
                         &vv, &sl, &th_bsum, &th_tmp, &th_pos, &th_map, &th_offs, &part, &far, &far_nodes, &out};
        for (DevBuf* b : all) dev_release(*b, &bytes);
        stage.release();
        rows = 0;
        row_stride = 0;
    }
};

constexpr int kScanTmp = 4096 + 16;   // u64 scan scratch per core row (total at [4096])

}  // namespace

struct TimedRange {
    hipEvent_t a, b;
    int kind;   // 0 forward, 1 core, 2 prep, 3 combine
    int ntp;    // (T, P) results covered (forward launches)
};

struct xs_plan {
    xs_opts o{};
    bool timing = false;
    std::vector<TimedRange> timed;
    double acc_ms[5] = {0, 0, 0, 0, 0};
    int64_t acc_n[5] = {0, 0, 0, 0, 0};
    int64_t acc_tp = 0;
    xs::Geometry geo{};
    int P = 2;
    int waves = 4;
    int n_split = 0;        // 0: chosen per call
    int tp_block = 0;       // 0: chosen per call
    int th_mode = 0;        // intensity threshold: 0 none, 1 constant, 2 HITRAN
    double th_icrit = 0.0, th_nucrit = 0.0;
    int emission = 0;       // 1: cross sections sum emissivities instead of Eq. 1 intensities
    bool has_vib = false;   // non-LTE: states carry vibrational energies (xs_set_vibrational_labels)
    bool lines_vib = false; // the line set carries its states' vibrational energies
    int last_split = 0, last_block = 0;
    uint64_t generation = 1;   // bumped whenever captured graphs become invalid
    // FP32 Voigt: bound of one (T, P)'s core values over the line set (any Lorentz width,
    // any T up to core_bound_T), valid while generation == core_bound_gen
    long long core_bound = 0;
    double core_bound_T = 0.0;
    uint64_t core_bound_gen = 0;
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
    DevBuf p_rec;              // prepared lines in the caller's order (xs::PrepRec)
    DevBuf s_nu, s_elow, s_cA, s_gref, s_nexp, s_kc, s_klo, s_khi, s_orig;
    DevBuf k1, v1, k2, v2, hist, hoff, tsum;
    DevBuf off, flag;
    DevBuf adj_pT, adj_pP, adj_part, adj_rec, adj_sums;
    int xcd_contiguous = 0;
    int lpt_order = 1;
    DevBuf tile_order;
    int n_order = 0, order_W = 0;
    std::vector<int> off_host;     // offsets table (host copy) for tile costs
    uint32_t* sorted_keys = nullptr;
    // partition function (xs_partition_function and the adjoint)
    int q_cap = 0;
    DevBuf T_dev, Q, dQ, qpart;
    static constexpr int kQBlocks = 256;
    // state reductions (moments, lifetimes, cooling function)
    int st_cap = 0;
    DevBuf st_T, st_part, st_sumA, st_power;
    // non-LTE: per-state vibrational energies, manifold minima, per sorted line E_vib
    DevBuf Ev, vmin, s_evl, s_evu;
    // bucketed per-state sums: histogram, offsets, scan scratch, records
    DevBuf st_bhist, st_bhoff, st_btsum, st_brec;
    // batched cross-section pipeline of direct calls
    Workset ws;
    // tables
    xs::Tables tabs{};
    DevBuf tab_dev;

    void release(DevBuf& b) { dev_release(b, &total_bytes); }
    xs_status ensure(DevBuf& b, size_t bytes, const char* what) { return dev_ensure(b, bytes, what, &total_bytes); }
    void drop_timed() {
        for (auto& t : timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
        timed.clear();
    }
    void release_all() {
        drop_timed();
        DevBuf* all[] = {&E, &g, &J, &tab_g, &tab_n, &p_rec, &s_nu, &s_elow, &s_cA, &s_gref, &s_nexp, &s_kc, &s_klo,
                         &s_khi, &s_orig, &k1, &v1, &k2, &v2, &hist, &hoff, &tsum, &off, &flag,
                         &T_dev, &Q, &dQ, &qpart, &tab_dev, &tile_order, &adj_pT, &adj_pP, &adj_part, &adj_rec,
                         &adj_sums, &st_T, &st_part, &st_sumA, &st_power, &Ev, &vmin, &s_evl, &s_evu, &st_bhist, &st_bhoff, &st_btsum, &st_brec};
        for (DevBuf* b : all) release(*b);
        ws.release();
    }
};

// A captured launch sequence of xs_cross_section for fixed (T, P) capacities.
struct xs_graph {
    xs_plan* p = nullptr;
    uint64_t generation = 0;
    int n_tp = 0;
    std::vector<double> T_cap;
    std::vector<xs::TPParam> tps;
    Workset ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Line-list streaming: chunks of transitions from host memory, accumulated on device.
struct xs_stream {
    xs_plan* p = nullptr;
    int n_tp = 0;
    std::vector<double> T, P;
    void* sigma = nullptr;        // caller's output [n_tp][n_points]
    hipStream_t compute = nullptr;
    hipStream_t copy = nullptr;   // host-to-device copies of chunks
    hipEvent_t copied[2] = {nullptr, nullptr};
    DevBuf acc, tmp;              // (sum, compensation) per value; last chunk's cross sections
    DevBuf raw[2][5];             // per slot: upper, lower, A, gamma_ref, n_exp
    int64_t raw_cap[2] = {0, 0};
    bool have_pending = false;    // a copied chunk awaiting its computation
    int pending_slot = 0;
    int64_t pending_n = 0;
    bool pending_broad = false;
    int64_t chunks = 0, lines = 0, kept = 0;
    int emission = 0;             // the plan's intensity kind when the stream began
    size_t bytes = 0;
};

namespace {

template <class T>
T* as(DevBuf& b) { return static_cast<T*>(b.p); }

// Event pair around a launch sequence when timing is on.
struct Timer {
    xs_plan* p;
    hipStream_t s;
    int kind, ntp;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(xs_plan* p_, hipStream_t s_, int k, int ntp_ = 0, bool on = true) : p(p_), s(s_), kind(k), ntp(ntp_) {
        if (on && p->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else {
            if (a) (void)hipEventDestroy(a);
            a = b = nullptr;
        }
    }
    void stop() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            p->timed.push_back({a, b, kind, ntp});
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
    if (o->profile < XS_DOPPLER || o->profile > XS_SUPERLINES) return fail(XS_ERR_UNSUPPORTED, "unknown profile");
    if (o->vv_beta != 0 && o->vv_beta != 1) return fail(XS_ERR_ARG, "vv_beta must be 0 or 1");
    if (!(o->vv_radius >= 0.0) || !std::isfinite(o->vv_radius)) return fail(XS_ERR_ARG, "vv_radius must be >= 0");
    if (o->precision != XS_FP64 && o->precision != XS_FP32) return fail(XS_ERR_ARG, "unknown precision");
    if (o->broadening < XS_BROAD_CONST || o->broadening > XS_BROAD_A0_JLOWER)
        return fail(XS_ERR_ARG, "unknown broadening scheme");
    if (o->index_base != 0 && o->index_base != 1) return fail(XS_ERR_ARG, "index_base must be 0 or 1");
    if (o->profile == XS_GAUSS_FIXED && !(o->alpha_fixed > 0.0))
        return fail(XS_ERR_ARG, "alpha_fixed must be > 0 for XS_GAUSS_FIXED");
    if (o->broadening == XS_BROAD_CONST && !(o->gamma_const >= 0.0 && std::isfinite(o->n_const)))
        return fail(XS_ERR_ARG, "gamma_const must be >= 0 and n_const finite");
    if (o->slices_per_wave != 0 && o->slices_per_wave != 1 && o->slices_per_wave != 2 && o->slices_per_wave != 4 &&
        o->slices_per_wave != 8)
        return fail(XS_ERR_ARG, "slices_per_wave must be 0, 1, 2, 4 or 8");
    if (o->slices_per_wave == 8 && (o->precision != XS_FP32 || o->waves_per_block > 2))
        return fail(XS_ERR_ARG, "8 slices per wavefront need XS_FP32 and 1 or 2 wavefronts per workgroup");
    if (o->a_is_log != 0 && o->a_is_log != 1) return fail(XS_ERR_ARG, "a_is_log must be 0 or 1");
    if (o->waves_per_block != 0 && o->waves_per_block != 1 && o->waves_per_block != 2 && o->waves_per_block != 4 &&
        o->waves_per_block != 8)
        return fail(XS_ERR_ARG, "waves_per_block must be 0, 1, 2, 4 or 8");
    if (o->n_split < 0 || o->n_split > 64) return fail(XS_ERR_ARG, "n_split must be in [0, 64]");
    if (o->tp_block < 0 || o->tp_block > 256) return fail(XS_ERR_ARG, "tp_block must be in [0, 256]");
    if (o->gh_nodes < 0 || o->gh_nodes > xs::kMaxGHConv) return fail(XS_ERR_ARG, "gh_nodes must be in [0, 64]");
    const double dnu = (o->nu_b - o->nu_a) / (double)(o->n_points - 1);
    if (!(dnu > 0.0)) return fail(XS_ERR_ARG, "grid step underflows");
    const double hw = o->cutoff / dnu;
    if (hw > 4.0e8) return fail(XS_ERR_ARG, "cutoff spans more than 4e8 grid steps");
    if ((double)o->n_points + 2.0 * (hw + 3.0) > 2.0e9) return fail(XS_ERR_ARG, "grid plus cut-off halo too large");
    return XS_OK;
}

// ------------------------------------------------------------ batched pipeline
int tile_width(const xs_plan* p) { return xs::tile_points(p->P, p->o.precision == XS_FP64 ? 4 : p->waves); }

int n_tiles(const xs_plan* p) {
    const int W = tile_width(p);
    return (p->geo.n_points + W - 1) / W;
}

// Dispatch order of the tiles of the current width: decreasing number of overlapping
// lines (longest processing time first).  Synchronous (the table is small).
xs_status build_tile_order(xs_plan* p) {
    const int W = tile_width(p);
    const int nt = n_tiles(p);
    if (p->order_W == W && p->n_order == nt) return XS_OK;
    p->n_order = 0;
    p->order_W = 0;
    if (!p->lpt_order || p->n_kept <= 0 || (int64_t)p->off_host.size() != (int64_t)p->geo.nkeys + 1) return XS_OK;
    const xs::Geometry& G = p->geo;
    std::vector<std::pair<int, int>> cost(nt);
    for (int t = 0; t < nt; ++t) {
        const int64_t k0 = std::min<int64_t>((int64_t)t * W, G.nkeys);           // key of kc = t0 - hmax
        const int64_t k1 = std::min<int64_t>((int64_t)t * W + W + 2 * G.hmax, G.nkeys);
        cost[t] = {p->off_host[k1] - p->off_host[k0], t};
    }
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first > b.first; });
    std::vector<int> order(nt);
    for (int t = 0; t < nt; ++t) order[t] = cost[t].second;
    XS_TRY(p->ensure(p->tile_order, nt * sizeof(int), "tile order"));
    XS_HIP(hipMemcpy(p->tile_order.p, order.data(), nt * sizeof(int), hipMemcpyHostToDevice));
    p->n_order = nt;
    p->order_W = W;
    return XS_OK;
}

bool is_vv(const xs_plan* p) { return p->o.profile == XS_VVOIGT || p->o.profile == XS_VVOIGT_NORM; }

// Voigt-like profiles: the Voigt zones (and, on the FP32 path, its core pre-pass) apply
bool voigt_like(const xs_plan* p) { return p->o.profile == XS_VOIGT || is_vv(p); }

double beta_of(const xs_opts& o, double T) {
    // Eq. 16: alpha_D = nu sqrt(2 k T ln2 / m) / c
    return std::sqrt(2.0 * xs::kKB * T * xs::kLN2 / (o.mass_da * xs::kAMU)) / xs::kC_SI;
}

// Radius in grid steps beyond which every point of a line is in the FP32 path's far
// zone (Voigt: |x| >= 40) or a Gaussian has underflowed (x^2 >= 110), for every
// temperature up to T_rm (the Doppler width grows with T).  Lorentz lines need none.
double rm_steps(const xs_plan* p, double T_rm) {
    const xs_opts& o = p->o;
    const double numax = std::max(std::fabs(o.nu_b), std::fabs(o.nu_a)) + o.cutoff;
    double xr = 0.0, alpha = 0.0;
    if (o.profile == XS_VOIGT || o.profile == XS_VVOIGT || o.profile == XS_VVOIGT_NORM) {
        xr = 40.0;
        alpha = numax * beta_of(o, T_rm);
    }
    else if (o.profile == XS_DOPPLER) { xr = 10.5; alpha = numax * beta_of(o, T_rm); }
    else if (o.profile == XS_GAUSS_FIXED) { xr = 10.5; alpha = o.alpha_fixed; }
    return xr * alpha / (xs::kSQRT_LN2 * p->geo.dnu) + 2.0;
}

xs::TPParam make_tp(const xs_plan* p, double T, double P, int iq, double T_rm) {
    const xs_opts& o = p->o;
    xs::TPParam tp{};
    tp.T = T;
    tp.P = P;
    tp.Tv = T;   // LTE unless the call gives vibrational temperatures
    tp.c2_over_T = xs::kC2 / T;
    tp.beta = beta_of(o, T);
    tp.ln_T0_T = std::log(o.T0 / T);
    tp.p_over_p0 = P / o.P0;
    tp.iq = iq;
    tp.emission = p->emission;
    const double rmd = rm_steps(p, T_rm);
    tp.rm = rmd > 1.0e9 ? 1000000000 : (int)std::ceil(rmd);
    // the same radius for a line of wavenumber nu: xr alpha_D(nu) / (sqrt(ln2) dnu)
    const double xr = voigt_like(p) ? 40.0 : p->o.profile == XS_DOPPLER ? 10.5 : 0.0;
    tp.rm_scale = xr * beta_of(p->o, T_rm) / (xs::kSQRT_LN2 * p->geo.dnu);
    return tp;
}

// Vectorized Voigt pre-pass needed: continuity factors or area normalisation
bool vv_needed(const xs_plan* p) { return is_vv(p) && (p->o.vv_beta || p->o.profile == XS_VVOIGT_NORM); }

// FP32 Voigt: the segmented sweep leaves lines far from a wavefront to the node-sampled
// far-wing kernel, whose per-share node totals need a buffer of at most kFarShares shares
constexpr int kFarShares = 256;
// grid steps between a wavefront of ww points and the nearest node-sampled line centre (the
// kernels' far_reach: 0.57 (ww - 1), rounded up, for the 16 Chebyshev nodes across it)
int far_reach_steps(int ww) { return (57 * (ww - 1) + 99) / 100; }
bool far_sampled(const xs_plan* p) { return p->o.precision == XS_FP32 && p->o.profile == XS_VOIGT; }

// Profile index of the kernels (the area-normalised form differs in its intensities only)
int kernel_profile(const xs_plan* p) {
    switch (p->o.profile) {
        case XS_VVOIGT:
        case XS_VVOIGT_NORM: return xs::kVVoigt;
        case XS_DOPPLER_BINNED: return xs::kDopplerBinned;
        case XS_LORENTZ_BINNED: return xs::kLorentzBinned;
        case XS_SUPERLINES: return xs::kSuperLines;
        default: return p->o.profile;
    }
}

bool superlines(const xs_plan* p) { return p->o.profile == XS_SUPERLINES; }

int hot_words(const xs_plan* p) { return is_vv(p) ? 12 : 8; }

bool core_path(const xs_plan* p) { return p->o.precision == XS_FP32 && voigt_like(p); }

bool fp32_path(const xs_plan* p) { return p->o.precision == XS_FP32; }

// FP32 line records (every profile of the FP32 tile kernel; super-lines read the lines)
bool records_path(const xs_plan* p) { return fp32_path(p) && !superlines(p); }

bool threshold_on(const xs_plan* p) { return p->th_mode != 0; }

// The Vectorized Voigt wing uses the Lorentzian (FP32) or the 2-node rule (FP64) for the
// reference profile: both need x_ref = sqrt(ln2) R / alpha_ref >= 2e4 at every temperature.
xs_status check_vv(const xs_plan* p, int n, const double* T) {
    if (!is_vv(p) || !(p->geo.vv_radius < p->o.cutoff)) return XS_OK;
    for (int i = 0; i < n; ++i) {
        const double xr = xs::kSQRT_LN2 * p->geo.vv_radius / beta_of(p->o, T[i]);
        if (!(xr >= 2.0e4))
            return fail(XS_ERR_ARG, "vv_radius too small for the reference profile at T = " + std::to_string(T[i]) +
                                        " K (needs sqrt(ln2) R / alpha_ref >= 2e4)");
    }
    return XS_OK;
}

// Bytes of per-(line, T, P) workspace: FP32 line records (104 or 120 B), Voigt core rows
// (16 B) and Vectorized Voigt factors (16 B).
int64_t row_bytes_per_line(const xs_plan* p) {
    return (records_path(p) ? 72 + 4 * hot_words(p) : 0) + (core_path(p) ? 16 : 0) + (vv_needed(p) ? 16 : 0) +
           (threshold_on(p) ? 8 : 0);
}

int pick_block(const xs_plan* p, int n_tp) {
    int B = p->tp_block > 0 ? p->tp_block : 8;
    if (p->tp_block <= 0 && row_bytes_per_line(p) > 0) {
        // keep the per-(T, P) rows of a block within 24 GiB
        const int64_t cap = ((int64_t)24 << 30) / std::max<int64_t>(row_bytes_per_line(p) * p->n_kept, 1);
        B = (int)std::max<int64_t>(1, std::min<int64_t>(B, cap));
    }
    return std::max(1, std::min(B, n_tp));
}

// Workgroups per tile: ~24000 workgroups per (T, P) (the chip holds ~1300 at once, so
// the heavy-first order ends with a short tail), each share keeping at least four LDS
// batches of lines.  It depends on the plan only, so a (T, P) result does not depend
// on the other points of its call.
int pick_split(const xs_plan* p) {
    if (superlines(p)) return 1;   // one thread per grid point, no shares
    if (p->n_split > 0) return p->n_split;
    const int nt = n_tiles(p);
    const xs::Geometry& G = p->geo;
    const double per_tile = (double)p->n_kept * (double)(tile_width(p) + 2 * G.hmax) / std::max(1, G.nkeys);
    const double batch = 64.0 * (p->o.precision == XS_FP64 ? 4 : p->waves);
    int S = 1;
    while (S < 32 && (int64_t)nt * S < 24000 && per_tile / (2.0 * S) >= 4.0 * batch) S *= 2;
    return S;
}

// FP32 sweep mode of a (T, P): per-wavefront line segments when the fast-path radius
// leaves room inside the half window, per-slice codes otherwise.
bool seg_mode(const xs_plan* p, const xs::TPParam& tp) {
    // (Vectorized Voigt: the windows' outer ends must also lie beyond R)
    return p->o.precision == XS_FP32 && (p->o.profile <= XS_VOIGT || is_vv(p)) &&
           64.0 * p->P + (double)tp.rm + 1.0 <= (double)p->geo.hmin &&
           (!is_vv(p) || 64.0 * p->P + (double)p->geo.rvmax + 1.0 <= (double)p->geo.hmin);
}

// Core rows and per-part buffers for blocks of B (T, P) split S ways.
xs_status ensure_rows(xs_plan* p, Workset& ws, int B, int S) {
    const int64_t n = std::max<int64_t>(p->n_kept, 1);
    if (vv_needed(p)) {
        XS_TRY(ws.ensure(ws.vv, (size_t)B * n * 2 * sizeof(double), "Vectorized Voigt factors"));
        ws.rows = B;
        ws.row_stride = n;
    }
    if (threshold_on(p)) {
        const int64_t nb = xs::core_blocks(n);
        XS_TRY(ws.ensure(ws.th_bsum, (size_t)B * nb * sizeof(unsigned long long), "threshold block counts"));
        XS_TRY(ws.ensure(ws.th_tmp, (size_t)B * kScanTmp * sizeof(unsigned long long), "threshold scan"));
        XS_TRY(ws.ensure(ws.th_pos, (size_t)B * (n + 1) * sizeof(unsigned), "threshold positions"));
        XS_TRY(ws.ensure(ws.th_map, (size_t)B * n * sizeof(int), "threshold map"));
        XS_TRY(ws.ensure(ws.th_offs, (size_t)B * ((size_t)p->geo.nkeys + 1) * sizeof(int), "threshold offsets"));
        ws.rows = B;
        ws.row_stride = n;
    }
    if (superlines(p)) {
        XS_TRY(ws.ensure(ws.sl, (size_t)B * n * sizeof(double), "super-line intensities"));
        ws.rows = B;
        ws.row_stride = n;
    }
    if (records_path(p)) {
        XS_TRY(ws.ensure(ws.hot, (size_t)B * n * hot_words(p) * sizeof(float), "line records"));
        XS_TRY(ws.ensure(ws.cold, (size_t)B * n * 16 * sizeof(int), "line records"));
        XS_TRY(ws.ensure(ws.xscale, (size_t)B * n * sizeof(double), "line records"));
        ws.rows = B;
        ws.row_stride = n;
    }
    if (core_path(p)) {
        const int64_t nb = xs::core_blocks(n);
        XS_TRY(ws.ensure(ws.rc, (size_t)B * n * sizeof(int), "core radii"));
        XS_TRY(ws.ensure(ws.cnt, (size_t)B * n * sizeof(int), "core counts"));
        XS_TRY(ws.ensure(ws.coff, (size_t)B * n * sizeof(long long), "core offsets"));
        XS_TRY(ws.ensure(ws.bsum, (size_t)B * nb * sizeof(unsigned long long), "core block sums"));
        XS_TRY(ws.ensure(ws.tmp, (size_t)B * kScanTmp * sizeof(unsigned long long), "core scan"));
        ws.rows = B;
        ws.row_stride = n;
    }
    if (S > 1) {
        const size_t elem = p->o.precision == XS_FP64 ? sizeof(double) : 2 * sizeof(float);
        XS_TRY(ws.ensure(ws.part, (size_t)B * S * (size_t)p->geo.n_points * elem, "split partial sums"));
    }
    if (far_sampled(p)) {
        XS_TRY(ws.ensure(ws.far, (size_t)B * 2 * (size_t)p->geo.n_points * sizeof(double), "far-wing sums"));
        // wavefronts of 64 points or more over the grid, a whole tile of them past its end
        const size_t waves = (size_t)p->geo.n_points / 64 + 2 + 8;
        XS_TRY(ws.ensure(ws.far_nodes, (size_t)B * waves * 16 * kFarShares * sizeof(double), "far-wing node sums"));
    }
    return XS_OK;
}

xs::SortedLines sorted_lines(xs_plan* p) {
    xs::SortedLines L{};
    L.nu = as<double>(p->s_nu); L.elow = as<double>(p->s_elow); L.cA = as<double>(p->s_cA);
    L.gref = as<float>(p->s_gref); L.nexp = as<float>(p->s_nexp); L.kc = as<int>(p->s_kc);
    L.klo = as<int>(p->s_klo); L.khi = as<int>(p->s_khi); L.orig = as<int>(p->s_orig);
    L.evl = p->lines_vib ? as<double>(p->s_evl) : nullptr;
    L.evu = p->lines_vib ? as<double>(p->s_evu) : nullptr;
    return L;
}

// Core pre-pass arguments of the call's (T, P) point `it` in core row `row`.
xs::CoreArgs core_args(xs_plan* p, Workset& ws, int it, int row) {
    xs::CoreArgs c{};
    const int64_t n = ws.row_stride, nb = xs::core_blocks(n);
    c.L = sorted_lines(p);
    c.G = p->geo;
    c.tp = as<xs::TPParam>(ws.tps) + it;
    c.Q = as<double>(ws.Q);
    c.n_lines = (int)p->n_kept;
    c.kept_pos = threshold_on(p) ? as<unsigned>(ws.th_pos) + (int64_t)row * (n + 1) : nullptr;
    c.tab = as<xs::Tables>(p->tab_dev);
    c.rc = as<int>(ws.rc) + row * n;
    c.cnt = as<int>(ws.cnt) + row * n;
    c.coff = as<long long>(ws.coff) + row * n;
    c.bsum = as<unsigned long long>(ws.bsum) + row * nb;
    c.scan_tmp = as<unsigned long long>(ws.tmp) + (int64_t)row * kScanTmp;
    c.val = as<float>(ws.val);
    c.vv = vv_needed(p) ? as<double2>(ws.vv) + row * n : nullptr;
    return c;
}

// Forward launch arguments for the (T, P) points [f, f + nb) of the call, whose core
// rows start at row0, writing sigma rows f.. of the call's output.
xs::FwdArgs fwd_args(xs_plan* p, Workset& ws, const std::vector<xs::TPParam>& tps, int f, int nb, int row0,
                     int S, void* sigma) {
    const xs_opts& o = p->o;
    const bool fp64 = o.precision == XS_FP64;
    const size_t elem = fp64 ? sizeof(double) : sizeof(float);
    xs::FwdArgs a{};
    a.L = sorted_lines(p);
    a.G = p->geo;
    a.tps = as<xs::TPParam>(ws.tps) + f;
    a.Q = as<double>(ws.Q);
    a.off = as<int>(p->off);
    a.sigma = static_cast<char*>(sigma) + (size_t)f * (size_t)p->geo.n_points * elem;
    a.part = ws.part.p;
    a.n_lines = (int)p->n_kept;
    a.n_tiles = n_tiles(p);
    a.n_tp = nb;
    a.n_split = S;
    a.seg = 1;
    for (int t = f; t < f + nb; ++t) a.seg = a.seg && seg_mode(p, tps[t]);
    a.xcd_contiguous = p->xcd_contiguous;
    a.tile_order = (p->n_order == a.n_tiles && p->order_W == tile_width(p)) ? as<int>(p->tile_order) : nullptr;
    a.alpha_fixed = o.alpha_fixed;
    a.tab = as<xs::Tables>(p->tab_dev);
    if (vv_needed(p) && fp64) {
        a.vv = as<double2>(ws.vv) + (int64_t)row0 * ws.row_stride;
        a.vv_stride = ws.row_stride;
    }
    if (threshold_on(p)) {
        a.map = as<int>(ws.th_map) + (int64_t)row0 * ws.row_stride;
        a.map_stride = ws.row_stride;
        a.offs = as<int>(ws.th_offs) + (int64_t)row0 * ((int64_t)p->geo.nkeys + 1);
        a.offs_stride = (int64_t)p->geo.nkeys + 1;
    }
    if (records_path(p)) {
        a.hot = as<float>(ws.hot) + (int64_t)row0 * ws.row_stride * hot_words(p);
        a.cold = as<int>(ws.cold) + (int64_t)row0 * ws.row_stride * 16;
        a.xscale = as<double>(ws.xscale) + (int64_t)row0 * ws.row_stride;
        a.rec_stride = ws.row_stride;
        a.core_val = as<float>(ws.val);
    }
    if (superlines(p)) {
        a.line_S = as<double>(ws.sl) + (int64_t)row0 * ws.row_stride;
        a.line_S_stride = ws.row_stride;
    }
    if (far_sampled(p) && a.seg && records_path(p)) {
        // shares of each wavefront's far lines, about 16 lines per lane each: many short
        // wavefronts spread the far wing evenly over the chip (at most kFarShares)
        const double per_wave = (double)p->n_kept * (2.0 * p->geo.hmin + 64.0 * p->P) / std::max(1, p->geo.nkeys);
        a.far = as<double>(ws.far);
        a.far_nodes = as<double>(ws.far_nodes);
        a.far_share = (int)std::min<double>(kFarShares, std::max(1.0, std::ceil(per_wave / 1024.0)));
        // the window ends go to the far kernel too when every window-end line lies beyond both
        // the far reach and the |z| < 40 radius of any wavefront it ends in: such lines are
        // at least hmin - WW + 2 steps from it
        const int WW = 64 * p->P;
        int rm = 0;
        for (int t = f; t < f + nb; ++t) rm = std::max(rm, tps[t].rm);
        a.far_ends = (int64_t)p->geo.hmin - WW + 2 >= (int64_t)std::max(far_reach_steps(WW), rm) ? 1 : 0;
        a.far_slots = 1 + a.far_ends;
    }
    return a;
}

// Line records of the call's (T, P) point `it` into row `row` (after its core values).
xs::RecArgs rec_args(xs_plan* p, Workset& ws, int it, int row) {
    xs::RecArgs r{};
    const int64_t n = ws.row_stride;
    r.L = sorted_lines(p);
    r.G = p->geo;
    r.tp = as<xs::TPParam>(ws.tps) + it;
    r.Q = as<double>(ws.Q);
    r.n_lines = (int)p->n_kept;
    r.tab = as<xs::Tables>(p->tab_dev);
    r.alpha_fixed = p->o.alpha_fixed;
    if (core_path(p)) {
        r.core_rc = as<int>(ws.rc) + row * n;
        r.core_off = as<long long>(ws.coff) + row * n;
    }
    r.vv = vv_needed(p) ? as<double2>(ws.vv) + row * n : nullptr;
    if (threshold_on(p)) {
        r.map = as<int>(ws.th_map) + row * n;
        r.count = as<unsigned long long>(ws.th_tmp) + (int64_t)row * kScanTmp + 4096;
    }
    r.hot = as<float>(ws.hot) + row * n * hot_words(p);
    r.cold = as<int>(ws.cold) + row * n * 16;   // a row: words 0-7 of its n records, then words 8-15
    r.cold_b = r.cold + n * 8;
    r.xscale = as<double>(ws.xscale) + row * n;
    return r;
}

// Per-(T, P) parameters and temperatures to the device (through pinned staging), then
// Q(T) for every temperature of the call.  With enqueue_q false the partition sum is
// left to the caller (graph capture records it).
// Q of the call's temperatures (ws.T: T then T_vib); non-LTE when the line set is.
hipError_t enqueue_q_of_call(xs_plan* p, Workset& ws, int n, hipStream_t s) {
    const double* Ev = p->lines_vib ? as<double>(p->Ev) : nullptr;
    return xs::launch_partition(as<double>(p->E), as<int>(p->g), Ev, p->n_states, as<double>(ws.T),
                                as<double>(ws.T) + n, n, as<double>(ws.qpart), xs_plan::kQBlocks, as<double>(ws.Q),
                                as<double>(ws.dQ), s);
}

xs_status upload_tps(xs_plan* p, Workset& ws, const std::vector<xs::TPParam>& tps, hipStream_t s, bool enqueue_q) {
    const int n = (int)tps.size();
    XS_TRY(ws.ensure(ws.T, 2 * n * sizeof(double), "temperatures"));
    XS_TRY(ws.ensure(ws.Q, n * sizeof(double), "Q(T)"));
    XS_TRY(ws.ensure(ws.dQ, n * sizeof(double), "dQ/dT"));
    XS_TRY(ws.ensure(ws.qpart, (size_t)2 * n * xs_plan::kQBlocks * sizeof(double), "Q partials"));
    XS_TRY(ws.ensure(ws.tps, n * sizeof(xs::TPParam), "(T, P) parameters"));
    void* h = nullptr;
    XS_TRY(ws.stage.get(n * (2 * sizeof(double) + sizeof(xs::TPParam)), &h));
    double* hT = static_cast<double*>(h);
    xs::TPParam* hp = reinterpret_cast<xs::TPParam*>(hT + 2 * n);
    for (int i = 0; i < n; ++i) { hT[i] = tps[i].T; hT[n + i] = tps[i].Tv; hp[i] = tps[i]; }
    XS_HIP(hipMemcpyAsync(ws.T.p, hT, 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
    XS_HIP(hipMemcpyAsync(ws.tps.p, hp, n * sizeof(xs::TPParam), hipMemcpyHostToDevice, s));
    XS_TRY(ws.stage.record(s));
    if (enqueue_q) XS_HIP(enqueue_q_of_call(p, ws, n, s));
    return XS_OK;
}

// Read back the u64 totals at scan_tmp[4096] of core rows [0, nb) (synchronous).
xs_status read_totals(Workset& ws, int nb, hipStream_t s, std::vector<unsigned long long>& out) {
    void* h = nullptr;
    XS_TRY(ws.stage.get(nb * sizeof(unsigned long long), &h));
    unsigned long long* ht = static_cast<unsigned long long*>(h);
    for (int t = 0; t < nb; ++t)
        XS_HIP(hipMemcpyAsync(ht + t, as<unsigned long long>(ws.tmp) + (int64_t)t * kScanTmp + 4096,
                              sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    XS_HIP(hipStreamSynchronize(s));
    out.assign(ht, ht + nb);
    return XS_OK;
}

// Core evaluation (optionally preceded by the count) of rows [0, nb) for the (T, P)
// points [f, f + nb), then the block's forward launch and, when split, the combine.
// Enqueue only: no allocation and no synchronisation (graph-capturable).
// Per-(T, P) pre-passes of the call's point `it` into row `row`: Vectorized Voigt factors,
// then (FP32) the Voigt core values and the line records.  Enqueue only.
// Intensity threshold: the kept lines of (T, P) point `it` compacted into row `row`.
xs_status enqueue_cull(xs_plan* p, Workset& ws, int it, int row, hipStream_t s) {
    xs::CullArgs c{};
    const int64_t n = ws.row_stride;
    c.L = sorted_lines(p);
    c.G = p->geo;
    c.tp = as<xs::TPParam>(ws.tps) + it;
    c.Q = as<double>(ws.Q);
    c.n_lines = (int)p->n_kept;
    c.mode = p->th_mode;
    c.i_crit = p->th_icrit;
    c.nu_crit = p->th_nucrit;
    c.bsum = as<unsigned long long>(ws.th_bsum) + (int64_t)row * xs::core_blocks(n);
    c.scan_tmp = as<unsigned long long>(ws.th_tmp) + (int64_t)row * kScanTmp;
    c.pos = as<unsigned>(ws.th_pos) + (int64_t)row * (n + 1);
    c.map = as<int>(ws.th_map) + (int64_t)row * n;
    c.off = as<int>(p->off);
    c.offs = as<int>(ws.th_offs) + (int64_t)row * ((int64_t)p->geo.nkeys + 1);
    XS_HIP(xs::launch_cull(c, s));
    return XS_OK;
}

// Pre-passes of (T, P) point `it` in row `row`.  count: the core counts are not computed
// yet (graph capture); otherwise count_block has run the cull and the counts.
xs_status enqueue_prepass(xs_plan* p, Workset& ws, int it, int row, bool count, const std::vector<long long>& vbase,
                          const std::vector<long long>& vend, hipStream_t s) {
    if (p->n_kept <= 0) return XS_OK;
    if (threshold_on(p) && (count || !core_path(p))) XS_TRY(enqueue_cull(p, ws, it, row, s));
    if (vv_needed(p)) {
        xs::VVArgs v{};
        v.L = sorted_lines(p);
        v.G = p->geo;
        v.tp = as<xs::TPParam>(ws.tps) + it;
        v.tab = as<xs::Tables>(p->tab_dev);
        v.n_lines = (int)p->n_kept;
        v.use_beta = p->o.vv_beta;
        v.normalise = p->o.profile == XS_VVOIGT_NORM ? 1 : 0;
        v.fp64 = p->o.precision == XS_FP64 ? 1 : 0;
        v.out = as<double2>(ws.vv) + (int64_t)row * ws.row_stride;
        XS_HIP(xs::launch_vv_prep(v, s));
    }
    if (!records_path(p)) return XS_OK;
    if (core_path(p)) {
        xs::CoreArgs c = core_args(p, ws, it, row);
        c.val_base = vbase[it];
        c.val_end = vend[it];
        if (count) XS_HIP(xs::launch_core_count(c, s));
        XS_HIP(xs::launch_core_eval(c, s));
    }
    XS_HIP(xs::launch_records(kernel_profile(p), rec_args(p, ws, it, row), s));
    return XS_OK;
}

xs_status enqueue_block(xs_plan* p, Workset& ws, const std::vector<xs::TPParam>& tps, int f, int nb, int S,
                        bool count, const std::vector<long long>& vbase, const std::vector<long long>& vend,
                        void* sigma, hipStream_t s, bool timed) {
    const bool fp64 = p->o.precision == XS_FP64;
    if ((records_path(p) || vv_needed(p) || threshold_on(p)) && p->n_kept > 0) {
        for (int t = 0; t < nb; ++t) {
            Timer tc(p, s, 1, 0, timed);
            XS_TRY(enqueue_prepass(p, ws, f + t, t, count, vbase, vend, s));
            tc.stop();
        }
    }
    // one launch per run of consecutive (T, P) sharing the sweep mode
    for (int r0 = f; r0 < f + nb;) {
        int r1 = r0 + 1;
        while (r1 < f + nb && seg_mode(p, tps[r1]) == seg_mode(p, tps[r0])) ++r1;
        const xs::FwdArgs a = fwd_args(p, ws, tps, r0, r1 - r0, r0 - f, S, sigma);
        {
            Timer tf(p, s, 0, r1 - r0, timed);
            XS_HIP(xs::launch_forward(kernel_profile(p), fp64 ? 1 : 0, p->waves, p->P, a, s));
            tf.stop();
        }
        if (a.far) {
            Timer tw(p, s, 4, r1 - r0, timed);
            XS_HIP(xs::launch_far(p->waves, p->P, a, s));
            tw.stop();
        }
        if (S > 1 || a.far) {
            Timer tm(p, s, 3, r1 - r0, timed);
            XS_HIP(xs::launch_combine(fp64 ? 1 : 0, a, s));
            tm.stop();
        }
        r0 = r1;
    }
    return XS_OK;
}

// Exact core counts of the block [f, f + nb) (one wait), value offsets, capacity.
xs_status count_block(xs_plan* p, Workset& ws, const std::vector<xs::TPParam>& tps, int f, int nb, hipStream_t s,
                      std::vector<long long>& vbase, std::vector<long long>& vend) {
    for (int t = 0; t < nb; ++t) {
        xs::CoreArgs c = core_args(p, ws, f + t, t);
        Timer tc(p, s, 1);
        if (threshold_on(p)) XS_TRY(enqueue_cull(p, ws, f + t, t, s));   // counts cover kept lines only
        XS_HIP(xs::launch_core_count(c, s));
        tc.stop();
    }
    std::vector<unsigned long long> tot;
    XS_TRY(read_totals(ws, nb, s, tot));
    long long base = 0;
    for (int t = 0; t < nb; ++t) {
        vbase[f + t] = base;
        base += (long long)tot[t];
        vend[f + t] = base;
    }
    return ws.ensure(ws.val, (size_t)std::max<long long>(base, 1) * sizeof(float), "core values");
}

xs_status validate_tp(int n_tp, const double* T, const double* P) {
    if (!T || !P) return fail(XS_ERR_ARG, "NULL argument");
    if (n_tp <= 0) return fail(XS_ERR_ARG, "n_tp must be > 0");
    for (int i = 0; i < n_tp; ++i) {
        if (!(T[i] > 0.0) || !std::isfinite(T[i])) return fail(XS_ERR_ARG, "temperatures must be finite and > 0");
        if (!(P[i] >= 0.0) || !std::isfinite(P[i])) return fail(XS_ERR_ARG, "pressures must be finite and >= 0");
    }
    return XS_OK;
}

}  // namespace

namespace xs {

xs_status set_error(xs_status s, const std::string& msg) { return fail(s, msg); }

bool plan_states(const xs_plan* p, const double** E, const int** g, int64_t* n_states) {
    if (!p) return false;
    *E = static_cast<const double*>(p->E.p);
    *g = static_cast<const int*>(p->g.p);
    *n_states = p->n_states;
    return true;
}

}  // namespace xs

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
    p->waves = opts->precision == XS_FP64 ? 4 : (opts->waves_per_block ? opts->waves_per_block : 2);
    p->n_split = opts->n_split;
    p->tp_block = opts->tp_block;
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
    G.vv_radius = opts->vv_radius > 0.0 ? opts->vv_radius : 4.0;
    {
        // R beyond the cut-off covers every window point: bounds past the half window suffice
        const double rv = std::min(G.vv_radius, opts->cutoff + 2.0 * G.dnu) / G.dnu;
        G.rvmax = (int)std::ceil(rv) + 2;
        G.rvmin = (int)std::floor(rv) - 2;
    }
    xs::weideman_coefficients(24, &p->tabs.w24);
    xs::weideman_coefficients(40, &p->tabs.w40);
    xs::dawson_table(p->tabs.dawson);
    xs::make_gh_pairs(2, &p->tabs.gh2);
    xs::make_gh_pairs(4, &p->tabs.gh4);
    xs::make_gh_pairs(6, &p->tabs.gh6);
    xs::make_gh_pairs(12, &p->tabs.gh12);
    {
        // the convolution profiles' rule (Eq. 30-31): gh_nodes nodes, "usually 30"
        xs::Tables& t = p->tabs;
        t.nconv = opts->gh_nodes > 0 ? opts->gh_nodes : xs::kGHConvDefault;
        xs::gauss_hermite_rule(t.nconv, t.tconv, t.wconv);
        for (int j = 0; j < t.nconv; ++j) {
            t.tconvf[j] = (float)t.tconv[j];
            t.wconvf[j] = (float)t.wconv[j];
        }
        // pairs +-t_j from the upper half of the ascending nodes; an odd rule's middle node
        // (t = 0) enters the pair formula twice, so it carries half its weight
        t.npair = 0;
        for (int j = t.nconv / 2; j < t.nconv; ++j, ++t.npair) {
            const bool zero = (t.nconv % 2 == 1) && j == t.nconv / 2;
            t.tpair[t.npair] = zero ? 0.0 : t.tconv[j];
            t.wpair[t.npair] = zero ? 0.5 * t.wconv[j] : t.wconv[j];
            t.tpairf[t.npair] = (float)t.tpair[t.npair];
            t.wpairf[t.npair] = (float)t.wpair[t.npair];
        }
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
    p->has_vib = false;
    p->lines_vib = false;
    p->generation++;
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
    p->generation++;
    xs_status st;
    if (n > p->cap) {
        const size_t d = n * sizeof(double), f = n * sizeof(float), i4 = n * sizeof(int);
        struct { DevBuf* b; size_t sz; } req[] = {
            {&p->p_rec, n * sizeof(xs::PrepRec)},
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
    p->lines_vib = false;
    if (p->has_vib) {
        XS_TRY(p->ensure(p->s_evl, (size_t)std::max<int64_t>(n, 1) * sizeof(double), "line vibrational energies"));
        XS_TRY(p->ensure(p->s_evu, (size_t)std::max<int64_t>(n, 1) * sizeof(double), "line vibrational energies"));
    }
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
    a.p_rec = as<xs::PrepRec>(p->p_rec);
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
    ga.p_rec = a.p_rec;
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
    p->order_W = 0;
    p->off_host.assign(p->geo.nkeys + 1, 0);
    if (kept > 0) {
        XS_HIP(hipMemcpy(p->off_host.data(), p->off.p, p->off_host.size() * sizeof(int), hipMemcpyDeviceToHost));
        if ((st = build_tile_order(p)) != XS_OK) return st;
    }
    if (p->has_vib && kept > 0) {
        // the kept lines' vibrational energies, read through the caller's index arrays
        // (so the call waits for them once more before returning)
        XS_HIP(xs::launch_vib_gather(kept, as<int>(p->s_orig), n, upper, lower, p->o.index_base, as<double>(p->Ev),
                                     p->n_states, as<double>(p->s_evl), as<double>(p->s_evu), s));
        XS_HIP(hipStreamSynchronize(s));
    }
    p->lines_vib = p->has_vib;
    p->have_lines = true;
    return XS_OK;
}

xs_status xs_set_intensity_threshold(xs_plan* p, int32_t mode, double i_crit, double nu_crit) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (mode < XS_THRESHOLD_NONE || mode > XS_THRESHOLD_HITRAN) return fail(XS_ERR_ARG, "unknown threshold mode");
    if (mode != XS_THRESHOLD_NONE && !(i_crit >= 0.0 && std::isfinite(i_crit)))
        return fail(XS_ERR_ARG, "i_crit must be finite and >= 0");
    if (mode == XS_THRESHOLD_HITRAN && !(nu_crit > 0.0 && std::isfinite(nu_crit)))
        return fail(XS_ERR_ARG, "nu_crit must be finite and > 0");
    p->th_mode = mode;
    p->th_icrit = i_crit;
    p->th_nucrit = nu_crit;
    p->generation++;   // captured graphs were recorded without (or with another) threshold
    return XS_OK;
}

xs_status xs_set_intensity_kind(xs_plan* p, int32_t kind) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (kind != XS_ABSORPTION && kind != XS_EMISSION) return fail(XS_ERR_ARG, "unknown intensity kind");
    if (p->emission != kind) p->generation++;   // captured graphs hold the other kind
    p->emission = kind;
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
    XS_HIP(xs::launch_partition(as<double>(p->E), as<int>(p->g), nullptr, p->n_states, as<double>(p->T_dev),
                                nullptr, nT, as<double>(p->qpart), xs_plan::kQBlocks, as<double>(p->Q),
                                as<double>(p->dQ), s));
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

// Temperatures of a state reduction on the device, and its partial-sum buffer.
static xs_status stage_temperatures(xs_plan* p, int nT, const double* T, hipStream_t s) {
    if (!T) return fail(XS_ERR_ARG, "NULL argument");
    if (nT <= 0) return fail(XS_ERR_ARG, "n_T must be > 0");
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0) || !std::isfinite(T[i])) return fail(XS_ERR_ARG, "temperatures must be finite and > 0");
    if (nT > p->st_cap) {
        XS_TRY(p->ensure(p->st_T, nT * sizeof(double), "state-reduction temperatures"));
        XS_TRY(p->ensure(p->st_part, (size_t)3 * nT * xs_plan::kQBlocks * sizeof(double), "state partial sums"));
        p->st_cap = nT;
    }
    XS_HIP(hipMemcpyAsync(p->st_T.p, T, nT * sizeof(double), hipMemcpyHostToDevice, s));
    return XS_OK;
}

// Per-state sums over the caller's transitions (sum of A and/or of A nu), then a wait for
// the validation flags.
static xs_status state_rates(xs_plan* p, int64_t n, const int32_t* upper, const int32_t* lower, const float* A,
                             bool sum_A, bool power, hipStream_t s) {
    if (n < 0) return fail(XS_ERR_ARG, "n_lines must be >= 0");
    if (n > 0 && (!upper || !A || (power && !lower))) return fail(XS_ERR_ARG, "NULL transition array");
    if (sum_A) XS_TRY(p->ensure(p->st_sumA, (size_t)p->n_states * sizeof(double), "per-state A sums"));
    if (power) XS_TRY(p->ensure(p->st_power, (size_t)p->n_states * sizeof(double), "per-state A nu sums"));
    XS_TRY(p->ensure(p->flag, sizeof(int) * 4, "flags"));
    if (sum_A) XS_HIP(xs::launch_fill(as<double>(p->st_sumA), p->n_states, 0.0, s));
    if (power) XS_HIP(xs::launch_fill(as<double>(p->st_power), p->n_states, 0.0, s));
    XS_HIP(hipMemsetAsync(p->flag.p, 0, sizeof(int), s));
    xs::RateArgs a{};
    a.n = n;
    a.upper = upper;
    a.lower = lower;
    a.A = A;
    a.index_base = p->o.index_base;
    a.a_is_log = p->o.a_is_log;
    a.E = as<double>(p->E);
    a.n_states = p->n_states;
    a.flag = as<int>(p->flag);
    a.sum_A = sum_A ? as<double>(p->st_sumA) : nullptr;
    a.power = power ? as<double>(p->st_power) : nullptr;
    if (xs::bucket_rates_fits(n, p->n_states)) {
        const size_t nh = (size_t)xs::bucket_hist_len(n, p->n_states);
        XS_TRY(p->ensure(p->st_bhist, nh * sizeof(uint32_t), "bucket histogram"));
        XS_TRY(p->ensure(p->st_bhoff, nh * sizeof(uint32_t), "bucket offsets"));
        XS_TRY(p->ensure(p->st_btsum, 4096 * sizeof(uint32_t), "bucket scan"));
        XS_TRY(p->ensure(p->st_brec, (size_t)n * 16, "bucket records"));
        XS_HIP(xs::launch_bucket_rates(a, as<uint32_t>(p->st_bhist), as<uint32_t>(p->st_bhoff),
                                       as<uint32_t>(p->st_btsum), p->st_brec.p, s));
    } else {
        XS_HIP(xs::launch_rates(a, s));
    }
    int flag = 0;
    XS_HIP(hipMemcpyAsync(&flag, p->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    XS_HIP(hipStreamSynchronize(s));
    if (flag & xs::kFlagIndex) return fail(XS_ERR_INDEX, "a transition's state index is out of range");
    if (flag & xs::kFlagNu) return fail(XS_ERR_NU_NONPOS, "a transition has E[upper] - E[lower] <= 0");
    return XS_OK;
}

xs_status xs_partition_moments(xs_plan* p, int32_t nT, const double* T, double* Q, double* Q1, double* Q2,
                               double* Cp, void* stream) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    XS_TRY(stage_temperatures(p, nT, T, s));
    XS_HIP(xs::launch_moments(as<double>(p->E), as<int>(p->g), p->n_states, as<double>(p->st_T), nT,
                              as<double>(p->st_part), xs_plan::kQBlocks, Q, Q1, Q2, Cp, s));
    return XS_OK;
}

xs_status xs_lifetimes(xs_plan* p, int64_t n_lines, const int32_t* upper, const float* A, double* tau,
                       void* stream) {
    if (!p || !tau) return fail(XS_ERR_ARG, "NULL argument");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    XS_TRY(state_rates(p, n_lines, upper, nullptr, A, true, false, s));
    XS_HIP(xs::launch_lifetimes(as<double>(p->st_sumA), p->n_states, tau, s));
    return XS_OK;
}

xs_status xs_cooling_function(xs_plan* p, int64_t n_lines, const int32_t* upper, const int32_t* lower,
                              const float* A, int32_t nT, const double* T, double* W, void* stream) {
    if (!p || !W) return fail(XS_ERR_ARG, "NULL argument");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    XS_TRY(stage_temperatures(p, nT, T, s));
    XS_TRY(state_rates(p, n_lines, upper, lower, A, false, true, s));
    XS_HIP(xs::launch_cooling(as<double>(p->E), as<int>(p->g), as<double>(p->st_power), p->n_states,
                              as<double>(p->st_T), nT, as<double>(p->st_part), xs_plan::kQBlocks, W, s));
    return XS_OK;
}

// Cross sections of a call; Tv (vibrational temperatures of non-LTE populations) or NULL.
static xs_status cross_section_call(xs_plan* p, int32_t n_tp, const double* T, const double* Tv, const double* P,
                                    void* sigma, void* stream) {
    if (!p || !sigma) return fail(XS_ERR_ARG, "NULL argument");
    XS_TRY(validate_tp(n_tp, T, P));
    XS_TRY(check_vv(p, n_tp, T));
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workset& ws = p->ws;
    std::vector<xs::TPParam> tps(n_tp);
    for (int i = 0; i < n_tp; ++i) {
        tps[i] = make_tp(p, T[i], P[i], i, T[i]);
        if (Tv) tps[i].Tv = Tv[i];
    }
    XS_TRY(build_tile_order(p));
    XS_TRY(upload_tps(p, ws, tps, s, true));
    const int B = pick_block(p, n_tp), S = pick_split(p);
    p->last_block = B;
    p->last_split = S;
    XS_TRY(ensure_rows(p, ws, B, S));
    std::vector<long long> vbase(n_tp, 0), vend(n_tp, 0);
    const bool core = core_path(p) && p->n_kept > 0;
    if (core) {
        // every core row of a block gets the capacity of the count bound at the call's
        // highest temperature; the bound is kept with the line set, so only a call with a
        // new line set or a higher temperature waits (once) to read it back
        int imax = 0;
        for (int i = 1; i < n_tp; ++i)
            if (T[i] > T[imax]) imax = i;
        if (!(p->core_bound_gen == p->generation && p->core_bound_T >= T[imax])) {
            xs::CoreArgs c = core_args(p, ws, imax, 0);
            XS_HIP(xs::launch_core_bound(c, s));
            std::vector<unsigned long long> tot;
            XS_TRY(read_totals(ws, 1, s, tot));
            p->core_bound = (long long)tot[0];
            p->core_bound_T = T[imax];
            p->core_bound_gen = p->generation;
        }
        const long long slot = std::max<long long>(p->core_bound, 1);
        XS_TRY(ws.ensure(ws.val, (size_t)B * (size_t)slot * sizeof(float), "core values"));
        for (int f = 0; f < n_tp; f += B)
            for (int t = 0; t < std::min(B, n_tp - f); ++t) {
                vbase[f + t] = (long long)t * slot;
                vend[f + t] = (long long)(t + 1) * slot;
            }
    }
    for (int f = 0; f < n_tp; f += B) {
        const int nb = std::min(B, n_tp - f);
        XS_TRY(enqueue_block(p, ws, tps, f, nb, S, core, vbase, vend, sigma, s, true));
    }
    return XS_OK;
}

xs_status xs_cross_section(xs_plan* p, int32_t n_tp, const double* T, const double* P, void* sigma,
                           void* stream) {
    return cross_section_call(p, n_tp, T, nullptr, P, sigma, stream);
}

static xs_status validate_tvib(int32_t n, const double* Tv) {
    if (!Tv) return fail(XS_ERR_ARG, "T_vib is NULL");
    for (int i = 0; i < n; ++i)
        if (!(Tv[i] > 0.0) || !std::isfinite(Tv[i])) return fail(XS_ERR_ARG, "T_vib must be finite and > 0");
    return XS_OK;
}

xs_status xs_cross_section_nlte(xs_plan* p, int32_t n_tp, const double* T_rot, const double* T_vib,
                                const double* P, void* sigma, void* stream) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (n_tp > 0) XS_TRY(validate_tvib(n_tp, T_vib));
    if (p->have_lines && !p->lines_vib)
        return fail(XS_ERR_STATE, "the line set has no vibrational energies (xs_set_vibrational_labels, then "
                                  "xs_set_lines)");
    return cross_section_call(p, n_tp, T_rot, T_vib, P, sigma, stream);
}

xs_status xs_set_vibrational_labels(xs_plan* p, int32_t n_labels, const int32_t* labels, void* stream) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    p->have_lines = false;   // the line set must be rebuilt with (or without) E_vib
    p->lines_vib = false;
    p->generation++;
    if (!labels) {
        p->has_vib = false;
        return XS_OK;
    }
    p->has_vib = false;
    if (n_labels <= 0) return fail(XS_ERR_ARG, "n_labels must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    XS_TRY(p->ensure(p->Ev, (size_t)p->n_states * sizeof(double), "vibrational energies"));
    XS_TRY(p->ensure(p->vmin, (size_t)n_labels * sizeof(unsigned long long), "manifold minima"));
    XS_TRY(p->ensure(p->flag, sizeof(int) * 4, "flags"));
    XS_HIP(hipMemsetAsync(p->flag.p, 0, sizeof(int), s));
    XS_HIP(xs::launch_vib_energies(as<double>(p->E), labels, p->n_states, n_labels,
                                   as<unsigned long long>(p->vmin), as<double>(p->Ev), as<int>(p->flag), s));
    int flag = 0;
    XS_HIP(hipMemcpyAsync(&flag, p->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    XS_HIP(hipStreamSynchronize(s));
    if (flag & xs::kFlagIndex) return fail(XS_ERR_INDEX, "a manifold label is outside [0, n_labels)");
    if (flag & xs::kFlagNu) return fail(XS_ERR_ARG, "non-LTE needs state energies >= 0");
    p->has_vib = true;
    return XS_OK;
}

xs_status xs_partition_function_nlte(xs_plan* p, int32_t nT, const double* T_rot, const double* T_vib, double* Q,
                                     void* stream) {
    if (!p || !T_rot || !Q) return fail(XS_ERR_ARG, "NULL argument");
    if (nT <= 0) return fail(XS_ERR_ARG, "n_T must be > 0");
    if (!p->has_vib) return fail(XS_ERR_STATE, "xs_set_vibrational_labels must come first");
    XS_TRY(validate_tvib(nT, T_vib));
    for (int i = 0; i < nT; ++i)
        if (!(T_rot[i] > 0.0) || !std::isfinite(T_rot[i])) return fail(XS_ERR_ARG, "temperatures must be finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (2 * nT > p->st_cap) {
        XS_TRY(p->ensure(p->st_T, 2 * nT * sizeof(double), "state-reduction temperatures"));
        XS_TRY(p->ensure(p->st_part, (size_t)6 * nT * xs_plan::kQBlocks * sizeof(double), "state partial sums"));
        p->st_cap = 2 * nT;
    }
    XS_HIP(hipMemcpyAsync(p->st_T.p, T_rot, nT * sizeof(double), hipMemcpyHostToDevice, s));
    XS_HIP(hipMemcpyAsync(as<double>(p->st_T) + nT, T_vib, nT * sizeof(double), hipMemcpyHostToDevice, s));
    XS_HIP(xs::launch_partition(as<double>(p->E), as<int>(p->g), as<double>(p->Ev), p->n_states, as<double>(p->st_T),
                                as<double>(p->st_T) + nT, nT, as<double>(p->st_part), xs_plan::kQBlocks, Q, nullptr,
                                s));
    return XS_OK;
}

// ------------------------------------------------------------------ graphs
xs_status xs_graph_create(xs_plan* p, int32_t n_tp, const double* T, const double* P, void* sigma,
                          xs_graph** out) {
    if (!out) return fail(XS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !sigma) return fail(XS_ERR_ARG, "NULL argument");
    XS_TRY(validate_tp(n_tp, T, P));
    XS_TRY(check_vv(p, n_tp, T));
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    XS_TRY(build_tile_order(p));
    xs_graph* g = new (std::nothrow) xs_graph();
    if (!g) return fail(XS_ERR_OOM, "host allocation failed");
    g->p = p;
    g->n_tp = n_tp;
    g->T_cap.assign(T, T + n_tp);
    g->tps.resize(n_tp);
    for (int i = 0; i < n_tp; ++i) g->tps[i] = make_tp(p, T[i], P[i], i, T[i]);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) { delete g; return hip_fail(e, "hipStreamCreateWithFlags"); }
    auto cleanup = [&](xs_status st) {
        if (cs) (void)hipStreamSynchronize(cs);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        g->ws.release();
        delete g;
        if (cs) (void)hipStreamDestroy(cs);
        return st;
    };
    Workset& ws = g->ws;
    const int B = pick_block(p, n_tp), S = pick_split(p);
    xs_status st = upload_tps(p, ws, g->tps, cs, true);
    if (st == XS_OK) st = ensure_rows(p, ws, B, S);
    std::vector<long long> vbase(n_tp, 0), vend(n_tp, 0);
    if (st == XS_OK && core_path(p) && p->n_kept > 0) {
        // capacities from the width-independent bound (valid for any T up to T_cap)
        long long cap = 1;
        for (int f = 0; f < n_tp && st == XS_OK; f += B) {
            const int nb = std::min(B, n_tp - f);
            for (int t = 0; t < nb && st == XS_OK; ++t) {
                xs::CoreArgs c = core_args(p, ws, f + t, t);
                e = xs::launch_core_bound(c, cs);
                if (e != hipSuccess) st = hip_fail(e, "core bound");
            }
            std::vector<unsigned long long> tot;
            if (st == XS_OK) st = read_totals(ws, nb, cs, tot);
            long long base = 0;
            for (int t = 0; t < nb && st == XS_OK; ++t) {
                vbase[f + t] = base;
                base += (long long)tot[t];
                vend[f + t] = base;
            }
            cap = std::max(cap, base);
        }
        if (st == XS_OK) st = ws.ensure(ws.val, (size_t)cap * sizeof(float), "core values");
    }
    if (st == XS_OK && (e = hipStreamSynchronize(cs)) != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    if (st != XS_OK) return cleanup(st);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamBeginCapture"));
    e = enqueue_q_of_call(p, ws, n_tp, cs);
    if (e != hipSuccess) st = hip_fail(e, "partition function");
    for (int f = 0; f < n_tp && st == XS_OK; f += B) {
        const int nb = std::min(B, n_tp - f);
        st = enqueue_block(p, ws, g->tps, f, nb, S, true, vbase, vend, sigma, cs, false);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (st != XS_OK) return cleanup(st);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamEndCapture"));
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { g->exec = nullptr; return cleanup(hip_fail(e, "hipGraphInstantiate")); }
    (void)hipStreamDestroy(cs);
    g->generation = p->generation;
    *out = g;
    return XS_OK;
}

xs_status xs_graph_set_tp(xs_graph* g, const double* T, const double* P, void* stream) {
    if (!g) return fail(XS_ERR_ARG, "graph is NULL");
    XS_TRY(validate_tp(g->n_tp, T, P));
    XS_TRY(check_vv(g->p, g->n_tp, T));
    for (int i = 0; i < g->n_tp; ++i)
        if (T[i] > g->T_cap[i])
            return fail(XS_ERR_ARG, "a temperature exceeds the one the graph was captured with");
    for (int i = 0; i < g->n_tp; ++i) g->tps[i] = make_tp(g->p, T[i], P[i], i, g->T_cap[i]);
    const int n = g->n_tp;
    Workset& ws = g->ws;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* h = nullptr;
    XS_TRY(ws.stage.get(n * (2 * sizeof(double) + sizeof(xs::TPParam)), &h));
    double* hT = static_cast<double*>(h);
    xs::TPParam* hp = reinterpret_cast<xs::TPParam*>(hT + 2 * n);
    for (int i = 0; i < n; ++i) { hT[i] = g->tps[i].T; hT[n + i] = g->tps[i].Tv; hp[i] = g->tps[i]; }
    XS_HIP(hipMemcpyAsync(ws.T.p, hT, 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
    XS_HIP(hipMemcpyAsync(ws.tps.p, hp, n * sizeof(xs::TPParam), hipMemcpyHostToDevice, s));
    return ws.stage.record(s);
}

xs_status xs_graph_launch(xs_graph* g, void* stream) {
    if (!g) return fail(XS_ERR_ARG, "graph is NULL");
    if (g->generation != g->p->generation)
        return fail(XS_ERR_STATE, "the plan's states, lines or tile configuration changed since the capture");
    XS_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return XS_OK;
}

xs_status xs_graph_destroy(xs_graph* g) {
    if (!g) return XS_OK;
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->ws.release();
    delete g;
    return XS_OK;
}

size_t xs_graph_workspace_bytes(const xs_graph* g) { return g ? g->ws.bytes : 0; }

// ------------------------------------------------------------------ tile shape
xs_status xs_set_tile_config(xs_plan* p, int32_t waves, int32_t slices, int32_t n_split, int32_t tp_block) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    const bool fp64 = p->o.precision == XS_FP64;
    if (!(waves == 0 || waves == 4 || ((waves == 1 || waves == 2 || waves == 8) && !fp64)))
        return fail(XS_ERR_ARG, "waves must be 0 or 4 (or 1, 2, 8 for XS_FP32)");
    if (!(slices == 0 || slices == 1 || slices == 2 || slices == 4 || slices == 8))
        return fail(XS_ERR_ARG, "slices must be 0, 1, 2, 4 or 8");
    if (slices == 8 && (fp64 || !(waves == 1 || waves == 2)))
        return fail(XS_ERR_ARG, "8 slices per wavefront need XS_FP32 and 1 or 2 wavefronts per workgroup");
    if (n_split < 0 || n_split > 64) return fail(XS_ERR_ARG, "n_split must be in [0, 64]");
    if (tp_block < 0 || tp_block > 256) return fail(XS_ERR_ARG, "tp_block must be in [0, 256]");
    XS_HIP(hipDeviceSynchronize());
    p->waves = fp64 ? 4 : (waves ? waves : 2);
    p->P = slices ? slices : 2;
    p->n_split = n_split;
    p->tp_block = tp_block;
    p->generation++;
    if (p->have_lines) XS_TRY(build_tile_order(p));
    return XS_OK;
}

xs_status xs_get_tile_config(const xs_plan* p, int32_t out[6]) {
    if (!p || !out) return fail(XS_ERR_ARG, "NULL argument");
    out[0] = p->waves;
    out[1] = p->P;
    out[2] = p->n_split;
    out[3] = p->tp_block;
    out[4] = p->last_split;
    out[5] = p->last_block;
    return XS_OK;
}

xs_status xs_autotune(xs_plan* p, int32_t n_tp, const double* T, const double* P, double budget_ms, void* stream,
                      int32_t out[4]) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    XS_TRY(validate_tp(n_tp, T, P));
    XS_TRY(check_vv(p, n_tp, T));
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    if (!(budget_ms > 0.0)) return fail(XS_ERR_ARG, "budget_ms must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    const bool fp64 = p->o.precision == XS_FP64;
    const int save_w = p->waves, save_p = p->P, save_s = p->n_split, save_b = p->tp_block;
    // sample: the first (T, P) points, at most one default block
    const int ns = pick_block(p, std::min<int>(n_tp, 16));
    std::vector<xs::TPParam> tps(ns);
    for (int i = 0; i < ns; ++i) tps[i] = make_tp(p, T[i], P[i], i, T[i]);
    Workset& ws = p->ws;
    XS_TRY(upload_tps(p, ws, tps, s, true));
    XS_TRY(ensure_rows(p, ws, ns, 1));
    std::vector<long long> vbase(ns, 0), vend(ns, 0);
    if (core_path(p) && p->n_kept > 0) XS_TRY(count_block(p, ws, tps, 0, ns, s, vbase, vend));
    for (int t = 0; t < ns; ++t) XS_TRY(enqueue_prepass(p, ws, t, t, false, vbase, vend, s));
    const size_t elem = fp64 ? sizeof(double) : sizeof(float);
    XS_TRY(ws.ensure(ws.out, (size_t)ns * p->geo.n_points * elem, "autotune output"));
    hipEvent_t e0, e1;
    XS_HIP(hipEventCreate(&e0));
    XS_HIP(hipEventCreate(&e1));
    // time of the forward (+ combine) launches over the sample in blocks of B, per (T, P)
    auto run = [&](int w, int sl, int S, int B, double* ms) -> xs_status {
        p->waves = w;
        p->P = sl;
        XS_TRY(build_tile_order(p));
        XS_TRY(ensure_rows(p, ws, ns, S));
        XS_HIP(hipEventRecord(e0, s));
        for (int f = 0; f < ns; f += B) {
            const int nb = std::min(B, ns - f);
            const xs::FwdArgs a = fwd_args(p, ws, tps, f, nb, f, S, ws.out.p);
            XS_HIP(xs::launch_forward(kernel_profile(p), fp64 ? 1 : 0, w, sl, a, s));
            if (a.far) XS_HIP(xs::launch_far(w, sl, a, s));
            XS_HIP(xs::launch_combine(fp64 ? 1 : 0, a, s));
        }
        XS_HIP(hipEventRecord(e1, s));
        XS_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        XS_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = (double)t / ns;
        return XS_OK;
    };
    struct Cand { int w, sl, S, B; double ms; };
    Cand best{save_w, save_p, 1, ns, 1e300};
    xs_status st = XS_OK;
    int tried = 0;
    // the faster of two timings (the first launch of a kernel includes its load, and close
    // candidates differ by a few per cent, about the spread of a single timing)
    auto consider = [&](int w, int sl, int S, int B) {
        if (st != XS_OK || (tried > 0 && elapsed() > budget_ms)) return;
        ++tried;
        double a = 0.0, b = 0.0;
        st = run(w, sl, S, B, &a);
        if (st == XS_OK) st = run(w, sl, S, B, &b);
        a = std::min(a, b);
        if (st == XS_OK && a < best.ms) best = Cand{w, sl, S, B, a};
    };
    // coordinate search: tile shapes at their default split, then the split of the best
    // shape, then the (T, P) block size
    const int shapes[11][2] = {{2, 2}, {1, 2}, {4, 2}, {2, 4}, {2, 1}, {1, 4}, {4, 4}, {8, 2}, {4, 1}, {1, 8}, {2, 8}};
    for (const auto& sh : shapes) {
        if (fp64 && sh[0] != 4) continue;
        p->waves = sh[0];
        p->P = sh[1];
        p->n_split = 0;
        consider(sh[0], sh[1], pick_split(p), ns);
    }
    const int splits[7] = {1, 2, 4, 8, 16, 32, 64};
    const int s0 = best.S;
    for (int S : splits)
        if (S != s0) consider(best.w, best.sl, S, ns);
    for (int B = 1; B < ns; B *= 2) consider(best.w, best.sl, best.S, B);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_release(ws.out, &ws.bytes);
    if (st != XS_OK || best.ms >= 1e300) {
        p->waves = save_w; p->P = save_p; p->n_split = save_s; p->tp_block = save_b;
        (void)build_tile_order(p);
        return st != XS_OK ? st : fail(XS_ERR_STATE, "autotune timed no configuration");
    }
    p->waves = best.w;
    p->P = best.sl;
    p->n_split = best.S;
    p->tp_block = best.B;
    p->generation++;
    XS_TRY(build_tile_order(p));
    if (out) { out[0] = best.w; out[1] = best.sl; out[2] = best.S; out[3] = best.B; }
    return XS_OK;
}

// ------------------------------------------------------------------ streaming
namespace {

size_t stream_elem(const xs_plan* p) { return p->o.precision == XS_FP64 ? sizeof(double) : sizeof(float); }

void stream_free(xs_stream* st) {
    if (st->compute) (void)hipStreamSynchronize(st->compute);
    if (st->copy) (void)hipStreamSynchronize(st->copy);
    dev_release(st->acc, &st->bytes);
    dev_release(st->tmp, &st->bytes);
    for (auto& slot : st->raw)
        for (auto& b : slot) dev_release(b, &st->bytes);
    for (auto& e : st->copied)
        if (e) (void)hipEventDestroy(e);
    if (st->copy) (void)hipStreamDestroy(st->copy);
    delete st;
}

xs_status stream_create(xs_plan* p, int n_tp, const double* T, const double* P, void* sigma, void* stream,
                        xs_stream** out) {
    xs_stream* st = new (std::nothrow) xs_stream();
    if (!st) return fail(XS_ERR_OOM, "host allocation failed");
    st->p = p;
    st->n_tp = n_tp;
    st->T.assign(T, T + n_tp);
    st->P.assign(P, P + n_tp);
    st->sigma = sigma;
    st->emission = p->emission;
    st->compute = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
    if (e != hipSuccess) { st->copy = nullptr; stream_free(st); return hip_fail(e, "hipStreamCreateWithFlags"); }
    for (auto& ev : st->copied) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) { ev = nullptr; stream_free(st); return hip_fail(e, "hipEventCreate"); }
    }
    const int64_t n = (int64_t)n_tp * p->geo.n_points;
    xs_status r = dev_ensure(st->acc, (size_t)n * 2 * stream_elem(p), "stream accumulators", &st->bytes);
    if (r == XS_OK) r = dev_ensure(st->tmp, (size_t)n * stream_elem(p), "stream chunk result", &st->bytes);
    if (r != XS_OK) { stream_free(st); return r; }
    *out = st;
    return XS_OK;
}

// Chunk index at which XS_FAULT_INJECT=chunk:k asks xs_stream_chunk to fail, or -1.
int64_t injected_chunk() {
    const char* v = std::getenv("XS_FAULT_INJECT");
    if (!v || std::strncmp(v, "chunk:", 6) != 0) return -1;
    char* end = nullptr;
    const long long k = std::strtoll(v + 6, &end, 10);
    return (end && end != v + 6 && *end == '\0' && k >= 0) ? (int64_t)k : -1;
}

// Line preparation and cross sections of the copied chunk, added into the accumulators.
xs_status stream_process(xs_stream* st) {
    if (!st->have_pending) return XS_OK;
    st->have_pending = false;
    xs_plan* p = st->p;
    if (p->emission != st->emission)
        return fail(XS_ERR_STATE, "the plan's intensity kind changed while the stream was open");
    const int k = st->pending_slot;
    XS_HIP(hipStreamWaitEvent(st->compute, st->copied[k], 0));
    DevBuf* r = st->raw[k];
    XS_TRY(xs_set_lines(p, st->pending_n, as<int32_t>(r[0]), as<int32_t>(r[1]), as<float>(r[2]),
                        st->pending_broad ? as<float>(r[3]) : nullptr, st->pending_broad ? as<float>(r[4]) : nullptr,
                        st->compute));
    st->lines += st->pending_n;
    st->kept += p->n_kept;
    if (p->n_kept == 0) return XS_OK;
    XS_TRY(xs_cross_section(p, st->n_tp, st->T.data(), st->P.data(), st->tmp.p, st->compute));
    XS_HIP(xs::launch_acc_add(p->o.precision == XS_FP64 ? 1 : 0, st->tmp.p, st->acc.p,
                              (int64_t)st->n_tp * p->geo.n_points, st->compute));
    return XS_OK;
}

constexpr uint64_t kCkptMagic = 0x32544b4343455358ull;   // "XSECCKT2"

// What a checkpoint's sums depend on besides the (T, P) points: the grid, the cut-off, the
// profile and its options, the mass and the broadening scheme with its constants.  A resume
// refuses a plan that differs in any of them (the chunks would add onto sums of another
// geometry).
struct CkptGeometry {
    double nu_a, nu_b, cutoff, mass_da, T0, P0, alpha_fixed, gamma_const, n_const, vv_radius;
    int64_t profile, broadening, index_base, a_is_log, vv_beta, n_j;
};

CkptGeometry ckpt_geometry(const xs_plan* p) {
    const xs_opts& o = p->o;
    CkptGeometry c{};
    c.nu_a = o.nu_a; c.nu_b = o.nu_b; c.cutoff = o.cutoff; c.mass_da = o.mass_da; c.T0 = o.T0; c.P0 = o.P0;
    c.alpha_fixed = o.alpha_fixed; c.gamma_const = o.gamma_const; c.n_const = o.n_const;
    c.vv_radius = p->geo.vv_radius;
    c.profile = o.profile; c.broadening = o.broadening; c.index_base = o.index_base; c.a_is_log = o.a_is_log;
    c.vv_beta = o.vv_beta;
    c.n_j = o.broadening == XS_BROAD_A0_JLOWER ? p->n_j : 0;
    return c;
}

// first field of the two geometries that differs, or NULL
const char* ckpt_mismatch(const CkptGeometry& a, const CkptGeometry& b) {
    if (std::memcmp(&a.nu_a, &b.nu_a, sizeof(double)) || std::memcmp(&a.nu_b, &b.nu_b, sizeof(double)))
        return "grid range (nu_a, nu_b)";
    if (std::memcmp(&a.cutoff, &b.cutoff, sizeof(double))) return "cut-off";
    if (a.profile != b.profile || std::memcmp(&a.alpha_fixed, &b.alpha_fixed, sizeof(double)) ||
        a.vv_beta != b.vv_beta || std::memcmp(&a.vv_radius, &b.vv_radius, sizeof(double)))
        return "profile or its options";
    if (std::memcmp(&a.mass_da, &b.mass_da, sizeof(double))) return "molecular mass";
    if (a.broadening != b.broadening || std::memcmp(&a.T0, &b.T0, sizeof(double)) ||
        std::memcmp(&a.P0, &b.P0, sizeof(double)) || std::memcmp(&a.gamma_const, &b.gamma_const, sizeof(double)) ||
        std::memcmp(&a.n_const, &b.n_const, sizeof(double)) || a.n_j != b.n_j)
        return "broadening scheme or its constants";
    if (a.index_base != b.index_base || a.a_is_log != b.a_is_log) return "index base or A convention";
    return nullptr;
}

}  // namespace

xs_status xs_stream_begin(xs_plan* p, int32_t n_tp, const double* T, const double* P, void* sigma, void* stream,
                          xs_stream** out) {
    if (!out) return fail(XS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !sigma) return fail(XS_ERR_ARG, "NULL argument");
    XS_TRY(validate_tp(n_tp, T, P));
    XS_TRY(check_vv(p, n_tp, T));
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    if (p->o.broadening == XS_BROAD_A0_JLOWER && (p->n_j <= 0 || !p->J.p))
        return fail(XS_ERR_STATE, "a0 broadening needs xs_set_broadening_table and states J");
    xs_stream* st = nullptr;
    XS_TRY(stream_create(p, n_tp, T, P, sigma, stream, &st));
    hipError_t e = xs::launch_acc_zero(p->o.precision == XS_FP64 ? 1 : 0, st->acc.p,
                                       (int64_t)n_tp * p->geo.n_points, st->compute);
    if (e != hipSuccess) { stream_free(st); return hip_fail(e, "accumulator clear"); }
    *out = st;
    return XS_OK;
}

xs_status xs_stream_chunk(xs_stream* st, int64_t n, const int32_t* upper, const int32_t* lower, const float* A,
                          const float* gamma_ref, const float* n_exp) {
    if (!st) return fail(XS_ERR_ARG, "stream is NULL");
    xs_plan* p = st->p;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(XS_ERR_ARG, "chunk size must be in [0, 2^31-1]");
    if (n > 0 && (!upper || !lower || !A)) return fail(XS_ERR_ARG, "upper, lower and A must be non-NULL");
    const bool broad = p->o.broadening == XS_BROAD_PER_LINE;
    if (broad && n > 0 && (!gamma_ref || !n_exp)) return fail(XS_ERR_ARG, "per-line broadening needs gamma_ref and n_exp");
    if (injected_chunk() == st->chunks)
        return fail(XS_ERR_INJECTED, "fault injected before chunk " + std::to_string(st->chunks) +
                                         " (XS_FAULT_INJECT)");
    const int k = (int)(st->chunks & 1);
    // the slot's previous chunk was prepared (synchronously) two calls ago
    if (n > st->raw_cap[k]) {
        const size_t sz[5] = {n * sizeof(int32_t), n * sizeof(int32_t), n * sizeof(float), n * sizeof(float),
                              n * sizeof(float)};
        for (int a = 0; a < 5; ++a) {
            if (a >= 3 && !broad) continue;
            XS_TRY(dev_ensure(st->raw[k][a], sz[a], "stream chunk buffers", &st->bytes));
        }
        st->raw_cap[k] = n;
    }
    if (n > 0) {
        XS_HIP(hipMemcpyAsync(st->raw[k][0].p, upper, n * sizeof(int32_t), hipMemcpyHostToDevice, st->copy));
        XS_HIP(hipMemcpyAsync(st->raw[k][1].p, lower, n * sizeof(int32_t), hipMemcpyHostToDevice, st->copy));
        XS_HIP(hipMemcpyAsync(st->raw[k][2].p, A, n * sizeof(float), hipMemcpyHostToDevice, st->copy));
        if (broad) {
            XS_HIP(hipMemcpyAsync(st->raw[k][3].p, gamma_ref, n * sizeof(float), hipMemcpyHostToDevice, st->copy));
            XS_HIP(hipMemcpyAsync(st->raw[k][4].p, n_exp, n * sizeof(float), hipMemcpyHostToDevice, st->copy));
        }
    }
    XS_HIP(hipEventRecord(st->copied[k], st->copy));
    // the previous chunk computes while this one is copied
    XS_TRY(stream_process(st));
    st->have_pending = true;
    st->pending_slot = k;
    st->pending_n = n;
    st->pending_broad = broad;
    st->chunks++;
    return XS_OK;
}

xs_status xs_stream_chunk_device(xs_stream* st, int64_t n, const int32_t* upper, const int32_t* lower,
                                 const float* A, const float* gamma_ref, const float* n_exp) {
    if (!st) return fail(XS_ERR_ARG, "stream is NULL");
    xs_plan* p = st->p;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(XS_ERR_ARG, "chunk size must be in [0, 2^31-1]");
    if (n > 0 && (!upper || !lower || !A)) return fail(XS_ERR_ARG, "upper, lower and A must be non-NULL");
    const bool broad = p->o.broadening == XS_BROAD_PER_LINE;
    if (broad && n > 0 && (!gamma_ref || !n_exp)) return fail(XS_ERR_ARG, "per-line broadening needs gamma_ref and n_exp");
    if (injected_chunk() == st->chunks)
        return fail(XS_ERR_INJECTED, "fault injected before chunk " + std::to_string(st->chunks) +
                                         " (XS_FAULT_INJECT)");
    // a pending host chunk computes first, then this one straight from the caller's arrays
    XS_TRY(stream_process(st));
    st->chunks++;
    if (p->emission != st->emission)
        return fail(XS_ERR_STATE, "the plan's intensity kind changed while the stream was open");
    XS_TRY(xs_set_lines(p, n, upper, lower, A, broad ? gamma_ref : nullptr, broad ? n_exp : nullptr, st->compute));
    st->lines += n;
    st->kept += p->n_kept;
    if (p->n_kept == 0) return XS_OK;
    XS_TRY(xs_cross_section(p, st->n_tp, st->T.data(), st->P.data(), st->tmp.p, st->compute));
    XS_HIP(xs::launch_acc_add(p->o.precision == XS_FP64 ? 1 : 0, st->tmp.p, st->acc.p,
                              (int64_t)st->n_tp * p->geo.n_points, st->compute));
    return XS_OK;
}

xs_status xs_stream_end(xs_stream* st, int64_t* lines_kept) {
    if (!st) return fail(XS_ERR_ARG, "stream is NULL");
    xs_status r = stream_process(st);
    if (r == XS_OK) {
        hipError_t e = xs::launch_acc_finish(st->p->o.precision == XS_FP64 ? 1 : 0, st->acc.p, st->sigma,
                                             (int64_t)st->n_tp * st->p->geo.n_points, st->compute);
        if (e != hipSuccess) r = hip_fail(e, "accumulator read-out");
    }
    if (r == XS_OK && lines_kept) *lines_kept = st->kept;
    stream_free(st);
    return r;
}

// precision and intensity kind of a stream's cross sections, as one checkpoint field
int64_t ckpt_kind(const xs_stream* st) { return st->p->o.precision | (st->emission << 8); }

xs_status xs_stream_checkpoint(xs_stream* st, const char* path) {
    if (!st || !path) return fail(XS_ERR_ARG, "NULL argument");
    XS_TRY(stream_process(st));
    xs_plan* p = st->p;
    const int64_t n = (int64_t)st->n_tp * p->geo.n_points;
    const size_t bytes = (size_t)n * 2 * stream_elem(p);
    std::vector<char> host(bytes);
    XS_HIP(hipMemcpyAsync(host.data(), st->acc.p, bytes, hipMemcpyDeviceToHost, st->compute));
    XS_HIP(hipStreamSynchronize(st->compute));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(XS_ERR_ARG, std::string("cannot write ") + tmp);
    const int64_t hdr[8] = {(int64_t)kCkptMagic, XS_ABI_VERSION, st->n_tp, p->geo.n_points, ckpt_kind(st),
                            st->chunks, st->lines, st->kept};
    const CkptGeometry geo = ckpt_geometry(p);
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1;
    ok = ok && std::fwrite(&geo, sizeof(geo), 1, f) == 1;
    ok = ok && std::fwrite(st->T.data(), sizeof(double), st->n_tp, f) == (size_t)st->n_tp;
    ok = ok && std::fwrite(st->P.data(), sizeof(double), st->n_tp, f) == (size_t)st->n_tp;
    ok = ok && std::fwrite(host.data(), 1, bytes, f) == bytes;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(XS_ERR_ARG, std::string("writing the checkpoint failed: ") + path);
    }
    return XS_OK;
}

xs_status xs_stream_resume(xs_plan* p, const char* path, void* sigma, void* stream, xs_stream** out) {
    if (!out) return fail(XS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !path || !sigma) return fail(XS_ERR_ARG, "NULL argument");
    if (p->n_states <= 0) return fail(XS_ERR_STATE, "xs_set_states must come first");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(XS_ERR_ARG, std::string("cannot read ") + path);
    int64_t hdr[8];
    if (std::fread(hdr, sizeof(hdr), 1, f) != 1 || hdr[0] != (int64_t)kCkptMagic || hdr[1] != XS_ABI_VERSION) {
        std::fclose(f);
        return fail(XS_ERR_ARG, "not a checkpoint of this library version");
    }
    const int n_tp = (int)hdr[2];
    if (n_tp <= 0 || hdr[3] != p->geo.n_points || hdr[4] != (p->o.precision | (p->emission << 8))) {
        std::fclose(f);
        return fail(XS_ERR_ARG, "the checkpoint's grid, precision or intensity kind differs from the plan's");
    }
    CkptGeometry geo{};
    if (std::fread(&geo, sizeof(geo), 1, f) != 1) {
        std::fclose(f);
        return fail(XS_ERR_ARG, "truncated checkpoint");
    }
    if (const char* what = ckpt_mismatch(geo, ckpt_geometry(p))) {
        std::fclose(f);
        return fail(XS_ERR_ARG, std::string("the checkpoint's ") + what + " differs from the plan's");
    }
    std::vector<double> T(n_tp), P(n_tp);
    const size_t bytes = (size_t)n_tp * p->geo.n_points * 2 * stream_elem(p);
    std::vector<char> host(bytes);
    bool ok = std::fread(T.data(), sizeof(double), n_tp, f) == (size_t)n_tp &&
              std::fread(P.data(), sizeof(double), n_tp, f) == (size_t)n_tp &&
              std::fread(host.data(), 1, bytes, f) == bytes;
    std::fclose(f);
    if (!ok) return fail(XS_ERR_ARG, "truncated checkpoint");
    XS_TRY(validate_tp(n_tp, T.data(), P.data()));
    xs_stream* st = nullptr;
    XS_TRY(stream_create(p, n_tp, T.data(), P.data(), sigma, stream, &st));
    hipError_t e = hipMemcpyAsync(st->acc.p, host.data(), bytes, hipMemcpyHostToDevice, st->compute);
    if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
    if (e != hipSuccess) { stream_free(st); return hip_fail(e, "checkpoint upload"); }
    st->chunks = hdr[5];
    st->lines = hdr[6];
    st->kept = hdr[7];
    *out = st;
    return XS_OK;
}

xs_status xs_stream_stats(const xs_stream* st, int64_t out[3]) {
    if (!st || !out) return fail(XS_ERR_ARG, "NULL argument");
    out[0] = st->chunks;
    out[1] = st->lines;
    out[2] = st->kept;
    return XS_OK;
}

xs_status xs_cross_section_adjoint(xs_plan* p, double T, double P, const void* gbar, double* dT, double* dP,
                                   void* dlnA, void* dgref, void* dn, void* stream) {
    if (!p || !gbar) return fail(XS_ERR_ARG, "NULL argument");
    if (!p->have_lines) return fail(XS_ERR_STATE, "xs_set_lines must succeed first");
    if (p->o.profile != XS_VOIGT) return fail(XS_ERR_UNSUPPORTED, "the adjoint is implemented for XS_VOIGT");
    if (threshold_on(p)) return fail(XS_ERR_UNSUPPORTED, "the adjoint does not apply an intensity threshold");
    if (p->emission) return fail(XS_ERR_UNSUPPORTED, "the adjoint differentiates absorption intensities (Eq. 1)");
    if (p->lines_vib) return fail(XS_ERR_UNSUPPORTED, "the adjoint differentiates LTE intensities");
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
    if (p->o.precision == XS_FP32) {
        if ((st = p->ensure(p->adj_rec, n * xs::kAdjRec * sizeof(float), "adjoint records")) != XS_OK) return st;
        if ((st = p->ensure(p->adj_sums, n * 6 * sizeof(double), "adjoint sums")) != XS_OK) return st;
    }
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
    a.rec = as<float>(p->adj_rec);
    a.sums = as<double>(p->adj_sums);
    Timer tf(p, s, 0, 1);
    XS_HIP(xs::launch_adjoint(a, o.precision == XS_FP64 ? 1 : 0, p->n_lines, as<double>(p->adj_part), dT, dP, s));
    tf.stop();
    return XS_OK;
}

xs_status xs_set_timing(xs_plan* p, int enable) {
    if (!p) return fail(XS_ERR_ARG, "plan is NULL");
    if (enable) {
        p->drop_timed();
        for (int k = 0; k < 5; ++k) { p->acc_ms[k] = 0; p->acc_n[k] = 0; }
        p->acc_tp = 0;
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
        if (t.kind == 0) p->acc_tp += t.ntp;
    }
    p->drop_timed();
    out->forward_ms = p->acc_ms[0];
    out->core_ms = p->acc_ms[1];
    out->prep_ms = p->acc_ms[2];
    out->forward_launches = p->acc_n[0];
    out->core_launches = p->acc_n[1];
    out->prep_launches = p->acc_n[2];
    out->combine_ms = p->acc_ms[3];
    out->combine_launches = p->acc_n[3];
    out->forward_tp = p->acc_tp;
    out->far_ms = p->acc_ms[4];
    out->far_launches = p->acc_n[4];
    return XS_OK;
}

size_t xs_workspace_bytes(const xs_plan* p) { return p ? p->total_bytes + p->ws.bytes : 0; }

const char* xs_last_error(void) { return g_err.c_str(); }

int xs_version(void) { return XS_ABI_VERSION; }

}  // extern "C"
