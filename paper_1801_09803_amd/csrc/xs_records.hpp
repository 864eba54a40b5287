// Line records of the FP32 path (written by record_kernel once per (line, T, P), read by
// the tile kernel and the node-sampled far-wing kernels): their word layouts.
#pragma once

#include "xs_forward_common.hpp"

namespace xs {

// hot record words: scale h, 2-node coefficients C0 C1 AMP B, centre offset XC, window
// bounds JLO JHI relative to kc; the Vectorized Voigt adds its wing term Y and amplitude VB
// and the R-region bounds JVLO JVHI, and puts {h, Y, VB, XC} first so that its wing loop
// reads one float4 per line
template <int PROF>
struct HotOf {
    static constexpr int H = 0, C0 = 1, C1 = 2, AMP = 3, B = 4, XC = 5, JLO = 6, JHI = 7;
    static constexpr int VY = -1, VB = -1, JVLO = -1, JVHI = -1;
};
template <>
struct HotOf<kVVoigt> {
    static constexpr int H = 0, VY = 1, VB = 2, XC = 3, C0 = 4, C1 = 5, AMP = 6, B = 7;
    static constexpr int JLO = 8, JHI = 9, JVLO = 10, JVHI = 11;
};
// cold record words (ints unless noted; C_CBASE is int64, C_M up to 8 floats: the Voigt
// zones' 4-node rule coefficients m0..m7 (struct Mid); the Gauss-Hermite profiles five).
// A row of records keeps words 0-7 of all its lines, then words 8-15 (two planes); Voigt
// records leave the second plane unwritten (mid_from_hot rebuilds m0..m7).
enum : int { C_CSC = 0, C_KC = 1, C_RAD = 2, C_KCL = 3, C_KCH = 4, C_FLAG = 5, C_CBASE = 6, C_M = 8 };
constexpr int kHot = 8;
constexpr int kCold = 16;
constexpr bool is_voigt(int prof) { return prof == kVoigt || prof == kVVoigt; }

// The 4-node rule's node pairs (t_a, w_a), (t_b, w_b) as t^2 and w, single precision.
struct MidNodes {
    float t2a, t2b, wa, wb;
};
__device__ __forceinline__ MidNodes mid_nodes(const Tables* tab) {
    MidNodes n;
    n.t2a = (float)(tab->gh4.t[0] * tab->gh4.t[0]);
    n.t2b = (float)(tab->gh4.t[1] * tab->gh4.t[1]);
    n.wa = (float)tab->gh4.w[0];
    n.wb = (float)tab->gh4.w[1];
    return n;
}

// The 4-node rule coefficients m0..m7 of a Voigt line in unscaled x (p_j = x^2 + y^2 - t_j^2,
// d_j = p_j^2 + 4 t_j^2 y^2, n_j = amp w_j (p_j + 2 t_j^2), amp = 2 a y / pi) from its hot
// words C1 = 2 y^2 sc^4 and AMP = a y sc^2 / sqrt(pi) and its x scale csc = 1/sc, a power of
// two: y^2 = C1 csc^4 / 2 and amp = (2/sqrt(pi)) AMP csc^2, both exact up to the words' own
// rounding.
__device__ __forceinline__ void mid_from_hot(float c1, float ampw, float csc, const MidNodes& n, float (&m)[8]) {
    const float csc2 = csc * csc;
    const float y2 = 0.5f * (c1 * (csc2 * csc2));
    const float amp = (ampw * csc2) * 1.1283791670955126f;   // 2 / sqrt(pi)
    const float ma = amp * n.wa, mb = amp * n.wb;
    m[0] = y2 - n.t2a;
    m[1] = 4.0f * n.t2a * y2;
    m[2] = ma;
    m[3] = ma * (2.0f * n.t2a);
    m[4] = y2 - n.t2b;
    m[5] = 4.0f * n.t2b * y2;
    m[6] = mb;
    m[7] = mb * (2.0f * n.t2b);
}
constexpr int hot_words(int prof) { return prof == kVVoigt ? 12 : kHot; }
// segmented sweep: keep per-wavefront anchors in the LDS record (saves two operations per
// line and wavefront) or rebuild them (a smaller LDS image)
constexpr bool anchors_in_lds(int prof) { return prof != kVVoigt; }

}  // namespace xs
