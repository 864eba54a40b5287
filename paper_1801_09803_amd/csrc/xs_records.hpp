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
// zones' 4-node rule coefficients m0..m7 (struct Mid); the Gauss-Hermite profiles five)
enum : int { C_CSC = 0, C_KC = 1, C_RAD = 2, C_KCL = 3, C_KCH = 4, C_FLAG = 5, C_CBASE = 6, C_M = 8 };
constexpr int kHot = 8;
constexpr int kCold = 16;
constexpr bool is_voigt(int prof) { return prof == kVoigt || prof == kVVoigt; }
constexpr int hot_words(int prof) { return prof == kVVoigt ? 12 : kHot; }
// segmented sweep: keep per-wavefront anchors in the LDS record (saves two operations per
// line and wavefront) or rebuild them (a smaller LDS image)
constexpr bool anchors_in_lds(int prof) { return prof != kVVoigt; }

}  // namespace xs
