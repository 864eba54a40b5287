// Prints the core pre-pass's Dawson table as the library's host code builds it at plan
// creation (xs::dawson_table), one coefficient per line, for tests/test_dawson_table.py.
#include "xs_internal.hpp"

#include <cstdio>

int main() {
    double t[xs::kDawsonIv * xs::kDawsonNc];
    xs::dawson_table(t);
    std::printf("%d %d\n", xs::kDawsonIv, xs::kDawsonNc);
    for (int i = 0; i < xs::kDawsonIv * xs::kDawsonNc; ++i) std::printf("%.17g\n", t[i]);
    return 0;
}
