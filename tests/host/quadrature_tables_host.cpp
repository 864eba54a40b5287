// Prints the quadrature tables the library's host code builds at plan creation, for
// tests/test_quadrature_tables.py:
//   dawson                  the core pre-pass's Dawson table (xs::dawson_table)
//   gh <n>                  the n-point Gauss-Hermite rule (xs::gauss_hermite_rule)
//   weideman <n>            Weideman's n coefficients and L (xs::weideman_coefficients)
// one header line of sizes, then one value per line.
#include "xs_internal.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

int main(int argc, char** argv) {
    if (argc >= 2 && !std::strcmp(argv[1], "dawson")) {
        double t[xs::kDawsonIv * xs::kDawsonNc];
        xs::dawson_table(t);
        std::printf("%d %d\n", xs::kDawsonIv, xs::kDawsonNc);
        for (double v : t) std::printf("%.17g\n", v);
        return 0;
    }
    if (argc >= 3 && !std::strcmp(argv[1], "gh")) {
        const int n = std::atoi(argv[2]);
        if (n < 1 || n > xs::kMaxGHConv) return 2;
        std::vector<double> t(n), w(n);
        xs::gauss_hermite_rule(n, t.data(), w.data());
        std::printf("%d\n", n);
        for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", t[i], w[i]);
        return 0;
    }
    if (argc >= 3 && !std::strcmp(argv[1], "weideman")) {
        const int n = std::atoi(argv[2]);
        if (n < 3 || n > xs::kMaxWeideman) return 2;
        xs::WeidemanCoef c;
        xs::weideman_coefficients(n, &c);
        std::printf("%d %.17g\n", c.n, c.L);
        for (int i = 0; i < n; ++i) std::printf("%.17g\n", c.a[i]);
        return 0;
    }
    std::fprintf(stderr, "usage: %s dawson | gh <n> | weideman <n>\n", argv[0]);
    return 2;
}
