// stencil_dump.cpp -- prints the library's 1-D transfer stencils (the
// Hermite tables built by ch_plan.h) for the host tests (test
// infrastructure).
//
// stdin:  "kind n" then n source coordinates, then "m" and m targets
//         (kind 0 periodic with period 1, 1 mirrored cell centres between
//         walls at 0 and 1, 2 face values including both walls, continued
//         oddly)
// stdout: one line per target, "i0 i1 i2 i3 w0 w1 w2 w3", or "FAIL"
#include <cstdio>
#include <vector>

#include "../../paper_2105_01865_amd/csrc/ch_plan.h"

int main()
{
    chp::SrcAxis a;
    int n = 0;
    if (scanf("%d %d", &a.kind, &n) != 2 || n < 1) return 2;
    a.s.resize(n);
    for (int i = 0; i < n; ++i)
        if (scanf("%lf", &a.s[i]) != 1) return 2;
    int m = 0;
    if (scanf("%d", &m) != 1 || m < 0) return 2;
    std::vector<double> t(m);
    for (int i = 0; i < m; ++i)
        if (scanf("%lf", &t[i]) != 1) return 2;
    std::vector<int> idx;
    std::vector<double> w;
    if (!chp::hermite_stencils(a, t, &idx, &w)) {
        printf("FAIL\n");
        return 0;
    }
    for (int q = 0; q < m; ++q)
        printf("%d %d %d %d %.17g %.17g %.17g %.17g\n", idx[4 * q], idx[4 * q + 1],
               idx[4 * q + 2], idx[4 * q + 3], w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    return 0;
}
