// Host checks of the WENO5 face arithmetic of the device code (ch_device.h),
// in single and double precision:
//  1. the increment is odd in the differences, bit for bit;
//  2. reading a stencil from the downwind side equals the centre minus the
//     increment of the forward differences in reverse order, bit for bit;
//  3. the shared-difference face flux u*C_up + |u|*inc equals u times the
//     value-based face (upwinded by the sign of u) to a few units in the
//     last place of the terms;
//  4. the fourth difference from first differences equals the 5-point
//     (1, -4, 6, -4, 1) stencil: exactly on integer data, to rounding on
//     random data;
//  5. the face value equals the Jiang-Shu WENO5 formula written out plainly
//     (three candidate parabolas, smoothness indicators, weights
//     0.1 / 0.6 / 0.3 over (eps + beta)^2), in double precision to 1e-12.
// Prints one line per failure and "ok" at the end; exits 1 on any failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "../../paper_2105_01865_amd/csrc/ch_device.h"

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ull;

// splitmix64: a deterministic stream of doubles in [0, 1)
double uniform()
{
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
bool same_bits(T a, T b)
{
    return std::memcmp(&a, &b, sizeof(T)) == 0;
}

int failures = 0;

template <typename T>
void fail(const char* what, int trial, double a, double b)
{
    if (failures < 20)
        std::printf("%s (%s) trial %d: %.17g vs %.17g\n", what, sizeof(T) == 4 ? "fp32" : "fp64",
                    trial, a, b);
    ++failures;
}

// six cell values: smooth, a jump, a tanh-like front or noise
template <typename T>
void stencil(int kind, T c[6])
{
    const double a = uniform() * 2 - 1, b = uniform() * 2 - 1, off = uniform();
    for (int i = 0; i < 6; ++i) {
        double v;
        switch (kind) {
        case 0: v = off + a * 0.05 * i + b * 0.002 * i * i; break;
        case 1: v = i < 3 ? off : off + a; break;
        case 2: v = 0.5 + 0.5 * std::tanh(4.0 * (i - 2.5 + b)); break;
        default: v = uniform(); break;
        }
        c[i] = T(v);
    }
}

// Jiang-Shu WENO5 at the face between c and d (upwind side a), as printed
// in textbooks: candidates, smoothness indicators, normalised weights.
double weno5_textbook(double a, double b, double c, double d, double e, double eps)
{
    const double q0 = (2 * a - 7 * b + 11 * c) / 6, q1 = (-b + 5 * c + 2 * d) / 6,
                 q2 = (2 * c + 5 * d - e) / 6;
    const double b0 = 13.0 / 12 * (a - 2 * b + c) * (a - 2 * b + c) +
                      0.25 * (a - 4 * b + 3 * c) * (a - 4 * b + 3 * c);
    const double b1 = 13.0 / 12 * (b - 2 * c + d) * (b - 2 * c + d) + 0.25 * (b - d) * (b - d);
    const double b2 = 13.0 / 12 * (c - 2 * d + e) * (c - 2 * d + e) +
                      0.25 * (3 * c - 4 * d + e) * (3 * c - 4 * d + e);
    const double a0 = 0.1 / ((eps + b0) * (eps + b0)), a1 = 0.6 / ((eps + b1) * (eps + b1)),
                 a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

template <typename T>
void run(int trials)
{
    const T eps = T(1e-6 * 12.0 / 13.0);
    const double ulp = sizeof(T) == 4 ? 1.1920929e-07 : 2.220446049250313e-16;
    for (int n = 0; n < trials; ++n) {
        T c[6];
        stencil<T>(n % 4, c);
        T D[6];   // D[j] = c[j] - c[j-1], j = 1 .. 5
        for (int j = 1; j < 6; ++j) D[j] = c[j] - c[j - 1];
        // 1: oddness
        const T inc = chd::weno5_inc<T>(D[1], D[2], D[3], D[4], eps);
        const T neg = chd::weno5_inc<T>(-D[1], -D[2], -D[3], -D[4], eps);
        if (!same_bits<T>(neg, -inc)) fail<T>("increment not odd", n, neg, -inc);
        // 2: downwind reading
        const T back = chd::weno5<T>(c[5], c[4], c[3], c[2], c[1], eps);
        const T back_d = c[3] - chd::weno5_inc<T>(D[5], D[4], D[3], D[2], eps);
        if (!same_bits<T>(back, back_d)) fail<T>("downwind reading", n, back, back_d);
        // 3: flux through the face, both signs and zero
        const double speeds[3] = {uniform() + 0.01, -(uniform() + 0.01), 0.0};
        for (double sp : speeds) {
            const T vel = T(sp);
            const T f_val = vel * chd::face_weno<T>(vel, c[0], c[1], c[2], c[3], c[4], c[5], eps);
            const T f_d = chd::flux_weno_d<T>(vel, D[1], D[2], D[3], D[4], D[5], c[2], c[3], eps);
            const T cen = vel >= T(0) ? c[2] : c[3];
            const double scale =
                std::fabs((double)vel) *
                (std::fabs((double)cen) + std::fabs((double)inc) + std::fabs((double)back - c[3]));
            if (std::fabs((double)f_val - (double)f_d) > 8 * ulp * scale)
                fail<T>("face flux", n, f_val, f_d);
        }
        // 4: fourth difference, random data
        const double d4ref = (double)c[0] - 4.0 * c[1] + 6.0 * c[2] - 4.0 * c[3] + (double)c[4];
        const T d4 = chd::d4_d<T>(D[1], D[2], D[3], D[4]);
        double mag = 0;
        for (int i = 0; i < 5; ++i) mag += std::fabs((double)c[i]);
        if (std::fabs((double)d4 - d4ref) > 32 * ulp * mag)
            fail<T>("fourth difference", n, d4, d4ref);
    }
    // 5: against the textbook formula (double precision only)
    if constexpr (sizeof(T) == 8) {
        for (int n = 0; n < trials; ++n) {
            T c[6];
            stencil<T>(n % 4, c);
            const double eps = 1e-6;
            const double ref = weno5_textbook(c[0], c[1], c[2], c[3], c[4], eps);
            const double got = chd::weno5<double>(c[0], c[1], c[2], c[3], c[4], eps * 12.0 / 13.0);
            double mag = 0;
            for (int i = 0; i < 5; ++i) mag += std::fabs(c[i]);
            if (std::fabs(got - ref) > 1e-12 * mag) fail<T>("textbook WENO5", n, got, ref);
        }
    }
    // 4: fourth difference, small integers (every operation exact)
    for (int n = 0; n < trials; ++n) {
        T c[5];
        for (int i = 0; i < 5; ++i) c[i] = T(std::floor(uniform() * 200.0) - 100.0);
        const T d4 = chd::d4_d<T>(c[1] - c[0], c[2] - c[1], c[3] - c[2], c[4] - c[3]);
        const T ref = c[0] - T(4) * c[1] + T(6) * c[2] - T(4) * c[3] + c[4];
        if (!same_bits<T>(d4, ref)) fail<T>("fourth difference, integers", n, d4, ref);
    }
}

}  // namespace

int main()
{
    run<float>(20000);
    run<double>(20000);
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
