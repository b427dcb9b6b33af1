// Every radix of the tile kernel's butterflies (radix.h over butterfly.h),
// compiled for the host, against the definition eq. dft evaluated in long
// double with the index product reduced exactly.  Prints the worst error per
// radix; exits non-zero above 1e-14 (FP64 butterflies).
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "radix.h"

using namespace mfft;

template <int R>
static double check()
{
    std::mt19937 g(R);
    std::uniform_real_distribution<double> u(-1, 1);
    double worst = 0;
    for (int trial = 0; trial < 4; ++trial) {
        cpx<double> v[R];
        std::complex<long double> x[R];
        for (int i = 0; i < R; ++i) {
            v[i] = {u(g), u(g)};
            x[i] = {v[i].re, v[i].im};
        }
        dftx<double, R>(v);
        for (int k = 0; k < R; ++k) {
            std::complex<long double> s = 0;
            for (int l = 0; l < R; ++l)
                s += x[l] * std::polar(1.0L, -2.0L * 3.14159265358979323846264338327950288L *
                                                 ((l * k) % R) / R);
            worst = std::fmax(worst, (double)std::abs(std::complex<long double>(v[k].re, v[k].im) - s));
        }
    }
    std::printf("radix %2d max error %.3e\n", R, worst);
    return worst;
}

int main()
{
    const double w[] = {check<2>(), check<3>(), check<4>(),  check<5>(),  check<6>(),
                        check<7>(), check<8>(), check<9>(),  check<10>(), check<12>(),
                        check<14>(), check<15>(), check<16>(), check<11>(), check<13>(),
                        check<17>(), check<19>(), check<23>()};
    double m = 0;
    for (double e : w) m = std::fmax(m, e);
    return m < 1e-14 ? 0 : 1;
}
