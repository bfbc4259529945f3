// Host check of sincos_cw: reads x values from stdin, prints sin and cos.
#include <cstdio>

#include "../fastmath.hpp"

int main()
{
    double x;
    while (std::scanf("%lf", &x) == 1) {
        double s, c;
        nfq::sincos_cw(x, &s, &c);
        std::printf("%.17g %.17g\n", s, c);
    }
    return 0;
}
