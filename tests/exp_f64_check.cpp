// Test helper: the fused logistic kernel's FP64 exponential compiled for the
// host.  Reads doubles from stdin and writes exp_lds(x) for each to stdout.
#include "exp_f64.hpp"

#include <cstdio>

int main() {
    double cf[hmc::EXP_NC];
    for (int n = 0; n < hmc::EXP_NC; ++n) cf[n] = hmc::exp_coef(n);
    double x;
    while (std::fread(&x, sizeof(double), 1, stdin) == 1) {
        const double y = hmc::exp_lds(x, cf);
        std::fwrite(&y, sizeof(double), 1, stdout);
    }
    return 0;
}
