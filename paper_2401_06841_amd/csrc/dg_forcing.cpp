// dg_forcing.cpp -- Ornstein-Uhlenbeck driving modes (Sec. 4.2), host side, FP64.
//
// The acceleration field is built from the Fourier modes with 1 <= |n| <= 2 (box units,
// k_min = 2 pi / L to k_max = 2 k_min), one complex 3-vector per +/- pair (the half
// space whose first non-zero component is positive: 16 vectors).  Each real and
// imaginary component follows x <- f x + sigma sqrt(1 - f^2) z, f = exp(-dt/t_c), with
// stationary standard deviation sigma; the installed amplitudes are the components
// perpendicular to n (purely solenoidal driving).
#include <cmath>
#include <cstring>

#include "dg.h"
#include "dg_ctx.hpp"

namespace {

constexpr int NMODES = 16;

int shell(int (*n)[3])
{
    int m = 0;
    for (int a = -2; a <= 2; ++a)
        for (int b = -2; b <= 2; ++b)
            for (int c = -2; c <= 2; ++c) {
                const int n2 = a * a + b * b + c * c;
                if (n2 < 1 || n2 > 4) continue;
                const int first = a != 0 ? a : (b != 0 ? b : c);
                if (first <= 0) continue;
                n[m][0] = a; n[m][1] = b; n[m][2] = c;
                ++m;
            }
    return m;
}

}  // namespace

int dg_forcing_ou_ndraws(void) { return NMODES * 6; }

int dg_forcing_ou_init(dg_ctx *c, double t_c, double sigma)
{
    if (!c) return DG_EINVAL;
    if (!(t_c > 0.0) || !(sigma >= 0.0)) return dg_fail(c, DG_EINVAL, "t_c must be > 0 and sigma >= 0");
    c->ou_tc = t_c;
    c->ou_sigma = sigma;
    std::memset(c->ou_x, 0, sizeof(c->ou_x));
    c->ou_ready = 1;
    return DG_OK;
}

int dg_forcing_ou_advance(dg_ctx *c, const double *z, double dt_drive)
{
    if (!c) return DG_EINVAL;
    if (!c->ou_ready) return dg_fail(c, DG_ESTATE, "dg_forcing_ou_init was not called");
    if (!z || !(dt_drive >= 0.0)) return dg_fail(c, DG_EINVAL, "bad draws or dt_drive");
    const double f = std::exp(-dt_drive / c->ou_tc);
    const double g = c->ou_sigma * std::sqrt(1.0 - f * f);
    for (int i = 0; i < NMODES * 6; ++i) c->ou_x[i] = f * c->ou_x[i] + g * z[i];
    int n[NMODES][3];
    const int nm = shell(n);
    double tab[NMODES * 9];
    for (int m = 0; m < nm; ++m) {
        const double nn = n[m][0] * n[m][0] + n[m][1] * n[m][1] + n[m][2] * n[m][2];
        double *row = tab + 9 * m;
        row[0] = n[m][0]; row[1] = n[m][1]; row[2] = n[m][2];
        for (int ri = 0; ri < 2; ++ri) {          // real and imaginary parts
            const double *x = c->ou_x + 6 * m + 3 * ri;
            const double dot = (n[m][0] * x[0] + n[m][1] * x[1] + n[m][2] * x[2]) / nn;
            for (int d = 0; d < 3; ++d) row[3 + 2 * d + ri] = x[d] - dot * n[m][d];
        }
    }
    return dg_set_forcing(c, tab, nm);
}

int dg_forcing_ou_get(const dg_ctx *c, double *x)
{
    if (!c || !x) return DG_EINVAL;
    std::memcpy(x, c->ou_x, sizeof(c->ou_x));
    return DG_OK;
}

int dg_forcing_ou_set(dg_ctx *c, const double *x)
{
    if (!c) return DG_EINVAL;
    if (!x) return dg_fail(c, DG_EINVAL, "x is null");
    if (!c->ou_ready) return dg_fail(c, DG_ESTATE, "dg_forcing_ou_init was not called");
    std::memcpy(c->ou_x, x, sizeof(c->ou_x));
    double z[NMODES * 6] = {};
    return dg_forcing_ou_advance(c, z, 0.0);   // f = 1, no noise: installs the table of x
}
