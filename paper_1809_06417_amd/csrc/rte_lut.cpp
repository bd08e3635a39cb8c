// Host-side FP64 construction of the colour-temperature LUT (Eq. 13 and the
// colour-temperature mapping of Sec. 3.3). Runs on the CPU once per set of
// temperature parameters; the table is then held in device memory as FP32.
//
// Band radiance: the Planck spectrum seen through a Gaussian camera band,
//   band(T) = int B(lambda, T) exp(-z^2 / 2) dlambda,  z = (lambda - mu) / sd,
// over the band window |z| <= 6 (the window is part of the definition: at
// 800 K the blue band's integrand still grows towards the window's red end,
// so a wider window changes the table there by up to 7e-6 relative),
// integrated in z by composite Gauss-Legendre quadrature. Only ratios of
// band radiances enter the table, so constant factors (the units of lambda,
// the Jacobian sd) cancel.
#include <cmath>
#include <thread>
#include <vector>

#include "rte_internal.h"

namespace rte {
namespace {

constexpr double kZ = 6.0;        // half-width of the band window, in standard deviations
constexpr int kGaussNodes = 4;    // nodes per sub-interval

// Planck's law written with the two radiation constants,
// B = c1 / (lambda^5 (exp(c2 / (lambda T)) - 1)), c1 = 2 h c^2, c2 = h c / k
// (exact SI values of h, c, k; vacuum speed of light), lambda in metres.
double planck_c1c2(double lambda_m, double T)
{
    const double h = 6.62607015e-34, c = 2.99792458e8, k = 1.380649e-23;
    const double c1 = 2.0 * h * c * c, c2 = h * c / k;
    const double l2 = lambda_m * lambda_m;
    return c1 / (l2 * l2 * lambda_m) / std::expm1(c2 / (lambda_m * T));
}

// Nodes and weights of n-point Gauss-Legendre quadrature on [-1, 1]: roots of
// the Legendre polynomial P_n by Newton's method (P_n and P_n' from the
// three-term recurrence), w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double r = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = r;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (r * p1 - p0) / (r * r - 1.0);
            const double dr = p1 / dp;
            r -= dr;
            if (std::fabs(dr) < 1e-16) break;
        }
        x[i] = r;
        w[i] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
}

// Band radiance in z (see above) on `parts` equal sub-intervals of [-kZ, kZ].
double band_radiance_gl(double T, double mu_nm, double sd_nm, int parts, const std::vector<double> &gx,
                        const std::vector<double> &gw)
{
    const double hz = 2.0 * kZ / parts;
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) {
        const double zc = -kZ + (p + 0.5) * hz;
        double part = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double z = zc + 0.5 * hz * gx[i];
            const double lam_nm = mu_nm + sd_nm * z;
            part += gw[i] * planck_c1c2(lam_nm * 1e-9, T) * std::exp(-0.5 * z * z);
        }
        acc += part;
    }
    return acc * 0.5 * hz;
}

}  // namespace

// `panels` sets the resolution: panels / kGaussNodes sub-intervals (at least
// one), i.e. about as many Planck evaluations per band as panels.
void build_temperature_lut(const rte_temp_params &tp, std::vector<float> &lut)
{
    const int L = tp.lut_size;
    lut.assign((size_t)3 * L, 0.0f);
    std::vector<double> gx, gw;
    gauss_legendre(kGaussNodes, gx, gw);
    const int parts = tp.panels / kGaussNodes > 1 ? tp.panels / kGaussNodes : 1;
    const double norm = band_radiance_gl(tp.t_norm, tp.band_nm[tp.channel], tp.band_std_nm, parts, gx, gw);
    const int n_workers = 8;
    std::vector<std::thread> pool;
    for (int w = 0; w < n_workers; ++w) {
        pool.emplace_back([&, w]() {
            for (int idx = w; idx < 3 * L; idx += n_workers) {
                const int c = idx / L, i = idx % L;
                const double T = (double)tp.t_min + ((double)tp.t_max - (double)tp.t_min) * (double)i / (double)(L - 1);
                lut[idx] = (float)(band_radiance_gl(T, tp.band_nm[c], tp.band_std_nm, parts, gx, gw) / norm);
            }
        });
    }
    for (auto &t : pool) t.join();
}

}  // namespace rte
