// Host-side FP64 construction of the colour-temperature LUT (Eq. 13 and the
// colour-temperature mapping of Sec. 3.3). Runs on the CPU once per set of
// temperature parameters; the table is then held in device memory as FP32.
#include <cmath>
#include <thread>
#include <vector>

#include "rte_internal.h"

namespace rte {
namespace {

// Planck's law: spectral radiance of a black body at wavelength lam [m] and
// temperature T [K]; exact SI constants, vacuum speed of light.
double planck_radiance(double lam, double T)
{
    const double h = 6.62607015e-34, c = 2.99792458e8, kb = 1.380649e-23;
    const double x = h * c / (lam * kb * T);
    return 2.0 * h * c * c / std::pow(lam, 5.0) / std::expm1(x);
}

// Radiance seen through a Gaussian band (centre mu, standard deviation sd, in
// nm): composite Simpson over mu +- 6 sd with an even number of panels.
double band_integral(double T, double mu, double sd, int panels)
{
    if (panels < 2) panels = 2;
    if (panels % 2) ++panels;
    const double a = mu - 6.0 * sd, b = mu + 6.0 * sd, step = (b - a) / panels;
    double acc = 0.0;
    for (int i = 0; i <= panels; ++i) {
        const double lam = a + i * step;
        const double z = (lam - mu) / sd;
        const double f = planck_radiance(lam * 1e-9, T) * std::exp(-0.5 * z * z);
        const double wgt = (i == 0 || i == panels) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
        acc += wgt * f;
    }
    return acc * step / 3.0;
}

}  // namespace

void build_temperature_lut(const rte_temp_params &tp, std::vector<float> &lut)
{
    const int L = tp.lut_size;
    lut.assign((size_t)3 * L, 0.0f);
    const double norm = band_integral(tp.t_norm, tp.band_nm[tp.channel], tp.band_std_nm, tp.panels);
    const int n_workers = 8;
    std::vector<std::thread> pool;
    for (int w = 0; w < n_workers; ++w) {
        pool.emplace_back([&, w]() {
            for (int idx = w; idx < 3 * L; idx += n_workers) {
                const int c = idx / L, i = idx % L;
                const double T = (double)tp.t_min + ((double)tp.t_max - (double)tp.t_min) * (double)i / (double)(L - 1);
                lut[idx] = (float)(band_integral(T, tp.band_nm[c], tp.band_std_nm, tp.panels) / norm);
            }
        });
    }
    for (auto &t : pool) t.join();
}

}  // namespace rte
