// tables.cpp -- host-side construction of the engine's cross-section tables (FP64 math,
// stored as FP32 on log-spaced energy nodes).
//
// Photons (Sec. 2.1.2 lists photoelectric absorption, Compton scattering and pair
// production): per material mu/rho and the cumulative process fractions; the phantom
// majorant used by delta tracking.  Electrons (Class II condensed history, Sec. 2.1.2):
// restricted range, hard-event cross section and its Moller share, radiation length.
// The models are the documented analytic readings: free-electron Klein-Nishina, a
// Z^4/E^3 photoelectric law, a log-growth pair law above 2 m c^2, restricted Bethe
// collision loss with a 200 keV Moller threshold, a 1/k bremsstrahlung spectrum with
// S_rad/S_col = Z_eff T / 800 MeV and a 10 keV hard-photon threshold, Dahl's X0.
#include "tables.hpp"

#include <algorithm>
#include <cmath>

namespace epidmc {

static const double PI = 3.14159265358979323846;

MatDerived derive(const HostMaterial &m)
{
    MatDerived d{};
    double wsum = 0;
    for (int i = 0; i < m.n; ++i) wsum += m.w[i];
    double ze = 0, zz = 0, inv_x0 = 0;
    for (int i = 0; i < m.n; ++i) {
        const double w = m.w[i] / wsum, Z = m.Z[i], A = m.A[i];
        const double atoms = NAVO * w / A;      // atoms of this element per gram
        d.ne += atoms * Z;
        d.pe_sum += atoms * Z * Z * Z * Z;
        d.pair_sum += atoms * Z * Z;
        ze += w * Z / A;
        zz += w * Z * Z / A;
        inv_x0 += w * (Z * (Z + 1.0) * std::log(287.0 / std::sqrt(Z))) / (716.4 * A);
    }
    d.zeff = zz / ze;
    d.x0 = 1.0 / inv_x0;
    d.ir = m.I_eV * 1e-6 / MEC2;
    return d;
}

double kn_total(double E)
{
    // Klein-Nishina cross section per free electron, cm^2
    const double k = E / MEC2, q = 1.0 + 2.0 * k, L = std::log(q);
    const double a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / q - L / k);
    return 2.0 * PI * RE_CM * RE_CM * (a + L / (2.0 * k) - (1.0 + 3.0 * k) / (q * q));
}

void photon_mu(const MatDerived &d, double E, uint32_t mask, double out[4])
{
    const double c = (mask & 1u) ? d.ne * kn_total(E) : 0.0;
    const double p = (mask & 2u) ? d.pe_sum * C_PE / (E * E * E) : 0.0;
    double q = 0.0;
    if ((mask & 4u) && E > 2.0 * MEC2) {
        const double r = 1.0 - 2.0 * MEC2 / E;
        q = d.pair_sum * (28.0 / 9.0) * ALPHA_FS * RE_CM * RE_CM * std::log(E / (2.0 * MEC2)) * r * r;
    }
    out[0] = c + p + q;
    out[1] = c;
    out[2] = p;
    out[3] = q;
}

double collision_power(const MatDerived &d, double T, bool restricted)
{
    // Bethe collision stopping power of electrons without density effect (MeV cm^2/g),
    // restricted to energy transfers below min(WCUT, T/2) when asked
    const double tau = T / MEC2, g = tau + 1.0, b2 = 1.0 - 1.0 / (g * g);
    const double D = restricted ? std::min(WCUT / MEC2, 0.5 * tau) : 0.5 * tau;
    const double F = -1.0 - b2 + std::log((tau - D) * D) + tau / (tau - D) +
                     (0.5 * D * D + (2.0 * tau + 1.0) * std::log(1.0 - D / tau)) / (g * g);
    return 2.0 * PI * RE_CM * RE_CM * MEC2 * d.ne / b2 * (std::log(2.0 * (tau + 2.0) / (d.ir * d.ir)) + F);
}

double radiative_power(const MatDerived &d, double T) { return collision_power(d, T, false) * d.zeff * T / BREM_K; }

double restricted_loss(const MatDerived &d, double T)
{
    return collision_power(d, T, true) + radiative_power(d, T) * KCUT / T;
}

double moller_xs(const MatDerived &d, double T)
{
    if (T <= 2.0 * WCUT) return 0.0;
    const double g = T / MEC2 + 1.0, b2 = 1.0 - 1.0 / (g * g), ec = WCUT / T;
    const double c1 = (g - 1.0) * (g - 1.0) / (g * g), c2 = (2.0 * g - 1.0) / (g * g);
    const double I = c1 * (0.5 - ec) + 1.0 / ec - 1.0 / (1.0 - ec) - c2 * std::log((1.0 - ec) / ec);
    return d.ne * 2.0 * PI * RE_CM * RE_CM * MEC2 / (b2 * T) * I;
}

double brems_xs(const MatDerived &d, double T)
{
    if (T <= KCUT) return 0.0;
    return radiative_power(d, T) / T * std::log(T / KCUT);
}

// composite Simpson integral of 1/L_res over [a, b], n panels
static double simpson_inv_loss(const MatDerived &d, double a, double b, int n)
{
    const double h = (b - a) / n;
    double s = 1.0 / restricted_loss(d, a) + 1.0 / restricted_loss(d, b);
    for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) / restricted_loss(d, a + i * h);
    return s * h / 3.0;
}

double range_between(const MatDerived &d, double a, double b)
{
    if (b <= a) return 0.0;
    const double kink = 2.0 * WCUT;   // restricted loss changes form at T = 2 WCUT
    if (a < kink && kink < b) return range_between(d, a, kink) + range_between(d, kink, b);
    return simpson_inv_loss(d, a, b, 64);
}

void build_photon_table(const MatDerived &d, uint32_t mask, double lnE0, double dl, float *out)
{
    for (int i = 0; i < NB_PH; ++i) {
        double mu[4];
        photon_mu(d, std::exp(lnE0 + i * dl), mask, mu);
        out[i] = (float)mu[0];
        out[NB_PH + i] = mu[0] > 0 ? (float)(mu[1] / mu[0]) : 1.0f;
        out[2 * NB_PH + i] = mu[0] > 0 ? (float)((mu[1] + mu[2]) / mu[0]) : 1.0f;
    }
}

void build_electron_table(const MatDerived &d, uint32_t mask, double lnT0, double dl, float *out)
{
    double R = 0.0, Tp = std::exp(lnT0);
    for (int i = 0; i < NB_EL; ++i) {
        const double T = std::exp(lnT0 + i * dl);
        if (i > 0) R += range_between(d, Tp, T);
        Tp = T;
        const double sm = (mask & 8u) ? 0.0 : moller_xs(d, T);
        const double sb = (mask & 8u) ? 0.0 : brems_xs(d, T);
        out[i] = (float)R;
        out[NB_EL + i] = (float)(sm + sb);
        out[2 * NB_EL + i] = (sm + sb) > 0 ? (float)(sm / (sm + sb)) : 0.0f;
    }
}

void build_alias(const std::vector<double> &w, std::vector<float> &prob, std::vector<int> &alias)
{
    // Vose's alias method: bin i keeps itself with probability prob[i], else alias[i]
    const int n = (int)w.size();
    prob.assign(n, 1.0f);
    alias.assign(n, 0);
    double tot = 0;
    for (double x : w) tot += x;
    if (n == 0 || tot <= 0) return;
    std::vector<double> p(n);
    std::vector<int> small, large;
    for (int i = 0; i < n; ++i) {
        p[i] = w[i] * n / tot;
        alias[i] = i;
        (p[i] < 1.0 ? small : large).push_back(i);
    }
    while (!small.empty() && !large.empty()) {
        const int s = small.back(), l = large.back();
        small.pop_back();
        prob[s] = (float)p[s];
        alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) { large.pop_back(); small.push_back(l); }
    }
    for (int i : large) { prob[i] = 1.0f; alias[i] = i; }
    for (int i : small) { prob[i] = 1.0f; alias[i] = i; }
    // a zero-weight bin left over by rounding must hand its slot to a weighted bin
    const int imax = (int)(std::max_element(w.begin(), w.end()) - w.begin());
    for (int i = 0; i < n; ++i)
        if (w[i] <= 0 && alias[i] == i) { prob[i] = 0.0f; alias[i] = imax; }
}

}  // namespace epidmc
