// tables.hpp -- host-side physics used to build the device tables.
#pragma once
#include <vector>

#include "engine.hpp"

namespace epidmc {

struct HostMaterial {
    int n;
    int Z[8];
    double A[8], w[8];
    double I_eV;
};

struct MatDerived {
    double ne;        // electrons per gram
    double pe_sum;    // sum over elements of atoms/g * Z^4
    double pair_sum;  // sum over elements of atoms/g * Z^2
    double zeff;      // electron-weighted mean Z
    double x0;        // radiation length, g/cm^2
    double ir;        // I / m c^2
};

MatDerived derive(const HostMaterial &m);
double kn_total(double E);
void photon_mu(const MatDerived &d, double E, uint32_t mask, double out[4]);
double collision_power(const MatDerived &d, double T, bool restricted);
double restricted_loss(const MatDerived &d, double T);
double moller_xs(const MatDerived &d, double T);
double brems_xs(const MatDerived &d, double T);
double range_between(const MatDerived &d, double a, double b);
void build_photon_table(const MatDerived &d, uint32_t mask, double lnE0, double dl, float *out);
void build_electron_table(const MatDerived &d, uint32_t mask, double lnT0, double dl, float *out);
void build_alias(const std::vector<double> &w, std::vector<float> &prob, std::vector<int> &alias);

}  // namespace epidmc
