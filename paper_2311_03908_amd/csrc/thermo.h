// Thermochemistry of the particle energy equation: species enthalpy and heat
// capacity (eqs. e3-22, e3-23, Table C1), gas conductivity (eqs. e3-58,
// e3-59, Table C3) and gas specific heat (eq. e3-57).
//
// Table C1 is printed to about three figures.  Taken literally its
// enthalpies jump at the range bounds (9 kJ/mol for Fe2O3 at 960 K) and Fe's
// 1000-1042 K range has a negative heat capacity.  Reading used here: every
// range keeps its printed heat capacity, and its enthalpy is shifted so that
// H is continuous, starting from the first range (whose constant gives the
// formation enthalpy at 298.15 K).  Fe's 1000-1042 K range instead takes a
// heat capacity linear between the neighbouring ranges' values at its ends.
// The shifts are computed once on the host (make_thermo) into a small table
// the kernels read from device memory.
#pragma once
#include "common.h"

namespace demrx {

enum Species { kH2 = 0, kH2O, kN2, kFe2O3, kFe3O4, kFeO, kFe, kNumSpecies };

struct ThermoPiece {
  double lo, hi;  // temperature range (K)
  double a[6];    // a1..a6 of Table C1 (kind 0); heat capacities at lo, hi in a[0], a[1] (kind 1)
  double h_lo;    // molar enthalpy at lo (J/mol), continuous with the range below
  int kind;       // 0: polynomial of Table C1; 1: heat capacity linear in T
};

struct ThermoTab {
  ThermoPiece p[kNumSpecies][4];
  int np[kNumSpecies];
};

// R (a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4): molar form of eq. e3-23
__host__ __device__ inline double poly_cp(const double *a, double T) {
  return kRg * (a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))));
}
// R (a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5), eq. e3-22 without a6
__host__ __device__ inline double poly_h(const double *a, double T) {
  return kRg * T * (a[0] + T * (a[1] / 2.0 + T * (a[2] / 3.0 + T * (a[3] / 4.0 + T * (a[4] / 5.0)))));
}

__host__ __device__ inline const ThermoPiece &piece_of(const ThermoTab &t, int sp, double T) {
  int r = 0;
  while (r < t.np[sp] - 1 && T > t.p[sp][r].hi) r++;
  return t.p[sp][r];
}

// molar heat capacity, J/(mol K)
__host__ __device__ inline double cp_mol(const ThermoTab &t, int sp, double T) {
  const ThermoPiece &q = piece_of(t, sp, T);
  if (q.kind == 1) return q.a[0] + (q.a[1] - q.a[0]) * (T - q.lo) / (q.hi - q.lo);
  return poly_cp(q.a, T);
}

// molar enthalpy (formation enthalpy included), J/mol
__host__ __device__ inline double h_mol(const ThermoTab &t, int sp, double T) {
  const ThermoPiece &q = piece_of(t, sp, T);
  if (q.kind == 1) {
    const double u = T - q.lo;
    return q.h_lo + q.a[0] * u + (q.a[1] - q.a[0]) * u * u / (2.0 * (q.hi - q.lo));
  }
  return q.h_lo + (poly_h(q.a, T) - poly_h(q.a, q.lo));
}

inline ThermoTab make_thermo() {
  // Table C1, molar form; species in Species order
  static const double A[kNumSpecies][4][8] = {
      {{298, 1000, 2.3443, 7.98e-3, -1.95e-5, 2.02e-8, -7.38e-12, -9.179e2},
       {1000, 6000, 2.9328, 8.27e-4, -1.46e-7, 1.54e-11, -6.89e-16, -8.131e2}},
      {{373, 1000, 4.1986, -2.04e-3, 6.52e-6, -5.49e-9, 1.77e-12, -3.03e4},
       {1000, 6000, 2.677, 2.97e-3, -7.74e-7, 9.44e-11, -4.27e-15, -2.989e4}},
      {{298, 1000, 3.531, -1.24e-4, -5.03e-7, 2.44e-9, -1.41e-12, -1.047e3},
       {1000, 6000, 2.9526, 1.40e-3, -4.93e-7, 7.86e-11, -4.61e-15, -9.239e2}},
      {{298, 960, 0.1522, 6.71e-2, -1.13e-4, 9.93e-8, -3.28e-11, -1.013e5},
       {960, 1700, 353.05, -0.9728, 1.05e-3, -4.96e-7, 8.74e-11, -1.96e5}},
      {{298, 850, 4.8445, 4.39e-2, 5.25e-5, -2.21e-7, 1.75e-10, -1.38e5},
       {850, 1870, 88.431, -0.149, 1.26e-4, -4.7e-8, 6.79e-12, -1.621e5}},
      {{298, 1000, 5.3195, 2.21e-3, 1.07e-6, -2.79e-9, 1.33e-12, -3.441e4},
       {1000, 1650, 5.8316, 1.43e-3, -9.32e-8, -6.6e-12, -2.25e-14, -3.457e4}},
      {{298, 1000, 2.4134, -1.58e-3, 2.15e-5, -3.8e-8, 2.20e-11, -774.38},
       {1000, 1042, 4690.8, -9.91, 2.69e-3, 5.54e-6, -3.02e-9, -1.415e6},
       {1042, 1184, 659.68, -1.14, 4.96e-4, 0, 0, -2.52e5},
       {1184, 1665, 61.011, -0.161, 1.68e-4, -7.75e-8, 1.33e-11, -1.65e4}}};
  static const int NP[kNumSpecies] = {2, 2, 2, 2, 2, 2, 4};
  ThermoTab t{};
  for (int s = 0; s < kNumSpecies; s++) {
    t.np[s] = NP[s];
    for (int r = 0; r < NP[s]; r++) {
      ThermoPiece &q = t.p[s][r];
      q.lo = A[s][r][0];
      q.hi = A[s][r][1];
      for (int k = 0; k < 6; k++) q.a[k] = A[s][r][2 + k];
      q.kind = 0;
    }
    // Fe, 1000-1042 K: heat capacity linear between its neighbours' values
    if (s == kFe) {
      ThermoPiece &q = t.p[s][1];
      q.a[0] = poly_cp(t.p[s][0].a, q.lo);
      q.a[1] = poly_cp(t.p[s][2].a, q.hi);
      q.kind = 1;
    }
    // enthalpy at each lower bound: the first range's own value, then continuity
    t.p[s][0].h_lo = poly_h(t.p[s][0].a, t.p[s][0].lo) + kRg * t.p[s][0].a[5];
    for (int r = 1; r < NP[s]; r++) {
      const ThermoPiece &b = t.p[s][r - 1];
      double h_top;
      if (b.kind == 1) {
        const double u = b.hi - b.lo;
        h_top = b.h_lo + 0.5 * (b.a[0] + b.a[1]) * u;
      } else {
        h_top = b.h_lo + (poly_h(b.a, b.hi) - poly_h(b.a, b.lo));
      }
      t.p[s][r].h_lo = h_top;
    }
  }
  return t;
}

// Gas mixture properties from true mole fractions (H2, H2O, N2): mass
// fractions Y_j = x_j M_j / sum x M, conductivity of eqs. e3-58, e3-59 (W/(m K))
// and specific heat of eq. e3-57 (J/(kg K))
__host__ __device__ inline void gas_heat_props(const ThermoTab &t, double T, double x1, double x2, double x3,
                                               double &lambda, double &cp) {
  const double M[3] = {2.016, 18.015, 28.013};
  const double L[3][5] = {{3.07e-3, 8.09e-4, -8.52e-7, 7.2e-10, -2.21e-13},
                          {6.84e-3, 6.25e-6, 1.31e-7, -5.99e-11, 1.12e-14},
                          {2.51e-3, 8.92e-5, -4.00e-8, 1.62e-11, -2.61e-15}};
  const double x[3] = {x1, x2, x3};
  const double Mg = x1 * M[0] + x2 * M[1] + x3 * M[2];
  lambda = 0.0;
  cp = 0.0;
  for (int j = 0; j < 3; j++) {
    const double Y = x[j] * M[j] / Mg;
    const double *c = L[j];
    lambda += Y * (c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4]))));
    cp += Y * cp_mol(t, j, T) / (M[j] * 1e-3);
  }
}

// Gunn's correlation (eq. e3-12) for the Nusselt number
template <typename T>
__host__ __device__ inline T gunn(T eps, T re02, T re07, T pr3) {
  return (T(7) - T(10) * eps + T(5) * eps * eps) * (T(1) + T(0.7) * re02 * pr3) +
         (T(1.33) - T(2.4) * eps + T(1.2) * eps * eps) * re07 * pr3;
}

}  // namespace demrx
