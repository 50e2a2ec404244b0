// Multi-interface unreacted-shrinking-core update of one parcel (Section 2 of
// the paper), shared by the coupled reaction kernel and the kinetic adjoint.
#pragma once
#include "common.h"

namespace demrx {

// Environment of one parcel for one reaction update.
template <typename S>
struct UscmEnv {
  S x;        // H2 fraction of the N2-free gas (Section 2.1)
  S xeq[3];   // equilibrium fractions of R1..R3 (eq. e2-1-3)
  S kk[3];    // K/(1+K) / k_r of R1..R3 (eqs. e2-12, e2-13)
  S rpD[3];   // r_p / D_eff of the Fe3O4, FeO, Fe layers (eqs. e2-14, e2-30)
  S F;        // gas-film resistance (eq. e2-20)
  S cad;      // A_p p / (R T) dt: moles of H2 per unit rate
};

template <typename S>
__device__ __forceinline__ S icbrt(S u);
template <>
__device__ __forceinline__ float icbrt<float>(float u) { return 1.0f / cbrtf(u); }
template <>
__device__ __forceinline__ double icbrt<double>(double u) { return 1.0 / cbrt(u); }

// One explicit update of the moles n = (Fe2O3, Fe3O4, FeO, Fe) per real
// particle: remaining fractions u = 1 - f (eqs. e2-15..e2-17), interface and
// layer resistances outside the innermost active interface (layer l spans
// interfaces l-1 and l; the last reaches the surface), series/parallel
// reduction of the resistance network of Figs. 2 and 4 from the innermost
// active interface outwards and back-substitution of the total flux over the
// active interfaces, then irreversible extents capped by the reactant present
// (Table 1 stoichiometry).  Returns the H2 extents, the network's Q = 1/R and
// S = Phi/R (eq. e4-8) and the number of negative rates clamped.
template <typename S>
__device__ __forceinline__ int uscm_step(S n[4], const UscmEnv<S> &e, S xi[3], S &Qn, S &Sn) {
  const S Nfe = S(2) * n[0] + S(3) * n[1] + n[2] + n[3];
  const S cum[3] = {S(2) * n[0], S(2) * n[0] + S(3) * n[1], S(2) * n[0] + S(3) * n[1] + n[2]};
  bool act[3];
  int inner = 3;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    act[q] = n[q] > S(1e-12) * Nfe && e.x > e.xeq[q];
    if (act[q] && inner == 3) inner = q;
  }
  S r[3] = {S(0), S(0), S(0)};
  Qn = S(0);
  Sn = S(0);
  int clamps = 0;
  if (inner < 3) {
    S ic[3], A[3], Bl[3];
#pragma unroll
    for (int q = 0; q < 3; q++) ic[q] = q >= inner ? icbrt<S>(cum[q] / Nfe) : S(0);
#pragma unroll
    for (int q = 0; q < 3; q++) {
      A[q] = act[q] ? ic[q] * ic[q] * e.kk[q] : S(0);
      const S outer = q < 2 ? ic[q + 1] : S(1);
      Bl[q] = q >= inner ? (ic[q] - outer) * e.rpD[q] : S(0);
    }
    // loops over the three interfaces are unrolled with static indices
    S Rin = inner == 0 ? A[0] : (inner == 1 ? A[1] : A[2]);
    S Phi = inner == 0 ? e.xeq[0] : (inner == 1 ? e.xeq[1] : e.xeq[2]);
#pragma unroll
    for (int q = 1; q < 3; q++) {
      if (q <= inner) continue;
      Rin += Bl[q - 1];
      if (act[q]) {
        const S g1 = S(1) / Rin, g2 = S(1) / A[q];
        Phi = (Phi * g1 + e.xeq[q] * g2) / (g1 + g2);
        Rin = S(1) / (g1 + g2);
      }
    }
    const S Rtot = Rin + Bl[2] + e.F;
    const S flux = (e.x - Phi) / Rtot;
    Qn = S(1) / Rtot;
    Sn = Phi / Rtot;
    S pot = e.x - flux * (e.F + Bl[2]);
    S rest = flux;
#pragma unroll
    for (int q = 2; q >= 0; q--) {
      if (q < inner) continue;
      if (act[q]) {
        r[q] = (pot - e.xeq[q]) / A[q];
        rest -= r[q];
      }
      if (q > inner) pot -= rest * Bl[q - 1];
    }
  }
  const S nu[3] = {S(3), S(1), S(1)};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    if (r[q] < S(0)) {
      r[q] = S(0);
      clamps++;
    }
    xi[q] = fmin(r[q] * e.cad, n[q] / nu[q]);
  }
  // an extent at its cap exhausts the reactant: 3 (n/3) may round above n
  n[0] = n[0] - S(3) * xi[0];
  if (n[0] < S(0)) n[0] = S(0);
  n[1] = n[1] + S(2) * xi[0] - xi[1];
  n[2] = n[2] + S(3) * xi[1] - xi[2];
  n[3] = n[3] + xi[2];
  return clamps;
}

// Overall reduction degree (eqs. e2-18, e2-19) of a state.
template <typename S>
__device__ __forceinline__ double fov_of(const S n[4], int kind) {
  const double a = n[0], b = n[1], c = n[2], d = n[3];
  const double N = 2.0 * a + 3.0 * b + c + d;
  const double fh = 1.0 - 2.0 * a / N, fm = 1.0 - (2.0 * a + 3.0 * b) / N, fw = 1.0 - (2.0 * a + 3.0 * b + c) / N;
  return kind == 1 ? 0.25 * fm + 0.75 * fw : fh / 9.0 + 2.0 * fm / 9.0 + 6.0 * fw / 9.0;
}

// Gas-side quantities shared by the reaction and the adjoint environment.
__device__ __forceinline__ double fuller_h2(double T, double p, double Mj, double Vj) {
  const double s = cbrt(7.07) + cbrt(Vj);
  return 1e-7 * pow(T, 1.75) * sqrt(1.0 / 2.016 + 1.0 / Mj) / ((p / 101325.0) * s * s);
}

// Molecular (Wilke, eq. e2-27) and pore (eqs. e2-28, e2-29) diffusivity of H2.
struct PoreDiff {
  double Dm, D;
};
__device__ __forceinline__ PoreDiff pore_diffusion(double T, double p, double a, double b, double nn, double d_pore_cm) {
  const double D_hw = fuller_h2(T, p, 18.015, 12.7);
  const double D_hn = fuller_h2(T, p, 28.013, 17.9);
  PoreDiff r;
  r.Dm = (b + nn < 1e-12) ? D_hw : (1.0 - a) / (b / D_hw + nn / D_hn);
  const double DK = 0.97 * (0.5 * d_pore_cm) * sqrt(T / 2.016);
  const double ratio = a > 0.0 ? (1.013 / (p * a)) / d_pore_cm : INFINITY;
  r.D = ratio <= 0.01 ? r.Dm : (ratio >= 10.0 ? DK : 1.0 / (1.0 / r.Dm + 1.0 / DK));
  return r;
}

__device__ __forceinline__ void gas_props_h2(double T, double p, double x1, double x2, double x3, double mu_fix,
                                             double &rho, double &mu) {
  // eq. e3-53 and eqs. e3-55/e3-56 with Table C2 (mass-weighted viscosity)
  const double M1 = 2.016, M2 = 18.015, M3 = 28.013;
  const double Mg = x1 * M1 + x2 * M2 + x3 * M3;
  rho = p * (Mg * 1e-3) / (kRg * T);
  if (mu_fix > 0.0) {
    mu = mu_fix;
    return;
  }
  const double m1 = 2.85e-6 + 2.16e-8 * T - 3.78e-12 * T * T;
  const double m2 = -4.44e-6 + 4.52e-8 * T - 3.20e-12 * T * T;
  const double m3 = 7.86e-6 + 3.87e-8 * T - 5.11e-12 * T * T;
  mu = (x1 * M1 * m1 + x2 * M2 * m2 + x3 * M3 * m3) / Mg;
}

// Gas-film resistance d_p / (Sh D_m) with Gunn's Sherwood number (eqs.
// e2-20..e2-24).
__device__ __forceinline__ double film_resistance(double rho, double mu, double Dm, double eps, double dp, double slip) {
  const double Re = rho * eps * dp * slip / mu;
  const double sc3 = cbrt(mu / (rho * Dm));
  const double Sh = (7.0 - 10.0 * eps + 5.0 * eps * eps) * (1.0 + 0.7 * pow(Re, 0.2) * sc3) +
                    (1.33 - 2.4 * eps + 1.2 * eps * eps) * pow(Re, 0.7) * sc3;
  return dp / (Sh * Dm);
}

}  // namespace demrx
