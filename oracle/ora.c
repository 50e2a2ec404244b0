/*
 * Oracle for the particle side of the coarse-grained CFD-DEM reduction model
 * of arxiv 2311.03908.  TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Plain FP64, ascending-id sums, built with -ffp-contract=off so that the
 * contact predicate is evaluated exactly as written.  Loops over independent
 * parcels or pairs may run on several threads (OpenMP); sums never do, so
 * the results do not depend on the thread count.  Function headers cite the paper's equations; readings of passages
 * the paper leaves open are marked "reading:".
 */
#include "ora.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RG 8.314 /* gas constant, Section 2.1 */
#define PI 3.14159265358979323846
#define HCAP 64  /* pair-history entries per parcel (partners with larger id) */

/* molar masses in g/mol: Fe2O3, Fe3O4, FeO, Fe and H2, H2O, N2 */
static const double MS[4] = {159.687, 231.531, 71.844, 55.845};
static const double MG[3] = {2.016, 18.015, 28.013};
/* Fuller diffusion volumes (cm3/mol) of H2, H2O, N2 (Section 2.3) */
static const double VD[3] = {7.07, 12.7, 17.9};
/* viscosity polynomials a1 + a2 T + a3 T^2 of H2, H2O, N2 (Table C2) */
static const double MUC[3][3] = {{2.85e-6, 2.16e-8, -3.78e-12},
                                 {-4.44e-6, 4.52e-8, -3.20e-12},
                                 {7.86e-6, 3.87e-8, -5.11e-12}};
/* K_eq = exp(a/T + b) of R1..R3 (Table 2) */
static const double KEQ[3][2] = {{1433.4, 9.08}, {-7393.9, 7.56}, {-2023.8, 1.24}};

typedef struct {
  int partner;
  double xi[3];
} hist_t;

struct ora_sys {
  ora_params P;
  ora_bed *beds;
  ora_ore *ores;
  int n, n_cells;
  double *pos, *vel, *omg; /* 3 per parcel */
  double *d, *k, *mass, *sp; /* sp: nh, nm, nw, nfe per parcel */
  int *ore, *bed;
  int *hcnt;
  hist_t *hist;
  double *wxi;          /* 6 walls x 3 per parcel */
  unsigned char *won;   /* 6 per parcel */
  double *eps;          /* gas voidage per cell from the last deposit */
  double *Tp;           /* particle temperature (K) */
  double *qrx;          /* k^3 (Q_r + Q_rm) of the last reaction update (W) */
  double *mcp;          /* m C_p,p of the parcel at the last reaction update (J/K) */
};

/* ------------------------------------------------------------ vectors */
static double dot3(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------ dual numbers
 * Forward-mode derivatives with respect to the six kinetic parameters. */
typedef struct {
  double v, d[6];
} dual;

static dual D(double v) {
  dual r;
  r.v = v;
  memset(r.d, 0, sizeof r.d);
  return r;
}
static dual dadd(dual a, dual b) {
  dual r;
  r.v = a.v + b.v;
  for (int i = 0; i < 6; i++) r.d[i] = a.d[i] + b.d[i];
  return r;
}
static dual dsub(dual a, dual b) {
  dual r;
  r.v = a.v - b.v;
  for (int i = 0; i < 6; i++) r.d[i] = a.d[i] - b.d[i];
  return r;
}
static dual dmul(dual a, dual b) {
  dual r;
  r.v = a.v * b.v;
  for (int i = 0; i < 6; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
static dual ddiv(dual a, dual b) {
  dual r;
  r.v = a.v / b.v;
  for (int i = 0; i < 6; i++) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
static dual dscale(dual a, double s) {
  dual r;
  r.v = a.v * s;
  for (int i = 0; i < 6; i++) r.d[i] = a.d[i] * s;
  return r;
}
static dual dpowc(dual a, double e) {
  dual r;
  r.v = pow(a.v, e);
  double f = e * pow(a.v, e - 1.0);
  for (int i = 0; i < 6; i++) r.d[i] = f * a.d[i];
  return r;
}
static dual dinv(dual a) { return ddiv(D(1.0), a); }

/* ------------------------------------------------------------ gas properties */

/* eq. e3-53 (ideal gas) and eqs. e3-55/e3-56 (mass-weighted viscosity, Table C2) */
void ora_gas_props(double T, double p, double xh2, double xh2o, double xn2, double mu_override,
                   double *rho, double *mu) {
  double xs[3] = {xh2, xh2o, xn2};
  double Mg = 0.0; /* g/mol, eq. e2-1-2 written with mole fractions */
  for (int j = 0; j < 3; j++) Mg += xs[j] * MG[j];
  *rho = p * (Mg * 1e-3) / (RG * T);
  if (mu_override > 0.0) {
    *mu = mu_override;
    return;
  }
  double m = 0.0;
  for (int j = 0; j < 3; j++) {
    double Y = xs[j] * MG[j] / Mg; /* mass fraction from eq. e2-1-1 */
    m += Y * (MUC[j][0] + MUC[j][1] * T + MUC[j][2] * T * T);
  }
  *mu = m;
}

/* eq. e2-26: Fuller-Schettler-Giddings binary diffusivity in m2/s (M in g/mol) */
double ora_fuller(double T, double p, int i, int j) {
  double a = pow(VD[i], 1.0 / 3.0) + pow(VD[j], 1.0 / 3.0);
  return 1e-7 * pow(T, 1.75) * sqrt(1.0 / MG[i] + 1.0 / MG[j]) / ((p / 101325.0) * a * a);
}

/* eq. e2-27: Wilke's molecular diffusivity of H2 in the mixture.
 * reading: for a gas with no species but H2 the expression is 0/0; the
 * binary H2-H2O coefficient is used. */
double ora_wilke_h2(double T, double p, double xh2, double xh2o, double xn2) {
  double others = xh2o + xn2;
  if (others < 1e-12) return ora_fuller(T, p, 0, 1);
  double s = xh2o / ora_fuller(T, p, 0, 1) + xn2 / ora_fuller(T, p, 0, 2);
  return (1.0 - xh2) / s;
}

/* eq. e2-28: Knudsen diffusivity of H2, r_a in cm, result in m2/s */
double ora_knudsen_h2(double T, double d_pore_cm) { return 0.97 * (0.5 * d_pore_cm) * sqrt(T / MG[0]); }

/* Section 2.3: regime by lambda/d_a with lambda = 1.013/(p x_H2) cm; eq. e2-29 in the transition */
double ora_pore_diff(double T, double p, double xh2, double xh2o, double xn2, double d_pore_cm) {
  double Dm = ora_wilke_h2(T, p, xh2, xh2o, xn2);
  double DK = ora_knudsen_h2(T, d_pore_cm);
  double ratio = (xh2 > 0.0) ? (1.013 / (p * xh2)) / d_pore_cm : INFINITY;
  if (ratio <= 0.01) return Dm;
  if (ratio >= 10.0) return DK;
  return 1.0 / (1.0 / Dm + 1.0 / DK);
}

/* eqs. e2-31..e2-36: porosity of the Fe2O3 core and of the Fe3O4, FeO, Fe layers */
void ora_layer_porosity(const ora_ore *o, double xi[4]) {
  double q_mh = 2.0 * MS[1] / (3.0 * MS[0]); /* 3Fe2O3 -> 2Fe3O4 */
  double q_wm = 3.0 * MS[2] / MS[1];         /* Fe3O4 -> 3FeO */
  double q_fw = MS[3] / MS[2];               /* FeO -> Fe */
  double re_h = (1.0 - o->xi0) * o->rho_true[0];
  double re_m = re_h * q_mh, re_w = re_m * q_wm, re_f = re_w * q_fw;
  xi[0] = 1.0 - re_h / o->rho_true[0];
  xi[1] = 1.0 - re_m / o->rho_true[1];
  xi[2] = 1.0 - re_w / o->rho_true[2];
  xi[3] = 1.0 - re_f / o->rho_true[3];
}

/* eq. e2-22 (Gunn) */
double ora_sherwood(double eps, double Re, double Sc) {
  double sc3 = pow(Sc, 1.0 / 3.0);
  return (7.0 - 10.0 * eps + 5.0 * eps * eps) * (1.0 + 0.7 * pow(Re, 0.2) * sc3) +
         (1.33 - 2.4 * eps + 1.2 * eps * eps) * pow(Re, 0.7) * sc3;
}

/* eqs. e2-20, e2-21, e2-23, e2-24: film resistance F = d_p / (Sh D_eff,f), with
 * D_eff,f the molecular diffusivity (eq. e2-27) */
double ora_film(double T, double p, double xh2, double xh2o, double xn2, double mu_override,
                double eps, double slip, double dp) {
  double rho, mu;
  ora_gas_props(T, p, xh2, xh2o, xn2, mu_override, &rho, &mu);
  double Df = ora_wilke_h2(T, p, xh2, xh2o, xn2);
  double Re = rho * eps * dp * slip / mu;
  double Sc = mu / (rho * Df);
  return dp / (ora_sherwood(eps, Re, Sc) * Df);
}

/* Table 2 equilibrium constants and eq. e2-1-3 */
double ora_keq(int i, double T) { return exp(KEQ[i][0] / T + KEQ[i][1]); }

/* ------------------------------------------------------------ thermochemistry */

/* Table C1: a1..a6 of eqs. e3-22 / e3-23 per temperature range (K), molar
 * form; species 0 H2, 1 H2O, 2 N2, 3 Fe2O3, 4 Fe3O4, 5 FeO, 6 Fe */
typedef struct {
  double lo, hi, a[6];
} c1_range;
static const int C1N[7] = {2, 2, 2, 2, 2, 2, 4};
static const c1_range C1[7][4] = {
    {{298, 1000, {2.3443, 7.98e-3, -1.95e-5, 2.02e-8, -7.38e-12, -9.179e2}},
     {1000, 6000, {2.9328, 8.27e-4, -1.46e-7, 1.54e-11, -6.89e-16, -8.131e2}}},
    {{373, 1000, {4.1986, -2.04e-3, 6.52e-6, -5.49e-9, 1.77e-12, -3.03e4}},
     {1000, 6000, {2.677, 2.97e-3, -7.74e-7, 9.44e-11, -4.27e-15, -2.989e4}}},
    {{298, 1000, {3.531, -1.24e-4, -5.03e-7, 2.44e-9, -1.41e-12, -1.047e3}},
     {1000, 6000, {2.9526, 1.40e-3, -4.93e-7, 7.86e-11, -4.61e-15, -9.239e2}}},
    {{298, 960, {0.1522, 6.71e-2, -1.13e-4, 9.93e-8, -3.28e-11, -1.013e5}},
     {960, 1700, {353.05, -0.9728, 1.05e-3, -4.96e-7, 8.74e-11, -1.96e5}}},
    {{298, 850, {4.8445, 4.39e-2, 5.25e-5, -2.21e-7, 1.75e-10, -1.38e5}},
     {850, 1870, {88.431, -0.149, 1.26e-4, -4.7e-8, 6.79e-12, -1.621e5}}},
    {{298, 1000, {5.3195, 2.21e-3, 1.07e-6, -2.79e-9, 1.33e-12, -3.441e4}},
     {1000, 1650, {5.8316, 1.43e-3, -9.32e-8, -6.6e-12, -2.25e-14, -3.457e4}}},
    {{298, 1000, {2.4134, -1.58e-3, 2.15e-5, -3.8e-8, 2.20e-11, -774.38}},
     {1000, 1042, {4690.8, -9.91, 2.69e-3, 5.54e-6, -3.02e-9, -1.415e6}},
     {1042, 1184, {659.68, -1.14, 4.96e-4, 0, 0, -2.52e5}},
     {1184, 1665, {61.011, -0.161, 1.68e-4, -7.75e-8, 1.33e-11, -1.65e4}}}};

/* eq. e3-23 times M: R (a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4), J/(mol K) */
static double c1_cp(const double *a, double T) {
  return RG * (a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T);
}
/* eq. e3-22 times M: R (a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5 + a6), J/mol */
static double c1_h(const double *a, double T) {
  double T2 = T * T, T3 = T2 * T, T4 = T3 * T, T5 = T4 * T;
  return RG * (a[0] * T + a[1] * T2 / 2.0 + a[2] * T3 / 3.0 + a[3] * T4 / 4.0 + a[4] * T5 / 5.0 + a[5]);
}
/* reading: Fe's 1000-1042 K coefficients give a negative heat capacity as
 * printed; there C_p is linear between the neighbouring ranges' values at
 * 1000 K and 1042 K */
static double fe_gap_cp(double T) {
  double c0 = c1_cp(C1[6][0].a, 1000.0), c1 = c1_cp(C1[6][2].a, 1042.0);
  return c0 + (c1 - c0) * (T - 1000.0) / 42.0;
}
static double fe_gap_h(double t) { /* integral of fe_gap_cp from 1000 K to t */
  double c0 = c1_cp(C1[6][0].a, 1000.0), c1 = c1_cp(C1[6][2].a, 1042.0);
  return c0 * (t - 1000.0) + (c1 - c0) * (t - 1000.0) * (t - 1000.0) / (2.0 * 42.0);
}

/* molar heat capacity of species sp (eq. e3-23) in the range holding T (the
 * nearest range outside the table) */
double ora_cp_mol(int sp, double T) {
  int r = 0;
  while (r < C1N[sp] - 1 && T > C1[sp][r].hi) r++;
  if (sp == 6 && r == 1) return fe_gap_cp(T);
  return c1_cp(C1[sp][r].a, T);
}

/* molar enthalpy of species sp (eq. e3-22).  reading: the printed
 * coefficients are rounded to about three figures, which leaves steps in H at
 * the range bounds (9 kJ/mol for Fe2O3 at 960 K); H is the first range's
 * eq. e3-22 (its a6 reproduces the formation enthalpy at 298.15 K) continued
 * upward by integrating each later range's heat capacity, i.e. each later
 * range's a6 is the one that makes H continuous at its lower bound */
double ora_h_mol(int sp, double T) {
  const c1_range *R = C1[sp];
  int nr = C1N[sp];
  double H = c1_h(R[0].a, (T <= R[0].hi || nr == 1) ? T : R[0].hi);
  for (int r = 1; r < nr && T > R[r].lo; r++) {
    double t1 = (T <= R[r].hi || r == nr - 1) ? T : R[r].hi;
    if (sp == 6 && r == 1)
      H += fe_gap_h(t1);
    else
      H += c1_h(R[r].a, t1) - c1_h(R[r].a, R[r].lo);
  }
  return H;
}

/* Table C3: thermal conductivity a1 + a2 T + ... + a5 T^4 (W/(m K)) of H2, H2O, N2 */
static const double LAMC[3][5] = {{3.07e-3, 8.09e-4, -8.52e-7, 7.2e-10, -2.21e-13},
                                  {6.84e-3, 6.25e-6, 1.31e-7, -5.99e-11, 1.12e-14},
                                  {2.51e-3, 8.92e-5, -4.00e-8, 1.62e-11, -2.61e-15}};

/* eqs. e3-58, e3-59: mass-weighted thermal conductivity of the gas */
double ora_lambda_g(double T, double xh2, double xh2o, double xn2) {
  double xs[3] = {xh2, xh2o, xn2}, Mg = 0.0, l = 0.0;
  for (int j = 0; j < 3; j++) Mg += xs[j] * MG[j];
  for (int j = 0; j < 3; j++) {
    const double *a = LAMC[j];
    l += xs[j] * MG[j] / Mg * (a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T);
  }
  return l;
}

/* eqs. e3-23, e3-57: mass-weighted specific heat of the gas, J/(kg K) */
double ora_cp_g(double T, double xh2, double xh2o, double xn2) {
  double xs[3] = {xh2, xh2o, xn2}, Mg = 0.0, c = 0.0;
  for (int j = 0; j < 3; j++) Mg += xs[j] * MG[j];
  for (int j = 0; j < 3; j++) c += xs[j] * MG[j] / Mg * ora_cp_mol(j, T) / (MG[j] * 1e-3);
  return c;
}

/* eq. e3-12: Gunn's correlation, the form of eq. e2-22 with Pr in place of Sc */
double ora_nusselt(double eps, double Re, double Pr) { return ora_sherwood(eps, Re, Pr); }

/* eq. e3-5-1 divided by eps_p = 1 - eps_g, so that F_d = (beta/eps_p) V (u_g - v)
 * (eq. e3-5) stays finite in a cell of unit voidage.  reading: Gidaspow's
 * inertial Ergun term carries eps_p (printed: eps_g, selectable); C_D is
 * Schiller-Naumann with the eps-weighted Re of eq. e2-23; eps = 0.8 takes the
 * Wen-Yu branch. */
double ora_beta_over_epsp(double eps, double rho, double mu, double slip, double dp, int printed) {
  double ep = 1.0 - eps;
  if (eps < 0.8) {
    double inertial = printed ? 1.75 * eps * rho * slip / (dp * ep) : 1.75 * rho * slip / dp;
    return 150.0 * ep * mu / (eps * dp * dp) + inertial;
  }
  double Re = rho * eps * dp * slip / mu;
  double cdre = (Re < 1000.0) ? 24.0 * (1.0 + 0.15 * pow(Re, 0.687)) : 0.44 * Re;
  return 0.75 * cdre * mu * pow(eps, -2.65) / (dp * dp);
}

/* Gidaspow-Ganser drag of non-spherical particles (eqs. e3-5-2..e3-5-5),
 * divided by eps_p like ora_beta_over_epsp, for sphericity psi in (0, 1] and
 * equivalent-area bed diameter Dbed.  The Ergun branch divides the viscous
 * term by psi^2 and the inertial one by psi (same eps reading as above); the
 * Wen-Yu branch takes Ganser's single-particle C_D with
 *   K1 = 1 / (1/3 + 2/3 psi^-1/2) - 2.25 dp / Dbed,
 *   K2 = 10^(1.8148 (-log10 psi)^0.5743),
 *   C_D Re = 24/K1 (1 + 0.1118 (Re K1 K2)^0.6567) + 0.4305 K2 Re / (1 + 3305 / (Re K1 K2)). */
double ora_beta_ganser_over_epsp(double eps, double rho, double mu, double slip, double dp, double psi,
                                 double Dbed, int printed) {
  double ep = 1.0 - eps;
  if (eps < 0.8) {
    double inertial = printed ? 1.75 * eps * rho * slip / (dp * psi * ep) : 1.75 * rho * slip / (dp * psi);
    return 150.0 * ep * mu / (eps * dp * dp * psi * psi) + inertial;
  }
  double Re = rho * eps * dp * slip / mu;
  double K1 = 1.0 / (1.0 / 3.0 + 2.0 / 3.0 / sqrt(psi)) - 2.25 * dp / Dbed;
  double K2 = pow(10.0, 1.8148 * pow(-log10(psi), 0.5743));
  double x = Re * K1 * K2;
  double cdre = 24.0 / K1 * (1.0 + 0.1118 * pow(x, 0.6567)) + (x > 0.0 ? 0.4305 * K2 * Re / (1.0 + 3305.0 / x) : 0.0);
  return 0.75 * cdre * mu * pow(eps, -2.65) / (dp * dp);
}

/* reading: the "equivalent-area bed diameter" of eq. e3-5-4 is that of the
 * bed's horizontal cross-section: 2R for a cylinder, sqrt(4 A / pi) for a box */
static double bed_diameter(const ora_bed *b) {
  if (b->wall_kind == 1) return 2.0 * b->R;
  return sqrt(4.0 * (b->hi[0] - b->lo[0]) * (b->hi[1] - b->lo[1]) / PI);
}

/* drag coefficient of parcel i (spheres: eq. e3-5-1; psi in (0, 1]: eq. e3-5-2) */
static double beta_of(const ora_sys *s, int i, double eps, double rho, double mu, double slip) {
  const ora_ore *o = &s->ores[s->ore[i]];
  double dp = s->d[i] / s->k[i]; /* reading: drag uses the real-particle diameter */
  if (o->psi > 0.0)
    return ora_beta_ganser_over_epsp(eps, rho, mu, slip, dp, o->psi, bed_diameter(&s->beds[s->bed[i]]),
                                     s->P.ergun_printed);
  return ora_beta_over_epsp(eps, rho, mu, slip, dp, s->P.ergun_printed);
}

/* eq. e3-45; reading: a non-positive radicand means a perfectly inelastic parcel */
double ora_e_cgp(double e_p, double k) {
  double a = 1.0 + k * (e_p * e_p - 1.0);
  return a > 0.0 ? sqrt(a) : 0.0;
}

/* eq. e3-44; e -> 0 gives critical damping */
double ora_zeta(double e) {
  if (e <= 0.0) return 1.0;
  double l = log(e);
  return -l / sqrt(PI * PI + l * l);
}

/* ------------------------------------------------------------ parcel / cell helpers */
static int cell_of(const ora_sys *s, int i) {
  const ora_bed *b = &s->beds[s->bed[i]];
  int c[3];
  for (int a = 0; a < 3; a++) {
    double f = floor((s->pos[3 * i + a] - b->origin[a]) / b->h);
    if (f < 0) f = 0;
    if (f > b->n[a] - 1) f = b->n[a] - 1;
    c[a] = (int)f;
  }
  return b->cell_off + c[0] + b->n[0] * (c[1] + b->n[1] * c[2]);
}
static double radius(const ora_sys *s, int i) { return 0.5 * s->d[i]; }
static double volume(const ora_sys *s, int i) { return PI / 6.0 * s->d[i] * s->d[i] * s->d[i]; }
static double inertia(const ora_sys *s, int i) {
  double r = radius(s, i);
  return 0.4 * s->mass[i] * r * r; /* eq. e3-7 */
}
/* eq. e3-4 with eq. e3-52: parcel mass = k^3 x real-particle mass */
static double parcel_mass(const ora_sys *s, int i) {
  const double *n = &s->sp[4 * i];
  double mp = (n[0] * MS[0] + n[1] * MS[1] + n[2] * MS[2] + n[3] * MS[3]) * 1e-3;
  double k = s->k[i];
  return k * k * k * mp;
}

/* eq. e3-9 times the parcel mass: m C_p,p = k^3 sum_z n_z C_p,z(T_p) (J/K) */
static double parcel_mcp(const ora_sys *s, int i) {
  const double *n = &s->sp[4 * i];
  double c = 0.0;
  for (int z = 0; z < 4; z++) c += n[z] * ora_cp_mol(3 + z, s->Tp[i]);
  double k = s->k[i];
  return k * k * k * c;
}

/* eqs. e3-10, e3-11, e3-12, e3-13 and e3-41: k^3 h_p A_p of parcel i (W/K)
 * from the gas of its cell, the voidage of the last deposit and its slip;
 * Re_p as in eq. e2-23, on the real-particle diameter */
static double parcel_hA(const ora_sys *s, const ora_gas *g, int i) {
  int c = cell_of(s, i);
  const ora_bed *B = &s->beds[s->bed[i]];
  double T = g->T[c], rho, mu;
  ora_gas_props(T, g->p[c], g->xH2[c], g->xH2O[c], g->xN2[c], B->mu_override, &rho, &mu);
  double lam = ora_lambda_g(T, g->xH2[c], g->xH2O[c], g->xN2[c]);
  double cp = ora_cp_g(T, g->xH2[c], g->xH2O[c], g->xN2[c]);
  double sl[3] = {g->ug[c] - s->vel[3 * i], g->vg[c] - s->vel[3 * i + 1], g->wg[c] - s->vel[3 * i + 2]};
  double slip = sqrt((sl[0] * sl[0] + sl[1] * sl[1]) + sl[2] * sl[2]);
  double k = s->k[i], dp = s->d[i] / k;
  double Re = rho * s->eps[c] * dp * slip / mu;
  double Nu = ora_nusselt(s->eps[c], Re, cp * mu / lam);
  double h = Nu * lam / dp;
  return k * k * k * h * PI * dp * dp;
}

/* ------------------------------------------------------------ construction */
static void deposit(ora_sys *s, const ora_gas *g, double *np_, double *sumK, double *sumKu,
                    double *sumKv, double *sumKw, double *sumKs);

ora_sys *ora_new(const ora_params *P, const ora_bed *beds, const ora_ore *ores, int n,
                 const double *x, const double *y, const double *z, const double *vx,
                 const double *vy, const double *vz, const double *wx, const double *wy,
                 const double *wz, const double *d, const double *k, const int *ore,
                 const int *bed, const double *nh, const double *nm, const double *nw,
                 const double *nfe) {
  ora_sys *s = (ora_sys *)calloc(1, sizeof *s);
  s->P = *P;
  s->beds = (ora_bed *)malloc(sizeof(ora_bed) * P->n_beds);
  memcpy(s->beds, beds, sizeof(ora_bed) * P->n_beds);
  s->ores = (ora_ore *)malloc(sizeof(ora_ore) * P->n_ores);
  memcpy(s->ores, ores, sizeof(ora_ore) * P->n_ores);
  s->n = n;
  int nc = 0;
  for (int b = 0; b < P->n_beds; b++) {
    int e = beds[b].cell_off + beds[b].n[0] * beds[b].n[1] * beds[b].n[2];
    if (e > nc) nc = e;
  }
  s->n_cells = nc;
  s->pos = (double *)malloc(sizeof(double) * 3 * n);
  s->vel = (double *)malloc(sizeof(double) * 3 * n);
  s->omg = (double *)malloc(sizeof(double) * 3 * n);
  s->d = (double *)malloc(sizeof(double) * n);
  s->k = (double *)malloc(sizeof(double) * n);
  s->mass = (double *)malloc(sizeof(double) * n);
  s->sp = (double *)malloc(sizeof(double) * 4 * n);
  s->ore = (int *)malloc(sizeof(int) * n);
  s->bed = (int *)malloc(sizeof(int) * n);
  s->hcnt = (int *)calloc(n, sizeof(int));
  s->hist = (hist_t *)malloc(sizeof(hist_t) * (size_t)HCAP * n);
  s->wxi = (double *)calloc((size_t)18 * n, sizeof(double));
  s->won = (unsigned char *)calloc((size_t)6 * n, 1);
  s->eps = (double *)malloc(sizeof(double) * (nc > 0 ? nc : 1));
  s->Tp = (double *)calloc(n > 0 ? n : 1, sizeof(double));
  s->qrx = (double *)calloc(n > 0 ? n : 1, sizeof(double));
  s->mcp = (double *)calloc(n > 0 ? n : 1, sizeof(double));
  for (int i = 0; i < n; i++) {
    s->pos[3 * i] = x[i];
    s->pos[3 * i + 1] = y[i];
    s->pos[3 * i + 2] = z[i];
    s->vel[3 * i] = vx[i];
    s->vel[3 * i + 1] = vy[i];
    s->vel[3 * i + 2] = vz[i];
    s->omg[3 * i] = wx[i];
    s->omg[3 * i + 1] = wy[i];
    s->omg[3 * i + 2] = wz[i];
    s->d[i] = d[i];
    s->k[i] = k[i];
    s->ore[i] = ore[i];
    s->bed[i] = bed[i];
    s->sp[4 * i] = nh[i];
    s->sp[4 * i + 1] = nm[i];
    s->sp[4 * i + 2] = nw[i];
    s->sp[4 * i + 3] = nfe[i];
    s->mass[i] = parcel_mass(s, i);
  }
  deposit(s, NULL, NULL, NULL, NULL, NULL, NULL, NULL); /* voidage at t = 0 */
  return s;
}

void ora_free(ora_sys *s) {
  if (!s) return;
  free(s->beds); free(s->ores); free(s->pos); free(s->vel); free(s->omg); free(s->d);
  free(s->k); free(s->mass); free(s->sp); free(s->ore); free(s->bed); free(s->hcnt);
  free(s->hist); free(s->wxi); free(s->won); free(s->eps); free(s->Tp); free(s->qrx); free(s->mcp);
  free(s);
}

int ora_n_cells(const ora_sys *s) { return s->n_cells; }

/* Threads of the parallel loops (builds with OpenMP; 1 otherwise).  Every
 * result is the same for any thread count: loops run over independent
 * parcels or pairs, and every sum runs in ascending id order. */
void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------ contact detection */
static int in_contact(const ora_sys *s, int a, int b) {
  double dx = s->pos[3 * b] - s->pos[3 * a];
  double dy = s->pos[3 * b + 1] - s->pos[3 * a + 1];
  double dz = s->pos[3 * b + 2] - s->pos[3 * a + 2];
  double sr = radius(s, a) + radius(s, b);
  return ((dx * dx + dy * dy) + dz * dz) < sr * sr;
}

static int cmp_pair(const void *p, const void *q) {
  const int *a = (const int *)p, *b = (const int *)q;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* Bins of one bed: edge >= the bed's largest diameter, members contiguous in
 * bin order, with bin-ordered copies of their positions and radii. */
typedef struct {
  int nc[3];
  double lo[3], cs[3];
  long *first;   /* bin b holds sorted[first[b] .. first[b+1]) */
  int *sorted;   /* parcel ids in bin order */
  double *q;     /* x, y, z, r of sorted[t] */
} bins_t;

/* All contacting pairs a < b (same bed), sorted by (a, b).  *out is
 * malloc'ed.  The cell list collects each parcel's partners on its own (in
 * parallel when built with OpenMP: up to HCAP per parcel, each short list
 * sorted, then concatenated in id order), so the list does not depend on the
 * thread count. */
static long find_pairs(ora_sys *s, int brute, int **out) {
  long cap = 1024, cnt = 0;
  int *pr = NULL;
  if (brute) {
    pr = (int *)malloc(sizeof(int) * 2 * cap);
    for (int a = 0; a < s->n; a++)
      for (int b = a + 1; b < s->n; b++)
        if (s->bed[a] == s->bed[b] && in_contact(s, a, b)) {
          if (cnt == cap) { cap *= 2; pr = (int *)realloc(pr, sizeof(int) * 2 * cap); }
          pr[2 * cnt] = a; pr[2 * cnt + 1] = b; cnt++;
        }
    qsort(pr, cnt, 2 * sizeof(int), cmp_pair);
    *out = pr;
    return cnt;
  }
  int n = s->n, nb_ = s->P.n_beds;
  bins_t *bins = (bins_t *)calloc(nb_ > 0 ? nb_ : 1, sizeof(bins_t));
  /* bins of edge >= the largest diameter of each bed */
  for (int bd = 0; bd < nb_; bd++) {
    const ora_bed *Bd = &s->beds[bd];
    bins_t *B = &bins[bd];
    double hc = 0.0;
    int nb = 0;
    for (int i = 0; i < n; i++)
      if (s->bed[i] == bd) {
        nb++;
        if (s->d[i] > hc) hc = s->d[i];
      }
    if (nb == 0) continue;
    for (int a = 0; a < 3; a++) {
      B->nc[a] = (int)floor((Bd->hi[a] - Bd->lo[a]) / hc);
      if (B->nc[a] < 1) B->nc[a] = 1;
      B->lo[a] = Bd->lo[a];
      B->cs[a] = (Bd->hi[a] - Bd->lo[a]) / B->nc[a];
    }
    long ncell = (long)B->nc[0] * B->nc[1] * B->nc[2];
    B->first = (long *)calloc(ncell + 1, sizeof(long));
    long *cellof = (long *)malloc(sizeof(long) * nb);
    int *member = (int *)malloc(sizeof(int) * nb);
    int m = 0;
    for (int i = 0; i < n; i++) {
      if (s->bed[i] != bd) continue;
      int c3[3];
      for (int a = 0; a < 3; a++) {
        double f = floor((s->pos[3 * i + a] - B->lo[a]) / B->cs[a]);
        if (f < 0) f = 0;
        if (f > B->nc[a] - 1) f = B->nc[a] - 1;
        c3[a] = (int)f;
      }
      cellof[m] = c3[0] + (long)B->nc[0] * (c3[1] + (long)B->nc[1] * c3[2]);
      B->first[cellof[m] + 1]++;
      member[m++] = i;
    }
    for (long c = 0; c < ncell; c++) B->first[c + 1] += B->first[c];
    long *fill = (long *)malloc(sizeof(long) * ncell);
    memcpy(fill, B->first, sizeof(long) * ncell);
    B->sorted = (int *)malloc(sizeof(int) * nb);
    for (int t = 0; t < nb; t++) B->sorted[fill[cellof[t]]++] = member[t];
    B->q = (double *)malloc(sizeof(double) * 4 * nb);
    for (int t = 0; t < nb; t++) {
      int i = B->sorted[t];
      B->q[4 * t] = s->pos[3 * i];
      B->q[4 * t + 1] = s->pos[3 * i + 1];
      B->q[4 * t + 2] = s->pos[3 * i + 2];
      B->q[4 * t + 3] = radius(s, i);
    }
    free(cellof); free(member); free(fill);
  }
  long *off = (long *)malloc(sizeof(long) * (n + 1));
  int *part = (int *)malloc(sizeof(int) * (size_t)HCAP * (n > 0 ? n : 1));
  int over = 0;
  off[0] = 0;
  for (int a = 0; a < n; a++) off[a + 1] = 0;
  /* bin by bin: the members of a bin against those of its 27 neighbours,
   * each member a keeping its partners b > a (a bin's members are written
   * by one thread only) */
  for (int bd = 0; bd < nb_; bd++) {
    const bins_t *B = &bins[bd];
    if (!B->first) continue;
    long ncell = (long)B->nc[0] * B->nc[1] * B->nc[2];
#pragma omp parallel for schedule(dynamic, 64) reduction(| : over)
    for (long c = 0; c < ncell; c++) {
      if (B->first[c] == B->first[c + 1]) continue;
      int cx = (int)(c % B->nc[0]), cy = (int)((c / B->nc[0]) % B->nc[1]), cz = (int)(c / ((long)B->nc[0] * B->nc[1]));
      for (long ta = B->first[c]; ta < B->first[c + 1]; ta++) off[B->sorted[ta] + 1] = 0;
      for (int oz = -1; oz <= 1; oz++)
        for (int oy = -1; oy <= 1; oy++)
          for (int ox = -1; ox <= 1; ox++) {
            int x2 = cx + ox, y2 = cy + oy, z2 = cz + oz;
            if (x2 < 0 || y2 < 0 || z2 < 0 || x2 >= B->nc[0] || y2 >= B->nc[1] || z2 >= B->nc[2]) continue;
            long c2 = x2 + (long)B->nc[0] * (y2 + (long)B->nc[1] * z2);
            for (long ta = B->first[c]; ta < B->first[c + 1]; ta++) {
              int a = B->sorted[ta];
              long m = off[a + 1];
              for (long tb = B->first[c2]; tb < B->first[c2 + 1]; tb++) {
                int b = B->sorted[tb];
                if (b <= a) continue;
                /* the contact predicate of in_contact(), on the bin-ordered copies */
                double dx = B->q[4 * tb] - B->q[4 * ta];
                double dy = B->q[4 * tb + 1] - B->q[4 * ta + 1];
                double dz = B->q[4 * tb + 2] - B->q[4 * ta + 2];
                double sr = B->q[4 * ta + 3] + B->q[4 * tb + 3];
                if (!(((dx * dx + dy * dy) + dz * dz) < sr * sr)) continue;
                if (m < HCAP) part[(size_t)HCAP * a + m] = b;
                m++;
              }
              off[a + 1] = m;
            }
          }
      for (long ta = B->first[c]; ta < B->first[c + 1]; ta++) {
        int a = B->sorted[ta];
        long m = off[a + 1];
        if (m > HCAP) over = 1;
        int *seg = part + (size_t)HCAP * a;
        for (long u = 1; u < m && u < HCAP; u++) /* insertion sort of a's few partners */
          for (long v = u; v > 0 && seg[v - 1] > seg[v]; v--) {
            int tmp = seg[v]; seg[v] = seg[v - 1]; seg[v - 1] = tmp;
          }
      }
    }
  }
  if (over) abort(); /* more partners than the history holds */
  for (int a = 0; a < n; a++) off[a + 1] += off[a];
  cnt = off[n];
  pr = (int *)malloc(sizeof(int) * 2 * (cnt > 0 ? cnt : 1));
#pragma omp parallel for schedule(static)
  for (int a = 0; a < n; a++)
    for (long u = 0; u < off[a + 1] - off[a]; u++) {
      pr[2 * (off[a] + u)] = a;
      pr[2 * (off[a] + u) + 1] = part[(size_t)HCAP * a + u];
    }
  free(part); free(off);
  for (int bd = 0; bd < nb_; bd++) {
    free(bins[bd].first); free(bins[bd].sorted); free(bins[bd].q);
  }
  free(bins);
  *out = pr;
  return cnt;
}

long ora_pairs(ora_sys *s, int brute, int *ij, long cap) {
  int *pr;
  long cnt = find_pairs(s, brute, &pr);
  for (long q = 0; q < cnt && q < cap; q++) { ij[2 * q] = pr[2 * q]; ij[2 * q + 1] = pr[2 * q + 1]; }
  free(pr);
  return cnt;
}

/* ------------------------------------------------------------ contact law
 * reading (the paper defers the contact model to another work): linear
 * spring-dashpot in the normal direction with damping ratio zeta from the
 * coarse-grained restitution (eqs. e3-44, e3-45), no tensile clamp; Cundall
 * tangential spring k_t with Coulomb cap mu_s |F_n|; the spring is projected
 * onto the current tangent plane before the increment v_t dt.  F (on the
 * first body), the tangential part Ft, the new history and |F_n| are returned. */
static void contact_law(const ora_params *P, double mstar, double zeta, double delta,
                        const double n[3], const double vrel[3], const double xi_in[3],
                        double F[3], double Ft[3], double xi_out[3], double *fn_abs, double scale[2]) {
  double gn = 2.0 * zeta * sqrt(mstar * P->kn);
  double vn = dot3(vrel, n);
  double fn = -(P->kn * delta + gn * vn);
  double vt[3], xi[3];
  for (int a = 0; a < 3; a++) vt[a] = vrel[a] - vn * n[a];
  double xn = dot3(xi_in, n);
  for (int a = 0; a < 3; a++) xi[a] = (xi_in[a] - xn * n[a]) + vt[a] * P->dt;
  double kt = P->kt_over_kn * P->kn, gt = P->gt_over_gn * gn;
  for (int a = 0; a < 3; a++) Ft[a] = -kt * xi[a] - gt * vt[a];
  double ftm = norm3(Ft), cap = P->mu_s * fabs(fn);
  if (ftm > cap) {
    for (int a = 0; a < 3; a++) {
      Ft[a] = cap * Ft[a] / ftm;
      xi[a] = -(Ft[a] + gt * vt[a]) / kt;
    }
  }
  for (int a = 0; a < 3; a++) {
    F[a] = fn * n[a] + Ft[a];
    xi_out[a] = xi[a];
  }
  *fn_abs = fabs(fn);
  if (scale) {
    /* magnitudes of the products the normal and the tangential force are
     * built from (|v_n|, |v_t| <= |v_rel|): the spring and the dashpot cancel
     * as a contact ends, so |F| alone understates them */
    double vr = norm3(vrel);
    scale[0] = P->kn * fabs(delta) + gn * vr;
    scale[1] = kt * (norm3(xi_in) + vr * P->dt) + gt * vr;
  }
}

static void rolling(const ora_sys *s, int i, double fn_abs, double T[3]) {
  if (s->P.mu_r <= 0.0) return;
  double w = norm3(&s->omg[3 * i]);
  if (w <= 0.0) return;
  for (int a = 0; a < 3; a++) T[a] -= s->P.mu_r * fn_abs * s->omg[3 * i + a] / w;
}

static int n_walls(const ora_bed *b) { return b->wall_kind == 0 ? 6 : 3; }

/* signed distance from the wall surface into the domain and the unit vector
 * from the parcel centre towards the wall */
static double wall_geom(const ora_bed *b, int w, const double x[3], double nvec[3]) {
  nvec[0] = nvec[1] = nvec[2] = 0.0;
  if (b->wall_kind == 0) {
    int ax = w / 2;
    if (w % 2 == 0) { nvec[ax] = -1.0; return x[ax] - b->lo[ax]; }
    nvec[ax] = 1.0;
    return b->hi[ax] - x[ax];
  }
  if (w == 0) {
    double cx = 0.5 * (b->lo[0] + b->hi[0]), cy = 0.5 * (b->lo[1] + b->hi[1]);
    double rx = x[0] - cx, ry = x[1] - cy;
    double rho = sqrt(rx * rx + ry * ry);
    if (rho <= 0.0) return b->R;
    nvec[0] = rx / rho;
    nvec[1] = ry / rho;
    return b->R - rho;
  }
  if (w == 1) { nvec[2] = -1.0; return x[2] - b->lo[2]; }
  nvec[2] = 1.0;
  return b->hi[2] - x[2];
}

/* eq. e3-5 with e3-5-1 plus body forces of eq. e3-3 (gravity, -V grad p);
 * with scale, the magnitudes of the three terms are added to *scale */
static void gas_force(const ora_sys *s, const ora_gas *g, int i, double F[3], double *scale) {
  double m = s->mass[i];
  for (int a = 0; a < 3; a++) F[a] += m * s->P.g[a];
  if (scale) *scale += m * norm3(s->P.g);
  if (!s->P.drag_on) return;
  int c = cell_of(s, i);
  const ora_bed *B = &s->beds[s->bed[i]];
  double V = volume(s, i);
  F[0] -= V * g->dpdx[c];
  F[1] -= V * g->dpdy[c];
  F[2] -= V * g->dpdz[c];
  double rho, mu;
  ora_gas_props(g->T[c], g->p[c], g->xH2[c], g->xH2O[c], g->xN2[c], B->mu_override, &rho, &mu);
  double sl[3] = {g->ug[c] - s->vel[3 * i], g->vg[c] - s->vel[3 * i + 1], g->wg[c] - s->vel[3 * i + 2]};
  double be = beta_of(s, i, s->eps[c], rho, mu, norm3(sl));
  for (int a = 0; a < 3; a++) F[a] += be * V * sl[a];
  if (scale) {
    double gp[3] = {g->dpdx[c], g->dpdy[c], g->dpdz[c]};
    *scale += V * norm3(gp) + be * V * norm3(sl);
  }
}

static const double *hist_lookup(const ora_sys *s, int a, int b) {
  for (int q = 0; q < s->hcnt[a]; q++)
    if (s->hist[(size_t)a * HCAP + q].partner == b) return s->hist[(size_t)a * HCAP + q].xi;
  return NULL;
}

/* One contact pair's terms in canonical orientation (a < b): force on a,
 * the cross product n x F_t (torques r_a n x F_t on a and r_b n x F_t on b),
 * |F_n|, the new tangential history and the force-term scales. */
typedef struct {
  double Fa[3], tq[3], fnabs, xi[3], sc[2];
} pair_t;

static void pair_terms(const ora_sys *s, int a, int b, pair_t *o) {
  static const double zero3[3] = {0, 0, 0};
  double dx[3], nv[3];
  for (int c = 0; c < 3; c++) dx[c] = s->pos[3 * b + c] - s->pos[3 * a + c];
  double dist = sqrt((dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]);
  double ra = radius(s, a), rb = radius(s, b);
  for (int c = 0; c < 3; c++) nv[c] = dx[c] / dist;
  double delta = (ra + rb) - dist;
  double ma = s->mass[a], mb = s->mass[b];
  double mstar = ma * mb / (ma + mb);
  double kk = s->k[a] > s->k[b] ? s->k[a] : s->k[b];
  double zeta = ora_zeta(ora_e_cgp(s->P.e_p, kk));
  double wsum[3], cr[3], vrel[3];
  for (int c = 0; c < 3; c++) wsum[c] = ra * s->omg[3 * a + c] + rb * s->omg[3 * b + c];
  cross3(wsum, nv, cr);
  for (int c = 0; c < 3; c++) vrel[c] = s->vel[3 * a + c] - s->vel[3 * b + c] + cr[c];
  const double *xo = hist_lookup(s, a, b);
  double Ft[3];
  contact_law(&s->P, mstar, zeta, delta, nv, vrel, xo ? xo : zero3, o->Fa, Ft, o->xi, &o->fnabs, o->sc);
  cross3(nv, Ft, o->tq);
}

/* Forces and torques of one DEM step from the step-start state; with commit,
 * the tangential histories are replaced by the new ones.  Fs and Ts (may be
 * NULL) receive per parcel the sum of the magnitudes of the products that
 * make up F and T (per contact: k_n |delta| + gamma_n |v_rel| normal, and
 * k_t (|xi| + |v_rel| dt) + gamma_t |v_rel| tangential; gravity, pressure
 * gradient and drag): the scale of the rounding error of F and T when they
 * are evaluated in a lower precision.
 *
 * Each pair is evaluated once (+F on a, -F on b); every parcel then adds its
 * pairs in ascending partner id, then its walls, then the gas force, so the
 * sums are the same for any thread count. */
static void compute_forces(ora_sys *s, const ora_gas *g, double *F, double *T, double *Fs, double *Ts,
                           int commit) {
  int n = s->n;
  static const double zero3[3] = {0, 0, 0};
  int *pr;
  long np_ = find_pairs(s, 0, &pr);
  pair_t *pt = (pair_t *)malloc(sizeof(pair_t) * (np_ > 0 ? np_ : 1));
#pragma omp parallel for schedule(static)
  for (long q = 0; q < np_; q++) pair_terms(s, pr[2 * q], pr[2 * q + 1], &pt[q]);
  /* pairs of each parcel: as the first member (pair list sorted by (a, b):
   * one run per a) and as the second (in ascending a) */
  long *first = (long *)calloc((size_t)n + 1, sizeof(long));
  long *sec_off = (long *)calloc((size_t)n + 1, sizeof(long));
  for (long q = 0; q < np_; q++) {
    first[pr[2 * q] + 1]++;
    sec_off[pr[2 * q + 1] + 1]++;
  }
  for (int i = 0; i < n; i++) {
    first[i + 1] += first[i];
    sec_off[i + 1] += sec_off[i];
  }
  long *sec = (long *)malloc(sizeof(long) * (np_ > 0 ? np_ : 1));
  long *fill = (long *)malloc(sizeof(long) * ((size_t)n + 1));
  memcpy(fill, sec_off, sizeof(long) * ((size_t)n + 1));
  for (long q = 0; q < np_; q++) sec[fill[pr[2 * q + 1]]++] = q;
  free(fill);
  int *ncnt = (int *)calloc(n, sizeof(int));
  hist_t *nh = (hist_t *)malloc(sizeof(hist_t) * (size_t)HCAP * n);
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : overflow)
  for (int i = 0; i < n; i++) {
    double Fi[3] = {0, 0, 0}, Ti[3] = {0, 0, 0}, fs = 0.0, ts = 0.0;
    double r = radius(s, i);
    int roll_on = s->P.mu_r > 0.0;
    /* partners with a smaller id (i second in their pair), then larger */
    for (long u = sec_off[i]; u < sec_off[i + 1]; u++) {
      const pair_t *p = &pt[sec[u]];
      for (int c = 0; c < 3; c++) {
        Fi[c] -= p->Fa[c];
        Ti[c] += r * p->tq[c];
      }
      rolling(s, i, p->fnabs, Ti);
      fs += p->sc[0] + p->sc[1];
      ts += r * p->sc[1] + (roll_on ? s->P.mu_r * p->sc[0] : 0.0);
    }
    for (long q = first[i]; q < first[i + 1]; q++) {
      const pair_t *p = &pt[q];
      for (int c = 0; c < 3; c++) {
        Fi[c] += p->Fa[c];
        Ti[c] += r * p->tq[c];
      }
      rolling(s, i, p->fnabs, Ti);
      fs += p->sc[0] + p->sc[1];
      ts += r * p->sc[1] + (roll_on ? s->P.mu_r * p->sc[0] : 0.0);
      if (ncnt[i] >= HCAP) {
        overflow = 1;
        continue;
      }
      nh[(size_t)i * HCAP + ncnt[i]].partner = pr[2 * q + 1];
      memcpy(nh[(size_t)i * HCAP + ncnt[i]].xi, p->xi, sizeof p->xi);
      ncnt[i]++;
    }
    /* walls: same law with m* = m, infinite radius and zero velocity */
    const ora_bed *B = &s->beds[s->bed[i]];
    for (int w = 0; w < n_walls(B); w++) {
      double nv[3];
      double phi = wall_geom(B, w, &s->pos[3 * i], nv);
      double delta = r - phi;
      if (!(delta > 0.0)) {
        if (commit) s->won[6 * i + w] = 0;
        continue;
      }
      double zeta = ora_zeta(ora_e_cgp(s->P.e_p, s->k[i]));
      double wr[3], cr[3], vrel[3];
      for (int c = 0; c < 3; c++) wr[c] = r * s->omg[3 * i + c];
      cross3(wr, nv, cr);
      for (int c = 0; c < 3; c++) vrel[c] = s->vel[3 * i + c] + cr[c];
      const double *xo = s->won[6 * i + w] ? &s->wxi[18 * i + 3 * w] : zero3;
      double Fa[3], Ft[3], xin[3], fnabs, tq[3], sc[2];
      contact_law(&s->P, s->mass[i], zeta, delta, nv, vrel, xo, Fa, Ft, xin, &fnabs, sc);
      cross3(nv, Ft, tq);
      for (int c = 0; c < 3; c++) {
        Fi[c] += Fa[c];
        Ti[c] += r * tq[c];
      }
      rolling(s, i, fnabs, Ti);
      fs += sc[0] + sc[1];
      ts += r * sc[1] + (roll_on ? s->P.mu_r * sc[0] : 0.0);
      if (commit) {
        memcpy(&s->wxi[18 * i + 3 * w], xin, sizeof xin);
        s->won[6 * i + w] = 1;
      }
    }
    gas_force(s, g, i, Fi, Fs ? &fs : NULL);
    for (int c = 0; c < 3; c++) {
      F[3 * i + c] = Fi[c];
      T[3 * i + c] = Ti[c];
    }
    if (Fs) Fs[i] = fs;
    if (Ts) Ts[i] = ts;
  }
  if (overflow) abort();
  free(pr);
  free(pt);
  free(first);
  free(sec_off);
  free(sec);
  if (commit) {
    free(s->hist);
    free(s->hcnt);
    s->hist = nh;
    s->hcnt = ncnt;
  } else {
    free(nh);
    free(ncnt);
  }
}

void ora_forces(ora_sys *s, const ora_gas *g, double *F, double *T) { compute_forces(s, g, F, T, NULL, NULL, 0); }

void ora_force_scale(ora_sys *s, const ora_gas *g, double *Fs, double *Ts) {
  double *F = (double *)malloc(sizeof(double) * 3 * (s->n > 0 ? s->n : 1));
  double *T = (double *)malloc(sizeof(double) * 3 * (s->n > 0 ? s->n : 1));
  compute_forces(s, g, F, T, Fs, Ts, 0);
  free(F);
  free(T);
}

/* Test harness: a fixed pseudo-random sign (+1 or -1) per parcel, component
 * and seed (splitmix64 of the three), for ora_step_perturbed. */
static double fixed_sign(unsigned long long seed, int i, int c) {
  unsigned long long z = seed * 0x9E3779B97F4A7C15ull + (unsigned long long)i * 6 + (unsigned long long)c + 1;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (z & 1ull) ? 1.0 : -1.0;
}

/* eq. e3-3 and e3-6 advanced by semi-implicit Euler (reading: the paper does
 * not name its integrator): v += dt F/m, w += dt T/I, x += dt v_new.  With
 * rel > 0 (test harness only: ora_step_perturbed) every force and torque
 * component is biased by rel times the parcel's force-term scale, with a
 * sign fixed per parcel and component, every step; with round32 the
 * velocities, spins and tangential springs are rounded to FP32 after every
 * step (the storage of a mixed-precision evaluation). */
static void step_impl(ora_sys *s, int nsteps, const ora_gas *g, double rel, unsigned long long seed,
                      int round32) {
  int n = s->n;
  double *F = (double *)malloc(sizeof(double) * 3 * n);
  double *T = (double *)malloc(sizeof(double) * 3 * n);
  double *Fs = rel > 0.0 ? (double *)malloc(sizeof(double) * n) : NULL;
  double *Ts = rel > 0.0 ? (double *)malloc(sizeof(double) * n) : NULL;
  for (int st = 0; st < nsteps; st++) {
    compute_forces(s, g, F, T, Fs, Ts, 1);
    if (rel > 0.0)
      for (int i = 0; i < n; i++)
        for (int c = 0; c < 3; c++) {
          F[3 * i + c] += rel * Fs[i] * fixed_sign(seed, i, c);
          T[3 * i + c] += rel * Ts[i] * fixed_sign(seed, i, 3 + c);
        }
    double dt = s->P.dt;
    /* eq. e3-8 with conduction and radiation left out: m C_p dT_p/dt =
     * k^3 (Q_conv + Q_r + Q_rm) (eqs. e3-41, e3-49, e3-50), explicit in the
     * step-start state; reading: m C_p,p and Q_r + Q_rm are those of the last
     * reaction update (masses change only at coupling, Section 4) */
    if (s->P.energy_on)
#pragma omp parallel for schedule(static)
      for (int i = 0; i < n; i++) {
        int c = cell_of(s, i);
        double q = parcel_hA(s, g, i) * (g->T[c] - s->Tp[i]) + s->qrx[i];
        s->Tp[i] += dt * q / s->mcp[i];
      }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
      double m = s->mass[i], I = inertia(s, i);
      for (int c = 0; c < 3; c++) {
        s->vel[3 * i + c] += dt * F[3 * i + c] / m;
        s->omg[3 * i + c] += dt * T[3 * i + c] / I;
        if (round32) { /* test harness: velocities and spins stored in FP32 */
          s->vel[3 * i + c] = (double)(float)s->vel[3 * i + c];
          s->omg[3 * i + c] = (double)(float)s->omg[3 * i + c];
        }
        s->pos[3 * i + c] += dt * s->vel[3 * i + c];
      }
      if (round32) { /* and the tangential springs */
        for (int q = 0; q < s->hcnt[i]; q++)
          for (int c = 0; c < 3; c++)
            s->hist[(size_t)i * HCAP + q].xi[c] = (double)(float)s->hist[(size_t)i * HCAP + q].xi[c];
        for (int c = 0; c < 18; c++) s->wxi[18 * i + c] = (double)(float)s->wxi[18 * i + c];
      }
    }
  }
  free(F);
  free(T);
  free(Fs);
  free(Ts);
}

void ora_step(ora_sys *s, int nsteps, const ora_gas *g) { step_impl(s, nsteps, g, 0.0, 0, 0); }

void ora_step_perturbed(ora_sys *s, int nsteps, const ora_gas *g, double rel, unsigned long long seed,
                        int round32) {
  step_impl(s, nsteps, g, rel, seed, round32);
}

/* ------------------------------------------------------------ deposition
 * eq. e3-25 / e3-27a summed over the parcels whose centre lies in the cell
 * (reading: nearest-grid-point both ways, V_cell = h^3, eps_g clamped below
 * by eps_min).  K_p = beta V_p / (1 - eps_g) uses the newly deposited eps_g. */
static void deposit(ora_sys *s, const ora_gas *g, double *np_, double *sumK, double *sumKu,
                    double *sumKv, double *sumKw, double *sumKs) {
  int nc = s->n_cells;
  double *sv = (double *)calloc(nc > 0 ? nc : 1, sizeof(double));
  double *cnt = (double *)calloc(nc > 0 ? nc : 1, sizeof(double));
  for (int i = 0; i < s->n; i++) {
    int c = cell_of(s, i);
    sv[c] += volume(s, i);
    cnt[c] += 1.0;
  }
  for (int b = 0; b < s->P.n_beds; b++) {
    const ora_bed *B = &s->beds[b];
    int ncb = B->n[0] * B->n[1] * B->n[2];
    double vc = B->h * B->h * B->h;
    for (int q = 0; q < ncb; q++) {
      int c = B->cell_off + q;
      double e = 1.0 - sv[c] / vc;
      if (e < s->P.eps_min) e = s->P.eps_min;
      if (e > 1.0) e = 1.0;
      s->eps[c] = e;
    }
  }
  if (np_) memcpy(np_, cnt, sizeof(double) * nc);
  if (g && (sumK || sumKu || sumKv || sumKw || sumKs)) {
    double *a[5] = {sumK, sumKu, sumKv, sumKw, sumKs};
    for (int j = 0; j < 5; j++) if (a[j]) memset(a[j], 0, sizeof(double) * nc);
    /* K_p and |u_g - v_p| per parcel (independent), then the cell sums in
     * ascending id */
    double *Kp = (double *)malloc(sizeof(double) * 2 * (s->n > 0 ? s->n : 1));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; i++) {
      int c = cell_of(s, i);
      const ora_bed *B = &s->beds[s->bed[i]];
      double rho, mu;
      ora_gas_props(g->T[c], g->p[c], g->xH2[c], g->xH2O[c], g->xN2[c], B->mu_override, &rho, &mu);
      double sl[3] = {g->ug[c] - s->vel[3 * i], g->vg[c] - s->vel[3 * i + 1], g->wg[c] - s->vel[3 * i + 2]};
      double slip = norm3(sl);
      Kp[2 * i] = beta_of(s, i, s->eps[c], rho, mu, slip) * volume(s, i);
      Kp[2 * i + 1] = slip;
    }
    for (int i = 0; i < s->n; i++) {
      int c = cell_of(s, i);
      double K = Kp[2 * i], slip = Kp[2 * i + 1];
      if (sumK) sumK[c] += K;
      if (sumKu) sumKu[c] += K * s->vel[3 * i];
      if (sumKv) sumKv[c] += K * s->vel[3 * i + 1];
      if (sumKw) sumKw[c] += K * s->vel[3 * i + 2];
      if (sumKs) sumKs[c] += K * slip;
    }
    free(Kp);
  }
  free(sv);
  free(cnt);
}

void ora_couple(ora_sys *s, const ora_gas *g, double *eps, double *np_, double *sumK,
                double *sumKu, double *sumKv, double *sumKw, double *sumKs) {
  deposit(s, g, np_, sumK, sumKu, sumKv, sumKw, sumKs);
  if (eps) memcpy(eps, s->eps, sizeof(double) * s->n_cells);
}

/* ------------------------------------------------------------ reaction (USCM) */

/* Kirchhoff solution of the resistance network of Fig. 2 / Fig. 4 for any set
 * of active interfaces, as a ladder from the innermost active interface
 * outwards (each stage a Thevenin pair (Phi, R)), then back-substitution
 * inwards.  It reproduces the paper's closed forms e2-2..e2-10 (with the
 * determinant corrected), eb1..eb3 and ea1..ea2.  A[i], B[] and x_eq[i] of
 * layers inside the innermost active interface are never used. */
static void ladder_dual(const int act[3], const dual A[3], const dual B[3], double F, double x,
                        const double xeq[3], dual r[3], dual *Q, dual *S) {
  int i0 = -1;
  for (int i = 0; i < 3; i++) { r[i] = D(0.0); if (act[i] && i0 < 0) i0 = i; }
  if (i0 < 0) { *Q = D(0.0); *S = D(0.0); return; }
  dual R = A[i0], Phi = D(xeq[i0]);
  for (int i = i0 + 1; i < 3; i++) {
    R = dadd(R, B[i - 1]);
    if (act[i]) {
      dual g1 = dinv(R), g2 = dinv(A[i]);
      Phi = ddiv(dadd(dmul(Phi, g1), dscale(g2, xeq[i])), dadd(g1, g2));
      R = dinv(dadd(g1, g2));
    }
  }
  dual Rt = dadd(dadd(R, B[2]), D(F));
  dual N = ddiv(dsub(D(x), Phi), Rt);
  *Q = dinv(Rt);
  *S = ddiv(Phi, Rt);
  dual phi = dsub(D(x), dmul(N, dadd(D(F), B[2])));
  dual flow = N;
  for (int i = 2; i >= i0; i--) {
    if (act[i]) {
      r[i] = ddiv(dsub(phi, D(xeq[i])), A[i]);
      flow = dsub(flow, r[i]);
    }
    if (i > i0) phi = dsub(phi, dmul(flow, B[i - 1]));
  }
}

void ora_ladder(const int active[3], const double A[3], const double B[3], double F, double x,
                const double xeq[3], double r[3], double *Q, double *S) {
  dual Ad[3], Bd[3], rd[3], q, sv;
  for (int i = 0; i < 3; i++) { Ad[i] = D(A[i]); Bd[i] = D(B[i]); }
  ladder_dual(active, Ad, Bd, F, x, xeq, rd, &q, &sv);
  for (int i = 0; i < 3; i++) r[i] = rd[i].v;
  *Q = q.v;
  *S = sv.v;
}

/* Per-parcel environment of one reaction update.  kr carries the kinetic
 * parameters' tangents. */
typedef struct {
  double x, xeq[3], kappa[3], c_mol, Ap, rp, Deff[3], F, dt;
  dual kr[3];
} renv;

/* One explicit reaction update of a parcel (eqs. e2-1..e2-19, e2-25, e3-1,
 * e3-2): shell geometry from the remaining fractions u = 1 - f (eqs.
 * e2-15..e2-17), interface resistances (eq. e2-12), layer diffusion
 * resistances (eq. e2-14; reading: layer m spans the h and m interfaces, layer
 * w the m and w interfaces, layer Fe the w interface and the surface), the
 * network solve, then H2 extents xi_i = A_p c r_i dt (moles per real particle;
 * reading: negative rates clamp to zero, the reactions being irreversible,
 * assumption (i), and each extent is capped by its reactant at the step start)
 * and the stoichiometry of Table 1.  Returns the number of clamped rates. */
static int react_core(const renv *e, dual sp[4], dual *Q, dual *S, dual xi[3]) {
  dual N = dadd(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), dadd(sp[2], sp[3]));
  dual u[3];
  u[0] = ddiv(dscale(sp[0], 2.0), N);
  u[1] = ddiv(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), N);
  u[2] = ddiv(dadd(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), sp[2]), N);
  int act[3];
  for (int i = 0; i < 3; i++) act[i] = (sp[i].v > 1e-12 * N.v) && (e->x > e->xeq[i]);
  int i0 = -1;
  for (int i = 0; i < 3; i++) if (act[i] && i0 < 0) i0 = i;
  dual A[3], B[3], r[3];
  for (int i = 0; i < 3; i++) { A[i] = D(1.0); B[i] = D(0.0); }
  int clamps = 0;
  if (i0 < 0) {
    *Q = D(0.0);
    *S = D(0.0);
    for (int i = 0; i < 3; i++) xi[i] = D(0.0);
    return 0;
  }
  for (int i = i0; i < 3; i++)
    if (act[i]) A[i] = ddiv(dscale(dpowc(u[i], -2.0 / 3.0), e->kappa[i]), e->kr[i]);
  /* layers outside i0: m (between interfaces 0 and 1), w (1..2), Fe (2..surface) */
  if (i0 <= 0) B[0] = dscale(dsub(dpowc(u[0], -1.0 / 3.0), dpowc(u[1], -1.0 / 3.0)), e->rp / e->Deff[0]);
  if (i0 <= 1) B[1] = dscale(dsub(dpowc(u[1], -1.0 / 3.0), dpowc(u[2], -1.0 / 3.0)), e->rp / e->Deff[1]);
  B[2] = dscale(dsub(dpowc(u[2], -1.0 / 3.0), D(1.0)), e->rp / e->Deff[2]);
  ladder_dual(act, A, B, e->F, e->x, e->xeq, r, Q, S);
  double cad = e->Ap * e->c_mol * e->dt;
  static const double nu[3] = {3.0, 1.0, 1.0};
  for (int i = 0; i < 3; i++) {
    if (r[i].v < 0.0) { r[i] = D(0.0); clamps++; }
    xi[i] = dscale(r[i], cad);
    dual lim = dscale(sp[i], 1.0 / nu[i]);
    if (xi[i].v > lim.v) xi[i] = lim;
  }
  dual n0 = dsub(sp[0], dscale(xi[0], 3.0));
  if (n0.v < 0.0) n0 = D(0.0); /* a capped extent exhausts Fe2O3; 3 (n/3) may round above n */
  dual n1 = dsub(dadd(sp[1], dscale(xi[0], 2.0)), xi[1]);
  dual n2 = dsub(dadd(sp[2], dscale(xi[1], 3.0)), xi[2]);
  dual n3 = dadd(sp[3], xi[2]);
  sp[0] = n0; sp[1] = n1; sp[2] = n2; sp[3] = n3;
  return clamps;
}

int ora_react_point(const double env[18], double sp[4]) {
  renv e;
  e.x = env[0];
  for (int i = 0; i < 3; i++) { e.xeq[i] = env[1 + i]; e.kappa[i] = env[4 + i]; e.kr[i] = D(env[7 + i]); }
  e.c_mol = env[10];
  e.Ap = env[11];
  e.rp = env[12];
  for (int i = 0; i < 3; i++) e.Deff[i] = env[13 + i];
  e.F = env[16];
  e.dt = env[17];
  dual d[4], Q, S, xi[3];
  for (int q = 0; q < 4; q++) d[q] = D(sp[q]);
  int c = react_core(&e, d, &Q, &S, xi);
  for (int q = 0; q < 4; q++) sp[q] = d[q].v;
  return c;
}

/* eqs. e2-18 / e2-19 from the remaining fractions */
static dual fov_of(const dual sp[4], int kind) {
  dual N = dadd(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), dadd(sp[2], sp[3]));
  dual fh = dsub(D(1.0), ddiv(dscale(sp[0], 2.0), N));
  dual fm = dsub(D(1.0), ddiv(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), N));
  dual fw = dsub(D(1.0), ddiv(dadd(dadd(dscale(sp[0], 2.0), dscale(sp[1], 3.0)), sp[2]), N));
  if (kind == 1) return dadd(dscale(fm, 0.25), dscale(fw, 0.75));
  return dadd(dadd(dscale(fh, 1.0 / 9.0), dscale(fm, 2.0 / 9.0)), dscale(fw, 6.0 / 9.0));
}

/* eqs. e2-18 / e2-19 for one state (nh, nm, nw, nfe); kind 0 hematite, 1 magnetite */
double ora_fov(const double sp[4], int kind) {
  dual d[4];
  for (int q = 0; q < 4; q++) d[q] = D(sp[q]);
  return fov_of(d, kind).v;
}

/* Environment of parcel i from its cell (NGP) and its slip. */
static void make_env(const ora_sys *s, const ora_gas *g, int i, double dt, const double *theta,
                     int tangents, renv *e) {
  int c = cell_of(s, i);
  const ora_bed *B = &s->beds[s->bed[i]];
  const ora_ore *o = &s->ores[s->ore[i]];
  double T = g->T[c], p = g->p[c], xh2 = g->xH2[c], xh2o = g->xH2O[c], xn2 = g->xN2[c];
  /* reading: with the energy equation, equilibria, rate constants and pore
   * diffusion take the particle temperature; the film, the gas density and
   * the molar concentration stay at the gas temperature */
  double Tk = s->P.energy_on ? s->Tp[i] : T;
  /* Section 2.1: H2 fraction of the N2-free gas */
  if (xh2o <= 0.0) e->x = xh2 > 0.0 ? 1.0 : 0.0;
  else e->x = xh2 / (xh2 + xh2o);
  for (int q = 0; q < 3; q++) {
    double K = ora_keq(q, Tk);
    e->xeq[q] = 1.0 / (K + 1.0);   /* eq. e2-1-3 */
    e->kappa[q] = K / (1.0 + K);   /* eq. e2-12 factor */
    const double *th = theta ? theta : B->theta;
    double kr = exp(th[2 * q] - th[2 * q + 1] / (RG * Tk)); /* eq. e2-13 */
    e->kr[q] = D(kr);
    if (tangents) {
      e->kr[q].d[2 * q] = kr;
      e->kr[q].d[2 * q + 1] = -kr / (RG * Tk);
    }
  }
  e->c_mol = p / (RG * T);
  double dp = s->d[i] / s->k[i];
  e->Ap = PI * dp * dp;
  e->rp = 0.5 * dp;
  double xi[4];
  ora_layer_porosity(o, xi);
  double Dp = ora_pore_diff(Tk, p, xh2, xh2o, xn2, o->d_pore_cm);
  for (int q = 0; q < 3; q++) e->Deff[q] = Dp * xi[q + 1] / o->tau; /* eq. e2-30 */
  double sl[3] = {g->ug[c] - s->vel[3 * i], g->vg[c] - s->vel[3 * i + 1], g->wg[c] - s->vel[3 * i + 2]};
  e->F = ora_film(T, p, xh2, xh2o, xn2, B->mu_override, s->eps[c], norm3(sl), dp);
  e->dt = dt;
}

long ora_react(ora_sys *s, double dt, const ora_gas *g, int update_mass, double *mdotH2,
               double *mdotH2O, double *sumEQ, double *sumES, double *fov, double *bed_fov,
               double *hA, double *hAT, double *Qrm, double *Hr) {
  int nc = s->n_cells, n = s->n;
  double *outs[8] = {mdotH2, mdotH2O, sumEQ, sumES, hA, hAT, Qrm, Hr};
  for (int j = 0; j < 8; j++) if (outs[j]) memset(outs[j], 0, sizeof(double) * nc);
  double *bw = (double *)calloc(s->P.n_beds, sizeof(double));
  double *bf = (double *)calloc(s->P.n_beds, sizeof(double));
  /* per parcel (independent): the update and its 8 cell terms, f_ov and the
   * bed weight; then the cell and bed sums in ascending id */
  double *pp = (double *)malloc(sizeof(double) * 10 * (n > 0 ? n : 1));
  long clamps = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : clamps)
  for (int i = 0; i < n; i++) {
    double *o = &pp[10 * i];
    renv e;
    make_env(s, g, i, dt, NULL, 0, &e);
    int c = cell_of(s, i);
    dual sp[4], Q, S, xi[3];
    for (int q = 0; q < 4; q++) sp[q] = D(s->sp[4 * i + q]);
    clamps += react_core(&e, sp, &Q, &S, xi);
    double dn[4];
    for (int q = 0; q < 4; q++) {
      dn[q] = sp[q].v - s->sp[4 * i + q];
      s->sp[4 * i + q] = sp[q].v;
    }
    double k3 = s->k[i] * s->k[i] * s->k[i];
    double xs = xi[0].v + xi[1].v + xi[2].v;
    for (int q = 4; q < 8; q++) o[q] = 0.0;
    if (s->P.energy_on) {
      /* eqs. e3-18, e3-19 (solids) and e3-20, e3-21 (gases) at T_p, with the
       * k^3 of eqs. e3-49, e3-50; the moles changed over dt per real
       * particle; reading: the gas species of a reaction are the H2 it takes
       * from and the H2O it gives to the gas */
      double Tp = s->Tp[i], Qr = 0.0;
      for (int z = 0; z < 4; z++) Qr -= ora_h_mol(3 + z, Tp) * dn[z] / dt;
      double Qm = -(ora_h_mol(1, Tp) - ora_h_mol(0, Tp)) * xs / dt;
      s->qrx[i] = k3 * (Qr + Qm);
      s->mcp[i] = parcel_mcp(s, i);
      /* eqs. e4-4, e4-5 (times V_cell), e3-38 and e3-39 (times -V_cell) */
      double ha = parcel_hA(s, g, i);
      o[4] = ha;
      o[5] = ha * Tp;
      o[6] = k3 * Qm;
      o[7] = k3 * (ora_h_mol(1, g->T[c]) - ora_h_mol(0, g->T[c])) * xs / dt;
    }
    /* eqs. e2-1, e2-25, e3-25, e3-52: kg/s per parcel, summed per cell */
    o[0] = -k3 * MG[0] * 1e-3 * xs / dt;
    o[1] = k3 * MG[1] * 1e-3 * xs / dt;
    /* eqs. e4-7..e4-11 with E = eta A_p / T, eta_H2 = -1 */
    double E = -e.Ap / g->T[c];
    o[2] = k3 * E * Q.v;
    o[3] = k3 * E * S.v;
    o[8] = fov_of(sp, s->ores[s->ore[i]].kind).v;
    o[9] = k3 * (2.0 * sp[0].v + 3.0 * sp[1].v + sp[2].v + sp[3].v);
    if (update_mass) s->mass[i] = parcel_mass(s, i);
  }
  for (int i = 0; i < n; i++) {
    const double *o = &pp[10 * i];
    int c = cell_of(s, i);
    for (int j = 0; j < 8; j++)
      if (outs[j] && (j < 4 || s->P.energy_on)) outs[j][c] += o[j];
    if (fov) fov[i] = o[8];
    bw[s->bed[i]] += o[9];
    bf[s->bed[i]] += o[9] * o[8];
  }
  free(pp);
  if (bed_fov)
    for (int b = 0; b < s->P.n_beds; b++) bed_fov[b] = bw[b] > 0 ? bf[b] / bw[b] : 0.0;
  free(bw);
  free(bf);
  return clamps;
}

void ora_grad(ora_sys *s, const ora_gas *g, int n_sub, double dt_react, int dyn_every,
              const double theta[6], double *J, double grad[6]) {
  int n = s->n;
  dual *sp = (dual *)malloc(sizeof(dual) * 4 * n);
  for (int i = 0; i < 4 * n; i++) sp[i] = D(s->sp[i]);
  for (int st = 0; st < n_sub; st++) {
    if (st % dyn_every == 0) {
      ora_step(s, 1, g);
      deposit(s, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < n; i++) {
      renv e;
      make_env(s, g, i, dt_react, theta, 1, &e);
      dual Q, S, xi[3];
      react_core(&e, &sp[4 * i], &Q, &S, xi);
    }
  }
  dual num = D(0.0);
  double den = 0.0;
  for (int i = 0; i < n; i++) {
    double k3 = s->k[i] * s->k[i] * s->k[i];
    double w = k3 * (2.0 * sp[4 * i].v + 3.0 * sp[4 * i + 1].v + sp[4 * i + 2].v + sp[4 * i + 3].v);
    num = dadd(num, dscale(fov_of(&sp[4 * i], s->ores[s->ore[i]].kind), w));
    den += w;
  }
  *J = num.v / den;
  for (int q = 0; q < 6; q++) grad[q] = num.d[q] / den;
  for (int i = 0; i < 4 * n; i++) s->sp[i] = sp[i].v;
  free(sp);
}

void ora_get(const ora_sys *s, double *x, double *y, double *z, double *vx, double *vy,
             double *vz, double *wx, double *wy, double *wz, double *nh, double *nm,
             double *nw, double *nfe, double *mass, double *eps) {
  for (int i = 0; i < s->n; i++) {
    if (x) x[i] = s->pos[3 * i];
    if (y) y[i] = s->pos[3 * i + 1];
    if (z) z[i] = s->pos[3 * i + 2];
    if (vx) vx[i] = s->vel[3 * i];
    if (vy) vy[i] = s->vel[3 * i + 1];
    if (vz) vz[i] = s->vel[3 * i + 2];
    if (wx) wx[i] = s->omg[3 * i];
    if (wy) wy[i] = s->omg[3 * i + 1];
    if (wz) wz[i] = s->omg[3 * i + 2];
    if (nh) nh[i] = s->sp[4 * i];
    if (nm) nm[i] = s->sp[4 * i + 1];
    if (nw) nw[i] = s->sp[4 * i + 2];
    if (nfe) nfe[i] = s->sp[4 * i + 3];
    if (mass) mass[i] = s->mass[i];
  }
  if (eps) memcpy(eps, s->eps, sizeof(double) * s->n_cells);
}

/* Test harness: the tangential springs held, for setting up both sides of a
 * comparison from the same contact history.  Pairs (i < j, the spring in the
 * orientation of i) go to ij / xi up to cap of them (the count is returned);
 * won (6 per parcel) and wxi (18 per parcel) take the wall springs. */
long ora_contacts(const ora_sys *s, int *ij, double *xi, long cap, unsigned char *won, double *wxi) {
  long m = 0;
  for (int i = 0; i < s->n; i++)
    for (int q = 0; q < s->hcnt[i]; q++) {
      if (m < cap) {
        ij[2 * m] = i;
        ij[2 * m + 1] = s->hist[(size_t)i * HCAP + q].partner;
        for (int c = 0; c < 3; c++) xi[3 * m + c] = s->hist[(size_t)i * HCAP + q].xi[c];
      }
      m++;
    }
  if (won) memcpy(won, s->won, (size_t)6 * s->n);
  if (wxi) memcpy(wxi, s->wxi, sizeof(double) * 18 * (size_t)s->n);
  return m;
}

/* Test harness: replace the springs by the given ones (the layout of
 * ora_contacts); returns -1 for a pair out of order or range, or when a
 * parcel would hold more than HCAP partners. */
int ora_set_contacts(ora_sys *s, const int *ij, const double *xi, long np, const unsigned char *won,
                     const double *wxi) {
  for (long m = 0; m < np; m++)
    if (ij[2 * m] < 0 || ij[2 * m] >= ij[2 * m + 1] || ij[2 * m + 1] >= s->n) return -1;
  for (int i = 0; i < s->n; i++) s->hcnt[i] = 0;
  for (long m = 0; m < np; m++) {
    const int i = ij[2 * m];
    if (s->hcnt[i] == HCAP) return -1;
    hist_t *h = &s->hist[(size_t)i * HCAP + s->hcnt[i]++];
    h->partner = ij[2 * m + 1];
    for (int c = 0; c < 3; c++) h->xi[c] = xi[3 * m + c];
  }
  memcpy(s->won, won, (size_t)6 * s->n);
  memcpy(s->wxi, wxi, sizeof(double) * 18 * (size_t)s->n);
  return 0;
}

/* particle temperatures (K, by id); m C_p,p follows, Q_r + Q_rm restarts at 0 */
void ora_set_temperature(ora_sys *s, const double *Tp) {
  for (int i = 0; i < s->n; i++) {
    s->Tp[i] = Tp[i];
    s->qrx[i] = 0.0;
    s->mcp[i] = parcel_mcp(s, i);
  }
}

void ora_get_energy(const ora_sys *s, double *Tp, double *qrx, double *mcp) {
  for (int i = 0; i < s->n; i++) {
    if (Tp) Tp[i] = s->Tp[i];
    if (qrx) qrx[i] = s->qrx[i];
    if (mcp) mcp[i] = s->mcp[i];
  }
}

/* ------------------------------------------------------------ gas species (two-way coupling)
 * One explicit step dt of H2 and H2O transport (eq. e3-40 with eqs. e4-9..e4-11)
 * on the frozen flow: reading: first-order upwind convection along z only (no
 * molecular or pseudo-turbulent diffusion), face velocity the mean of the two
 * cells' w, the inlet composition xin entering through each bed's bottom face,
 * zero gradient at the top; the H2 source semi-implicit through
 * C0 = sum(k^3 E Q)/V_cell and C1 = -(M_H2/R) sum(k^3 E S)/V_cell; the H2O
 * source the H2 taken, converted 1:1 in moles (Table 1); eps_g the voidage of
 * the last deposit, T and p frozen.  Outputs the new true mole fractions. */
void ora_gas_species(const ora_sys *s, const ora_gas *g, double dt, const double *sumEQ,
                     const double *sumES, const double xin[2], double *xh2_out, double *xh2o_out,
                     double *xn2_out) {
  for (int b = 0; b < s->P.n_beds; b++) {
    const ora_bed *B = &s->beds[b];
    int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    double V = B->h * B->h * B->h;
    for (int iz = 0; iz < nz; iz++)
      for (int iy = 0; iy < ny; iy++)
        for (int ix = 0; ix < nx; ix++) {
          int c = B->cell_off + ix + nx * (iy + ny * iz);
          /* partial densities eps rho Y_j (kg/m3 of cell) of H2, H2O, N2 in a cell
           * with composition x (true mole fractions), at the cell's T, p */
          double u[3], flux_lo[3], flux_hi[3];
          for (int side = 0; side < 3; side++) {
            /* side 0: this cell; side 1: the cell below (or the inlet); side 2: above */
            int cc = c;
            double x[3];
            if (side == 1) cc = iz > 0 ? c - nx * ny : -1;
            if (side == 2) cc = iz < nz - 1 ? c + nx * ny : -1;
            if (cc < 0 && side == 1) {
              x[0] = xin[0]; x[1] = xin[1]; x[2] = 1.0 - xin[0] - xin[1];
              cc = c;
            } else {
              if (cc < 0) cc = c; /* top: zero gradient */
              x[0] = g->xH2[cc]; x[1] = g->xH2O[cc]; x[2] = g->xN2[cc];
            }
            double Mg = 0.0;
            for (int j = 0; j < 3; j++) Mg += x[j] * MG[j];
            double rho = g->p[cc] * Mg * 1e-3 / (RG * g->T[cc]); /* eq. e3-53 */
            double e = s->eps[cc];
            double pd[3];
            for (int j = 0; j < 3; j++) pd[j] = e * rho * x[j] * MG[j] / Mg;
            if (side == 0) for (int j = 0; j < 3; j++) u[j] = pd[j];
            if (side == 1) {
              double wf = iz > 0 ? 0.5 * (g->wg[c - nx * ny] + g->wg[c]) : g->wg[c];
              for (int j = 0; j < 3; j++) flux_lo[j] = wf * (wf >= 0.0 ? pd[j] : 0.0);
            }
            if (side == 2) {
              double wf = iz < nz - 1 ? 0.5 * (g->wg[c] + g->wg[c + nx * ny]) : g->wg[c];
              for (int j = 0; j < 3; j++) flux_hi[j] = wf * (wf < 0.0 ? pd[j] : 0.0);
            }
          }
          /* upwind: the lower face carries the lower state upwards (w >= 0) or
           * this cell's state downwards; the upper face the reverse */
          {
            double wl = iz > 0 ? 0.5 * (g->wg[c - nx * ny] + g->wg[c]) : g->wg[c];
            double wu = iz < nz - 1 ? 0.5 * (g->wg[c] + g->wg[c + nx * ny]) : g->wg[c];
            for (int j = 0; j < 3; j++) {
              if (wl < 0.0) flux_lo[j] = wl * u[j];
              if (wu >= 0.0) flux_hi[j] = wu * u[j];
            }
          }
          double rhs[3];
          for (int j = 0; j < 3; j++) rhs[j] = u[j] - dt / B->h * (flux_hi[j] - flux_lo[j]);
          /* H2 semi-implicit (eq. e4-9): u1' (1 - dt C0 T / (X eps)) = rhs1 + dt C1 p */
          double x1 = g->xH2[c], x2 = g->xH2O[c];
          double X = x1 + x2;
          double C0 = sumEQ[c] / V, C1 = -(MG[0] * 1e-3 / RG) * sumES[c] / V;
          double e = s->eps[c];
          double u1 = rhs[0] + dt * C1 * g->p[c];
          if (X > 0.0) u1 = u1 / (1.0 - dt * C0 * g->T[c] / (X * e));
          if (u1 < 0.0) u1 = 0.0;
          /* H2 taken by the particles over dt (kg/m3), returned as H2O */
          double taken = rhs[0] - u1;
          double u2 = rhs[1] + taken * MG[1] / MG[0];
          double u3 = rhs[2];
          double n1 = u1 / MG[0], n2 = u2 / MG[1], n3 = u3 / MG[2], nt = n1 + n2 + n3;
          xh2_out[c] = n1 / nt;
          xh2o_out[c] = n2 / nt;
          xn2_out[c] = n3 / nt;
        }
  }
}

/* Gas-side momentum step of the two-way coupling (eqs. e4-1, e4-2 with the
 * interphase source of eqs. e3-27, e3-27a), on the frozen pressure field:
 *   eps rho (u' - u) / dt = -eps grad p + eps rho g + K_gp u' - K_gp u_p,
 * the source K_gp u_g implicit and K_gp u_p explicit.  reading: K_gp =
 * -sum_p K_p / V_cell and K_gp u_p = -sum_p K_p v_p / V_cell with K_p =
 * beta V_p / (1 - eps) of the last deposit, so the gas takes exactly the
 * drag the parcels feel (the printed form weights the sum by |u_g - v_p| /
 * |u_g - u_p| and equals this one when the parcels of a cell move
 * together).  eps is that of the last deposit, rho from eq. e3-53 at the
 * cell's T, p and composition; convection, viscous and pseudo-turbulent
 * stresses belong to the gas solver and are left out. */
void ora_gas_momentum(const ora_sys *s, const ora_gas *g, double dt, const double *sumK, const double *sumKu,
                      const double *sumKv, const double *sumKw, double *u_out, double *v_out, double *w_out) {
  for (int b = 0; b < s->P.n_beds; b++) {
    const ora_bed *B = &s->beds[b];
    int ncb = B->n[0] * B->n[1] * B->n[2];
    double V = B->h * B->h * B->h;
    for (int q = 0; q < ncb; q++) {
      int c = B->cell_off + q;
      double rho, mu;
      ora_gas_props(g->T[c], g->p[c], g->xH2[c], g->xH2O[c], g->xN2[c], 0.0, &rho, &mu);
      double e = s->eps[c];
      double u[3] = {g->ug[c], g->vg[c], g->wg[c]};
      double gp[3] = {g->dpdx[c], g->dpdy[c], g->dpdz[c]};
      double Kv[3] = {sumKu[c], sumKv[c], sumKw[c]};
      double *out[3] = {u_out, v_out, w_out};
      for (int a = 0; a < 3; a++) {
        double num = e * rho * u[a] / dt - e * gp[a] + e * rho * s->P.g[a] + Kv[a] / V;
        out[a][c] = num / (e * rho / dt + sumK[c] / V);
      }
    }
  }
}
