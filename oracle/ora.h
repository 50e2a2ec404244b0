/*
 * Oracle: a plain, slow, FP64 CPU implementation of the particle side of the
 * coarse-grained CFD-DEM reduction model (arxiv 2311.03908).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, constant or table
 * with the GPU library.
 *
 * Every quantity is SI and double precision.  Parcels are kept in original id
 * order; every sum over parcels, pairs or cells runs in ascending id order.
 * Loops over independent parcels or pairs may run on several threads
 * (OpenMP), which changes no result.
 *
 * Parity unpinned (conventions with no independent pin; the tests check only
 * their use, limits or finiteness): the tortuosity, eps_min, kt/kn, the
 * tangential damping, the neighbour skin and clamp thresholds, the mixture
 * viscosity correlation of Table C2, the magnitude of the Ergun branch of the
 * drag, the rolling-friction torque, the species coefficients E Q, E S of
 * eqs. e4-7..e4-11, and the gas conductivity correlation of Table C3 (pinned
 * only to textbook values of the pure gases).
 */
#ifndef ORA_H
#define ORA_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int wall_kind;          /* 0 = box (six planes), 1 = cylinder (side, floor, lid) */
  double lo[3], hi[3];    /* box; for a cylinder: floor lo[2], lid hi[2], axis at xy centre */
  double R;               /* cylinder radius */
  double origin[3];       /* gas grid origin */
  double h;               /* gas cell edge */
  int n[3];               /* gas cells per axis */
  int cell_off;           /* first cell of this bed in the concatenated gas arrays */
  double theta[6];        /* ln k0_i, Ea_i (J/mol) for R1..R3 */
  double mu_override;     /* > 0: gas viscosity fixed */
} ora_bed;

typedef struct {
  double xi0;             /* initial porosity */
  double d_pore_cm;       /* pore diameter d_a in cm */
  double tau;             /* tortuosity */
  double rho_true[4];     /* true densities of Fe2O3, Fe3O4, FeO, Fe */
  int kind;               /* 0 hematite ore (eq. e2-18), 1 magnetite ore (eq. e2-19) */
  double psi;             /* sphericity: 0 spheres (eq. e3-5-1), (0, 1] Gidaspow-Ganser (eq. e3-5-2) */
} ora_ore;

typedef struct {
  double kn, e_p, mu_s, mu_r, kt_over_kn, gt_over_gn, eps_min, dt;
  double g[3];
  int ergun_printed;      /* 1: inertial Ergun term with eps_g as printed */
  int drag_on;            /* 0: no gas-side forces (test switch) */
  int n_beds, n_ores;
  int energy_on;          /* 1: particle energy equation (set temperatures with ora_set_temperature) */
} ora_params;

typedef struct {
  const double *ug, *vg, *wg, *p, *dpdx, *dpdy, *dpdz, *T, *xH2, *xH2O, *xN2;
} ora_gas;

typedef struct ora_sys ora_sys;

ora_sys *ora_new(const ora_params *P, const ora_bed *beds, const ora_ore *ores, int n,
                 const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz,
                 const double *wx, const double *wy, const double *wz,
                 const double *d, const double *k, const int *ore, const int *bed,
                 const double *nh, const double *nm, const double *nw, const double *nfe);
void ora_free(ora_sys *s);
int ora_n_cells(const ora_sys *s);
/* threads of the parallel loops; results are identical for any count */
void ora_set_threads(int n);
int ora_threads(void);

/* canonical contact pairs (a < b by id) at the current positions, sorted;
 * brute = 1 uses the O(N^2) scan instead of the cell list.  Returns the count
 * (may exceed cap; only cap pairs are written). */
long ora_pairs(ora_sys *s, int brute, int *ij, long cap);
/* total force and torque the next step would apply (state is not changed) */
void ora_forces(ora_sys *s, const ora_gas *g, double *F, double *T);
/* per parcel, the sums of the magnitudes of the products that ora_forces
 * builds the force and the torque from (per contact and wall: spring,
 * dashpot, tangential spring and dashpot, rolling; gravity, pressure
 * gradient, drag): the scale of the rounding error of F and T when they are
 * evaluated in a lower precision */
void ora_force_scale(ora_sys *s, const ora_gas *g, double *Fs, double *Ts);
void ora_step(ora_sys *s, int nsteps, const ora_gas *g);
/* test harness only: ora_step with every force and torque component biased by
 * rel times the parcel's force-term scale (ora_force_scale), with a sign fixed
 * per parcel, component and seed: a deterministic emulation of a lower-precision
 * evaluation that errs by rel of the products the forces are built from; with
 * round32 the velocities, spins and tangential springs are also rounded to FP32
 * after every step (the state a mixed-precision evaluation stores) */
void ora_step_perturbed(ora_sys *s, int nsteps, const ora_gas *g, double rel, unsigned long long seed,
                        int round32);
/* voidage + drag deposition; outputs may be NULL */
void ora_couple(ora_sys *s, const ora_gas *g, double *eps, double *np_, double *sumK,
                double *sumKu, double *sumKv, double *sumKw, double *sumKs);
/* USCM update over dt; per-cell sources and per-parcel / per-bed f_ov (may be NULL);
 * update_mass = 0 keeps the DEM mass frozen.  Returns the number of clamped rates. */
long ora_react(ora_sys *s, double dt, const ora_gas *g, int update_mass, double *mdotH2,
               double *mdotH2O, double *sumEQ, double *sumES, double *fov, double *bed_fov,
               double *hA, double *hAT, double *Qrm, double *Hr);
/* energy equation: per-parcel temperatures (K, by id; Q_r + Q_rm restarts at 0)
 * and the current temperature, k^3 (Q_r + Q_rm) and m C_p,p of every parcel */
/* test harness: export / import of the tangential springs (pairs i < j with
 * the spring in i's orientation; 6 wall flags and 18 wall-spring components
 * per parcel); ora_contacts returns the pair count, ora_set_contacts -1 on a
 * bad pair */
long ora_contacts(const ora_sys *s, int *ij, double *xi, long cap, unsigned char *won, double *wxi);
int ora_set_contacts(ora_sys *s, const int *ij, const double *xi, long np, const unsigned char *won,
                     const double *wxi);
void ora_set_temperature(ora_sys *s, const double *Tp);
void ora_get_energy(const ora_sys *s, double *Tp, double *qrx, double *mcp);
void ora_get(const ora_sys *s, double *x, double *y, double *z, double *vx, double *vy,
             double *vz, double *wx, double *wy, double *wz, double *nh, double *nm,
             double *nw, double *nfe, double *mass, double *eps);
/* kinetic gradient by forward-mode dual numbers: n_sub reaction substeps of
 * dt_react with one DEM step (and a voidage deposit) before every dyn_every-th;
 * the DEM mass stays frozen.  Writes J (bed-mean f_ov of bed 0 weighted by
 * k^3 N_Fe over all parcels) and dJ/dtheta (6).  theta replaces every bed's
 * kinetic parameters. The system state is advanced. */
void ora_grad(ora_sys *s, const ora_gas *g, int n_sub, double dt_react, int dyn_every,
              const double theta[6], double *J, double grad[6]);

/* two-way coupling stand-in: one explicit step dt of H2 / H2O transport on the
 * frozen flow (upwind along z, inlet composition xin = (x_H2, x_H2O) at each bed's
 * floor) with the particle sources of the last ora_react (semi-implicit H2 through
 * sums of k^3 E Q and k^3 E S, eqs. e4-9..e4-11); new true mole fractions out */
void ora_gas_species(const ora_sys *s, const ora_gas *g, double dt, const double *sumEQ,
                     const double *sumES, const double xin[2], double *xh2_out, double *xh2o_out,
                     double *xn2_out);

/* two-way coupling, momentum: one step dt of the gas velocity on the frozen
 * pressure field with the interphase source of the last deposit's drag sums
 * (eqs. e4-1, e4-2: K_gp u_g implicit, K_gp u_p explicit); new velocities out */
void ora_gas_momentum(const ora_sys *s, const ora_gas *g, double dt, const double *sumK, const double *sumKu,
                      const double *sumKv, const double *sumKw, double *u_out, double *v_out, double *w_out);

/* ---- point functions, exported for the pins ---- */
double ora_e_cgp(double e_p, double k);
double ora_zeta(double e);
void ora_gas_props(double T, double p, double xh2, double xh2o, double xn2, double mu_override,
                   double *rho, double *mu);
double ora_fuller(double T, double p, int i, int j);   /* 0 H2, 1 H2O, 2 N2 */
double ora_wilke_h2(double T, double p, double xh2, double xh2o, double xn2);
double ora_knudsen_h2(double T, double d_pore_cm);
double ora_pore_diff(double T, double p, double xh2, double xh2o, double xn2, double d_pore_cm);
void ora_layer_porosity(const ora_ore *o, double xi[4]);
double ora_sherwood(double eps, double Re, double Sc);
double ora_film(double T, double p, double xh2, double xh2o, double xn2, double mu_override,
                double eps, double slip, double dp);
double ora_keq(int i, double T);
/* species 0 H2, 1 H2O, 2 N2, 3 Fe2O3, 4 Fe3O4, 5 FeO, 6 Fe (Table C1) */
double ora_h_mol(int sp, double T);    /* J/mol, eq. e3-22 times M */
double ora_cp_mol(int sp, double T);   /* J/(mol K), eq. e3-23 times M */
double ora_lambda_g(double T, double xh2, double xh2o, double xn2);  /* eqs. e3-58, e3-59 */
double ora_cp_g(double T, double xh2, double xh2o, double xn2);      /* eq. e3-57, J/(kg K) */
double ora_nusselt(double eps, double Re, double Pr);                /* eq. e3-12 */
double ora_beta_over_epsp(double eps, double rho, double mu, double slip, double dp, int printed);
double ora_beta_ganser_over_epsp(double eps, double rho, double mu, double slip, double dp, double psi,
                                 double Dbed, int printed);
/* resistance ladder: active[3] (hm, mw, wFe), A[3], B[3] = (B_m, B_w, B_Fe), F,
 * x, xeq[3] -> rates r[3] (unclamped) and the network's Q = 1/R, S = Phi/R */
void ora_ladder(const int active[3], const double A[3], const double B[3], double F, double x,
                const double xeq[3], double r[3], double *Q, double *S);
/* one parcel, explicit environment:
 *   env = {x, xeq0..2, kappa0..2, kr0..2, c_mol, Ap, rp, Deff_m, Deff_w, Deff_Fe, F, dt}
 * sp[4] (nh, nm, nw, nfe) updated in place; returns the number of clamped rates */
int ora_react_point(const double env[18], double sp[4]);
/* overall reduction degree of one state (nh, nm, nw, nfe): eq. e2-18 (kind 0) or e2-19 (kind 1) */
double ora_fov(const double sp[4], int kind);

#ifdef __cplusplus
}
#endif
#endif
