/*
 * demrx -- C-ABI of the MI355X (gfx950) particle side of the coarse-grained
 * CFD-DEM reduction model of arxiv 2311.03908 ("Direct reduction of iron ore
 * with hydrogen in fluidized beds: a coarse-grained CFD-DEM-IBM study").
 *
 * The calls follow the paper's statement of the particle/gas exchange
 * (Section 4, Fig. 5): the gas solver supplies per-cell fields; the particle
 * side advances parcel velocities every DEM step and returns the voidage and
 * the cell-summed momentum and species sources every n = dt_CFD / dt_DEM
 * steps, when the layer masses of the parcels are also updated.
 *
 * Conventions
 *  - SI units throughout; gas arrays hold one value per gas cell, the cells of
 *    all beds concatenated bed by bed, each bed x-fastest (c = ix + nx (iy + ny iz)).
 *  - Every array pointer in dem_parcels, dem_gas and dem_sources is a DEVICE
 *    pointer owned by the caller; the library never frees caller memory and
 *    keeps no caller pointer after a call returns.  Parcel arrays are in the
 *    caller's original parcel order.
 *  - All work is enqueued on the HIP stream given to dem_init; calls return
 *    as soon as the work is enqueued unless stated otherwise.  A context is
 *    not thread-safe; use one context per stream.
 *  - Return value: DEMRX_OK (0) or a negative DEMRX_E* code; dem_last_error()
 *    gives a message.  Errors detected on the device (slot overflow, a parcel
 *    leaving its grid, a non-finite state, a neighbour-list skin violation)
 *    are latched in a device status word and reported by the next call that
 *    synchronises (dem_sync, dem_pairs, dem_get_state, dem_react with a host
 *    result, dem_grad).
 */
#ifndef DEMRX_H
#define DEMRX_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DEMRX_OK 0
#define DEMRX_EINVAL -1     /* invalid argument (null pointer, bad size, bad parameter) */
#define DEMRX_EHIP -2       /* a HIP runtime call failed */
#define DEMRX_EOVERFLOW -3  /* a parcel has more neighbour candidates than max_nbr */
#define DEMRX_EDOMAIN -4    /* a parcel centre left its bed's grid */
#define DEMRX_ENONFINITE -5 /* non-finite parcel state, or gas input in a cell whose drag row is computed */
#define DEMRX_ENOMEM -6     /* device allocation failed */
#define DEMRX_ESKIN -7      /* displacement bound since the last neighbour build exceeded skin/2 */

#define DEM_FP64 0  /* forces, velocities and spins in FP64 */
#define DEM_MIXED 1 /* FP32 forces, velocities and spins; FP64 positions, grid and reaction */

#define DEM_WALL_BOX 0 /* six planes lo/hi */
#define DEM_WALL_CYL 1 /* cylinder of radius R about the vertical axis through the xy centre of
                          lo/hi, floor z = lo[2], lid z = hi[2] */
#define DEM_MAX_ORES 8
#define DEM_MAX_BEDS 4096
#define DEM_MAX_NBR 48
#define DEM_NOALLOC_MAX_PAIRS (1 << 21) /* pairs dem_pairs_noalloc can return */

typedef struct dem_ctx dem_ctx;

/* One bed: reactor walls, frozen gas grid and kinetic parameters. */
typedef struct {
  int32_t wall_kind;   /* DEM_WALL_BOX or DEM_WALL_CYL */
  double lo[3], hi[3]; /* walls (box) or bounding box of the cylinder */
  double R;            /* cylinder radius */
  double origin[3];    /* gas grid origin */
  double h;            /* gas cell edge; the grid must contain lo..hi */
  int32_t n[3];        /* gas cells per axis */
  int32_t refine;      /* DEM cells per gas-cell edge (1..4); h/refine must be >= the largest
                          parcel diameter of the bed plus the skin */
  double theta[6];     /* (ln k0, Ea) of R1 Fe2O3->Fe3O4, R2 Fe3O4->FeO, R3 FeO->Fe; eq. e2-13 */
  double mu_override;  /* > 0: gas viscosity fixed to this value instead of eq. e3-56 */
} dem_bed;

/* One ore type (Section 2.3, Table 3). */
typedef struct {
  double xi0;         /* initial particle porosity, eq. e2-32 */
  double d_pore_cm;   /* pore diameter d_a in cm (Section 2.3) */
  double tau;         /* tortuosity of eq. e2-30 */
  double rho_true[4]; /* true densities of Fe2O3, Fe3O4, FeO, Fe (kg/m3) */
  int32_t kind;       /* 0: hematite ore (f_ov by eq. e2-18), 1: magnetite ore (eq. e2-19) */
  double psi;         /* sphericity: 0 spheres (Gidaspow, eq. e3-5-1); in (0, 1]: Gidaspow-Ganser
                         drag of non-spherical particles (eqs. e3-5-2..e3-5-5, Table 3: 0.85, 0.86),
                         with the bed's equivalent-area diameter (2R, or sqrt(4 A / pi) for a box) */
} dem_ore;

typedef struct {
  int32_t precision;     /* DEM_FP64 or DEM_MIXED */
  int32_t n_beds;        /* 1..DEM_MAX_BEDS; host array copied at init */
  const dem_bed *beds;
  int32_t n_ores;        /* 1..DEM_MAX_ORES; host array copied at init */
  const dem_ore *ores;
  double kn;             /* normal spring stiffness (N/m) */
  double e_p;            /* restitution of the real particle; parcels use eq. e3-45 */
  double mu_s;           /* sliding friction */
  double mu_r;           /* rolling friction length (m); 0 disables */
  double kt_over_kn;     /* tangential / normal stiffness */
  double gt_over_gn;     /* tangential / normal damping */
  double eps_min;        /* lower clamp of the deposited voidage */
  double skin;           /* neighbour-list skin (m) */
  double dt;             /* DEM time step (s) */
  double g[3];           /* gravity (m/s2) */
  int32_t max_nbr;       /* neighbour slots per parcel, 1..DEM_MAX_NBR */
  int32_t check_every;   /* steps between neighbour-list checks (>= 1): at a check the lists are
                            rebuilt if the largest displacement since the last build plus twice the
                            largest speed times the steps to the next check could reach skin/2 */
  int32_t ergun_printed; /* 1: inertial Ergun term with eps_g as printed in eq. e3-5-1 */
  int32_t drag_on;       /* 0: no gas-side forces on parcels (gravity only) */
  int32_t energy_on;     /* 1: particle energy equation (eqs. e3-8..e3-13, e3-18..e3-23, e3-41,
                            e3-49, e3-50): each parcel carries T_p, heated by convection (Gunn Nu)
                            and by the reaction heats of the last dem_react; equilibria, rate
                            constants and pore diffusion then take T_p.  Conduction and
                            radiation are not modelled.  dem_grad requires 0. */
} dem_params;

/* Parcel state (device pointers, original order).  v and w point to float in
 * DEM_MIXED and to double in DEM_FP64.  d is the parcel diameter k * d_p
 * (FP32), k the coarse-graining ratio of Section 3.3, n_* the moles of
 * Fe2O3, Fe3O4, FeO and Fe per real particle, Tp the particle temperature
 * (K, double; read and written only with energy_on, required then). */
typedef struct {
  double *x, *y, *z;
  void *vx, *vy, *vz, *wx, *wy, *wz;
  float *d, *k;
  int32_t *ore, *bed;
  double *nh, *nm, *nw, *nfe;
  double *Tp;
} dem_parcels;

/* Frozen gas fields per cell (device pointers, double): velocity, pressure,
 * pressure gradient, temperature (also the particle temperature unless
 * energy_on) and the true mole fractions of H2, H2O and N2. */
typedef struct {
  const double *ug, *vg, *wg, *p, *dpdx, *dpdy, *dpdz, *T, *xH2, *xH2O, *xN2;
} dem_gas;

/* Per-cell outputs (device pointers, double, any may be NULL):
 *  eps     voidage (eq. e3-25 reading: 1 - sum V_p / h^3, clamped to [eps_min, 1])
 *  np      parcels per cell
 *  sumK    sum of K_p = beta V_p / (1 - eps_g) (eqs. e3-5, e3-27a), kg/s
 *  sumKu/v/w  sum of K_p v_p, sumKs sum of K_p |u_g - v_p|
 *  mdotH2, mdotH2O  parcel mass sources of eq. e3-25 times V_cell (kg/s, eqs. e2-25, e3-52)
 *  sumEQ, sumES     sums of k^3 E Q and k^3 E S of eqs. e4-8..e4-11 with E = eta_H2 A_p / T
 * and, written by dem_react with energy_on only (W/K or W, at the reaction update):
 *  hA      sum of k^3 h_p A_p = H0 V_cell (eqs. e3-10..e3-13, e3-41, e4-4)
 *  hAT     sum of k^3 h_p A_p T_p = H1 V_cell (eq. e4-5)
 *  Qrm     sum of k^3 Q_rm (eqs. e3-20, e3-21, e3-50); the gas takes -Qrm / V_cell in eq. e3-38
 *  Hr      sum over gas species of H_j(T_g) times mdot_j, = -M_r V_cell of eq. e3-39 */
typedef struct {
  double *eps, *np, *sumK, *sumKu, *sumKv, *sumKw, *sumKs, *mdotH2, *mdotH2O, *sumEQ, *sumES;
  double *hA, *hAT, *Qrm, *Hr;
} dem_sources;

/* Kinetic-gradient protocol: n_substeps reaction updates of dt_react, each
 * block of dyn_every substeps preceded by one DEM step and a voidage deposit;
 * the DEM mass stays frozen (the trajectory does not depend on theta).
 * Reaction state is checkpointed every ckpt_every substeps. */
typedef struct {
  int32_t n_substeps;
  double dt_react;
  int32_t dyn_every;
  int32_t ckpt_every;
  int32_t state_fp32; /* 1: FP32 reaction state (FP64 adjoint accumulation); 0: FP64 */
} dem_grad_spec;

typedef struct {
  int64_t n_parcels, n_contacts, n_wall_contacts, rebuilds, steps, clamps;
  double mean_coordination;      /* 2 n_contacts / n_parcels in the last step */
  int32_t max_nbr_used;
  uint32_t status;
  double step_kernel_ms;         /* mean duration of the timed DEM-step kernel launches */
  int64_t step_kernel_launches;  /* launches behind step_kernel_ms (see dem_profile) */
  int32_t step_block;            /* launch shape in use (dem_autotune): step-kernel block size, */
  int32_t step_xcd;              /* blocks per XCD chunk (1: plain round-robin), */
  int32_t build_grid;            /* persistent grid of the neighbour build, */
  int32_t check_period;          /* steps between neighbour-list checks (check_every) */
  int32_t build_threads;         /* neighbour build in use: threads per block, */
  int32_t build_tile;            /* LDS tile (candidate records staged at a time), */
  int32_t build_item_x;          /* DEM cells along x per work item */
  int32_t tune_cached;           /* 1: the shapes came from the autotuner cache */
} dem_stats;

/* Create a context holding n parcels.  Copies the parcel state (device, original
 * order) into internal cell-sorted storage, computes parcel masses (eq. e3-4)
 * and the voidage at t = 0.  stream: a hipStream_t (NULL = default stream).
 * Synchronises once.  Errors: EINVAL (nulls, n <= 0, bad params or grid),
 * ENOMEM, EDOMAIN (a parcel outside its bed's grid). */
int dem_init(const dem_params *p, const dem_parcels *in, int32_t n, void *stream, dem_ctx **out);

/* Advance n_steps DEM steps with the gas frozen (eq. e3-3, e3-6; semi-implicit
 * Euler): contact detection, soft-sphere parcel-parcel and parcel-wall forces,
 * Gidaspow drag with the voidage of the last deposit, gravity and -V grad p.
 * The neighbour lists are checked at every step count that is a multiple of
 * check_every (right after the step that reaches it, or before the next step
 * when that count has not been checked yet) and rebuilt on the device when
 * the displacement bound requires it (no host synchronisation);
 * a step that still finds a parcel moved by skin/2 since the last build
 * latches DEMRX_ESKIN.  The per-cell drag rows (gas velocity, voidage,
 * pressure gradient, density, viscosity) are computed once per call; right
 * after a coupling deposit only for each bed's gas layers that parcels can
 * reach in n_steps steps (the occupied layers widened by
 * (n_steps / check_every + 3) skin / 2 and one layer), else for every cell. */
int dem_step(dem_ctx *c, int32_t n_steps, const dem_gas *g);

/* Coupling deposit (eqs. e3-25, e3-27a, e4-1): voidage and drag sums per gas
 * cell from the current parcel state; the new voidage is used by later steps. */
int dem_couple(dem_ctx *c, const dem_gas *g, dem_sources *out);

/* Reaction update over dt_cfd (eqs. e2-1..e2-36, e3-1..e3-4, e3-52): the
 * multi-interface unreacted-shrinking-core rates of every parcel, the species
 * and mass update and the cell sources mdotH2, mdotH2O, sumEQ, sumES; with
 * energy_on also each parcel's reaction heat k^3 (Q_r + Q_rm) and heat
 * capacity m C_p,p (eq. e3-9), held by the DEM steps until the next update,
 * and the heat sums hA, hAT, Qrm, Hr.
 * bed_fov (host, n_beds doubles, may be NULL): bed-mean overall reduction
 * degree weighted by k^3 N_Fe (eqs. e2-18/e2-19); when given, the call
 * synchronises.  fov (device, n doubles, original order, may be NULL):
 * per-parcel overall reduction degree. */
int dem_react(dem_ctx *c, double dt_cfd, const dem_gas *g, dem_sources *out, double *bed_fov,
              double *fov);

/* Gas-side step of the two-way coupling for species (eq. e3-40 with the
 * semi-implicit sources of eqs. e4-9..e4-11), on the frozen flow of g: one
 * explicit step dt of H2 and H2O by first-order upwind convection along z
 * (face velocity the mean of the two cells' wg; xin = true mole fractions of
 * H2 and H2O (host, 2 doubles) entering through each bed's floor; zero
 * gradient at the lid), with the particle sources of the last dem_react:
 * H2 semi-implicit through C0 = sumEQ / V_cell and C1 = -(M_H2 / R) sumES /
 * V_cell, the H2 taken returned as H2O one to one in moles.  eps_g is the
 * voidage of the last deposit; T and p stay frozen.  Molecular and
 * pseudo-turbulent diffusion and the momentum and energy coupling belong to
 * the gas solver and are not modelled.  sumEQ, sumES: device, one double per
 * gas cell (as written by dem_react).  Writes the new true mole fractions to
 * xH2, xH2O, xN2 (device, one double per cell, distinct from g's arrays; the
 * caller copies them into its gas fields for the next interval).  A Courant
 * number |w| dt / h above one is reported as EINVAL by the next
 * synchronising call.  Errors: EINVAL (nulls, dt <= 0, xin outside [0, 1]). */
int dem_gas_species(dem_ctx *c, double dt, const dem_gas *g, const double *sumEQ, const double *sumES,
                    const double xin[2], double *xH2, double *xH2O, double *xN2);

/* Gas-side momentum step of the two-way coupling: one step dt of the gas
 * velocity of every cell on the frozen pressure field (eqs. e4-1, e4-2 with
 * the interphase source of eqs. e3-27, e3-27a),
 *   eps rho (u' - u) / dt = -eps grad p + eps rho g + K_gp u' - K_gp u_p,
 * the source K_gp u_g implicit and K_gp u_p explicit, where K_gp = -sumK /
 * V_cell and K_gp u_p = -(sumKu, sumKv, sumKw) / V_cell are the drag sums of
 * a dem_couple (device, one double per gas cell): the gas takes exactly the
 * drag the parcels feel.  eps is the voidage of the last deposit, rho that of
 * eq. e3-53 at the cell's T, p and composition, g the gravity of dem_params.
 * Convection and the viscous and pseudo-turbulent stresses belong to the gas
 * solver and are not modelled.  Writes the new velocities to ug, vg, wg
 * (device, one double per cell; each cell reads only itself, so they may be
 * g's own velocity arrays).  Errors: EINVAL (nulls, dt <= 0); a non-finite
 * result is reported by the next synchronising call. */
int dem_gas_momentum(dem_ctx *c, double dt, const dem_gas *g, const double *sumK, const double *sumKu,
                     const double *sumKv, const double *sumKw, double *ug, double *vg, double *wg);

/* Gradient of the bed-mean reduction degree J (all parcels, weight k^3 N_Fe)
 * after the protocol of spec with respect to theta (used for every bed) by a
 * reverse (adjoint) sweep with checkpointing; grad may be NULL for a plain
 * forward run.  J and grad are host pointers; the call synchronises.  The DEM
 * and reaction state of the context are left unchanged. */
int dem_grad(dem_ctx *c, const dem_grad_spec *s, const dem_gas *g, const double theta[6], double *J,
             double *grad);

/* Total force and torque (device, 3 n doubles each, original order, [3 i + axis])
 * that the next DEM step applies; the state is not changed. */
int dem_forces(dem_ctx *c, const dem_gas *g, double *F, double *T);

/* Copy the parcel state into caller arrays (original order; only non-null
 * members of out are written; d, k, ore, bed are ignored).  Synchronises. */
int dem_get_state(dem_ctx *c, dem_parcels *out);

/* Replace positions, velocities, spins and species (original order, all
 * members required except d, k, ore, bed, which are ignored); masses follow
 * the species; contact histories are cleared (dem_set_contacts restores
 * them).  Synchronises. */
int dem_set_state(dem_ctx *c, const dem_parcels *in);

/* Contact history, for checkpoint and resume: the tangential springs of the
 * contact model (the Cundall spring of the soft-sphere law, which the paper
 * takes from its DEM reference; eqs. e3-42..e3-45 fix the coarse-grained
 * stiffness and damping it acts with).  Host arrays:
 *   ids[2 * cap]  original ids (a, b) of each pair, a < b, ascending (a, b);
 *   xi[3 * cap]   its spring (m), with the contact normal from a to b;
 *   cap           capacity of ids and xi in pairs;
 *   count         pairs written (get: the total, which may exceed cap, in
 *                 which case only cap are written) or given (set);
 *   wall_on[6 n]  1 where parcel id (original order) has a spring on wall w
 *                 (index id * 6 + w; box walls -x, +x, -y, +y, -z, +z;
 *                 cylinder: mantle, bottom, top), else 0;
 *   wall_xi[18 n] that spring, index (id * 6 + w) * 3 + axis (0 if off). */
typedef struct {
  int64_t cap, count;
  uint32_t *ids;
  double *xi;
  uint8_t *wall_on;
  double *wall_xi;
} dem_contacts;

/* Export the springs of the pairs and walls in contact at the last step
 * (both partners of a pair hold the same spring; the record comes from the
 * one with the lower id).  Synchronises.  EINVAL on null arrays. */
int dem_get_contacts(dem_ctx *c, dem_contacts *io);

/* Load springs exported by dem_get_contacts (usually after dem_init or
 * dem_set_state with the same checkpoint): rebuilds the neighbour lists at the
 * current positions and gives every listed pair that still touches its
 * spring, as a rebuild carries springs over.  Pairs that no longer touch
 * drop theirs, as in a step.  Synchronises.  EINVAL unless every pair has
 * a < b < n and every spring is finite; EOVERFLOW (latched) when a parcel is
 * given more pairs than max_nbr. */
int dem_set_contacts(dem_ctx *c, const dem_contacts *in);

/* Contacting pairs at the current positions (exact FP64 test
 * ((dx dx + dy dy) + dz dz) < (r_i + r_j)^2), canonical (i < j by original id),
 * sorted by (i, j), written to the host array ij (2 * cap uint32).  *n_pairs
 * receives the total count (may exceed cap).  Synchronises. */
int dem_pairs(dem_ctx *c, uint32_t *ij, int64_t cap, int64_t *n_pairs);

/* dem_pairs for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same pairs, found through a
 * static device scratch of DEM_NOALLOC_MAX_PAIRS pairs (16 MiB, held by each
 * GPU the library runs on until the process ends) instead of a buffer the
 * context allocates; calls no hipMalloc or hipFree.  The pairs are copied
 * into ij and sorted there, so ij (host, 2 * cap uint32) must hold all of
 * them: *n_pairs always receives the count, and the call returns EINVAL when
 * it exceeds cap and EOVERFLOW when it exceeds DEM_NOALLOC_MAX_PAIRS (ij
 * untouched in both cases).  Calls on one GPU share its scratch: calls that
 * overlap on one GPU (contexts on different streams or threads) race.
 * Synchronises. */
int dem_pairs_noalloc(dem_ctx *c, uint32_t *ij, int64_t cap, int64_t *n_pairs);

/* Counters of the last step (host).  Synchronises. */
int dem_get_stats(dem_ctx *c, dem_stats *out);

/* Replay the full hot path -- couple_every DEM steps with the neighbour-list
 * check (and, when the displacement bound requires it, the rebuild) at every
 * step count that is a multiple of check_every, the coupling deposit and the
 * reaction update (dt_cfd = couple_every * dt) -- n_intervals times from a
 * HIP graph of the fewest intervals whose steps are a multiple of 2 and of
 * check_every, captured on first use (recaptured if the arguments change).
 * Whether a check rebuilds is decided on the device, so the replays need no
 * host synchronisation; a coupling right after a rebuild reuses its sort of
 * the parcels by cell.  out and
 * bed_fov (host) may be NULL; bed_fov receives the values after the last
 * interval and makes the call synchronise. */
int dem_run(dem_ctx *c, int32_t n_intervals, int32_t couple_every, const dem_gas *g,
            dem_sources *out, double *bed_fov);

/* Choose launch shapes for this context's kernels by timing candidates on
 * its own data (state unchanged): the DEM-step block size and XCD chunk (a
 * full step whose springs and contact masks go to internal spare buffers),
 * and the neighbour build's block size, LDS tile and work-item width (whole
 * rebuild chains are timed).  Synchronises.  With the environment variable
 * DEMRX_TUNE_LOG set, every candidate's timing goes to stderr.  With
 * DEMRX_TUNE_CACHE naming a JSON file, shapes stored there under the key of
 * this device architecture and configuration (parcel count, beds and their
 * grids, precision, list capacity, skin, energy equation) are applied without
 * timing, and newly chosen shapes are stored (the file is rewritten). */
int dem_autotune(dem_ctx *c, const dem_gas *g);

/* Set the launch shapes directly (instead of dem_autotune), e.g. to repeat a
 * measurement in a known shape: step_block threads per block of the DEM-step
 * kernel (64, 128, 256 or 512), step_xcd_chunk consecutive blocks kept on one
 * XCD by the block remap (1..64; 1 = no remap), build_grid blocks of the
 * persistent neighbour build (1..65536; 0 = as many as are resident on every
 * compute unit).  Results do not depend on the shapes.  DEMRX_EINVAL outside
 * these ranges (nothing changed).  No device work. */
int dem_set_launch(dem_ctx *c, int32_t step_block, int32_t step_xcd_chunk, int32_t build_grid);

/* Set the neighbour build's shape directly (instead of dem_autotune):
 * threads per block and LDS tile in candidate records, one of 512/2048,
 * 256/1024, 256/2048, 1024/4096, and the work-item width item_x, 8, 16 or 32
 * DEM cells along x.  The lists, and so all results, do not depend on the
 * shape.  DEMRX_EINVAL for other values (nothing changed).  Uploads the work
 * items of a new width on the context's stream. */
int dem_set_build(dem_ctx *c, int32_t threads, int32_t tile, int32_t item_x);

/* Enable (1) or disable (0) HIP-event timing of every DEM-step kernel launch,
 * recorded on the stream the kernel runs on (inside dem_run graphs too: the
 * events of the last replay are kept).  Resets the timings; dem_get_stats
 * reports their mean. */
int dem_profile(dem_ctx *c, int32_t enable);

/* Wait for all work of the context; report a latched device error. */
int dem_sync(dem_ctx *c);
const char *dem_last_error(const dem_ctx *c);
void dem_destroy(dem_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
