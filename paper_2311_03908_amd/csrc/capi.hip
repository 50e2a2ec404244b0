// Host side of the demrx C-ABI: validation, device memory, the rebuild /
// step / coupling sequence, HIP-graph replay of the full hot path and the
// launch-shape autotuner.  Numerics live in the kernel files.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "launch.h"

using namespace demrx;

struct dem_ctx {
  std::string err;
  virtual ~dem_ctx() = default;
  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
  virtual int step(int n, const dem_gas *g) = 0;
  virtual int couple(const dem_gas *g, dem_sources *o) = 0;
  virtual int react(double dt, const dem_gas *g, dem_sources *o, double *bed_fov, double *fov) = 0;
  virtual int gas_species(double dt, const dem_gas *g, const double *eq, const double *es, const double *xin,
                          double *x1, double *x2, double *x3) = 0;
  virtual int gas_momentum(double dt, const dem_gas *g, const double *sK, const double *sKu, const double *sKv,
                           const double *sKw, double *u, double *v, double *w) = 0;
  virtual int forces(const dem_gas *g, double *F, double *T) = 0;
  virtual int get_state(dem_parcels *o) = 0;
  virtual int set_state(const dem_parcels *in) = 0;
  virtual int pairs(uint32_t *ij, int64_t cap, int64_t *np) = 0;
  virtual int pairs_noalloc(uint32_t *ij, int64_t cap, int64_t *np) = 0;
  virtual int get_contacts(dem_contacts *io) = 0;
  virtual int set_contacts(const dem_contacts *in) = 0;
  virtual int stats(dem_stats *o) = 0;
  virtual int run(int n_int, int S, const dem_gas *g, dem_sources *o, double *bed_fov) = 0;
  virtual int autotune(const dem_gas *g) = 0;
  virtual int set_launch(int step_block, int step_xcd_chunk, int build_grid) = 0;
  virtual int set_build(int threads, int tile, int item_x) = 0;
  virtual int grad(const dem_grad_spec *s, const dem_gas *g, const double *theta, double *J, double *grad) = 0;
  virtual int profile(int enable) = 0;
  virtual int sync() = 0;
};

// Scratch of dem_pairs_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends) holding the pair
// counter in its first 256 bytes and up to DEM_NOALLOC_MAX_PAIRS pairs after
// it.  Host code uses only the address hipGetSymbolAddress returns for the
// current device (taken once per device at dem_init), never the symbol itself.
static __device__ __align__(256) unsigned char scratch[256 + (size_t)DEM_NOALLOC_MAX_PAIRS * 8];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the scratch address of the current device (resolved once per device)
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(DEMRX_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

GasArgs gas_args(const dem_gas *g) {
  GasArgs a;
  a.ug = g->ug; a.vg = g->vg; a.wg = g->wg; a.p = g->p;
  a.dpdx = g->dpdx; a.dpdy = g->dpdy; a.dpdz = g->dpdz; a.T = g->T;
  a.xH2 = g->xH2; a.xH2O = g->xH2O; a.xN2 = g->xN2;
  return a;
}

bool gas_ok(const dem_gas *g) {
  return g && g->ug && g->vg && g->wg && g->p && g->dpdx && g->dpdy && g->dpdz && g->T && g->xH2 && g->xH2O && g->xN2;
}

// Porosities of the product layers (eqs. e2-31..e2-36): effective densities
// scale by q_b,a = |eta_b| M_b / (|eta_a| M_a) down the Fe2O3 -> Fe3O4 -> FeO
// -> Fe chain.
OreDev make_ore(const dem_ore &o) {
  const double Mh = 159.687, Mm = 231.531, Mw = 71.844, Mf = 55.845;
  const double qmh = 2.0 * Mm / (3.0 * Mh), qwm = 3.0 * Mw / Mm, qfw = Mf / Mw;
  const double reh = (1.0 - o.xi0) * o.rho_true[0];
  const double rem = reh * qmh, rew = rem * qwm, ref = rew * qfw;
  OreDev d;
  d.xi_layer[0] = 1.0 - rem / o.rho_true[1];
  d.xi_layer[1] = 1.0 - rew / o.rho_true[2];
  d.xi_layer[2] = 1.0 - ref / o.rho_true[3];
  d.d_pore_cm = o.d_pore_cm;
  d.tau = o.tau;
  d.kind = o.kind;
  d.psi = o.psi;
  d.k1_shape = o.psi > 0.0 ? 1.0 / (1.0 / 3.0 + 2.0 / 3.0 / std::sqrt(o.psi)) : 0.0;
  d.k2 = o.psi > 0.0 ? std::pow(10.0, 1.8148 * std::pow(-std::log10(o.psi), 0.5743)) : 0.0;
  return d;
}

int status_code(uint32_t st) {
  if (st & 16u) return DEMRX_EINVAL;
  if (st & ST_NONFINITE) return DEMRX_ENONFINITE;
  if (st & ST_DOMAIN) return DEMRX_EDOMAIN;
  if (st & ST_OVERFLOW) return DEMRX_EOVERFLOW;
  if (st & ST_SKIN) return DEMRX_ESKIN;
  return DEMRX_OK;
}
const char *status_text(uint32_t st) {
  if (st & 16u) return "invalid parcel input (bed/ore index out of range, non-positive diameter or k < 1)";
  if (st & ST_NONFINITE) return "non-finite parcel state or gas field";
  if (st & ST_DOMAIN) return "a parcel centre lies outside its bed's gas grid";
  if (st & ST_OVERFLOW) return "neighbour candidates exceed max_nbr (or a stencil plane exceeds the LDS tile)";
  if (st & ST_SKIN) return "displacement bound since the last neighbour build exceeded skin/2";
  return "";
}

}  // namespace

template <typename T>
struct Ctx final : dem_ctx {
  dem_params P{};
  std::vector<dem_bed> hbeds;
  std::vector<dem_ore> hores;
  std::vector<BedDev> hbd;
  Phys ph{};
  int n = 0, n_gas = 0, n_keys = 0, n_items = 0, n_items_max = 0;
  hipStream_t st = nullptr, user_st = nullptr, cap_st = nullptr;
  std::vector<void *> allocs;
  BedDev *beds = nullptr;
  OreDev *ores = nullptr;
  int32_t *cell_bed = nullptr;
  Item *items = nullptr;
  Dyn<T> dyn[2]{};  // step buffers: a step reads dyn[cur] and writes dyn[cur ^ 1]
  Props<T> pr{}, pr_sp{};  // properties and the spare the rebuild permutes into
  Nbr<T> nb{};
  Spring<T> *carry = nullptr;      // springs carried across a rebuild (launch_permute)
  uint64_t *carry_mask = nullptr;  // old contact masks by new position (launch_permute)
  uint32_t *rb_flag = nullptr;     // set by the rebuild check: [0] rebuild at this check point, [1] its complement
  unsigned long long *rb_count = nullptr;  // rebuilds done (device counter)
  int cur = 0;
  int32_t *key = nullptr, *slot = nullptr, *count = nullptr, *start = nullptr, *perm = nullptr, *scan_scr = nullptr;
  int32_t *perm2 = nullptr;
  CellOrd cord{};  // cell-ordered x, id, key of the last scatter
  // cell order of the current positions for the deposits (refreshed at every
  // coupling without permuting the parcels or rebuilding neighbour lists)
  int32_t *start_d = nullptr, *order_d = nullptr;
  bool dep_fresh = false;
  bool occ_fresh = false;  // occupied-cell list of the current cell order
  int32_t *occ_flags = nullptr, *occ_offs = nullptr, *occ_list = nullptr, *occ_count = nullptr;
  int4 *bchunks = nullptr;
  bool bchunks_ready = false;  // chunk table of the bed means built (it never changes)
  double *bpartial = nullptr;
  int max_chunks = 0;
  int32_t *ilist = nullptr, *icount = nullptr;  // work items holding parcels; [0] count, [1] build queue
  int32_t *ibcount = nullptr;                    // items holding parcels per 256 (launch_items)
  T *gtab = nullptr;
  ThermoTab *thermo = nullptr;    // energy equation only
  const double *gas_T = nullptr;  // gas temperature of the last gas table (energy equation)
  double *rtab = nullptr;  // per-cell reaction quantities (launch_react_table)
  int2 *zrange = nullptr;  // per bed, the gas layers the drag table covers
  double *eps = nullptr, *pm = nullptr, *pw = nullptr, *bed_fov_d = nullptr, *theta_d = nullptr;
  uint32_t *status = nullptr;
  void *scratch_ptr = nullptr;       // this device's static scratch (dem_pairs_noalloc)
  float4 *xref = nullptr;            // positions at the last rebuild
  unsigned *dslot = nullptr;         // per-step displacement maxima (kSlots x 2, padded)
  unsigned long long *cslot = nullptr;  // contact counts of the counted step (kSlots, padded)

  unsigned long long *counters = nullptr;  // pp contacts, wall contacts, clamps, pairs
  uint32_t *pairs_buf = nullptr;
  long pairs_cap = 0;
  long step_count = 0;
  bool built = false;
  // step count of the last rebuild check: while no step has followed it,
  // rb_flag tells whether the parcels were sorted at the current positions
  long chain_step = -1;
  int step_block = 64, step_xcd = 1;
  // neighbour build: variant (block size, LDS tile), item width, grid
  // (0: resident blocks per CU x CUs)
  int build_variant = 0, item_x = 16, build_grid = 0;
  int n_cu = 256;
  std::string arch;
  bool tune_cached = false;
  std::vector<Item> hitems;  // host copy of the work items (kept alive for the async upload)
  int bpc[kBuildVariants] = {0, 0, 0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const void *> gkey;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  // step-kernel timing: event pairs of eager launches and of the captured graph
  bool prof = false, capturing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_eager, prof_graph, prof_capture;

  ~Ctx() override {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (cap_st) (void)hipStreamDestroy(cap_st);
    for (void *p : allocs) (void)hipFree(p);
    if (gscr.base) (void)hipFree(gscr.base);
  }

  template <typename P_>
  int dalloc(P_ *&p, size_t cnt) {
    void *q = nullptr;
    if (cnt == 0) cnt = 1;
    if (hipMalloc(&q, cnt * sizeof(P_)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DEMRX_ENOMEM, "device allocation of " + std::to_string(cnt * sizeof(P_)) + " bytes failed");
    }
    allocs.push_back(q);
    p = (P_ *)q;
    return DEMRX_OK;
  }

#define TRY(x)                 \
  do {                         \
    int r_ = (x);              \
    if (r_ != DEMRX_OK) return r_; \
  } while (0)

  int alloc_dyn(Dyn<T> &d) {
    TRY(dalloc(d.pos, n));
    TRY(dalloc(d.vel, n));
    return DEMRX_OK;
  }
  int alloc_props(Props<T> &p, const Props<T> *shared) {
    TRY(dalloc(p.kcg, n)); TRY(dalloc(p.tag, n));
    TRY(dalloc(p.nh, n)); TRY(dalloc(p.nm, n)); TRY(dalloc(p.nw, n)); TRY(dalloc(p.nfe, n));
    if (P.energy_on) {
      TRY(dalloc(p.Tp, n)); TRY(dalloc(p.qrx, n)); TRY(dalloc(p.mcp, n));
    }
    if (shared) {  // wall springs are indexed by original id: one copy
      p.wh = shared->wh;
      return DEMRX_OK;
    }
    TRY(dalloc(p.wh, (size_t)3 * kMaxWalls * n));
    return DEMRX_OK;
  }
  int alloc_nbr(Nbr<T> &b) {
    TRY(dalloc(b.cnt, n));
    TRY(dalloc(b.idx, (size_t)kMaxNbr * n));
    TRY(dalloc(b.hist, (size_t)kMaxNbr * n));
    TRY(dalloc(b.mask, n));
    TRY(dalloc(carry, (size_t)kMaxNbr * n));
    TRY(dalloc(carry_mask, n));
    return DEMRX_OK;
  }

  int init(const dem_params *p, const dem_parcels *in, int n_, hipStream_t s) {
    HIPCHK(scratch_address(&scratch_ptr));
    P = *p;
    n = n_;
    user_st = st = s;
    hbeds.assign(p->beds, p->beds + p->n_beds);
    hores.assign(p->ores, p->ores + p->n_ores);
    P.beds = nullptr;
    P.ores = nullptr;
    ph.kn = p->kn; ph.e_p = p->e_p; ph.mu_s = p->mu_s; ph.mu_r = p->mu_r;
    ph.kt = p->kt_over_kn * p->kn; ph.gt_ratio = p->gt_over_gn; ph.eps_min = p->eps_min;
    ph.skin = p->skin; ph.dt = p->dt;
    for (int a = 0; a < 3; a++) ph.g[a] = p->g[a];
    ph.ergun_printed = p->ergun_printed; ph.drag_on = p->drag_on;
    ph.n_beds = p->n_beds; ph.n_ores = p->n_ores; ph.max_nbr = p->max_nbr;
    ph.ganser = 0;
    for (int o = 0; o < p->n_ores; o++) ph.ganser |= p->ores[o].psi > 0.0;
    ph.energy = p->energy_on != 0;
    if (p->energy_on && !in->Tp) return fail(DEMRX_EINVAL, "energy_on needs the particle temperatures Tp");
    // beds
    long goff = 0, doff = 0, items_total = 0;
    for (int b = 0; b < p->n_beds; b++) {
      const dem_bed &B = hbeds[b];
      BedDev d{};
      for (int a = 0; a < 3; a++) {
        d.lo[a] = B.lo[a]; d.hi[a] = B.hi[a]; d.origin[a] = B.origin[a];
        d.n[a] = B.n[a]; d.nd[a] = B.n[a] * B.refine;
      }
      d.R = B.R;
      d.dbed = B.wall_kind == DEM_WALL_CYL ? 2.0 * B.R
                                           : std::sqrt(4.0 * (B.hi[0] - B.lo[0]) * (B.hi[1] - B.lo[1]) / M_PI);
      d.cx = 0.5 * (B.lo[0] + B.hi[0]);
      d.cy = 0.5 * (B.lo[1] + B.hi[1]);
      d.h = B.h;
      d.hd = B.h / B.refine;
      d.refine = B.refine;
      d.wall_kind = B.wall_kind;
      d.n_walls = B.wall_kind == DEM_WALL_BOX ? 6 : 3;
      d.gas_off = (int)goff;
      d.dem_off = (int)doff;
      d.n_gas = B.n[0] * B.n[1] * B.n[2];
      // key tiles (see dem_key): one tile per bed plane (row-major keys).
      // Columns of 16 x 16 cells measured no faster on the 2M-parcel bed.
      // The neighbour build relies on this: the cells of a bed row have
      // consecutive keys, so a row is one run of the sorted order.
      d.tx = d.nd[0];
      d.ty = d.nd[1];
      d.ntx = (d.nd[0] + d.tx - 1) / d.tx;
      const long nty = (d.nd[1] + d.ty - 1) / d.ty;
      const long n_dem = (long)d.ntx * d.tx * nty * d.ty * d.nd[2];
      if (n_dem > (1L << 30)) return fail(DEMRX_EINVAL, "grid too large");
      d.n_dem = (int)n_dem;
      for (int q = 0; q < 6; q++) d.theta[q] = B.theta[q];
      d.mu_override = B.mu_override;
      goff += d.n_gas;
      doff += d.n_dem;
      // work items of the narrowest width (the most items any width makes)
      items_total += (long)d.nd[1] * d.nd[2] * ((d.nd[0] + kItemWidths[0] - 1) / kItemWidths[0]);
      hbd.push_back(d);
    }
    if (goff > (1L << 30) || doff > (1L << 30) || items_total > (1L << 30))
      return fail(DEMRX_EINVAL, "grid too large");
    n_gas = (int)goff;
    n_keys = (int)doff;
    n_items_max = (int)items_total;
    std::vector<OreDev> hod;
    for (auto &o : hores) hod.push_back(make_ore(o));
    std::vector<int32_t> hcb(n_gas);
    for (int b = 0; b < p->n_beds; b++) {
      const BedDev &d = hbd[b];
      for (int c = 0; c < d.n_gas; c++) hcb[d.gas_off + c] = b;
    }
    // largest parcel per bed against the DEM cell (checked on the host once)
    {
      std::vector<float> hd(n);
      std::vector<int32_t> hb(n);
      HIPCHK(hipMemcpyAsync(hd.data(), in->d, n * sizeof(float), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hb.data(), in->bed, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::vector<double> dmax(p->n_beds, 0.0);
      for (int i = 0; i < n; i++)
        if (hb[i] >= 0 && hb[i] < p->n_beds) dmax[hb[i]] = std::max(dmax[hb[i]], (double)hd[i]);
      for (int b = 0; b < p->n_beds; b++) {
        if (hbd[b].hd < dmax[b] + p->skin)
          return fail(DEMRX_EINVAL, "bed " + std::to_string(b) + ": DEM cell " + std::to_string(hbd[b].hd) +
                                        " m is smaller than the largest parcel plus skin (" +
                                        std::to_string(dmax[b] + p->skin) + " m)");
        hbd[b].rmax = 0.5 * dmax[b];
      }
    }
    TRY(dalloc(beds, hbd.size()));
    TRY(dalloc(ores, hod.size()));
    TRY(dalloc(cell_bed, n_gas));
    TRY(dalloc(items, n_items_max));
    for (int k = 0; k < 2; k++) TRY(alloc_dyn(dyn[k]));
    TRY(alloc_props(pr, nullptr));
    TRY(alloc_props(pr_sp, &pr));
    TRY(alloc_nbr(nb));
    TRY(dalloc(rb_flag, 2));
    TRY(dalloc(rb_count, 1));
    TRY(dalloc(key, n)); TRY(dalloc(slot, n)); TRY(dalloc(perm, n)); TRY(dalloc(perm2, n));
    TRY(dalloc(cord.x, n)); TRY(dalloc(cord.id, n)); TRY(dalloc(cord.key, n));
    max_chunks = n / kBedChunk + p->n_beds + 2;
    TRY(dalloc(bchunks, max_chunks));
    TRY(dalloc(bpartial, 2 * (size_t)max_chunks));
    TRY(dalloc(count, (size_t)n_keys + 1)); TRY(dalloc(start, (size_t)n_keys + 1));
    TRY(dalloc(start_d, (size_t)n_keys + 1)); TRY(dalloc(order_d, n));
    TRY(dalloc(occ_flags, (size_t)n_gas + 1)); TRY(dalloc(occ_offs, (size_t)n_gas + 1));
    TRY(dalloc(occ_list, n_gas)); TRY(dalloc(occ_count, 1));
    TRY(dalloc(scan_scr, scan_scratch_ints((long)n_keys + 1)));
    TRY(dalloc(ilist, n_items_max)); TRY(dalloc(icount, 2)); TRY(dalloc(ibcount, n_items_max / 256 + 1));
    TRY(dalloc(gtab, (size_t)n_gas * kGasRow));
    TRY(dalloc(eps, n_gas));
    TRY(dalloc(zrange, hbd.size()));
    TRY(dalloc(rtab, (size_t)n_gas * kReactRow));
    TRY(dalloc(pm, (size_t)(P.energy_on ? 8 : 4) * n)); TRY(dalloc(pw, (size_t)2 * n));
    if (P.energy_on) {
      TRY(dalloc(thermo, 1));
      static const ThermoTab tt = make_thermo();
      HIPCHK(hipMemcpyAsync(thermo, &tt, sizeof(ThermoTab), hipMemcpyHostToDevice, st));
    }
    TRY(dalloc(bed_fov_d, p->n_beds)); TRY(dalloc(theta_d, 6));
    TRY(dalloc(status, 1)); TRY(dalloc(counters, 4)); TRY(dalloc(xref, n));
    TRY(dalloc(dslot, 2 * kSlots * kSlotPad)); TRY(dalloc(cslot, kSlots * kSlotPad64));
    HIPCHK(hipMemcpyAsync(beds, hbd.data(), hbd.size() * sizeof(BedDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ores, hod.data(), hod.size() * sizeof(OreDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(cell_bed, hcb.data(), hcb.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    TRY(upload_items(item_x));
    {
      int dev = 0;
      hipDeviceProp_t prop;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipGetDeviceProperties(&prop, dev));
      n_cu = std::max(1, prop.multiProcessorCount);
      arch = prop.gcnArchName;
    }
    launch_fill_u32((uint32_t *)nb.mask, 0u, 2L * n, st);
    launch_fill_i32(nb.cnt, 0, n, st);
    launch_fill_u32((uint32_t *)rb_count, 0u, 2, st);
    launch_fill_u32(status, 0u, 1, st);
    launch_fill_u32(dslot, 0u, 2 * kSlots * kSlotPad, st);
    launch_fill_u32((uint32_t *)cslot, 0u, 2 * kSlots * kSlotPad64, st);
    launch_fill_u32((uint32_t *)counters, 0u, 8, st);
    launch_fill_i32(count, 0, (long)n_keys + 1, st);  // cell counters: zero between sorts
    launch_init<T>(*in, n, ph, p->n_ores, thermo, dyn[0], pr, status, st);
    HIPCHK(hipGetLastError());
    TRY(check_status());
    TRY(rebuild_chain(1, true));
    TRY(resort());
    DepositOut o{};
    o.eps_ctx = eps;
    TRY(deposit(GasArgs{}, false, o));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return check_status();
  }

  int check_status() {
    uint32_t h = 0;
    HIPCHK(hipMemcpy(&h, status, sizeof h, hipMemcpyDeviceToHost));
    if (h) {
      launch_fill_u32(status, 0u, 1, st);
      return fail(status_code(h), status_text(h));
    }
    return DEMRX_OK;
  }

  int sync() override {
    HIPCHK(hipStreamSynchronize(st));
    return check_status();
  }

  // Neighbour-list rebuild check and the rebuild chain behind it.  The check
  // kernel sets rb_flag when the lists could go stale within `horizon` steps
  // (or when forced); every kernel of the chain returns at once when it is
  // clear, so the chain's place in a captured graph is fixed while whether it
  // runs is decided on the device.  A rebuild sorts the parcels by DEM cell
  // (bin, scan, scatter, in-cell rank), permutes the state through the spare
  // buffers back into dyn[cur] and pr (moving the contact springs to the new
  // positions on the way), and builds the lists; no buffer parity changes.
  // Work items of `width` DEM cells along x, in key order (row by row), so
  // that the persistent build blocks work on neighbouring cells at a time.
  int upload_items(int width) {
    hitems.clear();
    for (size_t b = 0; b < hbd.size(); b++) {
      const BedDev &d = hbd[b];
      for (int iz = 0; iz < d.nd[2]; iz++)
        for (int iy = 0; iy < d.nd[1]; iy++)
          for (int x0 = 0; x0 < d.nd[0]; x0 += width) hitems.push_back(Item{(int)b, x0, iy, iz});
    }
    if ((long)hitems.size() > n_items_max) return fail(DEMRX_EINVAL, "internal: work-item count");
    n_items = (int)hitems.size();
    item_x = width;
    HIPCHK(hipMemcpyAsync(items, hitems.data(), hitems.size() * sizeof(Item), hipMemcpyHostToDevice, st));
    return DEMRX_OK;
  }
  int build_grid_now() {
    if (build_grid > 0) return std::max(1, std::min(n_items, build_grid));
    if (!bpc[build_variant]) bpc[build_variant] = build_blocks_per_cu<T>(build_variant);
    return std::max(1, std::min(n_items, bpc[build_variant] * n_cu));
  }
  int rebuild_chain(int horizon, bool force) {
    const uint32_t *G = rb_flag;
    chain_step = step_count;
    launch_rebuild_check(dslot, (int)((step_count & 1) ^ 1), P.skin, P.dt, horizon, force ? 1 : 0, rb_flag,
                         rb_count, icount, st);
    // the cell counters are zero here: every scan of them clears them
    launch_bin<T>(dyn[cur], pr, beds, n, key, slot, count, status, st, G);
    launch_scan(count, start, (long)n_keys + 1, scan_scr, st, G, true);
    launch_scatter(key, slot, start, dyn[cur].pos, n, perm2, cord, st, G);
    launch_cellrank(start, perm2, cord, n, perm, st, G);
    launch_permute<T>(perm, n, dyn[cur], pr, dyn[cur ^ 1], pr_sp, xref, dslot, nb, carry, carry_mask, st, G);
    launch_items(items, n_items, item_x, beds, start, ibcount, ilist, icount, st, G);
    NbrBuild<T> a;
    a.d = dyn[cur];
    a.p = pr;
    a.nb = nb;
    a.carry = carry;
    a.carry_mask = carry_mask;
    a.gate = G;
    a.beds = beds;
    a.start = start;
    a.items = items;
    a.list = ilist;
    a.list_count = icount;
    a.n = n;
    a.cap = P.max_nbr;
    a.item_x = item_x;
    a.skin = P.skin;
    a.status = status;
    a.queue = icount + 1;  // zeroed by the check
    launch_build_nbr<T>(a, build_variant, build_grid_now(), st);
    HIPCHK(hipGetLastError());
    built = true;
    dep_fresh = false;  // the parcels may have moved in memory
    return DEMRX_OK;
  }

  // Cell order of the current positions (bin, scan, scatter, in-cell rank):
  // the parcels stay where they are; deposits and cell sums read them through
  // order_d.  Deterministic like the full sort.  Right after a rebuild check
  // (no step since), a rebuild has left the parcels in exactly this order
  // when it ran: then the sort is skipped on the device and the order is
  // the identity over the rebuild's cell offsets.
  int resort() {
    const uint32_t *G = chain_step == step_count ? rb_flag + 1 : nullptr;
    if (G) launch_cell_identity(order_d, n, start, start_d, (long)n_keys + 1, st, rb_flag);
    launch_bin<T>(dyn[cur], pr, beds, n, key, slot, count, status, st, G);
    launch_scan(count, start_d, (long)n_keys + 1, scan_scr, st, G, true);
    launch_scatter(key, slot, start_d, dyn[cur].pos, n, perm2, cord, st, G);
    launch_cellrank(start_d, perm2, cord, n, order_d, st, G);
    HIPCHK(hipGetLastError());
    dep_fresh = true;
    occ_fresh = false;
    return DEMRX_OK;
  }

  int ensure_dep() {
    if (!built) TRY(rebuild_chain(1, true));
    if (!dep_fresh) TRY(resort());
    return DEMRX_OK;
  }

  // voidage (and drag sums) of every gas cell from the current cell order:
  // empty cells directly, occupied cells through their compacted list
  int deposit(const GasArgs &g, bool sums, const DepositOut &o) {
    launch_occupied(start_d, cell_bed, bsel(), n_gas, sums, o, occ_flags, occ_offs, scan_scr, occ_list, occ_count, st);
    occ_fresh = true;
    launch_deposit<T>(dyn[cur], pr, g, start_d, order_d, cell_bed, bsel(), ores, ph, occ_list, occ_count, n_gas,
                      sums, o, st);
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  // Occupied cells of the current positions (voidage untouched).
  int ensure_occ() {
    TRY(ensure_dep());
    if (!occ_fresh) {
      launch_occupied(start_d, cell_bed, bsel(), n_gas, false, DepositOut{}, occ_flags, occ_offs, scan_scr, occ_list,
                      occ_count, st);
      occ_fresh = true;
    }
    return DEMRX_OK;
  }

  // The drag table.  With a horizon (the steps it serves) and an occupied
  // list of the current positions, only each bed's layers that parcels can
  // reach are computed: within h steps, with the lists checked every C
  // steps, a parcel moves less than (h / C + 3) skin / 2 (at most h / C + 1
  // rebuilds, each window held below skin / 2 by the step's own check, plus
  // the window running at the start).  Otherwise every row is computed.
  int gas_table(const dem_gas *g, int horizon = -1) {
    const int2 *zr = nullptr;
    if (horizon >= 0 && occ_fresh && dep_fresh) {
      const double reach = ((double)(horizon / check_period()) + 3.0) * 0.5 * P.skin;
      launch_occ_zrange(occ_list, occ_count, beds, P.n_beds, reach, zrange, st);
      zr = zrange;
    }
    launch_gas_table<T>(gas_args(g), eps, cell_bed, beds, thermo, n_gas, zr, gtab, status, st);
    gas_T = g->T;
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  BedSel bsel() const {
    BedSel b;
    b.beds = beds;
    b.n_beds = (int)hbd.size();
    b.one = hbd[0];
    return b;
  }

  StepArgs<T> step_args(int mode) {
    StepArgs<T> a;
    a.in = dyn[cur];
    a.out = dyn[cur ^ 1];
    a.pr = pr;
    a.nb = nb;
    a.gtab = gtab;
    a.beds = beds;
    a.ores = ores;
    a.ph = ph;
    a.bed0 = hbd[0];
    a.status = status;
    a.Tg = gas_T;
    a.xref = xref;
    a.dslot = dslot;
    a.cslot = cslot;
    a.count = 0;
    a.n = n;
    a.par = (int)(step_count & 1);
    a.mode = mode;
    a.xcd = step_xcd;
    a.Fout = a.Tout = nullptr;
    a.hist_w = mode == 2 ? carry : nb.hist;
    a.mask_w = mode == 2 ? carry_mask : nb.mask;
    return a;
  }

  int new_event(hipEvent_t &e) {
    HIPCHK(hipEventCreate(&e));
    ev_pool.push_back(e);
    return DEMRX_OK;
  }

  int profile(int enable) override {
    prof = enable != 0;
    prof_eager.clear();
    prof_graph.clear();
    return DEMRX_OK;
  }

  // The lists are checked at every step count that is a multiple of
  // check_every: right after the step that reaches it (so that a coupling
  // there finds the parcels sorted when they were rebuilt), or before the
  // next step when no check has run at that count yet.  Eager calls and
  // graphs take the same decisions.
  int check_period() const { return std::max(1, P.check_every); }
  bool check_due() const { return !built || step_count % check_period() == 0; }
  // steps from a due check to the next one
  int check_horizon() const { return check_period() - (int)(step_count % check_period()); }

  // One DEM step (the lists must be valid for it).
  int step_one(bool count = false) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
      auto &lst = capturing ? prof_capture : prof_eager;
      if (!capturing && lst.size() >= 65536) return fail(DEMRX_EINVAL, "profile buffer full; call dem_get_stats");
      TRY(new_event(e0));
      TRY(new_event(e1));
      HIPCHK(hipEventRecord(e0, st));
      lst.emplace_back(e0, e1);
    }
    StepArgs<T> sa = step_args(0);
    sa.count = count ? 1 : 0;
    launch_step<T>(sa, step_block, st);
    HIPCHK(hipGetLastError());
    if (prof) HIPCHK(hipEventRecord(e1, st));
    cur ^= 1;
    step_count++;
    dep_fresh = false;
    return DEMRX_OK;
  }

  // One step with the list check in front of it when one is due.
  int step_checked(bool count = false) {
    if (check_due() && chain_step != step_count) TRY(rebuild_chain(check_horizon(), !built));
    TRY(step_one(count));
    if (check_due()) TRY(rebuild_chain(check_horizon(), false));
    return DEMRX_OK;
  }

  int step(int ns, const dem_gas *g) override {
    if (ns < 0) return fail(DEMRX_EINVAL, "n_steps < 0");
    if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
    if (ns == 0) return DEMRX_OK;
    TRY(gas_table(g, ns));
    for (int s = 0; s < ns; s++) {
      if (s == ns - 1) launch_fill_u32((uint32_t *)cslot, 0u, 2 * kSlots * kSlotPad64, st);
      TRY(step_checked(s == ns - 1));
    }
    return DEMRX_OK;
  }

  // Lists valid for the current positions (check with a one-step horizon).
  int ensure_lists() { return rebuild_chain(1, !built); }

  int couple(const dem_gas *g, dem_sources *o) override {
    if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
    TRY(ensure_dep());
    DepositOut d{};
    d.eps_ctx = eps;
    bool sums = false;
    if (o) {
      d.eps = o->eps; d.np = o->np; d.sumK = o->sumK; d.sumKu = o->sumKu; d.sumKv = o->sumKv;
      d.sumKw = o->sumKw; d.sumKs = o->sumKs;
      sums = o->sumK || o->sumKu || o->sumKv || o->sumKw || o->sumKs;
    }
    TRY(deposit(gas_args(g), sums, d));
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  int react_core(double dt, const dem_gas *g, dem_sources *o, double *fov, bool bed_sum, int update_mass,
                 const double *theta_dev) {
    TRY(ensure_dep());
    ReactArgs<T> a;
    a.d = dyn[cur];
    a.p = pr;
    a.g = gas_args(g);
    a.eps = eps;
    a.bs = bsel();
    a.ores = ores;
    a.thermo = thermo;
    a.theta = theta_dev;
    a.rtab = nullptr;
    if (P.n_ores <= kReactRow - 10) {
      // gas-cell quantities once per occupied cell of the current order
      if (!occ_fresh) {
        launch_occupied(start_d, cell_bed, bsel(), n_gas, false, DepositOut{}, occ_flags, occ_offs, scan_scr, occ_list,
                        occ_count, st);
        occ_fresh = true;
      }
      launch_react_table(a.g, cell_bed, beds, ores, P.n_ores, theta_dev, occ_list, occ_count, n_gas, rtab, st);
      a.rtab = rtab;
    }
    a.dt = dt;
    a.n = n;
    a.update_mass = update_mass;
    a.pm = pm;
    a.pw = pw;
    a.fov = fov;
    a.clamps = counters + 2;
    a.status = status;
    launch_react<T>(a, st);
    if (o) {
      CellSumOut cs{{o->mdotH2, o->mdotH2O, o->sumEQ, o->sumES, o->hA, o->hAT, o->Qrm, o->Hr}, thermo ? 8 : 4};
      bool any = false;
      for (int q = 0; q < cs.rows; q++) any |= cs.o[q] != nullptr;
      if (any) {
        if (!occ_fresh) {  // occupied cells of the current order, voidage untouched
          launch_occupied(start_d, cell_bed, bsel(), n_gas, false, DepositOut{}, occ_flags, occ_offs, scan_scr, occ_list,
                          occ_count, st);
          occ_fresh = true;
        }
        launch_cellsum(pm, n, start_d, order_d, cell_bed, bsel(), n_gas, occ_flags, occ_list, occ_count, n_gas, cs, st);
      }
    }
    if (bed_sum) {
      // the table is built at the first eager call (a graph being captured
      // builds its own until then: captured work runs only when launched)
      launch_bedsum(pw, n, start, beds, P.n_beds, bchunks, max_chunks, bpartial, bed_fov_d, !bchunks_ready, st);
      if (!capturing) bchunks_ready = true;
    }
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  int react(double dt, const dem_gas *g, dem_sources *o, double *bed_fov, double *fov) override {
    if (!(dt > 0.0)) return fail(DEMRX_EINVAL, "dt_cfd must be positive");
    if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
    TRY(react_core(dt, g, o, fov, bed_fov != nullptr, 1, nullptr));
    if (bed_fov) {
      HIPCHK(hipMemcpyAsync(bed_fov, bed_fov_d, P.n_beds * sizeof(double), hipMemcpyDeviceToHost, st));
      return sync();
    }
    return DEMRX_OK;
  }

  int gas_species(double dt, const dem_gas *g, const double *eq, const double *es, const double *xin, double *x1,
                  double *x2, double *x3) override {
    if (!gas_ok(g) || !eq || !es || !xin || !x1 || !x2 || !x3) return fail(DEMRX_EINVAL, "null argument");
    // the step reads neighbouring cells of g's mole fractions while it writes
    // the outputs, so an output that aliases an input would race
    for (const double *o : {(const double *)x1, (const double *)x2, (const double *)x3})
      if (o == g->xH2 || o == g->xH2O || o == g->xN2)
        return fail(DEMRX_EINVAL, "species outputs must be distinct from the gas mole-fraction inputs");
    if (x1 == x2 || x1 == x3 || x2 == x3) return fail(DEMRX_EINVAL, "species outputs must be distinct arrays");
    if (!(dt > 0.0) || !(xin[0] >= 0.0) || !(xin[1] >= 0.0) || !(xin[0] + xin[1] <= 1.0))
      return fail(DEMRX_EINVAL, "dt must be positive and xin fractions in [0, 1] with sum <= 1");
    TRY(ensure_dep());
    launch_gas_species(gas_args(g), eps, cell_bed, beds, n_gas, dt, eq, es, xin[0], xin[1], x1, x2, x3, status, st);
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  int gas_momentum(double dt, const dem_gas *g, const double *sK, const double *sKu, const double *sKv,
                   const double *sKw, double *u, double *v, double *w) override {
    if (!gas_ok(g) || !sK || !sKu || !sKv || !sKw || !u || !v || !w) return fail(DEMRX_EINVAL, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DEMRX_EINVAL, "dt must be positive");
    TRY(ensure_dep());
    launch_gas_momentum(gas_args(g), eps, cell_bed, beds, n_gas, dt, P.g, sK, sKu, sKv, sKw, u, v, w, status, st);
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  int forces(const dem_gas *g, double *F, double *Tq) override {
    if (!gas_ok(g) || !F || !Tq) return fail(DEMRX_EINVAL, "null argument");
    TRY(ensure_lists());
    TRY(gas_table(g, 0));
    StepArgs<T> a = step_args(1);
    a.Fout = F;
    a.Tout = Tq;
    launch_step<T>(a, step_block, st);
    HIPCHK(hipGetLastError());
    return DEMRX_OK;
  }

  int get_state(dem_parcels *o) override {
    if (!o) return fail(DEMRX_EINVAL, "null output");
    launch_export<T>(dyn[cur], pr, n, *o, st);
    HIPCHK(hipGetLastError());
    return sync();
  }

  int set_state(const dem_parcels *in) override {
    if (!in || !in->x || !in->y || !in->z || !in->vx || !in->vy || !in->vz || !in->wx || !in->wy || !in->wz ||
        !in->nh || !in->nm || !in->nw || !in->nfe)
      return fail(DEMRX_EINVAL, "null parcel array");
    launch_import<T>(*in, n, thermo, dyn[cur], pr, st);
    launch_fill_u32((uint32_t *)nb.mask, 0u, 2L * n, st);
    built = false;
    TRY(rebuild_chain(1, true));
    TRY(resort());
    DepositOut o{};
    o.eps_ctx = eps;
    TRY(deposit(GasArgs{}, false, o));
    HIPCHK(hipGetLastError());
    return sync();
  }

  int pairs(uint32_t *ij, int64_t cap, int64_t *np) override {
    if (!np || (cap > 0 && !ij) || cap < 0) return fail(DEMRX_EINVAL, "bad pair buffer");
    TRY(ensure_lists());
    for (int attempt = 0; attempt < 2; attempt++) {
      if (!pairs_buf) {
        pairs_cap = std::max<long>(1024, (long)n * 4);
        TRY(dalloc(pairs_buf, 2 * (size_t)pairs_cap));
      }
      launch_fill_u32((uint32_t *)(counters + 3), 0u, 2, st);
      launch_pairs<T>(dyn[cur], pr, nb, n, P.max_nbr, pairs_buf, pairs_cap, counters + 3, st);
      HIPCHK(hipGetLastError());
      unsigned long long c = 0;
      HIPCHK(hipMemcpyAsync(&c, counters + 3, sizeof c, hipMemcpyDeviceToHost, st));
      TRY(sync());
      if ((long)c > pairs_cap) {
        pairs_cap = (long)c;
        TRY(dalloc(pairs_buf, 2 * (size_t)pairs_cap));
        continue;
      }
      std::vector<uint32_t> h(2 * c);
      if (c) HIPCHK(hipMemcpy(h.data(), pairs_buf, 2 * c * sizeof(uint32_t), hipMemcpyDeviceToHost));
      std::vector<uint64_t> k(c);
      for (size_t q = 0; q < c; q++) k[q] = ((uint64_t)h[2 * q] << 32) | h[2 * q + 1];
      std::sort(k.begin(), k.end());
      for (size_t q = 0; q < c && (int64_t)q < cap; q++) {
        ij[2 * q] = (uint32_t)(k[q] >> 32);
        ij[2 * q + 1] = (uint32_t)(k[q] & 0xffffffffu);
      }
      *np = (int64_t)c;
      return DEMRX_OK;
    }
    return fail(DEMRX_EHIP, "pair buffer growth failed");
  }

  // Device buffers of one call, freed when it returns (hipFree waits for the
  // device).
  struct CallBufs {
    std::vector<void *> p;
    ~CallBufs() {
      for (void *q : p) (void)hipFree(q);
    }
    template <typename U>
    bool get(U *&out, size_t cnt) {
      void *q = nullptr;
      if (hipMalloc(&q, std::max<size_t>(cnt, 1) * sizeof(U)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      p.push_back(q);
      out = (U *)q;
      return true;
    }
  };

  int get_contacts(dem_contacts *io) override {
    if (!io || io->cap < 0 || (io->cap > 0 && (!io->ids || !io->xi)) || !io->wall_on || !io->wall_xi)
      return fail(DEMRX_EINVAL, "bad contact buffers");
    TRY(ensure_lists());
    CallBufs B;
    uint8_t *won = nullptr;
    double *wxi = nullptr;
    unsigned long long *cnt = nullptr;
    if (!B.get(won, (size_t)n * kMaxWalls) || !B.get(wxi, (size_t)n * kMaxWalls * 3) || !B.get(cnt, 1))
      return fail(DEMRX_ENOMEM, "contact export buffers");
    long cap = std::max<long>(1024, 3L * n);
    for (int attempt = 0; attempt < 2; attempt++) {
      uint32_t *ids = nullptr;
      double *xi = nullptr;
      CallBufs P2;
      if (!P2.get(ids, 2 * (size_t)cap) || !P2.get(xi, 3 * (size_t)cap)) return fail(DEMRX_ENOMEM, "contact buffers");
      launch_fill_u32((uint32_t *)cnt, 0u, 2, st);
      launch_contacts_export<T>(dyn[cur].pos, nb, pr.wh, n, P.max_nbr, ids, xi, cap, cnt, won, wxi, st);
      HIPCHK(hipGetLastError());
      unsigned long long c = 0;
      HIPCHK(hipMemcpyAsync(&c, cnt, sizeof c, hipMemcpyDeviceToHost, st));
      TRY(sync());
      if ((long)c > cap) {
        cap = (long)c;
        continue;
      }
      std::vector<uint32_t> hi(2 * c);
      std::vector<double> hx(3 * c);
      if (c) {
        HIPCHK(hipMemcpy(hi.data(), ids, 2 * c * sizeof(uint32_t), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hx.data(), xi, 3 * c * sizeof(double), hipMemcpyDeviceToHost));
      }
      // ascending (a, b): the order does not depend on the launch
      std::vector<uint64_t> k(c);
      for (size_t q = 0; q < c; q++) k[q] = ((uint64_t)hi[2 * q] << 32) | hi[2 * q + 1];
      std::vector<size_t> ord(c);
      std::iota(ord.begin(), ord.end(), (size_t)0);
      std::sort(ord.begin(), ord.end(), [&](size_t u, size_t v) { return k[u] < k[v]; });
      for (size_t q = 0; q < c && (int64_t)q < io->cap; q++) {
        const size_t o = ord[q];
        io->ids[2 * q] = hi[2 * o];
        io->ids[2 * q + 1] = hi[2 * o + 1];
        for (int d = 0; d < 3; d++) io->xi[3 * q + d] = hx[3 * o + d];
      }
      io->count = (int64_t)c;
      HIPCHK(hipMemcpy(io->wall_on, won, (size_t)n * kMaxWalls, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(io->wall_xi, wxi, (size_t)n * kMaxWalls * 3 * sizeof(double), hipMemcpyDeviceToHost));
      return DEMRX_OK;
    }
    return fail(DEMRX_EHIP, "contact buffer growth failed");
  }

  int set_contacts(const dem_contacts *in) override {
    if (!in || in->count < 0 || (in->count > 0 && (!in->ids || !in->xi)) || !in->wall_on || !in->wall_xi)
      return fail(DEMRX_EINVAL, "bad contact arrays");
    const long np = (long)in->count;
    for (long q = 0; q < np; q++) {
      const uint32_t a = in->ids[2 * q], b = in->ids[2 * q + 1];
      if (!(a < b && b < (uint32_t)n)) return fail(DEMRX_EINVAL, "contact pair " + std::to_string(q) + " is not a < b < n");
      for (int d = 0; d < 3; d++)
        if (!std::isfinite(in->xi[3 * q + d])) return fail(DEMRX_EINVAL, "non-finite contact spring");
    }
    for (long q = 0; q < (long)n * kMaxWalls * 3; q++)
      if (!std::isfinite(in->wall_xi[q])) return fail(DEMRX_EINVAL, "non-finite wall spring");
    CallBufs B;
    uint32_t *ids = nullptr, *cnt = nullptr;
    double *xi = nullptr, *wxi = nullptr;
    uint8_t *won = nullptr;
    int32_t *inv = nullptr;
    if (!B.get(ids, 2 * (size_t)np) || !B.get(xi, 3 * (size_t)np) || !B.get(won, (size_t)n * kMaxWalls) ||
        !B.get(wxi, (size_t)n * kMaxWalls * 3) || !B.get(inv, n) || !B.get(cnt, n))
      return fail(DEMRX_ENOMEM, "contact import buffers");
    if (np) {
      HIPCHK(hipMemcpyAsync(ids, in->ids, 2 * np * sizeof(uint32_t), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(xi, in->xi, 3 * np * sizeof(double), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(won, in->wall_on, (size_t)n * kMaxWalls, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(wxi, in->wall_xi, (size_t)n * kMaxWalls * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    launch_contacts_import<T>(dyn[cur].pos, n, P.max_nbr, ids, xi, np, won, wxi, inv, cnt, nb, pr.wh, status, st);
    HIPCHK(hipGetLastError());
    TRY(rebuild_chain(1, true));
    return sync();
  }

  // dem_pairs through the device's static scratch: no device allocation.  The
  // pairs are copied into ij and sorted there, so ij must hold them all.
  int pairs_noalloc(uint32_t *ij, int64_t cap, int64_t *np) override {
    if (!np || (cap > 0 && !ij) || cap < 0) return fail(DEMRX_EINVAL, "bad pair buffer");
    TRY(ensure_lists());
    unsigned long long *cnt = (unsigned long long *)scratch_ptr;
    uint32_t *buf = (uint32_t *)((unsigned char *)scratch_ptr + 256);
    launch_fill_u32((uint32_t *)cnt, 0u, 2, st);  // the array keeps the last call's contents
    launch_pairs<T>(dyn[cur], pr, nb, n, P.max_nbr, buf, (long)DEM_NOALLOC_MAX_PAIRS, cnt, st);
    HIPCHK(hipGetLastError());
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, cnt, sizeof c, hipMemcpyDeviceToHost, st));
    TRY(sync());
    *np = (int64_t)c;
    if (c > (unsigned long long)DEM_NOALLOC_MAX_PAIRS)
      return fail(DEMRX_EOVERFLOW, std::to_string(c) + " contact pairs exceed the " +
                                       std::to_string(DEM_NOALLOC_MAX_PAIRS) + " of the static scratch; use dem_pairs");
    if ((int64_t)c > cap) return fail(DEMRX_EINVAL, "ij holds fewer pairs than there are (see *n_pairs)");
    if (c) HIPCHK(hipMemcpy(ij, buf, 2 * c * sizeof(uint32_t), hipMemcpyDeviceToHost));
    struct Pr {
      uint32_t a, b;
    };
    Pr *pp = reinterpret_cast<Pr *>(ij);
    std::sort(pp, pp + c, [](const Pr &x, const Pr &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; });
    return DEMRX_OK;
  }

  int stats(dem_stats *o) override {
    if (!o) return fail(DEMRX_EINVAL, "null output");
    unsigned long long c[4], rbc = 0;
    std::vector<unsigned long long> cs((size_t)kSlots * kSlotPad64);
    HIPCHK(hipMemcpyAsync(c, counters, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&rbc, rb_count, sizeof rbc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(cs.data(), cslot, cs.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    int r = sync();
    c[0] = c[1] = 0;
    for (int q = 0; q < kSlots; q++) {
      c[0] += cs[(size_t)q * kSlotPad64];
      c[1] += cs[(size_t)q * kSlotPad64 + 1];
    }
    o->n_parcels = n;
    o->n_contacts = (int64_t)(c[0] / 2);
    o->n_wall_contacts = (int64_t)c[1];
    o->rebuilds = (int64_t)rbc;
    o->steps = step_count;
    o->clamps = (int64_t)c[2];
    o->mean_coordination = n ? (double)c[0] / n : 0.0;
    o->max_nbr_used = P.max_nbr;
    o->status = 0;
    double tot = 0.0;
    long cnt = 0;
    for (auto *lst : {&prof_eager, &prof_graph}) {
      for (auto &pr_ : *lst) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr_.first, pr_.second) == hipSuccess) {
          tot += ms;
          cnt++;
        } else {
          (void)hipGetLastError();
        }
      }
    }
    o->step_kernel_ms = cnt ? tot / cnt : 0.0;
    o->step_kernel_launches = cnt;
    o->step_block = step_block;
    o->step_xcd = step_xcd;
    o->build_grid = build_grid_now();
    o->check_period = check_period();
    o->build_threads = build_threads(build_variant);
    o->build_tile = build_tile(build_variant);
    o->build_item_x = item_x;
    o->tune_cached = tune_cached ? 1 : 0;
    return r;
  }

  // One coupling interval of the hot path: S DEM steps (each with the list
  // check in front of it when one is due), the deposit and the reaction.
  int interval(int S, const dem_gas *g, dem_sources *o) {
    TRY(ensure_occ());
    TRY(gas_table(g, S));
    for (int s = 0; s < S; s++) {
      if (s == S - 1) launch_fill_u32((uint32_t *)cslot, 0u, 2 * kSlots * kSlotPad64, st);  // last step counts
      TRY(step_checked(s == S - 1));
    }
    TRY(couple(g, o));
    TRY(react_core(S * P.dt, g, o, nullptr, true, 1, nullptr));
    return DEMRX_OK;
  }

  // Intervals per graph: the fewest whose steps are a multiple of 2 (the
  // step buffers flip every step) and of the check period, so every replay
  // starts at the same buffer parity and check phase as the capture.
  long graph_intervals(int S) const {
    const long a = std::lcm((long)S, 2L), b = std::lcm(a, (long)check_period());
    return b / S;
  }

  int run(int n_int, int S, const dem_gas *g, dem_sources *o, double *bed_fov) override {
    if (n_int < 0 || S < 1) return fail(DEMRX_EINVAL, "bad interval count");
    if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
    if (n_int == 0) return DEMRX_OK;
    std::vector<const void *> k = {(const void *)(intptr_t)S, g->ug, g->vg, g->wg, g->p, g->dpdx, g->dpdy,
                                   g->dpdz, g->T, g->xH2, g->xH2O, g->xN2};
    dem_sources oo{};
    if (o) oo = *o;
    for (double *q : {oo.eps, oo.np, oo.sumK, oo.sumKu, oo.sumKv, oo.sumKw, oo.sumKs, oo.mdotH2, oo.mdotH2O,
                      oo.sumEQ, oo.sumES})
      k.push_back(q);
    k.push_back((const void *)(intptr_t)step_block);
    k.push_back((const void *)(intptr_t)step_xcd);
    // the graph bakes in the buffer parities it was captured at
    k.push_back((const void *)(intptr_t)(cur | (int)((step_count & 1) << 1)));
    k.push_back((const void *)(intptr_t)(step_count % check_period()));
    if (graph_intervals(S) > 4096) return fail(DEMRX_EINVAL, "couple_every and check_every give a graph of more "
                                                             "than 4096 intervals");
    if (!cap_st) {
      HIPCHK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ev_a, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_b, hipEventDisableTiming));
    }
    if (!built) TRY(rebuild_chain(1, true));  // a forced first build stays out of the graph
    TRY(ensure_occ());  // every interval, the first included, starts from a fresh occupied list
    if (!bchunks_ready) {  // the chunk table of the bed means, once and outside the graph
      launch_bedsum(nullptr, n, start, beds, P.n_beds, bchunks, max_chunks, bpartial, bed_fov_d, true, st);
      bchunks_ready = true;
    }
    // whether the lists were checked at the current positions decides the
    // first step's check, so it is part of what the graph bakes in
    k.push_back((const void *)(intptr_t)(chain_step == step_count ? 1 : 0));
    HIPCHK(hipEventRecord(ev_a, user_st));
    HIPCHK(hipStreamWaitEvent(cap_st, ev_a, 0));
    st = cap_st;
    int r = run_on_cap(n_int, S, g, o ? &oo : nullptr, k);
    st = user_st;
    if (r != DEMRX_OK) return r;
    HIPCHK(hipEventRecord(ev_b, cap_st));
    HIPCHK(hipStreamWaitEvent(user_st, ev_b, 0));
    if (bed_fov) {
      HIPCHK(hipMemcpyAsync(bed_fov, bed_fov_d, P.n_beds * sizeof(double), hipMemcpyDeviceToHost, st));
      return sync();
    }
    return DEMRX_OK;
  }

  int run_on_cap(int n_int, int S, const dem_gas *g, dem_sources *o, const std::vector<const void *> &k) {
    const int G = (int)graph_intervals(S);
    if (!gexec || k != gkey) {
      if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
      if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
      const int s_cur = cur;
      const long s_sc = step_count;
      const bool s_dep = dep_fresh, s_occ = occ_fresh;
      const long s_chain = chain_step;
      HIPCHK(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed));
      capturing = true;
      prof_capture.clear();
      int r = DEMRX_OK;
      for (int q = 0; q < G && r == DEMRX_OK; q++) r = interval(S, g, o);
      capturing = false;
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(cap_st, &gr);
      if (r != DEMRX_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return r;
      }
      if (e != hipSuccess) return fail(DEMRX_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      if (cur != s_cur || ((step_count ^ s_sc) & 1))
        return fail(DEMRX_EHIP, "graph intervals do not restore buffer parity");
      graph = gr;
      HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      gkey = k;
      gprof = prof;
      dep_after_graph = dep_fresh;
      occ_after_graph = occ_fresh;
      chain_after_graph = chain_step == step_count;
      chain_step = s_chain;
      cur = s_cur;
      step_count = s_sc;
      dep_fresh = s_dep;
      occ_fresh = s_occ;
    }
    if (gprof != prof) {  // recapture with or without timing events
      gkey.clear();
      return run_on_cap(n_int, S, g, o, k);
    }
    if (prof && n_int >= G) prof_graph = prof_capture;
    for (int q = 0; q < n_int / G; q++) {
      HIPCHK(hipGraphLaunch(gexec, cap_st));
      step_count += (long)G * S;
      dep_fresh = dep_after_graph;
      occ_fresh = occ_after_graph;
      chain_step = chain_after_graph ? step_count : -1;
    }
    for (int q = 0; q < n_int % G; q++) TRY(interval(S, g, o));
    return DEMRX_OK;
  }
  bool dep_after_graph = false, occ_after_graph = false, chain_after_graph = false;
  bool gprof = false;

  // Autotuner cache: a JSON object whose members (one per line) map a key of
  // the device architecture and the context's configuration to the chosen
  // shapes.  Read and rewritten by dem_autotune when DEMRX_TUNE_CACHE names
  // the file.
  std::string tune_key() const {
    std::string k = arch + "|n=" + std::to_string(n) + "|beds=" + std::to_string(hbd.size()) +
                    "|fp=" + std::to_string((int)sizeof(T)) + "|cap=" + std::to_string(P.max_nbr) +
                    "|skin=" + std::to_string(P.skin) + "|energy=" + std::to_string(P.energy_on);
    for (const BedDev &d : hbd)
      k += "|" + std::to_string(d.nd[0]) + "x" + std::to_string(d.nd[1]) + "x" + std::to_string(d.nd[2]);
    return k;
  }
  static bool tune_field(const std::string &line, const char *name, int &v) {
    const std::string f = std::string("\"") + name + "\":";
    const size_t p = line.find(f);
    return p != std::string::npos && std::sscanf(line.c_str() + p + f.size(), " %d", &v) == 1;
  }
  static std::vector<std::string> tune_lines(const char *path) {
    std::vector<std::string> out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    char buf[4096];
    while (std::fgets(buf, sizeof buf, f)) {
      std::string l(buf);
      while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ',' || l.back() == ' ')) l.pop_back();
      if (l.size() > 2 && l[0] == '"') out.push_back(l);
    }
    std::fclose(f);
    return out;
  }
  bool tune_load(const char *path) {
    const std::string key = "\"" + tune_key() + "\":";
    for (const std::string &l : tune_lines(path)) {
      if (l.compare(0, key.size(), key) != 0) continue;
      int b, x, th, tl, ix;
      if (!(tune_field(l, "step_block", b) && tune_field(l, "step_xcd", x) && tune_field(l, "build_threads", th) &&
            tune_field(l, "build_tile", tl) && tune_field(l, "item_x", ix)))
        return false;
      if (set_launch(b, x, 0) != DEMRX_OK || set_build(th, tl, ix) != DEMRX_OK) return false;
      return true;
    }
    return false;
  }
  void tune_store(const char *path) {
    const std::string key = "\"" + tune_key() + "\":";
    std::vector<std::string> keep;
    for (const std::string &l : tune_lines(path))
      if (l.compare(0, key.size(), key) != 0) keep.push_back(l);
    keep.push_back(key + " {\"step_block\": " + std::to_string(step_block) + ", \"step_xcd\": " +
                   std::to_string(step_xcd) + ", \"build_threads\": " + std::to_string(build_threads(build_variant)) +
                   ", \"build_tile\": " + std::to_string(build_tile(build_variant)) +
                   ", \"item_x\": " + std::to_string(item_x) + "}");
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t q = 0; q < keep.size(); q++) std::fprintf(f, "%s%s\n", keep[q].c_str(), q + 1 < keep.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
  }

  int autotune(const dem_gas *g) override {
    if (!gas_ok(g)) return fail(DEMRX_EINVAL, "null gas field");
    const char *cache = std::getenv("DEMRX_TUNE_CACHE");
    if (cache && *cache && tune_load(cache)) {
      tune_cached = true;
      return DEMRX_OK;
    }
    tune_cached = false;
    TRY(ensure_lists());
    TRY(gas_table(g));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_b = step_block, best_x = step_xcd;
    const bool tune_log = std::getenv("DEMRX_TUNE_LOG") != nullptr;  // per-candidate timings on stderr
    for (int b : {64, 128, 256, 512}) {
      for (int x : {1, 4, 16, 64}) {
        step_xcd = x;
        // candidates lie within a few per cent of each other: eight timed
        // launches each (after one untimed) keep the pick above the noise
        float tot = 0.0f;
        for (int rep = 0; rep < 9; rep++) {
          HIPCHK(hipEventRecord(e0, st));
          launch_step<T>(step_args(2), b, st);
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.0f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (rep) tot += ms;
        }
        if (tune_log) std::fprintf(stderr, "[demrx] autotune step block %d xcd chunk %d: %.1f us\n", b, x, tot / 8 * 1e3f);
        if (tot < best) { best = tot; best_b = b; best_x = x; }
      }
    }
    step_block = best_b;
    step_xcd = best_x;
    // neighbour build: block size and LDS tile, item width (grid: resident
    // blocks on every CU); each candidate times whole forced rebuild chains
    best = 1e30f;
    int best_v = build_variant, best_w = item_x;
    build_grid = 0;
    for (int v = 0; v < kBuildVariants; v++) {
      for (int wdt : kItemWidths) {
        build_variant = v;
        TRY(upload_items(wdt));
        float tot = 0.0f;
        for (int rep = 0; rep < 3; rep++) {
          HIPCHK(hipEventRecord(e0, st));
          TRY(rebuild_chain(1, true));
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.0f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (rep) tot += ms;
        }
        if (tune_log)
          std::fprintf(stderr, "[demrx] autotune build %d threads, tile %d, item %d cells (grid %d): %.1f us\n",
                       build_threads(v), build_tile(v), wdt, build_grid_now(), tot / 2 * 1e3f);
        if (tot < best) { best = tot; best_v = v; best_w = wdt; }
      }
    }
    build_variant = best_v;
    TRY(upload_items(best_w));
    TRY(rebuild_chain(1, true));  // lists of the chosen shape (identical for every shape)
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; gkey.clear(); }
    TRY(sync());
    if (cache && *cache) tune_store(cache);
    return DEMRX_OK;
  }

  int set_launch(int b, int x, int gsz) override {
    if (!(b == 64 || b == 128 || b == 256 || b == 512) || x < 1 || x > 64 || gsz < 0 || gsz > 65536)
      return fail(DEMRX_EINVAL, "launch shape out of range (step block 64/128/256/512, XCD chunk 1..64, "
                                "build grid 0..65536)");
    step_block = b;
    step_xcd = x;
    build_grid = gsz;
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; gkey.clear(); }
    return DEMRX_OK;
  }

  int set_build(int threads, int tile, int width) override {
    int v = -1;
    for (int q = 0; q < kBuildVariants; q++)
      if (build_threads(q) == threads && build_tile(q) == tile) v = q;
    bool wok = false;
    for (int wdt : kItemWidths) wok |= wdt == width;
    if (v < 0 || !wok)
      return fail(DEMRX_EINVAL, "build shape not available (threads/tile 512/2048, 256/1024, 256/2048, "
                                "1024/4096; item width 8, 16 or 32)");
    build_variant = v;
    if (width != item_x) TRY(upload_items(width));
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; gkey.clear(); }
    return DEMRX_OK;
  }

  int grad(const dem_grad_spec *s, const dem_gas *g, const double *theta, double *J, double *gr) override;
  struct {
    void *base = nullptr;
    size_t cap = 0;
  } gscr;
};

#include "grad_impl.h"

// ------------------------------------------------------------------ C entry points
static int validate(const dem_params *p, const dem_parcels *in, int32_t n, std::string &m) {
  if (!p || !in) { m = "null params or parcels"; return DEMRX_EINVAL; }
  if (n <= 0) { m = "n_parcels must be positive"; return DEMRX_EINVAL; }
  if (p->precision != DEM_FP64 && p->precision != DEM_MIXED) { m = "unknown precision"; return DEMRX_EINVAL; }
  if (p->n_beds < 1 || p->n_beds > DEM_MAX_BEDS || !p->beds) { m = "bad n_beds/beds"; return DEMRX_EINVAL; }
  if (p->n_ores < 1 || p->n_ores > DEM_MAX_ORES || !p->ores) { m = "bad n_ores/ores"; return DEMRX_EINVAL; }
  if (!(p->kn > 0) || !(p->e_p > 0 && p->e_p <= 1) || !(p->mu_s >= 0) || !(p->mu_r >= 0) ||
      !(p->kt_over_kn > 0) || !(p->gt_over_gn >= 0) || !(p->eps_min > 0 && p->eps_min <= 1) ||
      !(p->skin >= 0) || !(p->dt > 0) || !std::isfinite(p->g[0] + p->g[1] + p->g[2])) {
    m = "bad physical parameter";
    return DEMRX_EINVAL;
  }
  if (p->max_nbr < 1 || p->max_nbr > DEM_MAX_NBR || p->check_every < 1) { m = "bad max_nbr/check_every"; return DEMRX_EINVAL; }
  for (int b = 0; b < p->n_beds; b++) {
    const dem_bed &B = p->beds[b];
    if (B.wall_kind != DEM_WALL_BOX && B.wall_kind != DEM_WALL_CYL) { m = "bad wall kind"; return DEMRX_EINVAL; }
    if (!(B.h > 0) || B.n[0] < 1 || B.n[1] < 1 || B.n[2] < 1 || B.refine < 1 || B.refine > 4) {
      m = "bad grid of bed " + std::to_string(b);
      return DEMRX_EINVAL;
    }
    for (int a = 0; a < 3; a++)
      if (!(B.lo[a] < B.hi[a]) || B.origin[a] > B.lo[a] + 1e-12 || B.origin[a] + B.n[a] * B.h < B.hi[a] - 1e-12) {
        m = "grid of bed " + std::to_string(b) + " does not contain its walls";
        return DEMRX_EINVAL;
      }
    if (B.wall_kind == DEM_WALL_CYL &&
        !(B.R > 0 && 2 * B.R <= (B.hi[0] - B.lo[0]) + 1e-12 && 2 * B.R <= (B.hi[1] - B.lo[1]) + 1e-12)) {
      m = "cylinder radius of bed " + std::to_string(b) + " does not fit its bounding box";
      return DEMRX_EINVAL;
    }
  }
  for (int o = 0; o < p->n_ores; o++) {
    const dem_ore &O = p->ores[o];
    if (!(O.xi0 >= 0 && O.xi0 < 1) || !(O.d_pore_cm > 0) || !(O.tau > 0) || (O.kind != 0 && O.kind != 1)) {
      m = "bad ore " + std::to_string(o);
      return DEMRX_EINVAL;
    }
  }
  if (!in->x || !in->y || !in->z || !in->vx || !in->vy || !in->vz || !in->wx || !in->wy || !in->wz || !in->d ||
      !in->k || !in->ore || !in->bed || !in->nh || !in->nm || !in->nw || !in->nfe) {
    m = "null parcel array";
    return DEMRX_EINVAL;
  }
  return DEMRX_OK;
}

static thread_local std::string g_init_err;

extern "C" {

int dem_init(const dem_params *p, const dem_parcels *in, int32_t n, void *stream, dem_ctx **out) {
  if (!out) return DEMRX_EINVAL;
  *out = nullptr;
  std::string m;
  int r = validate(p, in, n, m);
  if (r != DEMRX_OK) {
    g_init_err = m;
    return r;
  }
  dem_ctx *c = nullptr;
  if (p->precision == DEM_MIXED) {
    auto *q = new Ctx<float>();
    r = q->init(p, in, n, (hipStream_t)stream);
    c = q;
  } else {
    auto *q = new Ctx<double>();
    r = q->init(p, in, n, (hipStream_t)stream);
    c = q;
  }
  if (r != DEMRX_OK) {
    g_init_err = c->err;
    delete c;
    return r;
  }
  *out = c;
  return DEMRX_OK;
}

int dem_step(dem_ctx *c, int32_t n, const dem_gas *g) { return c ? c->step(n, g) : DEMRX_EINVAL; }
int dem_couple(dem_ctx *c, const dem_gas *g, dem_sources *o) { return c ? c->couple(g, o) : DEMRX_EINVAL; }
int dem_react(dem_ctx *c, double dt, const dem_gas *g, dem_sources *o, double *bed_fov, double *fov) {
  return c ? c->react(dt, g, o, bed_fov, fov) : DEMRX_EINVAL;
}
int dem_gas_species(dem_ctx *c, double dt, const dem_gas *g, const double *sumEQ, const double *sumES,
                    const double xin[2], double *xH2, double *xH2O, double *xN2) {
  return c ? c->gas_species(dt, g, sumEQ, sumES, xin, xH2, xH2O, xN2) : DEMRX_EINVAL;
}
int dem_gas_momentum(dem_ctx *c, double dt, const dem_gas *g, const double *sumK, const double *sumKu,
                     const double *sumKv, const double *sumKw, double *ug, double *vg, double *wg) {
  return c ? c->gas_momentum(dt, g, sumK, sumKu, sumKv, sumKw, ug, vg, wg) : DEMRX_EINVAL;
}
int dem_grad(dem_ctx *c, const dem_grad_spec *s, const dem_gas *g, const double theta[6], double *J, double *grad) {
  return c ? c->grad(s, g, theta, J, grad) : DEMRX_EINVAL;
}
int dem_forces(dem_ctx *c, const dem_gas *g, double *F, double *T) { return c ? c->forces(g, F, T) : DEMRX_EINVAL; }
int dem_get_state(dem_ctx *c, dem_parcels *o) { return c ? c->get_state(o) : DEMRX_EINVAL; }
int dem_set_state(dem_ctx *c, const dem_parcels *in) { return c ? c->set_state(in) : DEMRX_EINVAL; }
int dem_pairs(dem_ctx *c, uint32_t *ij, int64_t cap, int64_t *np) { return c ? c->pairs(ij, cap, np) : DEMRX_EINVAL; }
int dem_pairs_noalloc(dem_ctx *c, uint32_t *ij, int64_t cap, int64_t *np) {
  return c ? c->pairs_noalloc(ij, cap, np) : DEMRX_EINVAL;
}
int dem_get_stats(dem_ctx *c, dem_stats *o) { return c ? c->stats(o) : DEMRX_EINVAL; }
int dem_run(dem_ctx *c, int32_t n_int, int32_t S, const dem_gas *g, dem_sources *o, double *bed_fov) {
  return c ? c->run(n_int, S, g, o, bed_fov) : DEMRX_EINVAL;
}
int dem_autotune(dem_ctx *c, const dem_gas *g) { return c ? c->autotune(g) : DEMRX_EINVAL; }
int dem_set_launch(dem_ctx *c, int32_t step_block, int32_t step_xcd_chunk, int32_t build_grid) {
  return c ? c->set_launch(step_block, step_xcd_chunk, build_grid) : DEMRX_EINVAL;
}
int dem_get_contacts(dem_ctx *c, dem_contacts *io) { return c ? c->get_contacts(io) : DEMRX_EINVAL; }
int dem_set_contacts(dem_ctx *c, const dem_contacts *in) { return c ? c->set_contacts(in) : DEMRX_EINVAL; }
int dem_set_build(dem_ctx *c, int32_t threads, int32_t tile, int32_t item_x) {
  return c ? c->set_build(threads, tile, item_x) : DEMRX_EINVAL;
}
int dem_profile(dem_ctx *c, int32_t enable) { return c ? c->profile(enable) : DEMRX_EINVAL; }
int dem_sync(dem_ctx *c) { return c ? c->sync() : DEMRX_EINVAL; }
const char *dem_last_error(const dem_ctx *c) { return c ? c->err.c_str() : g_init_err.c_str(); }
void dem_destroy(dem_ctx *c) { delete c; }

}  // extern "C"
