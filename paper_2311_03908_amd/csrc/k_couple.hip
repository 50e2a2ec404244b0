// Coupling kernels: voidage/drag deposition onto the gas grid, the
// multi-interface unreacted-shrinking-core reaction update, per-cell and
// per-bed reductions (deterministic: fixed lane assignment and shuffle trees,
// no floating-point atomics), and state import/export.
#include <algorithm>

#include "launch.h"
#include "uscm.h"

namespace demrx {

constexpr int kGroup = 16;  // lanes per gas cell in the segmented reductions

__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = kGroup / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kGroup);
  return v;
}

// DEM-cell ranges of a gas cell: refine^2 rows of `refine` consecutive keys
// (key tiles hold a multiple of `refine` cells along x)
struct GasCellRanges {
  const BedDev &B;
  int gx, gy, gz, f;
  __device__ GasCellRanges(const BedDev &B_, int c) : B(B_) {
    const int lc = c - B.gas_off;
    gx = lc % B.n[0];
    gy = (lc / B.n[0]) % B.n[1];
    gz = lc / (B.n[0] * B.n[1]);
    f = B.refine;
  }
  __device__ int row_key(int r) const {  // r in [0, f*f)
    const int sy = r % f, sz = r / f;
    return dem_key(B, gx * f, gy * f + sy, gz * f + sz);
  }
};

// ------------------------------------------------------------------ gas table
// Ideal-gas density (eq. e3-53) and mass-weighted viscosity (eqs. e3-55,
// e3-56, Table C2) of each cell, with the cell's velocity, voidage and
// pressure gradient, packed in one row for the drag gather; with the energy
// equation also the conductivity and Pr^(1/3) (eqs. e3-13, e3-57..e3-59).
__device__ __forceinline__ void gas_rho_mu(double T, double p, double x1, double x2, double x3, double mu_fix,
                                           double &rho, double &mu) {
  const double M1 = 2.016, M2 = 18.015, M3 = 28.013;  // g/mol H2, H2O, N2
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

template <typename T>
__global__ void k_gas_table(GasArgs g, const double *eps, const int32_t *cell_bed, const BedDev *beds,
                            const ThermoTab *thermo, int n_gas, const int2 *zr, T *gtab, uint32_t *status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gas) return;
  if (zr) {  // only the layers of its bed that parcels can reach
    const int b = cell_bed[c];
    const BedDev &B = beds[b];
    const int z = (c - B.gas_off) / (B.n[0] * B.n[1]);
    if (z < zr[b].x || z > zr[b].y) return;
  }
  double rho, mu;
  gas_rho_mu(g.T[c], g.p[c], g.xH2[c], g.xH2O[c], g.xN2[c], beds[cell_bed[c]].mu_override, rho, mu);
  T *r = gtab + (long)c * kGasRow;
  r[0] = T(g.ug[c]);
  r[1] = T(g.vg[c]);
  r[2] = T(g.wg[c]);
  r[3] = T(eps[c]);
  r[4] = T(g.dpdx[c]);
  r[5] = T(g.dpdy[c]);
  r[6] = T(g.dpdz[c]);
  r[7] = T(rho);
  r[8] = T(mu);
  r[9] = r[10] = T(0);
  r[11] = T(eps[c] < 0.8 ? 1 : 0);  // drag branch, decided in FP64
  double lam = 1.0, cp = 1.0;
  if (thermo) {
    gas_heat_props(*thermo, g.T[c], g.xH2[c], g.xH2O[c], g.xN2[c], lam, cp);
    r[9] = T(lam);
    r[10] = T(cbrt(cp * mu / lam));
  }
  if (!(lam > 0.0 && cp > 0.0 && isfinite(g.T[c])) ||
      !(isfinite(rho) && isfinite(mu) && isfinite(g.ug[c] + g.vg[c] + g.wg[c]) &&
        isfinite(g.dpdx[c] + g.dpdy[c] + g.dpdz[c])) || !(rho > 0.0) || !(mu > 0.0))
    atomicOr(status, ST_NONFINITE);
}

template <typename T>
void launch_gas_table(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds,
                      const ThermoTab *thermo, int n_gas, const int2 *zr, T *gtab, uint32_t *status, hipStream_t s) {
  k_gas_table<T><<<(n_gas + 255) / 256, 256, 0, s>>>(g, eps, cell_bed, beds, thermo, n_gas, zr, gtab, status);
}

// Layers of each bed that parcels can reach: the occupied list is sorted by
// cell and cells are numbered bed by bed, z outermost, so a bed's first and
// last listed cells hold its lowest and highest occupied layers; the range
// is widened by `reach` metres and one layer.  An empty bed gets an empty
// range.
__global__ void __launch_bounds__(64) k_occ_zrange(const int32_t *list, const int32_t *count, const BedDev *beds,
                                                   int n_beds, double reach, int2 *zr) {
  const int b = blockIdx.x;  // one wave per bed
  const int l = threadIdx.x;
  const BedDev &B = beds[b];
  const int m = *count;
  // first list position holding a cell >= v: each round the wave samples 64
  // evenly spaced positions of the remaining range and keeps one stride
  auto first_at_least = [&](int v) {
    int lo = 0, hi = m;  // answer in [lo, hi]
    while (hi - lo > 64) {
      const long step = ((long)(hi - lo) + 63) / 64;
      const int q = (int)min((long)lo + (long)l * step, (long)hi - 1);
      const bool below = list[q] < v;
      const uint64_t bal = __ballot(below);  // below is monotone in l
      const int k = __popcll(bal);           // lanes whose sample lies below v
      const int nlo = k == 0 ? lo : (int)min((long)lo + (long)(k - 1) * step + 1, (long)hi);
      const int nhi = k == 64 ? hi : (int)min((long)lo + (long)k * step, (long)hi);
      lo = nlo;
      hi = nhi;
    }
    const int q = lo + l;
    const bool below = q < hi && list[q] < v;
    return lo + __popcll(__ballot(below));
  };
  const int i0 = first_at_least(B.gas_off), i1 = first_at_least(B.gas_off + B.n_gas);
  if (l != 0) return;
  if (i0 >= i1) {
    zr[b] = make_int2(1, 0);
    return;
  }
  const int layer = B.n[0] * B.n[1];
  const int margin = (int)ceil(reach / B.h) + 1;
  const int z0 = (list[i0] - B.gas_off) / layer, z1 = (list[i1 - 1] - B.gas_off) / layer;
  zr[b] = make_int2(max(z0 - margin, 0), min(z1 + margin, B.n[2] - 1));
}
void launch_occ_zrange(const int32_t *list, const int32_t *count, const BedDev *beds, int n_beds, double reach,
                       int2 *zr, hipStream_t s) {
  k_occ_zrange<<<n_beds, 64, 0, s>>>(list, count, beds, n_beds, reach, zr);
}

template void launch_gas_table<float>(const GasArgs &, const double *, const int32_t *, const BedDev *,
                                      const ThermoTab *, int, const int2 *, float *, uint32_t *, hipStream_t);
template void launch_gas_table<double>(const GasArgs &, const double *, const int32_t *, const BedDev *,
                                       const ThermoTab *, int, const int2 *, double *, uint32_t *, hipStream_t);


// ------------------------------------------------------------------ deposition
// Occupied gas cells: most cells of a tall reactor grid hold no parcel.  One
// thread per cell writes the outputs of an empty cell (voidage 1, zero sums)
// and flags the others, which are compacted (scan) into a list; the deposit
// then runs one 16-lane group per listed cell.
__global__ void k_occ_flags(const int32_t *start, const int32_t *cell_bed, BedSel bs, int n_gas, int sums,
                            DepositOut o, int32_t *flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_gas) return;
  if (c == n_gas) {
    flags[c] = 0;
    return;
  }
  bool any = false;
  on_bed(bs, [&] { return cell_bed[c]; }, [&](const BedDev &B) {
    const GasCellRanges R(B, c);
    for (int r = 0; r < R.f * R.f && !any; r++) {
      const int k0 = R.row_key(r);
      any = start[k0 + R.f] > start[k0];
    }
  });
  flags[c] = any ? 1 : 0;
  if (any) return;
  if (o.eps_ctx) o.eps_ctx[c] = 1.0;
  if (o.eps) o.eps[c] = 1.0;
  if (o.np) o.np[c] = 0.0;
  if (!sums) return;
  if (o.sumK) o.sumK[c] = 0.0;
  if (o.sumKu) o.sumKu[c] = 0.0;
  if (o.sumKv) o.sumKv[c] = 0.0;
  if (o.sumKw) o.sumKw[c] = 0.0;
  if (o.sumKs) o.sumKs[c] = 0.0;
}

__global__ void k_occ_compact(const int32_t *flags, const int32_t *offs, int n_gas, int32_t *list, int32_t *count) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_gas) return;
  if (c == n_gas) {
    *count = offs[n_gas];
    return;
  }
  if (flags[c]) list[offs[c]] = c;
}

template <typename T, bool kGanser>
__global__ void __launch_bounds__(256) k_deposit(Dyn<T> d, Props<T> p, GasArgs g, const int32_t *start,
                                                 const int32_t *order, const int32_t *cell_bed, BedSel bs,
                                                 const OreDev *ores, Phys ph, const int32_t *list, const int32_t *list_count, int sums,
                                                 DepositOut o) {
  const int sl = threadIdx.x % kGroup;
  const int n_list = *list_count;
  const int groups = gridDim.x * (blockDim.x / kGroup);
  // Each lane takes the parcels sl, sl + 16, ... of every row of the cell,
  // two per trip with both records requested before either is used; the
  // sums run in that order, then over the group's lanes.
  auto cell = [&](const BedDev &B, const int c) {
    const GasCellRanges R(B, c);
    // the cell's gas state, requested with the first parcel records
    double Tc = 0.0, pc = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0, ug = 0.0, vg = 0.0, wg = 0.0;
    if (sums) {
      Tc = g.T[c];
      pc = g.p[c];
      x1 = g.xH2[c];
      x2 = g.xH2O[c];
      x3 = g.xN2[c];
      ug = g.ug[c];
      vg = g.vg[c];
      wg = g.wg[c];
    }
    double sv = 0.0, cnt = 0.0;
    for (int r = 0; r < R.f * R.f; r++) {
      const int k0 = R.row_key(r);
      const int e = start[k0 + R.f];
      for (int q = start[k0] + sl; q < e; q += 2 * kGroup) {
        const bool two = q + kGroup < e;
        const int j0 = order[q], j1 = two ? order[q + kGroup] : j0;
        const double d0 = 2.0 * (double)d.pos[j0].r, d1 = 2.0 * (double)d.pos[j1].r;
        sv += kPi / 6.0 * d0 * d0 * d0;
        cnt += 1.0;
        if (two) {
          sv += kPi / 6.0 * d1 * d1 * d1;
          cnt += 1.0;
        }
      }
    }
    sv = group_sum(sv);
    cnt = group_sum(cnt);
    double eps = 1.0 - sv / (B.h * B.h * B.h);
    eps = eps < ph.eps_min ? ph.eps_min : (eps > 1.0 ? 1.0 : eps);
    if (sl == 0) {
      o.eps_ctx[c] = eps;
      if (o.eps) o.eps[c] = eps;
      if (o.np) o.np[c] = cnt;
    }
    if (!sums) return;
    double rho, mu;
    gas_props_h2(Tc, pc, x1, x2, x3, B.mu_override, rho, mu);
    // the drag branch and the dilute branch's eps^-2.65, once per cell
    const bool dense = eps < 0.8;
    const double epse = dense ? 0.0 : pow(eps, -2.65);
    double sK = 0, sKu = 0, sKv = 0, sKw = 0, sKs = 0;
    auto add = [&](const VelRec<T> &vr, float rj, float kj, int32_t tj) {
      const double vx = (double)vr.v[0], vy = (double)vr.v[1], vz = (double)vr.v[2];
      const double sx = ug - vx, sy = vg - vy, sz = wg - vz;
      const double slip = sqrt(sx * sx + sy * sy + sz * sz);
      const double dd = 2.0 * (double)rj;
      const double V = kPi / 6.0 * dd * dd * dd;
      const double dpj = dd / (double)kj;  // real-particle diameter
      double beta;
      if constexpr (kGanser)
        beta = drag_beta_e<double>(ph, ores[ore_of(tj)], B, dense, eps, epse, rho, mu, slip, dpj);
      else
        beta = beta_over_epsp_e<double>(dense, eps, epse, rho, mu, slip, dpj, ph.ergun_printed);
      const double K = beta * V;
      sK += K;
      sKu += K * vx;
      sKv += K * vy;
      sKw += K * vz;
      sKs += K * slip;
    };
    for (int r = 0; r < R.f * R.f; r++) {
      const int k0 = R.row_key(r);
      const int e = start[k0 + R.f];
      for (int q = start[k0] + sl; q < e; q += 2 * kGroup) {
        const bool two = q + kGroup < e;
        const int j0 = order[q], j1 = two ? order[q + kGroup] : j0;
        const VelRec<T> v0 = d.vel[j0], v1 = d.vel[j1];
        const float r0 = d.pos[j0].r, r1 = d.pos[j1].r;
        const float c0 = p.kcg[j0], c1 = p.kcg[j1];
        const int32_t t0 = kGanser ? p.tag[j0] : 0, t1 = kGanser ? p.tag[j1] : 0;
        add(v0, r0, c0, t0);
        if (two) add(v1, r1, c1, t1);
      }
    }
    sK = group_sum(sK);
    sKu = group_sum(sKu);
    sKv = group_sum(sKv);
    sKw = group_sum(sKw);
    sKs = group_sum(sKs);
    if (sl == 0) {
      if (o.sumK) o.sumK[c] = sK;
      if (o.sumKu) o.sumKu[c] = sKu;
      if (o.sumKv) o.sumKv[c] = sKv;
      if (o.sumKw) o.sumKw[c] = sKw;
      if (o.sumKs) o.sumKs[c] = sKs;
    }
  };
  for (int gi = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup; gi < n_list; gi += groups) {
    const int c = list[gi];
    on_bed(bs, [&] { return cell_bed[c]; }, [&](const BedDev &B) { cell(B, c); });
  }
}

void launch_occupied(const int32_t *start, const int32_t *cell_bed, const BedSel &bs, int n_gas, bool sums,
                     const DepositOut &o, int32_t *flags, int32_t *offs, int32_t *scratch, int32_t *list,
                     int32_t *count, hipStream_t s) {
  k_occ_flags<<<(n_gas + 256) / 256, 256, 0, s>>>(start, cell_bed, bs, n_gas, sums ? 1 : 0, o, flags);
  launch_scan(flags, offs, n_gas + 1, scratch, s);
  k_occ_compact<<<(n_gas + 256) / 256, 256, 0, s>>>(flags, offs, n_gas, list, count);
}

template <typename T>
void launch_deposit(const Dyn<T> &d, const Props<T> &p, const GasArgs &g, const int32_t *start,
                    const int32_t *order, const int32_t *cell_bed, const BedSel &bs, const OreDev *ores,
                    const Phys &ph, const int32_t *list, const int32_t *list_count, int max_list, bool sums,
                    const DepositOut &o, hipStream_t s) {
  const int groups_per_block = 256 / kGroup;
  const int blocks = std::max(1, std::min((max_list + groups_per_block - 1) / groups_per_block, 8192));
  // the drag law is a template parameter: the sphericity-corrected law
  // holds many more registers, which the spherical case does not pay for
  if (ph.ganser)
    k_deposit<T, true><<<blocks, 256, 0, s>>>(d, p, g, start, order, cell_bed, bs, ores, ph, list, list_count,
                                              sums ? 1 : 0, o);
  else
    k_deposit<T, false><<<blocks, 256, 0, s>>>(d, p, g, start, order, cell_bed, bs, ores, ph, list, list_count,
                                               sums ? 1 : 0, o);
}

// ------------------------------------------------------------------ reaction
// Environment of a parcel from its gas cell (NGP) and slip, then the update of
// its species (uscm_step), its mass (eq. e3-4), its cell sources (eqs. e2-25,
// e3-52, e4-8) and its weighted reduction degree.
// Quantities of the update that depend on the gas cell only, once per occupied
// cell (the same functions of the same inputs as per parcel, so the same
// values): H2 fraction, equilibria and rate constants at T_g (eqs. e2-1-3,
// e2-12, e2-13), density and viscosity (eqs. e3-53, e3-55, e3-56), the
// molecular and each ore's pore diffusivity (eqs. e2-27..e2-29).
__global__ void k_react_table(GasArgs g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores, int n_ores,
                              const double *theta, const int32_t *list, const int32_t *list_count, double *tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= *list_count) return;
  const int c = list[t];
  const BedDev &B = beds[cell_bed[c]];
  const double Tg = g.T[c], p = g.p[c], xa = g.xH2[c], xb = g.xH2O[c], xn = g.xN2[c];
  const double *th = theta ? theta : B.theta;
  double *r = tab + (long)c * kReactRow;
  r[0] = xb > 0.0 ? xa / (xa + xb) : (xa > 0.0 ? 1.0 : 0.0);
  const double RT = kRg * Tg;
  const double Kc[3] = {exp(1433.4 / Tg + 9.08), exp(-7393.9 / Tg + 7.56), exp(-2023.8 / Tg + 1.24)};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    r[1 + q] = 1.0 / (Kc[q] + 1.0);
    r[4 + q] = (Kc[q] / (1.0 + Kc[q])) / exp(th[2 * q] - th[2 * q + 1] / RT);
  }
  double rho, mu;
  gas_props_h2(Tg, p, xa, xb, xn, B.mu_override, rho, mu);
  r[7] = rho;
  r[8] = mu;
  for (int o = 0; o < n_ores; o++) {
    const PoreDiff Dd = pore_diffusion(Tg, p, xa, xb, xn, ores[o].d_pore_cm);
    r[9] = Dd.Dm;
    r[10 + o] = Dd.D;
  }
}

void launch_react_table(const GasArgs &g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores,
                        int n_ores, const double *theta, const int32_t *list, const int32_t *list_count, int max_list,
                        double *tab, hipStream_t s) {
  k_react_table<<<(max_list + 255) / 256, 256, 0, s>>>(g, cell_bed, beds, ores, n_ores, theta, list, list_count, tab);
}

// The energy equation (kThermo) moves the interface reactions and the pore
// diffusion to the particle temperature, so those stay per parcel; without it
// they come from the cell table when one is given.
template <typename T, bool kThermo>
__device__ __forceinline__ void react_parcel(const ReactArgs<T> &a, const int j, const int32_t tag, const BedDev &B) {
  const OreDev &O = a.ores[ore_of(tag)];
  const PosRec P = load_pos(a.d.pos, j);
  const VelRec<T> Vr = a.d.vel[j];
  Cells cl;
  locate(B, P.x, P.y, P.z, cl);
  const int c = cl.gas;
  const double Tg = a.g.T[c], p = a.g.p[c], xa = a.g.xH2[c], xb = a.g.xH2O[c], xn = a.g.xN2[c];
  const double *th = a.theta ? a.theta : B.theta;
  const double *rw = a.rtab ? a.rtab + (long)c * kReactRow : nullptr;
  // with the energy equation the interface reactions and the pore diffusion
  // run at the particle temperature; film, density and concentration at T_g
  const double Tk = kThermo ? a.p.Tp[j] : Tg;
  const double RT = kRg * Tg, RTk = kRg * Tk;
  UscmEnv<double> e;
  if (!kThermo && rw) {
    e.x = rw[0];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      e.xeq[q] = rw[1 + q];
      e.kk[q] = rw[4 + q];
    }
  } else {
    e.x = xb > 0.0 ? xa / (xa + xb) : (xa > 0.0 ? 1.0 : 0.0);
    // Table 2 equilibria (eq. e2-1-3) and Arrhenius constants (eq. e2-13)
    const double Kc[3] = {exp(1433.4 / Tk + 9.08), exp(-7393.9 / Tk + 7.56), exp(-2023.8 / Tk + 1.24)};
#pragma unroll
    for (int q = 0; q < 3; q++) {
      e.xeq[q] = 1.0 / (Kc[q] + 1.0);
      e.kk[q] = (Kc[q] / (1.0 + Kc[q])) / exp(th[2 * q] - th[2 * q + 1] / RTk);
    }
  }
  const double kcg = (double)a.p.kcg[j];
  const double dp = 2.0 * (double)P.r / kcg, rp = 0.5 * dp, Ap = kPi * dp * dp;
  PoreDiff Dd;
  double rho, mu;
  if (rw) {
    Dd.Dm = rw[9];
    Dd.D = rw[10 + ore_of(tag)];
    rho = rw[7];
    mu = rw[8];
  } else {
    Dd = pore_diffusion(Tg, p, xa, xb, xn, O.d_pore_cm);
    gas_props_h2(Tg, p, xa, xb, xn, B.mu_override, rho, mu);
  }
  const double Dpore = kThermo ? pore_diffusion(Tk, p, xa, xb, xn, O.d_pore_cm).D : Dd.D;
#pragma unroll
  for (int q = 0; q < 3; q++) e.rpD[q] = rp / (Dpore * O.xi_layer[q] / O.tau);
  const double sx = a.g.ug[c] - (double)Vr.v[0], sy = a.g.vg[c] - (double)Vr.v[1], sz = a.g.wg[c] - (double)Vr.v[2];
  const double slip = sqrt(sx * sx + sy * sy + sz * sz);
  e.F = film_resistance(rho, mu, Dd.Dm, a.eps[c], dp, slip);
  e.cad = Ap * (p / RT) * a.dt;
  double n[4] = {a.p.nh[j], a.p.nm[j], a.p.nw[j], a.p.nfe[j]};
  const double n0[4] = {n[0], n[1], n[2], n[3]};
  double xi[3], Qn, Sn;
  const int clamps = uscm_step<double>(n, e, xi, Qn, Sn);
  a.p.nh[j] = n[0];
  a.p.nm[j] = n[1];
  a.p.nw[j] = n[2];
  a.p.nfe[j] = n[3];
  const double k3 = kcg * kcg * kcg;
  const double xs = xi[0] + xi[1] + xi[2];
  const long N = a.n;
  a.pm[j] = -k3 * 2.016e-3 * xs / a.dt;      // eq. e3-52, kg/s
  a.pm[N + j] = k3 * 18.015e-3 * xs / a.dt;  // eq. e2-25
  const double E = -Ap / Tg;                 // eq. e4-8 with eta_H2 = -1
  a.pm[2 * N + j] = k3 * E * Qn;
  a.pm[3 * N + j] = k3 * E * Sn;
  if constexpr (kThermo) {
    const ThermoTab &tt = *a.thermo;
    // eqs. e3-18..e3-21 with the k^3 of eqs. e3-49, e3-50: enthalpies at T_p
    // of the solid species' mole changes and of the H2 taken / H2O given
    double Qr = 0.0, cp = 0.0;
#pragma unroll
    for (int z = 0; z < 4; z++) {
      Qr -= h_mol(tt, kFe2O3 + z, Tk) * (n[z] - n0[z]);
      cp += n[z] * cp_mol(tt, kFe2O3 + z, Tk);
    }
    const double Qm = -(h_mol(tt, kH2O, Tk) - h_mol(tt, kH2, Tk)) * xs;
    a.p.qrx[j] = k3 * (Qr + Qm) / a.dt;
    a.p.mcp[j] = k3 * cp;  // eq. e3-9 times the parcel mass
    // H0, H1 of eqs. e4-4, e4-5 (times V_cell), Q_rm of eq. e3-38 and the
    // gas-species enthalpy flow of eq. e3-39 at T_g
    double lam, cpg;
    gas_heat_props(tt, Tg, xa, xb, xn, lam, cpg);
    const double Re = rho * a.eps[c] * dp * slip / mu;
    const double nu = gunn<double>(a.eps[c], pow(Re, 0.2), pow(Re, 0.7), cbrt(cpg * mu / lam));
    const double hA = k3 * nu * lam * kPi * dp;
    a.pm[4 * N + j] = hA;
    a.pm[5 * N + j] = hA * Tk;
    a.pm[6 * N + j] = k3 * Qm / a.dt;
    a.pm[7 * N + j] = k3 * (h_mol(tt, kH2O, Tg) - h_mol(tt, kH2, Tg)) * xs / a.dt;
  }
  const double fov = fov_of<double>(n, O.kind);
  const double w = k3 * (2.0 * n[0] + 3.0 * n[1] + n[2] + n[3]);
  a.pw[j] = w * fov;
  a.pw[N + j] = w;
  if (a.fov) a.fov[P.id] = fov;
  if (a.update_mass)
    a.d.vel[j].m = T(k3 * 1e-3 * (n[0] * 159.687 + n[1] * 231.531 + n[2] * 71.844 + n[3] * 55.845));
  if (clamps) atomicAdd(a.clamps, (unsigned long long)clamps);
  if (!(isfinite(fov) && n[0] >= 0.0 && n[1] >= 0.0 && n[2] >= 0.0)) atomicOr(a.status, ST_NONFINITE);
}

template <typename T, bool kThermo>
__global__ void __launch_bounds__(256) k_react(ReactArgs<T> a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const int32_t tag = a.p.tag[j];
  on_bed(a.bs, [&] { return bed_of(tag); }, [&](const BedDev &B) { react_parcel<T, kThermo>(a, j, tag, B); });
}

template <typename T>
void launch_react(const ReactArgs<T> &a, hipStream_t s) {
  if (a.thermo)
    k_react<T, true><<<(a.n + 255) / 256, 256, 0, s>>>(a);
  else
    k_react<T, false><<<(a.n + 255) / 256, 256, 0, s>>>(a);
}

// Cell sums of the per-parcel sources in one launch: the first `be` blocks
// write zeros for the empty cells, the others sum each listed (occupied)
// cell with a 16-lane group (lanes take the parcels as in the deposit, two
// per trip).
__global__ void __launch_bounds__(256) k_cellsum(const double *pm, int n, const int32_t *start, const int32_t *order,
                                                 const int32_t *cell_bed, BedSel bs, const int32_t *flags,
                                                 int n_gas, int be, const int32_t *list, const int32_t *list_count,
                                                 CellSumOut o) {
  if ((int)blockIdx.x < be) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_gas; c += be * blockDim.x) {
      if (flags[c]) continue;
#pragma unroll
      for (int q = 0; q < 8; q++)
        if (q < o.rows && o.o[q]) o.o[q][c] = 0.0;
    }
    return;
  }
  const int sl = threadIdx.x % kGroup;
  const int n_list = *list_count;
  const int groups = ((int)gridDim.x - be) * (blockDim.x / kGroup);
  for (int gi = (((int)blockIdx.x - be) * blockDim.x + threadIdx.x) / kGroup; gi < n_list; gi += groups) {
    const int c = list[gi];
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    on_bed(bs, [&] { return cell_bed[c]; }, [&](const BedDev &B) {
      const GasCellRanges R(B, c);
      for (int r = 0; r < R.f * R.f; r++) {
        const int k0 = R.row_key(r);
        const int e = start[k0 + R.f];
        for (int t = start[k0] + sl; t < e; t += 2 * kGroup) {
          const bool two = t + kGroup < e;
          const int j0 = order[t], j1 = two ? order[t + kGroup] : j0;
          double v0[8], v1[8];
#pragma unroll
          for (int q = 0; q < 8; q++)
            if (q < o.rows) {
              v0[q] = pm[(long)q * n + j0];
              v1[q] = pm[(long)q * n + j1];
            }
#pragma unroll
          for (int q = 0; q < 8; q++)
            if (q < o.rows) {
              s[q] += v0[q];
              if (two) s[q] += v1[q];
            }
        }
      }
    });
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (q < o.rows) s[q] = group_sum(s[q]);
    if (sl == 0) {
#pragma unroll
      for (int q = 0; q < 8; q++)
        if (q < o.rows && o.o[q]) o.o[q][c] = s[q];
    }
  }
}

void launch_cellsum(const double *pm, int n, const int32_t *start, const int32_t *order, const int32_t *cell_bed,
                    const BedSel &bs, int n_gas, const int32_t *flags, const int32_t *list,
                    const int32_t *list_count, int max_list, const CellSumOut &o, hipStream_t s) {
  const int be = std::max(1, std::min((n_gas + 255) / 256, 2048));
  const int groups_per_block = 256 / kGroup;
  const int nbs = std::max(1, std::min((max_list + groups_per_block - 1) / groups_per_block, 8192));
  k_cellsum<<<be + nbs, 256, 0, s>>>(pm, n, start, order, cell_bed, bs, flags, n_gas, be, list, list_count, o);
}

// Bed-mean f_ov weighted by k^3 N_Fe: every bed's parcel range (contiguous,
// keys are bed-major) is cut into chunks of kBedChunk parcels; one block sums
// each chunk with a fixed shuffle/LDS tree, then one thread per bed adds its
// chunks in order.  Deterministic, and parallel for a single large bed.
__global__ void __launch_bounds__(256) k_bed_chunks(const int32_t *start, const BedDev *beds, int n_beds,
                                                    int4 *chunks, int max_chunks) {
  // beds in groups of 256: chunk counts, their prefix, then every thread
  // writes chunks of the group (its bed found by bisecting the prefix)
  __shared__ int cnt[256], off[257];
  int base = 0;
  for (int b0 = 0; b0 < n_beds; b0 += 256) {
    const int b = b0 + (int)threadIdx.x;
    int c = 0;
    if (b < n_beds) {
      const int s0 = start[beds[b].dem_off], e0 = start[beds[b].dem_off + beds[b].n_dem];
      c = (e0 - s0 + kBedChunk - 1) / kBedChunk;
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int o = base;
      for (int q = 0; q < 256; q++) {
        off[q] = o;
        o += cnt[q];
      }
      off[256] = o;
    }
    __syncthreads();
    for (int k = off[0] + (int)threadIdx.x; k < off[256]; k += 256) {
      int lo = 0, hi = 256;  // last q with off[q] <= k
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
      }
      const BedDev &B = beds[b0 + lo];
      const int sb = start[B.dem_off], eb = start[B.dem_off + B.n_dem];
      const int q0 = sb + (k - off[lo]) * kBedChunk;
      if (k < max_chunks - 1) chunks[k] = make_int4(b0 + lo, q0, min(q0 + kBedChunk, eb), 0);
    }
    base = off[256];
    __syncthreads();
  }
  if (threadIdx.x == 0) chunks[max_chunks - 1] = make_int4(min(base, max_chunks - 1), 0, 0, 0);  // chunk count
}

__global__ void __launch_bounds__(256) k_chunk_sum(const double *pw, int n, const int4 *chunks, int max_chunks,
                                                    double *partial) {
  const int nch = chunks[max_chunks - 1].x;
  if ((int)blockIdx.x >= nch) return;
  const int4 ch = chunks[blockIdx.x];
  double a = 0.0, b = 0.0;
  for (int j = ch.y + threadIdx.x; j < ch.z; j += blockDim.x) {
    a += pw[j];
    b += pw[(long)n + j];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  __shared__ double sa[4], sb[4];
  if ((threadIdx.x & 63) == 0) {
    sa[threadIdx.x >> 6] = a;
    sb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
    partial[2 * blockIdx.x + 1] = (sb[0] + sb[1]) + (sb[2] + sb[3]);
  }
}

__global__ void __launch_bounds__(256) k_bed_final(const int4 *chunks, int max_chunks, const double *partial,
                                                  double *bed_fov) {
  const int b = blockIdx.x;
  const int nch = chunks[max_chunks - 1].x;
  // chunks are ordered by bed: bisect for this bed's first and last chunk
  int lo = 0, hi = nch;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (chunks[mid].x < b) lo = mid + 1; else hi = mid;
  }
  int e0 = lo, e1 = nch;
  while (e0 < e1) {
    const int mid = (e0 + e1) >> 1;
    if (chunks[mid].x <= b) e0 = mid + 1; else e1 = mid;
  }
  double A = 0.0, Bs = 0.0;
  for (int c = lo + threadIdx.x; c < e0; c += blockDim.x) {
    A += partial[2 * c];
    Bs += partial[2 * c + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    A += __shfl_xor(A, o, 64);
    Bs += __shfl_xor(Bs, o, 64);
  }
  __shared__ double sa[4], sb[4];
  if ((threadIdx.x & 63) == 0) {
    sa[threadIdx.x >> 6] = A;
    sb[threadIdx.x >> 6] = Bs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a2 = (sa[0] + sa[1]) + (sa[2] + sa[3]);
    const double b2 = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    bed_fov[b] = b2 > 0.0 ? a2 / b2 : 0.0;
  }
}

void launch_bedsum(const double *pw, int n, const int32_t *start, const BedDev *beds, int n_beds, int4 *chunks,
                   int max_chunks, double *partial, double *bed_fov, bool table, hipStream_t s) {
  if (table) k_bed_chunks<<<1, 256, 0, s>>>(start, beds, n_beds, chunks, max_chunks);
  if (!pw) return;
  k_chunk_sum<<<max_chunks - 1, 256, 0, s>>>(pw, n, chunks, max_chunks, partial);
  k_bed_final<<<n_beds, 256, 0, s>>>(chunks, max_chunks, partial, bed_fov);
}

// ------------------------------------------------------------------ init / import / export
// heat capacity of a parcel, m C_p,p = k^3 sum_z n_z C_p,z(T_p) (eq. e3-9)
__device__ __forceinline__ double parcel_mcp(const ThermoTab &t, double k, const double n[4], double Tp) {
  double c = 0.0;
#pragma unroll
  for (int z = 0; z < 4; z++) c += n[z] * cp_mol(t, kFe2O3 + z, Tp);
  return k * k * k * c;
}

template <typename T>
__global__ void k_init(dem_parcels in, int n, Phys ph, int n_ores, const ThermoTab *thermo, Dyn<T> d, Props<T> p,
                       uint32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float dd = in.d[i], kk = in.k[i];
  PosRec P;
  P.x = in.x[i];
  P.y = in.y[i];
  P.z = in.z[i];
  P.r = 0.5f * dd;
  P.id = (uint32_t)i;
  store_pos(d.pos, i, P);
  VelRec<T> V;
  V.v[0] = ((const T *)in.vx)[i];
  V.v[1] = ((const T *)in.vy)[i];
  V.v[2] = ((const T *)in.vz)[i];
  V.w[0] = ((const T *)in.wx)[i];
  V.w[1] = ((const T *)in.wy)[i];
  V.w[2] = ((const T *)in.wz)[i];
  const int b = in.bed[i], o = in.ore[i];
  if (b < 0 || b >= ph.n_beds || o < 0 || o >= n_ores || !(dd > 0.0f) || !(kk >= 1.0f)) atomicOr(status, 16u);
  p.kcg[i] = kk;
  const bool ok = b >= 0 && b < ph.n_beds && o >= 0 && o < n_ores;
  p.tag[i] = ok ? b * 256 + o : 0;
  const double nh = in.nh[i], nm = in.nm[i], nw = in.nw[i], nfe = in.nfe[i];
  p.nh[i] = nh;
  p.nm[i] = nm;
  p.nw[i] = nw;
  p.nfe[i] = nfe;
  if (thermo) {
    const double Tp = in.Tp[i];
    if (!(Tp > 0.0 && Tp < 1e4)) atomicOr(status, 16u);
    const double ns[4] = {nh, nm, nw, nfe};
    p.Tp[i] = Tp;
    p.qrx[i] = 0.0;
    p.mcp[i] = parcel_mcp(*thermo, (double)kk, ns, Tp);
  }
  const double k3 = (double)kk * kk * kk;
  V.m = T(k3 * 1e-3 * (nh * 159.687 + nm * 231.531 + nw * 71.844 + nfe * 55.845));  // eq. e3-4
  // eq. e3-45 restitution of the parcel, eq. e3-44 damping ratio
  const double rad = 1.0 + (double)kk * (ph.e_p * ph.e_p - 1.0);
  const double e = rad > 0.0 ? sqrt(rad) : 0.0;
  double z = 1.0;
  if (e > 0.0) {
    const double l = log(e);
    z = -l / sqrt(kPi * kPi + l * l);
  }
  V.zeta = T(z);
  d.vel[i] = V;
#pragma unroll
  for (int k = 0; k < 3 * kMaxWalls; k++) p.wh[(long)k * n + i] = T(0);
}

template <typename T>
void launch_init(const dem_parcels &in, int n, const Phys &ph, int n_ores, const ThermoTab *thermo, const Dyn<T> &d,
                 const Props<T> &p, uint32_t *status, hipStream_t s) {
  k_init<T><<<(n + 255) / 256, 256, 0, s>>>(in, n, ph, n_ores, thermo, d, p, status);
}

template <typename T>
__global__ void k_export(Dyn<T> d, Props<T> p, int n, dem_parcels out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const PosRec P = load_pos(d.pos, j);
  const VelRec<T> V = d.vel[j];
  const uint32_t i = P.id;
  if (out.x) out.x[i] = P.x;
  if (out.y) out.y[i] = P.y;
  if (out.z) out.z[i] = P.z;
  if (out.vx) ((T *)out.vx)[i] = V.v[0];
  if (out.vy) ((T *)out.vy)[i] = V.v[1];
  if (out.vz) ((T *)out.vz)[i] = V.v[2];
  if (out.wx) ((T *)out.wx)[i] = V.w[0];
  if (out.wy) ((T *)out.wy)[i] = V.w[1];
  if (out.wz) ((T *)out.wz)[i] = V.w[2];
  if (out.nh) out.nh[i] = p.nh[j];
  if (out.nm) out.nm[i] = p.nm[j];
  if (out.nw) out.nw[i] = p.nw[j];
  if (out.nfe) out.nfe[i] = p.nfe[j];
  if (out.Tp && p.Tp) out.Tp[i] = p.Tp[j];
}

template <typename T>
void launch_export(const Dyn<T> &d, const Props<T> &p, int n, const dem_parcels &out, hipStream_t s) {
  k_export<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, n, out);
}

template <typename T>
__global__ void k_import(dem_parcels in, int n, const ThermoTab *thermo, Dyn<T> d, Props<T> p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  PosRec P = load_pos(d.pos, j);
  const uint32_t i = P.id;
  P.x = in.x[i];
  P.y = in.y[i];
  P.z = in.z[i];
  store_pos(d.pos, j, P);
  VelRec<T> V = d.vel[j];
  V.v[0] = ((const T *)in.vx)[i];
  V.v[1] = ((const T *)in.vy)[i];
  V.v[2] = ((const T *)in.vz)[i];
  V.w[0] = ((const T *)in.wx)[i];
  V.w[1] = ((const T *)in.wy)[i];
  V.w[2] = ((const T *)in.wz)[i];
  const double nh = in.nh[i], nm = in.nm[i], nw = in.nw[i], nfe = in.nfe[i];
  p.nh[j] = nh;
  p.nm[j] = nm;
  p.nw[j] = nw;
  p.nfe[j] = nfe;
  const double kk = (double)p.kcg[j];
  V.m = T(kk * kk * kk * 1e-3 * (nh * 159.687 + nm * 231.531 + nw * 71.844 + nfe * 55.845));
  if (thermo) {  // new temperature if given; the heat capacity follows, the reaction heat restarts
    const double Tp = in.Tp ? in.Tp[i] : p.Tp[j];
    const double ns[4] = {nh, nm, nw, nfe};
    p.Tp[j] = Tp;
    p.qrx[j] = 0.0;
    p.mcp[j] = parcel_mcp(*thermo, kk, ns, Tp);
  }
  d.vel[j] = V;
#pragma unroll
  for (int k = 0; k < 3 * kMaxWalls; k++) p.wh[(long)k * n + i] = T(0);
}

template <typename T>
void launch_import(const dem_parcels &in, int n, const ThermoTab *thermo, const Dyn<T> &d, const Props<T> &p,
                   hipStream_t s) {
  k_import<T><<<(n + 255) / 256, 256, 0, s>>>(in, n, thermo, d, p);
}

// ------------------------------------------------------------------ gas species
// Gas-side step of the two-way coupling: H2 and H2O transported on the frozen
// flow (eq. e3-40) by first-order upwind convection along z, with the
// particle sources of the last reaction update: H2 semi-implicit through the
// C0, C1 of eqs. e4-9..e4-11, the H2 taken returned as H2O one to one in
// moles.  One thread per gas cell; reads the old fractions, writes new ones.
struct GasPartial {
  double v[3];  // eps_g rho_g Y_j of H2, H2O, N2 (kg per m3 of cell)
};
__device__ __forceinline__ GasPartial gas_partial(double eps, double T, double p, double x1, double x2, double x3) {
  const double M[3] = {2.016e-3, 18.015e-3, 28.013e-3};  // kg/mol
  GasPartial g;
  // eps rho Y_j = eps p x_j M_j / (R T) (eq. e3-53 with Y_j = x_j M_j / M_g)
  const double c = eps * p / (kRg * T);
  g.v[0] = c * x1 * M[0];
  g.v[1] = c * x2 * M[1];
  g.v[2] = c * x3 * M[2];
  return g;
}

__global__ void k_gas_species(GasArgs g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                              double dt, const double *sumEQ, const double *sumES, double xin1, double xin2,
                              double *o1, double *o2, double *o3, uint32_t *status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gas) return;
  const BedDev &B = beds[cell_bed[c]];
  const int q = c - B.gas_off;
  const int layer = B.n[0] * B.n[1];
  const int iz = q / layer;
  const bool has_lo = iz > 0, has_hi = iz < B.n[2] - 1;
  const GasPartial me = gas_partial(eps[c], g.T[c], g.p[c], g.xH2[c], g.xH2O[c], g.xN2[c]);
  // lower face: the state below (or the inlet, at the cell's eps, T, p) moves up
  const double wl = has_lo ? 0.5 * (g.wg[c - layer] + g.wg[c]) : g.wg[c];
  GasPartial lo;
  if (has_lo) {
    const int d = c - layer;
    lo = gas_partial(eps[d], g.T[d], g.p[d], g.xH2[d], g.xH2O[d], g.xN2[d]);
  } else {
    lo = gas_partial(eps[c], g.T[c], g.p[c], xin1, xin2, 1.0 - xin1 - xin2);
  }
  // upper face: this state moves up, or the state above (zero gradient at the top) down
  const double wu = has_hi ? 0.5 * (g.wg[c] + g.wg[c + layer]) : g.wg[c];
  GasPartial hi = me;
  if (has_hi && wu < 0.0) {
    const int d = c + layer;
    hi = gas_partial(eps[d], g.T[d], g.p[d], g.xH2[d], g.xH2O[d], g.xN2[d]);
  }
  const double r = dt / B.h;
  if (fabs(wl) * r > 1.0 || fabs(wu) * r > 1.0) atomicOr(status, 16u);  // Courant number above one
  double rhs[3];
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const double f_lo = wl * (wl >= 0.0 ? lo.v[j] : me.v[j]);
    const double f_hi = wu * (wu >= 0.0 ? me.v[j] : hi.v[j]);
    rhs[j] = me.v[j] - r * (f_hi - f_lo);
  }
  // H2: u (1 - dt C0 T / (X eps)) = rhs + dt C1 p (eq. e4-9), C0 = sum E Q / V,
  // C1 = -(M_H2 / R) sum E S / V
  const double V = B.h * B.h * B.h;
  const double X = g.xH2[c] + g.xH2O[c];
  const double C0 = sumEQ[c] / V, C1 = -(2.016e-3 / kRg) * sumES[c] / V;
  double u1 = rhs[0] + dt * C1 * g.p[c];
  if (X > 0.0) u1 /= 1.0 - dt * C0 * g.T[c] / (X * eps[c]);
  u1 = fmax(u1, 0.0);
  const double u2 = rhs[1] + (rhs[0] - u1) * (18.015 / 2.016);
  const double n1 = u1 / 2.016, n2 = u2 / 18.015, n3 = rhs[2] / 28.013, nt = n1 + n2 + n3;
  o1[c] = n1 / nt;
  o2[c] = n2 / nt;
  o3[c] = n3 / nt;
}

void launch_gas_species(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                        double dt, const double *sumEQ, const double *sumES, double xin1, double xin2, double *o1,
                        double *o2, double *o3, uint32_t *status, hipStream_t s) {
  k_gas_species<<<(n_gas + 255) / 256, 256, 0, s>>>(g, eps, cell_bed, beds, n_gas, dt, sumEQ, sumES, xin1, xin2, o1,
                                                    o2, o3, status);
}

// Gas-side momentum step of the two-way coupling (eqs. e4-1, e4-2 with the
// interphase source of eqs. e3-27, e3-27a) on the frozen pressure field, one
// thread per cell:
//   eps rho (u' - u) / dt = -eps grad p + eps rho g + K_gp u' - K_gp u_p,
// K_gp u_g implicit, K_gp u_p explicit, with K_gp = -sum K / V_cell and
// K_gp u_p = -sum K v / V_cell from the drag sums of the last deposit, so the
// gas takes exactly the drag the parcels feel.  Convection and the viscous
// and pseudo-turbulent stresses belong to the gas solver.
__global__ void k_gas_momentum(GasArgs g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                               double dt, double gx, double gy, double gz, const double *sK, const double *sKu,
                               const double *sKv, const double *sKw, double *uo, double *vo, double *wo,
                               uint32_t *status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gas) return;
  const BedDev &B = beds[cell_bed[c]];
  const double V = B.h * B.h * B.h;
  double rho, mu;
  gas_props_h2(g.T[c], g.p[c], g.xH2[c], g.xH2O[c], g.xN2[c], 1.0, rho, mu);
  const double e = eps[c];
  const double den = e * rho / dt + sK[c] / V;
  const double u[3] = {g.ug[c], g.vg[c], g.wg[c]};
  const double gp[3] = {g.dpdx[c], g.dpdy[c], g.dpdz[c]};
  const double gv[3] = {gx, gy, gz};
  const double Kv[3] = {sKu[c], sKv[c], sKw[c]};
  double r[3];
#pragma unroll
  for (int a = 0; a < 3; a++) r[a] = (e * rho * u[a] / dt - e * gp[a] + e * rho * gv[a] + Kv[a] / V) / den;
  uo[c] = r[0];
  vo[c] = r[1];
  wo[c] = r[2];
  if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) atomicOr(status, ST_NONFINITE);
}

void launch_gas_momentum(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                         double dt, const double grav[3], const double *sK, const double *sKu, const double *sKv,
                         const double *sKw, double *uo, double *vo, double *wo, uint32_t *status, hipStream_t s) {
  k_gas_momentum<<<(n_gas + 255) / 256, 256, 0, s>>>(g, eps, cell_bed, beds, n_gas, dt, grav[0], grav[1], grav[2], sK,
                                                     sKu, sKv, sKw, uo, vo, wo, status);
}

#define INST(T)                                                                                                    \
  template void launch_deposit<T>(const Dyn<T> &, const Props<T> &, const GasArgs &, const int32_t *,             \
                                  const int32_t *, const int32_t *, const BedSel &, const OreDev *, const Phys &, \
                                  const int32_t *, const int32_t *, int, bool, const DepositOut &, hipStream_t);  \
  template void launch_react<T>(const ReactArgs<T> &, hipStream_t);                                               \
  template void launch_init<T>(const dem_parcels &, int, const Phys &, int, const ThermoTab *, const Dyn<T> &,    \
                               const Props<T> &, uint32_t *, hipStream_t);                                         \
  template void launch_export<T>(const Dyn<T> &, const Props<T> &, int, const dem_parcels &, hipStream_t);        \
  template void launch_import<T>(const dem_parcels &, int, const ThermoTab *, const Dyn<T> &, const Props<T> &,  \
                                 hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace demrx
