// Kinetic-parameter gradient of the bed-mean reduction degree by a reverse
// (adjoint) sweep over the reaction substeps.
//
// The DEM does not read the reaction state in this protocol (parcel masses
// are frozen), so the reaction environment of every parcel -- its gas cell
// and film resistance during each dynamics interval -- does not depend on the
// kinetic parameters theta = (ln k0_i, Ea_i) and is recorded once.  The
// reaction state lives in original-id order; every parcel is independent, so
// one thread carries a parcel through all substeps:
//   forward:  n_{s+1} = g(n_s; theta), checkpoints every ckpt_every substeps;
//   backward: for each checkpoint segment, last first, replay the segment into
//             a per-parcel buffer, then walk it backwards with
//             lambda_s = lambda_{s+1} dg/dn,  thetabar += lambda_{s+1} dg/dtheta.
// dg is formed by hand: stoichiometry, extent caps and clamps (the branch taken
// by the forward), the network solve differentiated by forward tangents over
// its six resistances, then the resistances' dependence on the remaining
// fractions u = 1 - f and on k_r = exp(ln k0 - Ea / (R T)).
#include "launch.h"
#include "uscm.h"

namespace demrx {

// Per-gas-cell reaction table: x, xeq[3], kk[3] (= K/(1+K)/k_r), 1/(R T), p/(R T)
constexpr int kCtab = 9;

// ------------------------------------------------------------------ tables
__global__ void k_adj_cells(GasArgs g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores, int n_ores,
                            int n_gas, const double *theta, double *ctab, double *dtab) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gas) return;
  const double T = g.T[c], p = g.p[c], xa = g.xH2[c], xb = g.xH2O[c], xn = g.xN2[c];
  const double RT = kRg * T;
  const double *th = theta ? theta : beds[cell_bed[c]].theta;
  double *r = ctab + (long)c * kCtab;
  r[0] = xb > 0.0 ? xa / (xa + xb) : (xa > 0.0 ? 1.0 : 0.0);
  const double Kc[3] = {exp(1433.4 / T + 9.08), exp(-7393.9 / T + 7.56), exp(-2023.8 / T + 1.24)};
  for (int q = 0; q < 3; q++) {
    r[1 + q] = 1.0 / (Kc[q] + 1.0);
    r[4 + q] = (Kc[q] / (1.0 + Kc[q])) / exp(th[2 * q] - th[2 * q + 1] / RT);
  }
  r[7] = 1.0 / RT;
  r[8] = p / RT;
  for (int o = 0; o < n_ores; o++) {
    const PoreDiff D = pore_diffusion(T, p, xa, xb, xn, ores[o].d_pore_cm);
    for (int q = 0; q < 3; q++) dtab[((long)c * n_ores + o) * 3 + q] = ores[o].tau / (D.D * ores[o].xi_layer[q]);
  }
}

// Static parcel data and the initial reaction state, scattered to original order.
template <typename T, typename S>
__global__ void k_adj_static(Dyn<T> d, Props<T> p, const OreDev *ores, int n, double *dp, double *k3, int32_t *ore,
                             int32_t *kind, S *state) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const PosRec P = load_pos(d.pos, j);
  const uint32_t id = P.id;
  const double kc = (double)p.kcg[j];
  dp[id] = 2.0 * (double)P.r / kc;
  k3[id] = kc * kc * kc;
  const int o = ore_of(p.tag[j]);
  ore[id] = o;
  kind[id] = ores[o].kind;
  state[id] = S(p.nh[j]);
  state[(long)n + id] = S(p.nm[j]);
  state[2L * n + id] = S(p.nw[j]);
  state[3L * n + id] = S(p.nfe[j]);
}

// Environment of one dynamics interval: gas cell (NGP) and film resistance.
template <typename T>
__global__ void k_adj_record(Dyn<T> d, Props<T> p, GasArgs g, const double *eps, const BedDev *beds, int n,
                             int32_t *rec_cell, double *rec_F) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const PosRec P = load_pos(d.pos, j);
  const VelRec<T> V = d.vel[j];
  const BedDev &B = beds[bed_of(p.tag[j])];
  Cells cl;
  locate(B, P.x, P.y, P.z, cl);
  const int c = cl.gas;
  const double T_ = g.T[c], pg = g.p[c], xa = g.xH2[c], xb = g.xH2O[c], xn = g.xN2[c];
  double rho, mu;
  gas_props_h2(T_, pg, xa, xb, xn, B.mu_override, rho, mu);
  const double Dm = pore_diffusion(T_, pg, xa, xb, xn, 1.0).Dm;
  const double sx = g.ug[c] - (double)V.v[0], sy = g.vg[c] - (double)V.v[1], sz = g.wg[c] - (double)V.v[2];
  const double dp = 2.0 * (double)P.r / (double)p.kcg[j];
  rec_cell[P.id] = c;
  rec_F[P.id] = film_resistance(rho, mu, Dm, eps[c], dp, sqrt(sx * sx + sy * sy + sz * sz));
}

template <typename S>
__device__ __forceinline__ void load_env(const AdjArgs &a, int i, int k, UscmEnv<S> &e, double &irt) {
  const long slot = k - a.k_base;
  const int c = a.rec_cell[slot * a.n + i];
  const double F = a.rec_F[slot * a.n + i];
  const double *r = a.ctab + (long)c * kCtab;
  const double *dt3 = a.dtab + ((long)c * a.n_ores + a.ore[i]) * 3;
  const double dp = a.dp[i];
  e.x = S(r[0]);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    e.xeq[q] = S(r[1 + q]);
    e.kk[q] = S(r[4 + q]);
    e.rpD[q] = S(0.5 * dp * dt3[q]);
  }
  e.F = S(F);
  e.cad = S(kPi * dp * dp * r[8] * a.dt);
  irt = r[7];
}

template <typename S>
__device__ __forceinline__ void block_sum8(double v[8], double *part) {
  __shared__ double sm[4][8];
#pragma unroll
  for (int k = 0; k < 8; k++) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 8; k++) sm[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = (sm[0][threadIdx.x] + sm[1][threadIdx.x]) +
                                                           (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
}

// ------------------------------------------------------------------ forward
template <typename S>
__global__ void __launch_bounds__(256) k_adj_forward(AdjArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < a.n) {
    S *st = (S *)a.state;
    S nn[4];
#pragma unroll
    for (int q = 0; q < 4; q++) nn[q] = st[(long)q * a.n + i];
    int kcur = -1;
    UscmEnv<S> e;
    double irt;
    for (int s = a.s_begin; s < a.s_end; s++) {
      if (a.ckpt && s % a.ckpt_every == 0) {
        S *ck = (S *)a.ckpt + (long)(s / a.ckpt_every) * 4 * a.n;
#pragma unroll
        for (int q = 0; q < 4; q++) ck[(long)q * a.n + i] = nn[q];
      }
      const int k = s / a.dyn_every;
      if (k != kcur) {
        load_env<S>(a, i, k, e, irt);
        kcur = k;
      }
      S xi[3], Q, Sv;
      uscm_step<S>(nn, e, xi, Q, Sv);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) st[(long)q * a.n + i] = nn[q];
    const double w = a.k3[i] * (2.0 * (double)nn[0] + 3.0 * (double)nn[1] + (double)nn[2] + (double)nn[3]);
    v[0] = w * fov_of<S>(nn, a.kind[i]);
    v[1] = w;
  }
  if (a.part) block_sum8<S>(v, a.part);
}

// ------------------------------------------------------------------ backward
template <typename C>
struct D6 {  // value and tangents w.r.t. (A0, A1, A2, B0, B1, B2)
  C v, d[6];
};
template <typename C>
__device__ __forceinline__ D6<C> dc(C v) {
  D6<C> r;
  r.v = v;
#pragma unroll
  for (int t = 0; t < 6; t++) r.d[t] = C(0);
  return r;
}
template <typename C>
__device__ __forceinline__ D6<C> dvar(C v, int t) {
  D6<C> r = dc<C>(v);
  r.d[t] = C(1);
  return r;
}
template <typename C>
__device__ __forceinline__ D6<C> operator+(const D6<C> &a, const D6<C> &b) {
  D6<C> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int t = 0; t < 6; t++) r.d[t] = a.d[t] + b.d[t];
  return r;
}
template <typename C>
__device__ __forceinline__ D6<C> operator-(const D6<C> &a, const D6<C> &b) {
  D6<C> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int t = 0; t < 6; t++) r.d[t] = a.d[t] - b.d[t];
  return r;
}
template <typename C>
__device__ __forceinline__ D6<C> operator*(const D6<C> &a, const D6<C> &b) {
  D6<C> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int t = 0; t < 6; t++) r.d[t] = a.d[t] * b.v + a.v * b.d[t];
  return r;
}
template <typename C>
__device__ __forceinline__ D6<C> operator/(const D6<C> &a, const D6<C> &b) {
  D6<C> r;
  const C ib = C(1) / b.v;
  r.v = a.v * ib;
#pragma unroll
  for (int t = 0; t < 6; t++) r.d[t] = (a.d[t] - r.v * b.d[t]) * ib;
  return r;
}

template <typename C>
__device__ __forceinline__ C icbrt_c(C u);
template <>
__device__ __forceinline__ float icbrt_c<float>(float u) { return 1.0f / cbrtf(u); }
template <>
__device__ __forceinline__ double icbrt_c<double>(double u) { return 1.0 / cbrt(u); }

// lam <- lam dg/dn, tb += lam dg/dtheta at state n (vector-Jacobian product of
// uscm_step).  The partial derivatives are formed in C (float for an FP32
// reaction state: their rounding is far below the state's own); lam and the
// theta accumulators stay in FP64.
template <typename C>
__device__ __forceinline__ void uscm_vjp(const double n[4], const UscmEnv<double> &e, double irt, double lam[4], double tb[6]) {
  const double Nfe = 2.0 * n[0] + 3.0 * n[1] + n[2] + n[3];
  const double cum[3] = {2.0 * n[0], 2.0 * n[0] + 3.0 * n[1], 2.0 * n[0] + 3.0 * n[1] + n[2]};
  bool act[3];
  int inner = 3;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    act[q] = n[q] > 1e-12 * Nfe && e.x > e.xeq[q];
    if (act[q] && inner == 3) inner = q;
  }
  if (inner == 3) return;
  C u[3], ic[3], A[3], Bv[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    u[q] = C(cum[q] / Nfe);
    ic[q] = q >= inner ? icbrt_c<C>(u[q]) : C(0);
  }
#pragma unroll
  for (int q = 0; q < 3; q++) {
    A[q] = act[q] ? ic[q] * ic[q] * C(e.kk[q]) : C(1);
    const C outer = q < 2 ? ic[q + 1] : C(1);
    Bv[q] = q >= inner ? (ic[q] - outer) * C(e.rpD[q]) : C(0);
  }
  // network solve with tangents over (A, B); loops unrolled over the three
  // interfaces so that every array index is static (no scratch)
  D6<C> Ad[3], Bd[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    Ad[q] = dvar<C>(A[q], q);
    Bd[q] = dvar<C>(Bv[q], 3 + q);
  }
  const C ex = C(e.x), eF = C(e.F);
  D6<C> R = inner == 0 ? Ad[0] : (inner == 1 ? Ad[1] : Ad[2]);
  D6<C> Phi = dc<C>(C(inner == 0 ? e.xeq[0] : (inner == 1 ? e.xeq[1] : e.xeq[2])));
#pragma unroll
  for (int q = 1; q < 3; q++) {
    if (q <= inner) continue;
    R = R + Bd[q - 1];
    if (act[q]) {
      const D6<C> one = dc<C>(C(1));
      const D6<C> g1 = one / R, g2 = one / Ad[q];
      Phi = (Phi * g1 + dc<C>(C(e.xeq[q])) * g2) / (g1 + g2);
      R = one / (g1 + g2);
    }
  }
  const D6<C> Rt = R + Bd[2] + dc<C>(eF);
  const D6<C> flux = (dc<C>(ex) - Phi) / Rt;
  D6<C> pot = dc<C>(ex) - flux * (dc<C>(eF) + Bd[2]);
  D6<C> rest = flux;
  D6<C> r[3] = {dc<C>(C(0)), dc<C>(C(0)), dc<C>(C(0))};
#pragma unroll
  for (int q = 2; q >= 0; q--) {
    if (q < inner) continue;
    if (act[q]) {
      r[q] = (pot - dc<C>(C(e.xeq[q]))) / Ad[q];
      rest = rest - r[q];
    }
    if (q > inner) pot = pot - rest * Bd[q - 1];
  }
  // stoichiometry and extents (the branch the forward took)
  const double xb[3] = {-3.0 * lam[0] + 2.0 * lam[1], -lam[1] + 3.0 * lam[2], -lam[2] + lam[3]};
  const double nu[3] = {3.0, 1.0, 1.0};
  double nl[4] = {lam[0], lam[1], lam[2], lam[3]};
  double Ab[3] = {0, 0, 0}, Bb[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    if (r[q].v < C(0)) continue;                         // clamped: no dependence
    if ((double)r[q].v * e.cad > n[q] / nu[q]) {         // capped by the reactant
      nl[q] += xb[q] / nu[q];
      continue;
    }
    const double rb = e.cad * xb[q];
#pragma unroll
    for (int t = 0; t < 3; t++) {
      Ab[t] += rb * (double)r[q].d[t];
      Bb[t] += rb * (double)r[q].d[3 + t];
    }
  }
  // resistances -> theta and remaining fractions
  double ab[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    if (act[q]) {
      tb[2 * q] += -Ab[q] * (double)A[q];
      tb[2 * q + 1] += Ab[q] * (double)A[q] * irt;
      ab[q] += Ab[q] * 2.0 * (double)ic[q] * e.kk[q];
    }
    if (q >= inner) {
      ab[q] += Bb[q] * e.rpD[q];
      if (q < 2) ab[q + 1] -= Bb[q] * e.rpD[q];
    }
  }
  // u_q = cum_q / N with dcum/dn = (2,0,0,0), (2,3,0,0), (2,3,1,0) and dN/dn = (2,3,1,1)
  const double dcum[3][4] = {{2, 0, 0, 0}, {2, 3, 0, 0}, {2, 3, 1, 0}};
  const double dN[4] = {2, 3, 1, 1};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    if (q < inner) continue;
    const double uq = cum[q] / Nfe;
    const double ub = ab[q] * (-(double)ic[q] / (3.0 * uq));
#pragma unroll
    for (int z = 0; z < 4; z++) nl[z] += ub * (dcum[q][z] - uq * dN[z]) / Nfe;
  }
  for (int z = 0; z < 4; z++) lam[z] = nl[z];
}

// d f_ov / d n at state n (eqs. e2-18, e2-19 through u = cum / N)
__device__ __forceinline__ void dfov_dn(const double n[4], int kind, double g[4]) {
  const double Nfe = 2.0 * n[0] + 3.0 * n[1] + n[2] + n[3];
  const double cum[3] = {2.0 * n[0], 2.0 * n[0] + 3.0 * n[1], 2.0 * n[0] + 3.0 * n[1] + n[2]};
  const double wq[3] = {kind == 1 ? 0.0 : 1.0 / 9.0, kind == 1 ? 0.25 : 2.0 / 9.0, kind == 1 ? 0.75 : 6.0 / 9.0};
  const double dcum[3][4] = {{2, 0, 0, 0}, {2, 3, 0, 0}, {2, 3, 1, 0}};
  const double dN[4] = {2, 3, 1, 1};
  for (int z = 0; z < 4; z++) g[z] = 0.0;
  for (int q = 0; q < 3; q++) {
    const double u = cum[q] / Nfe;
    for (int z = 0; z < 4; z++) g[z] -= wq[q] * (dcum[q][z] - u * dN[z]) / Nfe;  // f = 1 - u
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_adj_backward(AdjArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < a.n) {
    const long N = a.n;
    S *seg = (S *)a.seg;
    const int n_ckpt = (a.n_sub + a.ckpt_every - 1) / a.ckpt_every;
    double lam[4], tb[6] = {0, 0, 0, 0, 0, 0};
    for (int c = n_ckpt - 1; c >= 0; c--) {
      const int s0 = c * a.ckpt_every, s1 = min(s0 + a.ckpt_every, a.n_sub);
      const S *ck = (const S *)a.ckpt + (long)c * 4 * N;
      S nn[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        nn[q] = ck[(long)q * N + i];
        seg[(long)q * N + i] = nn[q];
      }
      int kcur = -1;
      UscmEnv<S> e;
      double irt;
      for (int s = s0; s < s1; s++) {
        const int k = s / a.dyn_every;
        if (k != kcur) {
          load_env<S>(a, i, k, e, irt);
          kcur = k;
        }
        S xi[3], Q, Sv;
        uscm_step<S>(nn, e, xi, Q, Sv);
        S *dst = seg + (long)(s - s0 + 1) * 4 * N;
#pragma unroll
        for (int q = 0; q < 4; q++) dst[(long)q * N + i] = nn[q];
      }
      if (c == n_ckpt - 1) {  // dJ/dn at the final state: (w / sum w) df_ov/dn
        const double nf[4] = {(double)nn[0], (double)nn[1], (double)nn[2], (double)nn[3]};
        double g[4];
        dfov_dn(nf, a.kind[i], g);
        const double w = a.k3[i] * (2.0 * nf[0] + 3.0 * nf[1] + nf[2] + nf[3]);
        for (int z = 0; z < 4; z++) lam[z] = a.inv_W * w * g[z];
      }
      // substeps of the segment, last first, grouped by dynamics interval so
      // that each interval's environment is loaded once
      for (int s = s1 - 1; s >= s0;) {
        const int k = s / a.dyn_every;
        const int s_lo = max(s0, k * a.dyn_every);
        UscmEnv<double> ed;
        double irt_k;
        load_env<double>(a, i, k, ed, irt_k);
        for (; s >= s_lo; s--) {
          const S *src = seg + (long)(s - s0) * 4 * N;
          const double ns[4] = {(double)src[i], (double)src[N + i], (double)src[2 * N + i], (double)src[3 * N + i]};
          uscm_vjp<S>(ns, ed, irt_k, lam, tb);
        }
      }
    }
    for (int t = 0; t < 6; t++) v[2 + t] = tb[t];
  }
  block_sum8<S>(v, a.part);
}

// ------------------------------------------------------------------ launchers
int adjoint_blocks(int n) { return (n + 255) / 256; }

void launch_adj_cells(const GasArgs &g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores, int n_ores,
                      int n_gas, const double *theta, double *ctab, double *dtab, hipStream_t s) {
  k_adj_cells<<<(n_gas + 255) / 256, 256, 0, s>>>(g, cell_bed, beds, ores, n_ores, n_gas, theta, ctab, dtab);
}

template <typename T, typename S>
void launch_adj_static(const Dyn<T> &d, const Props<T> &p, const OreDev *ores, int n, double *dp, double *k3,
                       int32_t *ore, int32_t *kind, S *state, hipStream_t s) {
  k_adj_static<T, S><<<(n + 255) / 256, 256, 0, s>>>(d, p, ores, n, dp, k3, ore, kind, state);
}

template <typename T>
void launch_adj_record(const Dyn<T> &d, const Props<T> &p, const GasArgs &g, const double *eps, const BedDev *beds,
                       int n, int32_t *rec_cell, double *rec_F, hipStream_t s) {
  k_adj_record<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, g, eps, beds, n, rec_cell, rec_F);
}

void launch_adjoint_forward(const AdjArgs &a, int fp32, hipStream_t s) {
  if (fp32)
    k_adj_forward<float><<<adjoint_blocks(a.n), 256, 0, s>>>(a);
  else
    k_adj_forward<double><<<adjoint_blocks(a.n), 256, 0, s>>>(a);
}

void launch_adjoint_backward(const AdjArgs &a, int fp32, hipStream_t s) {
  if (fp32)
    k_adj_backward<float><<<adjoint_blocks(a.n), 256, 0, s>>>(a);
  else
    k_adj_backward<double><<<adjoint_blocks(a.n), 256, 0, s>>>(a);
}

#define INST(T, S)                                                                                               \
  template void launch_adj_static<T, S>(const Dyn<T> &, const Props<T> &, const OreDev *, int, double *, double *, \
                                        int32_t *, int32_t *, S *, hipStream_t);
INST(float, float)
INST(float, double)
INST(double, float)
INST(double, double)
#undef INST
template void launch_adj_record<float>(const Dyn<float> &, const Props<float> &, const GasArgs &, const double *,
                                       const BedDev *, int, int32_t *, double *, hipStream_t);
template void launch_adj_record<double>(const Dyn<double> &, const Props<double> &, const GasArgs &, const double *,
                                        const BedDev *, int, int32_t *, double *, hipStream_t);

}  // namespace demrx
