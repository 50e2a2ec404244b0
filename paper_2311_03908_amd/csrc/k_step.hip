// One DEM step, fused: exact contact test over the Verlet candidates,
// soft-sphere parcel-parcel and parcel-wall forces with tangential springs,
// Gidaspow drag + gravity + pressure-gradient force, semi-implicit Euler.
// One thread per parcel in cell-sorted order; the step reads buffer `in` and
// writes buffer `out`, so no parcel sees a partner's updated state.  Mode 0
// integrates; mode 1 writes the forces and torques instead (state unchanged);
// mode 2 is the autotuner's timing run: it writes the springs and masks to
// the spare buffers of the rebuild (same addresses within them, so the same
// memory pattern) and skips the reductions.
#include "launch.h"

namespace demrx {

// Reciprocal, square root and reciprocal square root of the contact law: in
// mixed precision the hardware's single-precision instructions (about 1 ulp;
// the forces keep to the FP32 gate), in FP64 the correctly rounded ones.
template <typename T>
__device__ __forceinline__ T law_rcp(T a) {
  return T(1) / a;
}
template <>
__device__ __forceinline__ float law_rcp<float>(float a) {
  return __builtin_amdgcn_rcpf(a);
}
template <typename T>
__device__ __forceinline__ T law_sqrt(T a) {
  return tsqrt<T>(a);
}
template <>
__device__ __forceinline__ float law_sqrt<float>(float a) {
  return __builtin_amdgcn_sqrtf(a);
}
template <typename T>
__device__ __forceinline__ T law_rsq(T a) {
  return T(1) / tsqrt<T>(a);
}
template <>
__device__ __forceinline__ float law_rsq<float>(float a) {
  return __builtin_amdgcn_rsqf(a);
}

// Linear spring-dashpot normal force (no tensile clamp) and Cundall tangential
// spring with Coulomb cap, in the orientation of body a; n points from a to b;
// ikt = 1 / k_t.  The paper defers the contact model to another work; the
// damping ratio follows the coarse-grained restitution of eqs. e3-44/e3-45.
template <typename T>
__device__ __forceinline__ void contact_force(const Phys &ph, T mstar, T zeta, T delta, const T n[3], const T vrel[3],
                                              const T xin[3], T F[3], T Ft[3], T xo[3], T &fn_abs,
                                              T ikt) {
  const T kn = T(ph.kn), dt = T(ph.dt);
  const T gn = T(2) * zeta * law_sqrt<T>(mstar * kn);
  const T vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
  const T fn = -(kn * delta + gn * vn);
  T vt[3];
#pragma unroll
  for (int a = 0; a < 3; a++) vt[a] = vrel[a] - vn * n[a];
  const T xn = xin[0] * n[0] + xin[1] * n[1] + xin[2] * n[2];
#pragma unroll
  for (int a = 0; a < 3; a++) xo[a] = (xin[a] - xn * n[a]) + vt[a] * dt;
  const T kt = T(ph.kt), gt = T(ph.gt_ratio) * gn;
#pragma unroll
  for (int a = 0; a < 3; a++) Ft[a] = -kt * xo[a] - gt * vt[a];
  const T ft2 = Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2];
  const T cap = T(ph.mu_s) * fabs(fn);
  if (ft2 > cap * cap) {
    const T sc = cap * law_rsq<T>(ft2);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      Ft[a] *= sc;
      xo[a] = -(Ft[a] + gt * vt[a]) * ikt;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; a++) F[a] = fn * n[a] + Ft[a];
  fn_abs = fabs(fn);
}

template <typename T>
__device__ __forceinline__ void cross(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Neighbour position records requested kLand at a time land in LDS
// (global_load_lds: 16 B per lane and instruction, written lane-major as a
// 1 KB row) instead of registers.  That leaves the registers to the near
// slots' velocity records and springs, which are requested with the position
// records (mixed precision: 124 VGPRs, 4 waves per SIMD); each wave owns
// kLand record rows of 2 KB (8 KB; 16 waves take 128 KB of a CU's 160 KB).
// The rows are read back by the lane that requested them, after a wait on
// the vector-memory counter, which the LDS writes of these loads decrement.
constexpr int kLand = 4;
constexpr int kLandWaveBytes = kLand * 2048;
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void land_pos(const PosRec *p, int j, unsigned char *row) {
  const unsigned char *g = reinterpret_cast<const unsigned char *>(p + j);
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_void *)row, 16, 0, 0);
  __builtin_amdgcn_global_load_lds((const void *)(g + 16), (lds_void *)(row + 1024), 16, 0, 0);
}
__device__ __forceinline__ PosRec landed_pos(const unsigned char *row) {
  const int l = (int)(threadIdx.x & 63) * 16;
  const double2 a = *reinterpret_cast<const double2 *>(row + l);
  const double2 b = *reinterpret_cast<const double2 *>(row + 1024 + l);
  PosRec r;
  r.x = a.x;
  r.y = a.y;
  r.z = b.x;
  const uint64_t bits = (uint64_t)__double_as_longlong(b.y);
  r.r = __uint_as_float((uint32_t)bits);
  r.id = (uint32_t)(bits >> 32);
  return r;
}
// wait for every outstanding vector-memory load (the landed rows included)
__device__ __forceinline__ void land_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The DEM step of parcel i (sorted index): contacts over its candidate list,
// walls, body and gas forces, integration.  Accumulates the displacement
// maximum and the contact counts of the calling thread.
template <typename T>
__device__ __forceinline__ void step_parcel(const StepArgs<T> &a, const int i, float &dmax2, float &vmax2, int &n_pp,
                                            int &n_w, unsigned char *wl) {
  const long N = a.n;
  {
    const PosRec P = load_pos(a.in.pos, i);
    const VelRec<T> Vi = a.in.vel[i];
    const double xi = P.x, yi = P.y, zi = P.z;
    const float rif = P.r;
    const T ri = T(rif);
    const T mi = Vi.m;
    const T zi_ = Vi.zeta;
    const uint32_t idi = P.id;
    const int32_t tag = a.pr.tag[i];
    const uint64_t mold = a.nb.mask[i];
    uint64_t mnew = 0;
    T F[3] = {T(0), T(0), T(0)}, Tq[3] = {T(0), T(0), T(0)};
    const T wmag = tsqrt<T>(Vi.w[0] * Vi.w[0] + Vi.w[1] * Vi.w[1] + Vi.w[2] * Vi.w[2]);
    const bool roll = a.ph.mu_r > 0.0 && wmag > T(0);
    const T ikt = T(1.0 / a.ph.kt);  // 1 / k_t
    // The list holds the candidates touching at the last rebuild in slots
    // cap-1, cap-2, ... ("near") and the others in slots 0, 1, ... ("far").
    // Each region is visited in lockstep across the wave (near first, where
    // nearly every lane has a contact), so neighbour indices and the
    // slot-major tangential springs of one visit are contiguous rows.
    // Indices and position records are requested kPre slots at a time so
    // that the gathers overlap; the records land in the wave's LDS rows.
    // Both loops run to the wave's largest count (cmax), the same for every
    // lane, so the lanes leave them together.  A wave raises its issue
    // priority while it requests a group's records, so that its loads go
    // out ahead of other waves' arithmetic on the SIMD.
    const int cnt = a.nb.cnt[i];
    const int c_near = cnt >> 16, c_far = cnt & 0xffff;
    // the wave's largest near and far counts.  Active lanes are a prefix of
    // the wave (the parcels past the end sit in its top lanes); a value read
    // from an inactive lane counts 0.  In the xor butterfly, lane 0 then
    // still combines every active lane: whenever it (or a lane feeding it)
    // reads an inactive lane, every lane behind that one is past the end too.
    int2 cmax;
    {
      const uint64_t act = __builtin_amdgcn_read_exec();
      const int lane = (int)(threadIdx.x & 63);
      int cn = c_near, cf = c_far;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const bool on = (act >> (lane ^ o)) & 1ull;
        const int vn = __shfl_xor(cn, o, 64), vf = __shfl_xor(cf, o, 64);
        cn = max(cn, on ? vn : 0);
        cf = max(cf, on ? vf : 0);
      }
      cmax = make_int2(__builtin_amdgcn_readfirstlane(cn), __builtin_amdgcn_readfirstlane(cf));
    }
    const int cap = a.ph.max_nbr;
    uint64_t cbits = 0;
    // pv / ph: the partner's velocity record and the spring, when the caller
    // has already requested them (null: loaded here, after the test)
    auto pair = [&](int s, int j, const PosRec &Q, const VelRec<T> *pv, const Spring<T> *ph) {
      const double dx = Q.x - xi, dy = Q.y - yi, dz = Q.z - zi;
      const double d2 = dist2_exact(dx, dy, dz);
      const double sr = (double)rif + (double)Q.r;
      if (!(d2 < sq_exact(sr))) return;
      cbits |= 1ull << s;
      // pair evaluated in canonical orientation (lower original id first) so
      // both partners obtain bit-identical values with opposite signs
      const bool ifirst = idi < Q.id;
      const T sgn = ifirst ? T(1) : T(-1);
      // unit normal and overlap: in mixed precision from the single-precision
      // reciprocal square root of the FP64 d^2, with the overlap as
      // (s^2 - d^2) / (s + d) (the difference taken in FP64, the distance in
      // the denominator needed only to FP32 accuracy); in FP64 from the
      // correctly rounded distance
      T inv, delta;
      if constexpr (sizeof(T) == 4) {
        const float d2f = (float)d2;
        inv = law_rsq<float>(d2f);
        delta = (float)fma(sr, sr, -d2) * law_rcp<float>((float)sr + d2f * inv);
      } else {
        const double dist = sqrt(d2);
        inv = T(1) / T(dist);
        delta = T(sr - dist);
      }
      const T n[3] = {T(ifirst ? dx : -dx) * inv, T(ifirst ? dy : -dy) * inv, T(ifirst ? dz : -dz) * inv};
      const VelRec<T> Vj = pv ? *pv : a.in.vel[j];
      const T rj = T(Q.r);
      const T ra = ifirst ? ri : rj, rb = ifirst ? rj : ri;
      const T ma = ifirst ? mi : Vj.m, mb = ifirst ? Vj.m : mi;
      T vrel[3], ws[3], cr[3];
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const T va = ifirst ? Vi.v[c] : Vj.v[c], vb = ifirst ? Vj.v[c] : Vi.v[c];
        const T wa = ifirst ? Vi.w[c] : Vj.w[c], wb = ifirst ? Vj.w[c] : Vi.w[c];
        ws[c] = ra * wa + rb * wb;
        vrel[c] = va - vb;
      }
      cross(ws, n, cr);
#pragma unroll
      for (int c = 0; c < 3; c++) vrel[c] += cr[c];
      const T mstar = ma * mb * law_rcp<T>(ma + mb);
      const T zeta = zi_ > Vj.zeta ? zi_ : Vj.zeta;
      T xin[3] = {T(0), T(0), T(0)};
      if ((mold >> s) & 1ull) {
        const Spring<T> h = ph ? *ph : a.nb.hist[(long)s * N + i];
        xin[0] = h.x;
        xin[1] = h.y;
        xin[2] = h.z;
      }
      T Fa[3], Ft[3], xo[3], fnabs;
      contact_force<T>(a.ph, mstar, zeta, delta, n, vrel, xin, Fa, Ft, xo, fnabs, ikt);
      T tq[3];
      cross(n, Ft, tq);
#pragma unroll
      for (int c = 0; c < 3; c++) {
        F[c] += sgn * Fa[c];
        Tq[c] += ri * tq[c];
      }
      if (roll) {
#pragma unroll
        for (int c = 0; c < 3; c++) Tq[c] -= T(a.ph.mu_r) * fnabs * Vi.w[c] / wmag;
      }
      if (a.mode != 1) a.hist_w[(long)s * N + i] = Spring<T>{xo[0], xo[1], xo[2], spring_tag<T>(Q.id)};
      n_pp++;
    };
    constexpr int kPre = kLand;
    // in FP64 the requested records would take 64 more registers
    constexpr bool kNearPrefetch = sizeof(T) == 4;
    for (int t0 = 0; t0 < cmax.x; t0 += kPre) {
      int jj[kPre];
      __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int k = 0; k < kPre; k++) jj[k] = (t0 + k < c_near) ? a.nb.idx[(long)(cap - 1 - t0 - k) * N + i] : -1;
      // every row is requested (a slot past the lane's count lands parcel
      // 0's record, never read), so the requests go out back to back
#pragma unroll
      for (int k = 0; k < kPre; k++) land_pos(a.in.pos, jj[k] >= 0 ? jj[k] : 0, wl + k * 2048);
      if constexpr (kNearPrefetch) {
        // a near slot is nearly always a contact: its partner's velocity
        // record and its spring are requested with the position records,
        // so the group waits for memory once
        VelRec<T> vv[kPre];
        Spring<T> hh[kPre];
#pragma unroll
        for (int k = 0; k < kPre; k++)
          if (jj[k] >= 0) vv[k] = a.in.vel[jj[k]];
#pragma unroll
        for (int k = 0; k < kPre; k++) {
          const int s = cap - 1 - t0 - k;
          if (jj[k] >= 0 && ((mold >> s) & 1ull)) hh[k] = a.nb.hist[(long)s * N + i];
        }
        __builtin_amdgcn_s_setprio(0);
        land_wait();
#pragma unroll
        for (int k = 0; k < kPre; k++)
          if (jj[k] >= 0) pair(cap - 1 - t0 - k, jj[k], landed_pos(wl + k * 2048), &vv[k], &hh[k]);
      } else {
        __builtin_amdgcn_s_setprio(0);
        land_wait();
#pragma unroll
        for (int k = 0; k < kPre; k++)
          if (jj[k] >= 0) pair(cap - 1 - t0 - k, jj[k], landed_pos(wl + k * 2048), nullptr, nullptr);
      }
    }
    {
      // far region: the next group's indices are requested while the
      // current group's position records are in flight
      int jn[kPre];
#pragma unroll
      for (int k = 0; k < kPre; k++) jn[k] = (k < c_far) ? a.nb.idx[(long)k * N + i] : -1;
      for (int t0 = 0; t0 < cmax.y; t0 += kPre) {
        int jj[kPre];
#pragma unroll
        for (int k = 0; k < kPre; k++) jj[k] = jn[k];
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int k = 0; k < kPre; k++)
          if (jj[k] >= 0) land_pos(a.in.pos, jj[k], wl + k * 2048);
#pragma unroll
        for (int k = 0; k < kPre; k++) jn[k] = (t0 + kPre + k < c_far) ? a.nb.idx[(long)(t0 + kPre + k) * N + i] : -1;
        __builtin_amdgcn_s_setprio(0);
        land_wait();
#pragma unroll
        for (int k = 0; k < kPre; k++)
          if (jj[k] >= 0) pair(t0 + k, jj[k], landed_pos(wl + k * 2048), nullptr, nullptr);
      }
    }
    mnew = cbits;
    // walls, gravity, pressure gradient and drag, against the parcel's bed
    auto bed_terms = [&](const BedDev &B) {
      // walls: same law against a body of infinite mass and radius at rest
      for (int w = 0; w < B.n_walls; w++) {
        // a parcel well inside the cylinder's side wall (rho^2 below
        // (R - r)^2 by a relative margin far above rounding) cannot touch
        // it: the square root and the normal are computed only near it
        if (B.wall_kind == DEM_WALL_CYL && w == 0) {
          const double rx = xi - B.cx, ry = yi - B.cy, gap = B.R - (double)rif;
          if (gap > 0.0 && rx * rx + ry * ry < gap * gap * (1.0 - 1e-9)) continue;
        }
        double nv[3];
        const double phi = wall_clearance(B, w, xi, yi, zi, nv);
        const double delw = (double)rif - phi;
        if (!(delw > 0.0)) continue;
        const T n[3] = {T(nv[0]), T(nv[1]), T(nv[2])};
        T wr[3] = {ri * Vi.w[0], ri * Vi.w[1], ri * Vi.w[2]}, cr[3];
        cross(wr, n, cr);
        const T vrel[3] = {Vi.v[0] + cr[0], Vi.v[1] + cr[1], Vi.v[2] + cr[2]};
        T xin[3] = {T(0), T(0), T(0)};
        if ((mold >> (kWallBit + w)) & 1ull) {
#pragma unroll
          for (int c = 0; c < 3; c++) xin[c] = a.pr.wh[(long)(w * 3 + c) * N + idi];
        }
        T Fa[3], Ft[3], xo[3], fnabs;
        contact_force<T>(a.ph, mi, zi_, T(delw), n, vrel, xin, Fa, Ft, xo, fnabs, ikt);
        T tq[3];
        cross(n, Ft, tq);
#pragma unroll
        for (int c = 0; c < 3; c++) {
          F[c] += Fa[c];
          Tq[c] += ri * tq[c];
        }
        if (roll) {
#pragma unroll
          for (int c = 0; c < 3; c++) Tq[c] -= T(a.ph.mu_r) * fnabs * Vi.w[c] / wmag;
        }
        if (a.mode == 0) {
#pragma unroll
          for (int c = 0; c < 3; c++) a.pr.wh[(long)(w * 3 + c) * N + idi] = xo[c];
        }
        mnew |= 1ull << (kWallBit + w);
        n_w++;
      }
      // gravity, pressure gradient and drag (eqs. e3-3, e3-5), NGP gas cell
#pragma unroll
      for (int c = 0; c < 3; c++) F[c] += mi * T(a.ph.g[c]);
      if (a.ph.drag_on || a.ph.energy) {
        Cells cl;
        locate(B, xi, yi, zi, cl);
        const Quad<T> *gq = reinterpret_cast<const Quad<T> *>(a.gtab + (long)cl.gas * kGasRow);
        const Quad<T> g0 = gq[0], g1 = gq[1], g2 = gq[2];
        const T mu = g2.x;
        const T kcg = T(a.pr.kcg[i]);
        const T dpr = T(2) * ri / kcg;  // real-particle diameter
        const T s[3] = {g0.x - Vi.v[0], g0.y - Vi.v[1], g0.z - Vi.v[2]};
        const T slip = tsqrt<T>(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        if (a.ph.drag_on) {
          const T V = T(kPi / 6.0) * (T(2) * ri) * (T(2) * ri) * (T(2) * ri);
          const T be = drag_beta<T>(a.ph, a.ores[ore_of(tag)], B, g2.w != T(0), g0.w, g1.w, mu, slip, dpr);
          F[0] += be * V * s[0] - V * g1.x;
          F[1] += be * V * s[1] - V * g1.y;
          F[2] += be * V * s[2] - V * g1.z;
        }
        if (a.ph.energy && a.mode == 0) {
          // eqs. e3-8, e3-10..e3-13, e3-41: k^3 h_p A_p = k^3 Nu lambda_g pi d_p,
          // with the reaction heat and m C_p,p of the last reaction update
          const T re = g1.w * g0.w * dpr * slip / mu;
          const T nu = gunn<T>(g0.w, tpow<T>(re, T(0.2)), tpow<T>(re, T(0.7)), g2.z);
          const T hA = kcg * kcg * kcg * nu * g2.y * T(kPi) * dpr;
          const double Tp = a.pr.Tp[i];
          const double q = (double)hA * (a.Tg[cl.gas] - Tp) + a.pr.qrx[i];
          a.pr.Tp[i] = Tp + a.ph.dt * q / a.pr.mcp[i];
        }
      }
    };
    // with a single bed its record comes from the kernel arguments (scalar
    // loads, which need no wait on vector memory; a record in global memory
    // is read through vector loads, as the kernel also stores to global
    // memory, and each of its reads costs a memory round trip)
    if (a.ph.n_beds == 1)
      bed_terms(a.bed0);
    else
      bed_terms(a.beds[bed_of(tag)]);
    if (a.mode == 1) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        a.Fout[3 * (long)idi + c] = (double)F[c];
        a.Tout[3 * (long)idi + c] = (double)Tq[c];
      }
    } else {
      const T dt = T(a.ph.dt);
      const T im = T(1) / mi;
      const T iI = T(1) / (T(0.4) * mi * ri * ri);
      VelRec<T> Vo = Vi;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        Vo.v[c] = Vi.v[c] + dt * F[c] * im;
        Vo.w[c] = Vi.w[c] + dt * Tq[c] * iI;
      }
      PosRec Po = P;
      Po.x = xi + a.ph.dt * (double)Vo.v[0];
      Po.y = yi + a.ph.dt * (double)Vo.v[1];
      Po.z = zi + a.ph.dt * (double)Vo.v[2];
      store_pos(a.out.pos, i, Po);
      a.out.vel[i] = Vo;
      if (a.mode != 1 && mnew != mold) a.mask_w[i] = mnew;
      const float v2 = (float)(Vo.v[0] * Vo.v[0] + Vo.v[1] * Vo.v[1] + Vo.v[2] * Vo.v[2]);
      const float4 xr = a.xref[i];
      const float ex = (float)Po.x - xr.x, ey = (float)Po.y - xr.y, ez = (float)Po.z - xr.z;
      dmax2 = fmaxf(dmax2, ex * ex + ey * ey + ez * ez);
      vmax2 = fmaxf(vmax2, v2);
      if (!(isfinite(Po.x) && isfinite(Po.y) && isfinite(Po.z) && isfinite(v2) &&
            isfinite((float)(Vo.w[0] + Vo.w[1] + Vo.w[2]))))
        atomicOr(a.status, ST_NONFINITE);
    }
  }
}

// Wave maximum of the displacement and the contact counts, one no-return
// atomic per wave into one of kSlots padded slots (so waves rarely contend
// and retire independently, with no block barrier)
template <typename T>
__device__ __forceinline__ void step_flush(const StepArgs<T> &a, float dmax2, float vmax2, int n_pp, int n_w) {
  if (a.mode != 0) return;
  float m = dmax2, v = vmax2;
  int c0 = n_pp, c1 = n_w;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmaxf(m, __shfl_xor(m, o, 64));
    v = fmaxf(v, __shfl_xor(v, o, 64));
    c0 += __shfl_xor(c0, o, 64);
    c1 += __shfl_xor(c1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    const int sl = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kSlots - 1));
    atomicMax(a.dslot + (a.par * kSlots + sl) * kSlotPad, __float_as_uint(m));
    atomicMax(a.dslot + (a.par * kSlots + sl) * kSlotPad + 1, __float_as_uint(v));
    if (a.count) {
      if (c0) atomicAdd(a.cslot + sl * kSlotPad64, (unsigned long long)c0);
      if (c1) atomicAdd(a.cslot + sl * kSlotPad64 + 1, (unsigned long long)c1);
    }
  }
}

// Largest displacement of any parcel since the last rebuild, up to the
// positions this step starts from (the previous step's wave maxima are
// complete): the candidate lists hold every pair while it is below skin/2
template <typename T>
__device__ __forceinline__ void step_skin_check(const StepArgs<T> &a) {
  if (a.mode == 0 && blockIdx.x == 0 && threadIdx.x < 64) {
    unsigned *src = a.dslot + ((a.par ^ 1) * kSlots + threadIdx.x) * kSlotPad;
    float d2 = __uint_as_float(*src);
    src[0] = 0u;
    src[1] = 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, o, 64));
    const float lim = 0.5f * (float)a.ph.skin - 1e-7f;  // FP32 reference positions
    if (threadIdx.x == 0 && d2 > lim * lim) atomicOr(a.status, ST_SKIN);
  }
}

// One thread per parcel over the sorted order; (block / 64) * 8 KB of dynamic
// LDS for the landed neighbour records.
template <typename T>
__global__ void __launch_bounds__(512, sizeof(T) == 4 ? 4 : 1) k_step(StepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int i = (a.xcd > 1 ? xcd_block(a.xcd) : (int)blockIdx.x) * blockDim.x + threadIdx.x;
  step_skin_check(a);
  float dmax2 = 0.0f, vmax2 = 0.0f;
  int n_pp = 0, n_w = 0;
  unsigned char *wl = lds + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kLandWaveBytes;
  if (i < a.n) step_parcel(a, i, dmax2, vmax2, n_pp, n_w, wl);
  step_flush(a, dmax2, vmax2, n_pp, n_w);
}

template <typename T>
void launch_step(const StepArgs<T> &a, int block, hipStream_t s) {
  const int q = 8 * (a.xcd > 1 ? a.xcd : 1);  // grid: a multiple of 8 chunks for the XCD remap
  const int g = ((a.n + block - 1) / block + q - 1) / q * q;
  k_step<T><<<g, block, (size_t)(block / 64) * kLandWaveBytes, s>>>(a);
}


template void launch_step<float>(const StepArgs<float> &, int, hipStream_t);
template void launch_step<double>(const StepArgs<double> &, int, hipStream_t);
}  // namespace demrx
