// Device-side types and helpers shared by the demrx kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/demrx.h"

namespace demrx {

constexpr int kMaxNbr = DEM_MAX_NBR;  // neighbour slots per parcel; mask bits 0..47
constexpr int kWallBit = 48;          // mask bits 48..53: walls
constexpr int kMaxWalls = 6;
constexpr double kPi = 3.14159265358979323846;
constexpr double kRg = 8.314;  // J/(mol K), Section 2.1

enum : uint32_t { ST_OVERFLOW = 1u, ST_DOMAIN = 2u, ST_NONFINITE = 4u, ST_SKIN = 8u };

// One bed as the kernels see it.
struct BedDev {
  double lo[3], hi[3];
  double R, cx, cy;
  double origin[3];
  double h, hd;          // gas cell edge, DEM cell edge (h / refine)
  int n[3], nd[3];       // gas cells, DEM cells per axis
  int refine, wall_kind, n_walls;
  int gas_off, dem_off;  // first gas cell, first DEM cell key of the bed
  int n_gas, n_dem;
  double theta[6];
  double mu_override;
  double rmax;           // largest parcel radius in the bed
  double dbed;           // equivalent-area diameter of the horizontal cross-section
  int tx, ty, ntx;       // key tiles: tx x ty DEM cells in x, y; tiles per x row
};

// Sort key of a DEM cell.  Cells are grouped in columns of tx x ty cells that
// run through the whole bed height; columns follow each other x-fastest, and
// inside a column the order is z, then y, then x.  A run of neighbouring
// cells, and the parcels in them, then stays within a small window of
// memory: one z-plane of a column is tx * ty cells, so the planes above and
// below a cell (its contact neighbours) sit close to it in the sorted arrays.
// Keys of a bed span [dem_off, dem_off + n_dem) with n_dem counting padded
// columns; padding cells stay empty.
__host__ __device__ __forceinline__ int dem_key(const BedDev &b, int x, int y, int z) {
  const int cx = x / b.tx, cy = y / b.ty;
  return b.dem_off + (((cy * b.ntx + cx) * b.nd[2] + z) * b.ty + (y - cy * b.ty)) * b.tx + (x - cx * b.tx);
}

// Per-ore constants: porosities of the Fe3O4, FeO, Fe layers (eqs. e2-31..e2-36)
struct OreDev {
  double xi_layer[3];
  double d_pore_cm, tau;
  double psi;       // sphericity (0: spheres)
  double k1_shape;  // Ganser's Stokes shape factor before the wall correction
  double k2;        // Ganser's Newton shape factor
  int kind;
};

struct Phys {
  double kn, e_p, mu_s, mu_r, kt, gt_ratio, eps_min, skin, dt;
  double g[3];
  int ergun_printed, drag_on, n_beds, n_ores, max_nbr;
  int ganser;  // some ore has a sphericity in (0, 1]
  int energy;  // particle energy equation on
};

// Parcel records, double-buffered (the step reads one buffer and writes the
// other).  One 32-byte position record per parcel, so that a neighbour's
// position, radius and id arrive in one memory transaction; the velocity
// record holds what is only read for parcels in contact.
struct alignas(32) PosRec {
  double x, y, z;
  float r;      // parcel radius d/2 (FP32-representable)
  uint32_t id;  // original parcel id
};
template <typename T>
struct alignas(sizeof(T) * 8) VelRec {
  T v[3], w[3];
  T m;     // parcel mass
  T zeta;  // damping ratio of the parcel's coarse-grained restitution
};
template <typename T>
struct Dyn {
  PosRec *pos;
  VelRec<T> *vel;
};

// Per-parcel properties.  kcg, tag and the species are permuted with the
// parcels at every rebuild; the wall springs, touched only in wall contact,
// stay in original-id order.
template <typename T>
struct Props {
  float *kcg;
  int32_t *tag;  // bed * 256 + ore
  double *nh, *nm, *nw, *nfe;
  T *wh;         // wall tangential springs by original id: [(wall * 3 + axis) * N + id]
  // energy equation only (null otherwise): temperature (K), k^3 (Q_r + Q_rm)
  // of the last reaction update (W) and m C_p,p at that update (J/K)
  double *Tp, *qrx, *mcp;
};

// Four values loaded and stored as one vector record
template <typename T>
struct alignas(sizeof(T) * 4) Quad {
  T x, y, z, w;
};
// Tangential spring of one contact slot; w carries the partner's original id
// (bit pattern in FP32, exact value in FP64) so that a rebuild can match it
template <typename T>
using Spring = Quad<T>;
template <typename T>
__device__ __forceinline__ T spring_tag(uint32_t id);
template <>
__device__ __forceinline__ float spring_tag<float>(uint32_t id) { return __uint_as_float(id); }
template <>
__device__ __forceinline__ double spring_tag<double>(uint32_t id) { return (double)id; }
__device__ __forceinline__ uint32_t spring_partner(float w) { return __float_as_uint(w); }
__device__ __forceinline__ uint32_t spring_partner(double w) { return (uint32_t)w; }

// Neighbour list (slot-major) with the pair tangential springs of each slot
template <typename T>
struct Nbr {
  int32_t *cnt;
  int32_t *idx;       // [slot * N + i] sorted index of the partner
  Spring<T> *hist;    // [slot * N + i]
  uint64_t *mask;     // bit s: slot s in contact last step; bits 48..53: walls
};

// Vector loads of the records (one 16-byte transaction per half)
__device__ __forceinline__ PosRec load_pos(const PosRec *p, long i) {
  const double4 a = *reinterpret_cast<const double4 *>(p + i);
  PosRec r;
  r.x = a.x;
  r.y = a.y;
  r.z = a.z;
  const uint64_t bits = (uint64_t)__double_as_longlong(a.w);
  r.r = __uint_as_float((uint32_t)bits);
  r.id = (uint32_t)(bits >> 32);
  return r;
}
__device__ __forceinline__ void store_pos(PosRec *p, long i, const PosRec &r) {
  const uint64_t bits = ((uint64_t)r.id << 32) | (uint64_t)__float_as_uint(r.r);
  *reinterpret_cast<double4 *>(p + i) = make_double4(r.x, r.y, r.z, __longlong_as_double((long long)bits));
}

// Block index remapped for the 8 XCDs, which receive workgroups in turn:
// each XCD takes chunks of `chunk` consecutive blocks (chunk 1: no remap;
// chunk grid/8: one contiguous range per XCD).  Larger chunks keep a
// neighbourhood's records in one XCD's L2; smaller ones spread the requests
// over more L2 channels and balance the XCDs.  The grid is a multiple of
// 8 * chunk.
__device__ __forceinline__ int xcd_block(int chunk) {
  const int j = (int)(blockIdx.x >> 3), x = (int)(blockIdx.x & 7);
  return (j / chunk) * (8 * chunk) + x * chunk + (j % chunk);
}

__device__ __forceinline__ int bed_of(int32_t tag) { return tag >> 8; }
__device__ __forceinline__ int ore_of(int32_t tag) { return tag & 255; }

// Exact contact predicate terms, evaluated without contraction so that the
// result equals the FP64 reference bit for bit.
__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}
__device__ __forceinline__ double sq_exact(double s) {
#pragma clang fp contract(off)
  return s * s;
}

// Gas cell (nearest grid point) and nested DEM cell of a position.
// Returns false if the position lies outside the bed's grid (then clamped).
struct Cells {
  int gas, dem;  // global indices
  int d[3];      // DEM cell coordinates within the bed
};
__device__ __forceinline__ bool locate(const BedDev &b, double x, double y, double z, Cells &c) {
  const double p[3] = {x, y, z};
  bool inside = true;
  int g[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double rel = p[a] - b.origin[a];
    double f = floor(rel / b.h);
    if (!(f >= 0.0)) { f = 0.0; inside = false; }
    if (f > b.n[a] - 1) { f = b.n[a] - 1; inside = false; }
    g[a] = (int)f;
    int s = 0;
    if (b.refine > 1) {
      double fs = floor((rel - g[a] * b.h) / b.hd);
      s = fs < 0.0 ? 0 : (fs > b.refine - 1 ? b.refine - 1 : (int)fs);
    }
    c.d[a] = g[a] * b.refine + s;
  }
  c.gas = b.gas_off + g[0] + b.n[0] * (g[1] + b.n[1] * g[2]);
  c.dem = dem_key(b, c.d[0], c.d[1], c.d[2]);
  return inside;
}

// Wall w of a bed: signed clearance of the point from the wall surface and the
// unit vector from the point towards the wall.
__device__ __forceinline__ double wall_clearance(const BedDev &b, int w, double x, double y, double z,
                                                 double nv[3]) {
  nv[0] = nv[1] = nv[2] = 0.0;
  if (b.wall_kind == DEM_WALL_BOX) {
    const int ax = w >> 1;
    const double p = ax == 0 ? x : (ax == 1 ? y : z);
    if ((w & 1) == 0) { nv[ax] = -1.0; return p - b.lo[ax]; }
    nv[ax] = 1.0;
    return b.hi[ax] - p;
  }
  if (w == 0) {
    const double rx = x - b.cx, ry = y - b.cy;
    const double rho = sqrt(rx * rx + ry * ry);
    if (rho <= 0.0) return b.R;
    nv[0] = rx / rho;
    nv[1] = ry / rho;
    return b.R - rho;
  }
  if (w == 1) { nv[2] = -1.0; return z - b.lo[2]; }
  nv[2] = 1.0;
  return b.hi[2] - z;
}

template <typename T>
__device__ __forceinline__ T tsqrt(T a);
template <>
__device__ __forceinline__ float tsqrt<float>(float a) { return sqrtf(a); }
template <>
__device__ __forceinline__ double tsqrt<double>(double a) { return sqrt(a); }
template <typename T>
__device__ __forceinline__ T tpow(T a, T e);
template <>
__device__ __forceinline__ float tpow<float>(float a, float e) {
  // a^e for a >= 0 from the hardware's base-2 logarithm and exponential
  // (a few ulp, within the mixed path's FP32 gate; a = 0 gives 0 for e > 0)
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(a));
}
template <>
__device__ __forceinline__ double tpow<double>(double a, double e) { return pow(a, e); }

// Gidaspow drag coefficient divided by eps_p = 1 - eps_g (eq. e3-5-1), so
// that F_d = (beta/eps_p) V (u_g - v) (eq. e3-5) is finite at eps_g = 1.
// Wen-Yu with Schiller-Naumann C_D (Re of eq. e2-23) at eps_g >= 0.8.
// The branch is chosen by the caller (dense: eps_g < 0.8, decided on the
// FP64 voidage, so that an FP32 evaluation takes the branch the FP64 one does).
// The same with eps^-2.65 of the dilute branch passed in (epse), for callers
// that hold it per gas cell.
template <typename T>
__device__ __forceinline__ T beta_over_epsp_e(bool dense, T eps, T epse, T rho, T mu, T slip, T dp, int printed) {
  const T ep = T(1) - eps;
  if (dense) {
    const T inertial = printed ? T(1.75) * eps * rho * slip / (dp * ep) : T(1.75) * rho * slip / dp;
    return T(150) * ep * mu / (eps * dp * dp) + inertial;
  }
  const T re = rho * eps * dp * slip / mu;
  const T cdre = re < T(1000) ? T(24) * (T(1) + T(0.15) * tpow<T>(re, T(0.687))) : T(0.44) * re;
  return T(0.75) * cdre * mu * epse / (dp * dp);
}
template <typename T>
__device__ __forceinline__ T beta_over_epsp(bool dense, T eps, T rho, T mu, T slip, T dp, int printed) {
  return beta_over_epsp_e<T>(dense, eps, dense ? T(0) : tpow<T>(eps, T(-2.65)), rho, mu, slip, dp, printed);
}

// Gidaspow-Ganser drag of particles of sphericity psi (eqs. e3-5-2..e3-5-5),
// divided by eps_p like beta_over_epsp: the dense branch divides the viscous
// term by psi^2 and the inertial one by psi; the dilute branch takes Ganser's
// single-particle C_D with K1 = 1/(1/3 + 2/3 psi^-1/2) - 2.25 dp / Dbed and
// K2 = 10^(1.8148 (-log10 psi)^0.5743) (K1, K2 passed in, per parcel).
template <typename T>
__device__ __forceinline__ T beta_ganser_over_epsp_e(bool dense, T eps, T epse, T rho, T mu, T slip, T dp, T psi, T K1,
                                                     T K2, int printed) {
  const T ep = T(1) - eps;
  if (dense) {
    const T inertial =
        printed ? T(1.75) * eps * rho * slip / (dp * psi * ep) : T(1.75) * rho * slip / (dp * psi);
    return T(150) * ep * mu / (eps * dp * dp * psi * psi) + inertial;
  }
  const T re = rho * eps * dp * slip / mu;
  const T x = re * K1 * K2;
  const T cdre = T(24) / K1 * (T(1) + T(0.1118) * tpow<T>(x, T(0.6567))) +
                 (x > T(0) ? T(0.4305) * K2 * re / (T(1) + T(3305) / x) : T(0));
  return T(0.75) * cdre * mu * epse / (dp * dp);
}
template <typename T>
__device__ __forceinline__ T beta_ganser_over_epsp(bool dense, T eps, T rho, T mu, T slip, T dp, T psi, T K1, T K2,
                                                   int printed) {
  return beta_ganser_over_epsp_e<T>(dense, eps, dense ? T(0) : tpow<T>(eps, T(-2.65)), rho, mu, slip, dp, psi, K1, K2,
                                    printed);
}

// drag coefficient over eps_p of one parcel of ore O in bed B: Gidaspow for
// spheres, Gidaspow-Ganser for a sphericity in (0, 1]
template <typename T>
__device__ __forceinline__ T drag_beta_e(const Phys &ph, const OreDev &O, const BedDev &B, bool dense, T eps, T epse,
                                         T rho, T mu, T slip, T dp) {
  if (ph.ganser && O.psi > 0.0) {
    const T K1 = T(O.k1_shape) - T(2.25) * dp / T(B.dbed);
    return beta_ganser_over_epsp_e<T>(dense, eps, epse, rho, mu, slip, dp, T(O.psi), K1, T(O.k2), ph.ergun_printed);
  }
  return beta_over_epsp_e<T>(dense, eps, epse, rho, mu, slip, dp, ph.ergun_printed);
}
template <typename T>
__device__ __forceinline__ T drag_beta(const Phys &ph, const OreDev &O, const BedDev &B, bool dense, T eps, T rho,
                                       T mu, T slip, T dp) {
  return drag_beta_e<T>(ph, O, B, dense, eps, dense ? T(0) : tpow<T>(eps, T(-2.65)), rho, mu, slip, dp);
}

// Per-gas-cell drag table row, three quads: (ug vg wg eps) (dpdx dpdy dpdz rho)
// (mu lambda Pr^1/3 dense), dense = 1 where the FP64 voidage is below 0.8
constexpr int kGasRow = 12;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace demrx
