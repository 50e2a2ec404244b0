// Neighbour-list rebuild: counting sort of parcels by DEM cell (cells nest
// inside gas cells, bed-major keys), deterministic in-cell order by original
// id, permutation of the parcel state, and the LDS-staged 27-cell candidate
// scan with wave64 ballot compaction and tangential-spring carry-over.
#include "launch.h"

namespace demrx {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i32(int32_t *p, int32_t v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
static int grid_for(long n, int block, int cap = 65536) {
  long g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
void launch_fill_i32(int32_t *p, int32_t v, long n, hipStream_t s) {
  if (n > 0) k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_fill_u32(uint32_t *p, uint32_t v, long n, hipStream_t s) {
  if (n > 0) k_fill_u32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum: 256 threads x 16 items per block, block totals scanned
// by one block, then added back.
constexpr int kScanThreads = 256, kScanItems = 16, kScanTile = kScanThreads * kScanItems;

__device__ int block_exclusive_scan(int v, int *lds, int &total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
      int t = lds[w];
      lds[w] = acc;
      acc += t;
    }
    lds[15] = acc;
  }
  __syncthreads();
  int r = x - v + lds[wid];
  total = lds[15];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t *in, int32_t *out, int32_t *bsum, long m) {
  __shared__ int lds[16];
  const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    v[k] = (base + k < m) ? in[base + k] : 0;
    sum += v[k];
  }
  int total;
  int run = block_exclusive_scan(sum, lds, total);
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int32_t *bsum, int nb) {
  __shared__ int lds[16];
  int carry = 0;
  for (int base = 0; base < nb; base += kScanTile) {
    const int b0 = base + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      v[k] = (b0 + k < nb) ? bsum[b0 + k] : 0;
      sum += v[k];
    }
    int total;
    int run = block_exclusive_scan(sum, lds, total) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      if (b0 + k < nb) bsum[b0 + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

__global__ void k_scan_add(int32_t *out, const int32_t *bsum, long m) {
  const long i = (long)blockIdx.x * kScanTile + threadIdx.x;
  const int add = bsum[blockIdx.x];
  for (int k = 0; k < kScanItems; k++) {
    const long j = i + (long)k * kScanThreads;
    if (j < m) out[j] += add;
  }
}

long scan_scratch_ints(long m) { return (m + kScanTile - 1) / kScanTile + 1; }

void launch_scan(const int32_t *in, int32_t *out, long m, int32_t *scratch, hipStream_t s) {
  const int nb = (int)((m + kScanTile - 1) / kScanTile);
  k_scan_tiles<<<nb, kScanThreads, 0, s>>>(in, out, scratch, m);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(scratch, nb);
  k_scan_add<<<nb, kScanThreads, 0, s>>>(out, scratch, m);
}

// ------------------------------------------------------------------ binning
template <typename T>
__global__ void k_bin(Dyn<T> d, Props<T> p, const BedDev *beds, int n, int32_t *key, int32_t *slot,
                      int32_t *count, uint32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = d.x[i], y = d.y[i], z = d.z[i];
  const BedDev &B = beds[bed_of(p.tag[i])];
  Cells c;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) atomicOr(status, ST_NONFINITE);
  if (!locate(B, x, y, z, c)) atomicOr(status, ST_DOMAIN);
  key[i] = c.dem;
  slot[i] = atomicAdd(&count[c.dem], 1);
}

template <typename T>
void launch_bin(const Dyn<T> &d, const Props<T> &p, const BedDev *beds, int n, int32_t *key, int32_t *slot,
                int32_t *count, uint32_t *status, hipStream_t s) {
  k_bin<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, beds, n, key, slot, count, status);
}

__global__ void k_scatter(const int32_t *key, const int32_t *slot, const int32_t *start, int n, int32_t *perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[start[key[i]] + slot[i]] = i;
}
void launch_scatter(const int32_t *key, const int32_t *slot, const int32_t *start, int n, int32_t *perm,
                    hipStream_t s) {
  k_scatter<<<(n + 255) / 256, 256, 0, s>>>(key, slot, start, n, perm);
}

// Order the parcels of each cell by original id (the atomic slot order is not
// reproducible); cells hold tens of parcels, so one thread per cell sorts by
// insertion.
__global__ void k_cellsort(const int32_t *start, int n_keys, const uint32_t *id_old, int32_t *perm) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_keys) return;
  const int s = start[c], e = start[c + 1];
  for (int a = s + 1; a < e; a++) {
    const int v = perm[a];
    const uint32_t key = id_old[v];
    int b = a - 1;
    while (b >= s && id_old[perm[b]] > key) {
      perm[b + 1] = perm[b];
      b--;
    }
    perm[b + 1] = v;
  }
}
void launch_cellsort(const int32_t *start, int n_keys, const uint32_t *id_old, int32_t *perm, hipStream_t s) {
  k_cellsort<<<(n_keys + 255) / 256, 256, 0, s>>>(start, n_keys, id_old, perm);
}

template <typename T>
__global__ void k_permute(const int32_t *perm, int n, Dyn<T> din, Props<T> pin, Dyn<T> dout, Props<T> pout,
                          unsigned *vmax, double *disp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    vmax[0] = 0u;
    vmax[1] = 0u;
    disp[0] = 0.0;
  }
  if (j >= n) return;
  const int i = perm[j];
  dout.x[j] = din.x[i];
  dout.y[j] = din.y[i];
  dout.z[j] = din.z[i];
  dout.vx[j] = din.vx[i];
  dout.vy[j] = din.vy[i];
  dout.vz[j] = din.vz[i];
  dout.wx[j] = din.wx[i];
  dout.wy[j] = din.wy[i];
  dout.wz[j] = din.wz[i];
  pout.rad[j] = pin.rad[i];
  pout.kcg[j] = pin.kcg[i];
  pout.mass[j] = pin.mass[i];
  pout.zeta[j] = pin.zeta[i];
  pout.tag[j] = pin.tag[i];
  pout.id[j] = pin.id[i];
  pout.nh[j] = pin.nh[i];
  pout.nm[j] = pin.nm[i];
  pout.nw[j] = pin.nw[i];
  pout.nfe[j] = pin.nfe[i];
#pragma unroll
  for (int k = 0; k < 3 * kMaxWalls; k++) pout.wh[(long)k * n + j] = pin.wh[(long)k * n + i];
}

template <typename T>
void launch_permute(const int32_t *perm, int n, const Dyn<T> &din, const Props<T> &pin, const Dyn<T> &dout,
                    const Props<T> &pout, unsigned *vmax, double *disp, hipStream_t s) {
  k_permute<T><<<(n + 255) / 256, 256, 0, s>>>(perm, n, din, pin, dout, pout, vmax, disp);
}

// ------------------------------------------------------------------ work items
__device__ __forceinline__ int item_key(const BedDev &B, int x, int y, int z) {
  return B.dem_off + x + B.nd[0] * (y + B.nd[1] * z);
}

__global__ void k_item_flags(const Item *items, int n_items, const BedDev *beds, const int32_t *start,
                             int32_t *flags) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_items) return;
  if (t == n_items) {
    flags[t] = 0;
    return;
  }
  const Item it = items[t];
  const BedDev &B = beds[it.bed];
  const int xe = min(it.x0 + kItemX, B.nd[0]);
  const int k0 = item_key(B, it.x0, it.iy, it.iz);
  const int k1 = item_key(B, xe - 1, it.iy, it.iz) + 1;
  flags[t] = start[k1] > start[k0] ? 1 : 0;
}

__global__ void k_item_compact(const int32_t *flags, const int32_t *offs, int n_items, int32_t *list,
                               int32_t *count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_items) return;
  if (t == n_items) {
    *count = offs[n_items];
    return;
  }
  if (flags[t]) list[offs[t]] = t;
}

void launch_items(const Item *items, int n_items, const BedDev *beds, const int32_t *start, int32_t *flags,
                  int32_t *offs, int32_t *scratch, int32_t *list, int32_t *count, hipStream_t s) {
  k_item_flags<<<(n_items + 256) / 256, 256, 0, s>>>(items, n_items, beds, start, flags);
  launch_scan(flags, offs, n_items + 1, scratch, s);
  k_item_compact<<<(n_items + 256) / 256, 256, 0, s>>>(flags, offs, n_items, list, count);
}

// ------------------------------------------------------------------ neighbour build
// Work item: kItemX consecutive DEM cells of one row.  For each of the three
// z-planes of the stencil, the three rows (dy = -1..1) spanning x0-1 .. x0+kItemX
// are staged in LDS (relative FP32 positions and radii, one coalesced pass);
// each wave then takes centre parcels one at a time and its 64 lanes test the
// centre's own 3x3 candidate cells of that plane, compacting hits with a
// ballot.  Candidates are pairs closer than r_i + r_j + skin (conservative
// FP32 test); exact contact is decided each step.
constexpr int kCandMax = 3072;  // staged candidates per plane
constexpr int kCentMax = 512;   // centres per pass
constexpr int kBuildThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kBuildThreads) k_build_nbr(NbrBuild<T> a) {
  __shared__ float4 cpos[kCandMax];
  __shared__ int cidx[kCandMax];
  __shared__ int ccnt[kCentMax];
  __shared__ int rstart[3][kItemX + 3];  // global start of each staged cell (+ end)
  __shared__ int roff[4];                // LDS offset of each staged row
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int n_list = *a.list_count;
  const long N = a.n;
  const float cut_scale = 1.0f + 1e-5f;
  for (int w = blockIdx.x; w < n_list; w += gridDim.x) {
    const Item it = a.items[a.list[w]];
    const BedDev &B = a.beds[it.bed];
    const int xc = min(kItemX, B.nd[0] - it.x0);
    const int c0 = a.start[item_key(B, it.x0, it.iy, it.iz)];
    const int c1 = a.start[item_key(B, it.x0 + xc - 1, it.iy, it.iz) + 1];
    const int xa = max(it.x0 - 1, 0), xb = min(it.x0 + xc, B.nd[0] - 1);
    const int nx = xb - xa + 1;  // staged cells per row
    const double xr = B.origin[0] + it.x0 * B.hd, yr = B.origin[1] + it.iy * B.hd, zr = B.origin[2] + it.iz * B.hd;
    for (int cb = c0; cb < c1; cb += kCentMax) {
      const int nc = min(kCentMax, c1 - cb);
      for (int t = threadIdx.x; t < nc; t += blockDim.x) ccnt[t] = 0;
      for (int dz = -1; dz <= 1; dz++) {
        const int iz2 = it.iz + dz;
        if (iz2 < 0 || iz2 >= B.nd[2]) continue;
        __syncthreads();
        if (threadIdx.x < 3 * (nx + 1)) {
          const int r = threadIdx.x / (nx + 1), q = threadIdx.x % (nx + 1);
          const int iy2 = it.iy + r - 1;
          int v = 0;
          if (iy2 >= 0 && iy2 < B.nd[1]) v = a.start[item_key(B, xa + q, iy2, iz2)];
          rstart[r][q] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          int o = 0;
          for (int r = 0; r < 3; r++) {
            roff[r] = o;
            const int iy2 = it.iy + r - 1;
            if (iy2 >= 0 && iy2 < B.nd[1]) o += rstart[r][nx] - rstart[r][0];
          }
          roff[3] = o;
        }
        __syncthreads();
        const int tot = roff[3];
        if (tot > kCandMax) {
          if (threadIdx.x == 0) atomicOr(a.status, ST_OVERFLOW);
          continue;
        }
        for (int t = threadIdx.x; t < tot; t += blockDim.x) {
          const int r = t >= roff[2] ? 2 : (t >= roff[1] ? 1 : 0);
          const int j = rstart[r][0] + (t - roff[r]);
          cpos[t] = make_float4((float)(a.d.x[j] - xr), (float)(a.d.y[j] - yr), (float)(a.d.z[j] - zr), a.p.rad[j]);
          cidx[t] = j;
        }
        __syncthreads();
        for (int ci = wid; ci < nc; ci += nwave) {
          const int i = cb + ci;
          // x cell of the centre: first staged x whose cell range ends beyond i
          int cx = it.x0;
          while (cx < it.x0 + xc - 1 && a.start[item_key(B, cx, it.iy, it.iz) + 1] <= i) cx++;
          const float xi = (float)(a.d.x[i] - xr), yi = (float)(a.d.y[i] - yr), zi = (float)(a.d.z[i] - zr);
          const float ri = a.p.rad[i];
          const float rs = ri + (float)a.skin;
          const int qa = max(cx - 1, xa) - xa, qb = min(cx + 1, xb) - xa + 1;
          int seg_lo[3], pre[4];
          pre[0] = 0;
#pragma unroll
          for (int r = 0; r < 3; r++) {
            const int iy2 = it.iy + r - 1;
            int len = 0;
            seg_lo[r] = 0;
            if (iy2 >= 0 && iy2 < B.nd[1]) {
              seg_lo[r] = roff[r] + (rstart[r][qa] - rstart[r][0]);
              len = rstart[r][qb] - rstart[r][qa];
            }
            pre[r + 1] = pre[r] + len;
          }
          int cnt = ccnt[ci];
          for (int base = 0; base < pre[3]; base += 64) {
            const int t = base + lane;
            bool hit = false;
            int j = -1;
            if (t < pre[3]) {
              const int r = t >= pre[2] ? 2 : (t >= pre[1] ? 1 : 0);
              const int q = seg_lo[r] + (t - pre[r]);
              const float4 c = cpos[q];
              j = cidx[q];
              const float dx = c.x - xi, dy = c.y - yi, dz2 = c.z - zi;
              const float cut = (rs + c.w) * cut_scale;
              hit = (j != i) && (dx * dx + dy * dy + dz2 * dz2 < cut * cut);
            }
            const uint64_t bal = __ballot(hit);
            const int pos = cnt + __popcll(bal & ((1ull << lane) - 1ull));
            if (hit && pos < a.cap) a.nb_new.idx[(long)pos * N + i] = j;
            cnt += __popcll(bal);
          }
          if (lane == 0) ccnt[ci] = cnt;
        }
      }
      __syncthreads();
      // finalise: counts, overflow, spring carry-over from the old list
      for (int ci = wid; ci < nc; ci += nwave) {
        const int i = cb + ci;
        int cnt = ccnt[ci];
        if (cnt > a.cap) {
          if (lane == 0) atomicOr(a.status, ST_OVERFLOW);
          cnt = a.cap;
        }
        const int po = a.perm[i];
        const uint64_t mo = a.nb_old.mask[po];
        uint32_t my_id = 0xffffffffu;
        if (lane < cnt) my_id = a.p.id[a.nb_new.idx[(long)lane * N + i]];
        uint64_t bits = mo & ((1ull << kWallBit) - 1ull);
        uint64_t newbits = 0;
        while (bits) {
          const int q = __ffsll((unsigned long long)bits) - 1;
          bits &= bits - 1;
          const uint32_t oid = a.id_old[a.nb_old.idx[(long)q * N + po]];
          const bool m = (lane < cnt) && (my_id == oid);
          if (m) {
#pragma unroll
            for (int ax = 0; ax < 3; ax++)
              a.nb_new.hist[((long)ax * kMaxNbr + lane) * N + i] = a.nb_old.hist[((long)ax * kMaxNbr + q) * N + po];
          }
          newbits |= __ballot(m);
        }
        if (lane == 0) {
          a.nb_new.cnt[i] = cnt;
          a.nb_new.mask[i] = newbits | (mo & ~((1ull << kWallBit) - 1ull));
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
void launch_build_nbr(const NbrBuild<T> &a, int grid, hipStream_t s) {
  k_build_nbr<T><<<grid, kBuildThreads, 0, s>>>(a);
}

// ------------------------------------------------------------------ pairs
template <typename T>
__global__ void k_pairs(Dyn<T> d, Props<T> p, Nbr<T> nb, int n, uint32_t *out, long cap, unsigned long long *count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = d.x[i], yi = d.y[i], zi = d.z[i];
  const double ri = p.rad[i];
  const uint32_t idi = p.id[i];
  const int c = nb.cnt[i];
  for (int s = 0; s < c; s++) {
    const int j = nb.idx[(long)s * n + i];
    const uint32_t idj = p.id[j];
    if (idj <= idi) continue;
    const double d2 = dist2_exact(d.x[j] - xi, d.y[j] - yi, d.z[j] - zi);
    const double sr = ri + (double)p.rad[j];
    if (d2 < sq_exact(sr)) {
      const unsigned long long k = atomicAdd(count, 1ull);
      if ((long)k < cap) {
        out[2 * k] = idi;
        out[2 * k + 1] = idj;
      }
    }
  }
}
template <typename T>
void launch_pairs(const Dyn<T> &d, const Props<T> &p, const Nbr<T> &nb, int n, uint32_t *out, long cap,
                  unsigned long long *count, hipStream_t s) {
  k_pairs<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, nb, n, out, cap, count);
}

#define INST(T)                                                                                                   \
  template void launch_bin<T>(const Dyn<T> &, const Props<T> &, const BedDev *, int, int32_t *, int32_t *,       \
                              int32_t *, uint32_t *, hipStream_t);                                                \
  template void launch_permute<T>(const int32_t *, int, const Dyn<T> &, const Props<T> &, const Dyn<T> &,        \
                                  const Props<T> &, unsigned *, double *, hipStream_t);                          \
  template void launch_build_nbr<T>(const NbrBuild<T> &, int, hipStream_t);                                      \
  template void launch_pairs<T>(const Dyn<T> &, const Props<T> &, const Nbr<T> &, int, uint32_t *, long,         \
                                unsigned long long *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace demrx
