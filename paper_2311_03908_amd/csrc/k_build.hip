// Neighbour-list rebuild: counting sort of parcels by DEM cell (cells nest
// inside gas cells, bed-major keys), deterministic in-cell order by original
// id, permutation of the parcel state, and the LDS-staged 27-cell candidate
// scan with wave64 ballot compaction and tangential-spring carry-over.
#include <algorithm>

#include "launch.h"

namespace demrx {

// ------------------------------------------------------------------ fills
// Kernels of the neighbour rebuild take a gate: a device word that the
// rebuild check sets; with a non-null gate holding 0 they return at once, so
// a captured graph holds the rebuild chain and runs it only when needed.
__device__ __forceinline__ bool gated_off(const uint32_t *gate) { return gate && *gate == 0u; }

__global__ void k_fill_i32(int32_t *p, int32_t v, long n, const uint32_t *gate) {
  if (gated_off(gate)) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
static int grid_for(long n, int block, int cap = 65536) {
  long g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
void launch_fill_i32(int32_t *p, int32_t v, long n, hipStream_t s, const uint32_t *gate) {
  if (n > 0) k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n, gate);
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

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t *in, int32_t *out, int32_t *bsum, long m,
                                                              const uint32_t *gate) {
  if (gated_off(gate)) return;
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

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int32_t *bsum, int nb, const uint32_t *gate) {
  if (gated_off(gate)) return;
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

__global__ void k_scan_add(int32_t *out, const int32_t *bsum, long m, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const long i = (long)blockIdx.x * kScanTile + threadIdx.x;
  const int add = bsum[blockIdx.x];
  for (int k = 0; k < kScanItems; k++) {
    const long j = i + (long)k * kScanThreads;
    if (j < m) out[j] += add;
  }
}

long scan_scratch_ints(long m) { return (m + kScanTile - 1) / kScanTile + 1; }

void launch_scan(const int32_t *in, int32_t *out, long m, int32_t *scratch, hipStream_t s, const uint32_t *gate) {
  const int nb = (int)((m + kScanTile - 1) / kScanTile);
  k_scan_tiles<<<nb, kScanThreads, 0, s>>>(in, out, scratch, m, gate);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(scratch, nb, gate);
  k_scan_add<<<nb, kScanThreads, 0, s>>>(out, scratch, m, gate);
}

// ------------------------------------------------------------------ binning
// Bin parcels by DEM cell.  Parcels arrive in the order of the last sort, so
// runs of equal keys are common inside a wave: one atomic per run reserves
// the run's slots.
template <typename T>
__global__ void k_bin(Dyn<T> d, Props<T> p, const BedDev *beds, int n, int32_t *key, int32_t *slot,
                      int32_t *count, uint32_t *status, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int k = -1;
  if (i < n) {
    const PosRec q = load_pos(d.pos, i);
    const BedDev &B = beds[bed_of(p.tag[i])];
    Cells c;
    if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) atomicOr(status, ST_NONFINITE);
    if (!locate(B, q.x, q.y, q.z, c)) atomicOr(status, ST_DOMAIN);
    k = c.dem;
  }
  const int prev = __shfl_up(k, 1, 64);
  const bool head = (i < n) && (lane == 0 || prev != k);
  const uint64_t heads = __ballot(head);
  const uint64_t below = heads & ((2ull << lane) - 1ull);      // heads at or below this lane
  const int my_head = 63 - __clzll((long long)below);
  const uint64_t above = heads & ~((2ull << lane) - 1ull);     // heads after this lane
  const int next_head = above ? __ffsll((unsigned long long)above) - 1 : 64;
  int base = 0;
  if (head) {
    const int len = min(next_head, (int)((n - (i - lane)) < 64 ? (n - (i - lane)) : 64)) - lane;
    base = atomicAdd(&count[k], len);
  }
  base = __shfl(base, my_head, 64);
  if (i < n) {
    key[i] = k;
    slot[i] = base + (lane - my_head);
  }
}

template <typename T>
void launch_bin(const Dyn<T> &d, const Props<T> &p, const BedDev *beds, int n, int32_t *key, int32_t *slot,
                int32_t *count, uint32_t *status, hipStream_t s, const uint32_t *gate) {
  k_bin<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, beds, n, key, slot, count, status, gate);
}

// Counting-sort scatter: parcel i goes to its slot of its cell's range; its x
// and original id are copied along (cell order), for the in-cell rank.
__global__ void k_scatter(const int32_t *key, const int32_t *slot, const int32_t *start, const PosRec *pos, int n,
                          int32_t *perm, CellOrd co, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i];
  const int j = start[k] + slot[i];
  const PosRec P = load_pos(pos, i);
  perm[j] = i;
  co.x[j] = P.x;
  co.id[j] = P.id;
  co.key[j] = k;
}
void launch_scatter(const int32_t *key, const int32_t *slot, const int32_t *start, const PosRec *pos, int n,
                    int32_t *perm, const CellOrd &co, hipStream_t s, const uint32_t *gate) {
  k_scatter<<<(n + 255) / 256, 256, 0, s>>>(key, slot, start, pos, n, perm, co, gate);
}

// Order the parcels of each cell by x, ties by original id (the atomic slot
// order is not reproducible; x order makes every row of cells x-sorted for the
// candidate search): every parcel counts the members of its cell that precede
// it and moves to that rank.  The members' x and id are read from the
// cell-ordered copies of the scatter: one contiguous run per cell, shared by
// the neighbouring threads of the same cell.
__global__ void k_cellrank(const int32_t *start, const int32_t *perm, CellOrd co, int n, int32_t *perm_out,
                           const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = co.key[p];
  const int s = start[c], e = start[c + 1];
  const double x = co.x[p];
  const uint32_t id = co.id[p];
  int rank = 0;
#pragma unroll 4
  for (int q = s; q < e; q++) {
    const double xq = co.x[q];
    rank += (xq < x || (xq == x && co.id[q] < id)) ? 1 : 0;
  }
  perm_out[s + rank] = perm[p];
}
void launch_cellrank(const int32_t *start, const int32_t *perm, const CellOrd &co, int n, int32_t *perm_out,
                     hipStream_t s, const uint32_t *gate) {
  k_cellrank<<<(n + 255) / 256, 256, 0, s>>>(start, perm, co, n, perm_out, gate);
}

// Permutation into the spare buffers (the other step buffer and the spare
// properties), then a copy back: the parcels keep the buffers they live in,
// so no buffer parity depends on whether a rebuild ran.
template <typename T>
__global__ void k_permute(const int32_t *perm, int n, Dyn<T> din, Props<T> pin, Dyn<T> dout, Props<T> pout,
                          float4 *xref, unsigned *dslot, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 2 * kSlots) {  // displacement and speed maxima restart at the rebuild
    dslot[j * kSlotPad] = 0u;
    dslot[j * kSlotPad + 1] = 0u;
  }
  if (j >= n) return;
  const int i = perm[j];
  const PosRec P = load_pos(din.pos, i);
  store_pos(dout.pos, j, P);
  xref[j] = make_float4((float)P.x, (float)P.y, (float)P.z, 0.0f);
  dout.vel[j] = din.vel[i];
  pout.kcg[j] = pin.kcg[i];
  pout.tag[j] = pin.tag[i];
  pout.nh[j] = pin.nh[i];
  pout.nm[j] = pin.nm[i];
  pout.nw[j] = pin.nw[i];
  pout.nfe[j] = pin.nfe[i];
  if (pin.Tp) {
    pout.Tp[j] = pin.Tp[i];
    pout.qrx[j] = pin.qrx[i];
    pout.mcp[j] = pin.mcp[i];
  }
}

template <typename T>
__global__ void k_copy_back(int n, Dyn<T> src, Props<T> psrc, Dyn<T> dst, Props<T> pdst, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  store_pos(dst.pos, j, load_pos(src.pos, j));
  dst.vel[j] = src.vel[j];
  pdst.kcg[j] = psrc.kcg[j];
  pdst.tag[j] = psrc.tag[j];
  pdst.nh[j] = psrc.nh[j];
  pdst.nm[j] = psrc.nm[j];
  pdst.nw[j] = psrc.nw[j];
  pdst.nfe[j] = psrc.nfe[j];
  if (psrc.Tp) {
    pdst.Tp[j] = psrc.Tp[j];
    pdst.qrx[j] = psrc.qrx[j];
    pdst.mcp[j] = psrc.mcp[j];
  }
}

template <typename T>
void launch_permute(const int32_t *perm, int n, const Dyn<T> &d, const Props<T> &p, const Dyn<T> &spare,
                    const Props<T> &pspare, float4 *xref, unsigned *dslot, hipStream_t s, const uint32_t *gate) {
  const int g = (std::max(n, 2 * kSlots) + 255) / 256;
  k_permute<T><<<g, 256, 0, s>>>(perm, n, d, p, spare, pspare, xref, dslot, gate);
  k_copy_back<T><<<(n + 255) / 256, 256, 0, s>>>(n, spare, pspare, d, p, gate);
}

// Contact springs of every parcel (old sorted order) before a rebuild,
// compacted: carry[k * N + p] for its k-th contact (bits 0..47 of the mask in
// ascending slot), carry_meta[p] = (wall bits << 16) | count.  The build
// carries them to the new lists by matching partner ids.
template <typename T>
__global__ void k_carry(Nbr<T> nb, int n, Spring<T> *carry, uint32_t *carry_meta, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const long N = n;
  const uint64_t m = nb.mask[p];
  uint64_t b = m & ((1ull << kWallBit) - 1ull);
  uint32_t k = 0;
  for (; b; b &= b - 1, k++) {
    const int q = __ffsll((unsigned long long)b) - 1;
    carry[(long)k * N + p] = nb.hist[(long)q * N + p];
  }
  carry_meta[p] = ((uint32_t)(m >> kWallBit) << 16) | k;
}

template <typename T>
void launch_carry(const Nbr<T> &nb, int n, Spring<T> *carry, uint32_t *carry_meta, hipStream_t s,
                  const uint32_t *gate) {
  k_carry<T><<<(n + 255) / 256, 256, 0, s>>>(nb, n, carry, carry_meta, gate);
}

// Decide whether the lists must be rebuilt before the next `horizon` steps:
// D, the largest displacement of any parcel since the last rebuild (exact,
// from the FP32 reference positions), and V, the largest speed, both of the
// last step.  The lists hold every pair that can touch while D < skin/2, so
// they are rebuilt when D + grow V, with grow = 2 x horizon x dt (speeds may
// double within the horizon), could reach skin/2.  The step kernel's own
// exact check stays as the safety net.  One block of 64 threads.
__global__ void k_rebuild_check(const unsigned *dslot, int par_last, float lim, float grow, int force, uint32_t *flag,
                                unsigned long long *count) {
  const int t = threadIdx.x;
  float d2 = __uint_as_float(dslot[(par_last * kSlots + t) * kSlotPad]);
  float v2 = __uint_as_float(dslot[(par_last * kSlots + t) * kSlotPad + 1]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d2 = fmaxf(d2, __shfl_xor(d2, o, 64));
    v2 = fmaxf(v2, __shfl_xor(v2, o, 64));
  }
  if (t == 0) {
    const bool rb = force || !(sqrtf(d2) + grow * sqrtf(v2) < lim);
    *flag = rb ? 1u : 0u;
    if (rb) *count += 1ull;
  }
}

void launch_rebuild_check(const unsigned *dslot, int par_last, double skin, double dt, int horizon, int force,
                          uint32_t *flag, unsigned long long *count, hipStream_t s) {
  const float lim = 0.5f * (float)skin - 1e-7f;
  k_rebuild_check<<<1, 64, 0, s>>>(dslot, par_last, lim, (float)(2.0 * horizon * dt), force, flag, count);
}

// ------------------------------------------------------------------ work items
__global__ void k_item_flags(const Item *items, int n_items, const BedDev *beds, const int32_t *start,
                             int32_t *flags, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_items) return;
  if (t == n_items) {
    flags[t] = 0;
    return;
  }
  const Item it = items[t];
  const BedDev &B = beds[it.bed];
  const int xe = min(it.x0 + kItemX, B.nd[0]);
  const int k0 = dem_key(B, it.x0, it.iy, it.iz);
  const int k1 = dem_key(B, xe - 1, it.iy, it.iz) + 1;
  flags[t] = start[k1] > start[k0] ? 1 : 0;
}

__global__ void k_item_compact(const int32_t *flags, const int32_t *offs, int n_items, int32_t *list,
                               int32_t *count, const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_items) return;
  if (t == n_items) {
    *count = offs[n_items];
    return;
  }
  if (flags[t]) list[offs[t]] = t;
}

void launch_items(const Item *items, int n_items, const BedDev *beds, const int32_t *start, int32_t *flags,
                  int32_t *offs, int32_t *scratch, int32_t *list, int32_t *count, hipStream_t s,
                  const uint32_t *gate) {
  k_item_flags<<<(n_items + 256) / 256, 256, 0, s>>>(items, n_items, beds, start, flags, gate);
  launch_scan(flags, offs, n_items + 1, scratch, s, gate);
  k_item_compact<<<(n_items + 256) / 256, 256, 0, s>>>(flags, offs, n_items, list, count, gate);
}

// ------------------------------------------------------------------ neighbour build
// Work item: kItemX consecutive DEM cells of one row of a bed.  The nine rows
// of its 3x3 (y, z) stencil, each spanning x0-1 .. x0+kItemX, are staged in
// LDS (FP32 positions relative to the item corner, radii, sorted indices,
// original ids) as many rows at a time as fit; every thread owns one centre
// parcel of the item and tests the 3 cells of each staged row around its own
// cell, keeping the candidates closer than r_i + r_j + skin (conservative FP32
// test; the exact contact test runs every step).
//
// The list has two regions so that the step visits contacts in lockstep rows:
// candidates that touch now (FP32 test with a 1e-4 margin, a superset of the
// exact contacts) fill slots cap-1, cap-2, ... downwards, the others fill
// slots 0, 1, ... upwards; cnt packs (near << 16) | far.  The tangential
// springs of partners in contact before the rebuild, compacted by k_carry,
// are carried over to the near slots by matching original ids, which every
// spring record carries (read into registers for up to kCarry old contacts;
// more fall back to a loop).
constexpr int kCandMax = 2048;
constexpr int kBuildThreads = 512;
constexpr int kCarry = 8;  // 78 VGPRs: three 512-thread blocks per CU
constexpr float kNear = 1.0f + 1e-4f;

template <typename T>
__global__ void __launch_bounds__(kBuildThreads) k_build_nbr(NbrBuild<T> a) {
  if (gated_off(a.gate)) return;
  __shared__ float4 cpos[kCandMax];
  __shared__ int cidx[kCandMax];
  __shared__ uint32_t cid[kCandMax];
  // each stencil row is staged from up to three runs of keys: the halo cell
  // left of the item, the item's own cells, the halo cell right of it
  __shared__ int sst[9][3], sln[9][3];
  __shared__ int roff[10];
  const int n_list = *a.list_count;
  const long N = a.n;
  const float cut_scale = 1.0f + 1e-5f;
  const int tid = threadIdx.x;
  __shared__ int w_next;
  // blocks take work items from a queue (counter zeroed before the launch),
  // so that items of uneven cost balance over the persistent grid
  for (;;) {
    __syncthreads();
    if (tid == 0) w_next = atomicAdd(a.queue, 1);
    __syncthreads();
    const int w = w_next;
    if (w >= n_list) break;
    const Item it = a.items[a.list[w]];
    const BedDev &B = a.beds[it.bed];
    const int xc = min(kItemX, B.nd[0] - it.x0);
    __syncthreads();
    if (tid < 27) {
      const int r = tid / 3, k = tid % 3;
      const int iy2 = it.iy + (r % 3) - 1, iz2 = it.iz + (r / 3) - 1;
      const int xl = k == 0 ? it.x0 - 1 : (k == 1 ? it.x0 : it.x0 + xc);
      const int xh = k == 1 ? it.x0 + xc - 1 : xl;
      int s0 = 0, ln = 0;
      if (iy2 >= 0 && iy2 < B.nd[1] && iz2 >= 0 && iz2 < B.nd[2] && xl >= 0 && xh < B.nd[0]) {
        s0 = a.start[dem_key(B, xl, iy2, iz2)];
        ln = a.start[dem_key(B, xh, iy2, iz2) + 1] - s0;
      }
      sst[r][k] = s0;
      sln[r][k] = ln;
    }
    __syncthreads();
    const int c0 = sst[4][1], c1 = c0 + sln[4][1];
    const double xr = B.origin[0] + it.x0 * B.hd, yr = B.origin[1] + it.iy * B.hd, zr = B.origin[2] + it.iz * B.hd;
    for (int cb = c0; cb < c1; cb += blockDim.x) {
      const int i = cb + tid;
      const bool mine = i < c1;
      float xi = 0.f, yi = 0.f, zi = 0.f, rs = 0.f, ri = 0.f;
      int nn = 0, nf = 0;  // near / far candidates written
      bool over = false;
      float cut_hi = 0.f;
      // partners in contact before the rebuild: original ids of the first
      // kCarry carried springs (the rest are matched by a loop)
      uint32_t oid[kCarry];
      int po = 0, n_old = 0;
      uint32_t wallbits = 0;
      uint64_t newbits = 0;
#pragma unroll
      for (int k = 0; k < kCarry; k++) oid[k] = 0xffffffffu;
      if (mine) {
        const PosRec pi = load_pos(a.d.pos, i);
        xi = (float)(pi.x - xr);
        yi = (float)(pi.y - yr);
        zi = (float)(pi.z - zr);
        ri = pi.r;
        rs = pi.r + (float)a.skin;
        // widest candidate distance along x for this centre
        cut_hi = (rs + (float)B.rmax) * cut_scale + 1e-9f;
        po = a.perm[i];
        const uint32_t meta = a.carry_meta[po];
        n_old = (int)(meta & 0xffffu);
        wallbits = meta >> 16;
#pragma unroll
        for (int k = 0; k < kCarry; k++)
          if (k < n_old) oid[k] = spring_partner(a.carry[(long)k * N + po].w);
      }
      int row = 0;
      while (row < 9) {
        // as many consecutive rows as fit in LDS
        int re = row, tot = 0;
        while (re < 9) {
          const int len = sln[re][0] + sln[re][1] + sln[re][2];
          if (tot + len > kCandMax) break;
          tot += len;
          re++;
        }
        if (re == row) {  // one row alone exceeds the tile
          if (tid == 0) atomicOr(a.status, ST_OVERFLOW);
          row++;
          continue;
        }
        __syncthreads();
        if (tid == 0) {
          int o = 0;
          for (int r = row; r < re; r++) {
            roff[r] = o;
            o += sln[r][0] + sln[r][1] + sln[r][2];
          }
          roff[re] = o;
        }
        __syncthreads();
        for (int t = tid; t < tot; t += blockDim.x) {
          int r = row;
          while (r + 1 < re && roff[r + 1] <= t) r++;
          const int o = t - roff[r];
          const int j = o < sln[r][0] ? sst[r][0] + o
                                      : (o < sln[r][0] + sln[r][1] ? sst[r][1] + (o - sln[r][0])
                                                                   : sst[r][2] + (o - sln[r][0] - sln[r][1]));
          const PosRec pj = load_pos(a.d.pos, j);
          cpos[t] = make_float4((float)(pj.x - xr), (float)(pj.y - yr), (float)(pj.z - zr), pj.r);
          cidx[t] = j;
          cid[t] = pj.id;
        }
        __syncthreads();
        if (mine) {
          for (int r = row; r < re; r++) {
            // the staged row is sorted by x: bisect the window |x_j - x_i| < cut_hi
            int lo = roff[r], hi = roff[r + 1];
            {
              int a0 = lo, a1 = hi;
              const float xl = xi - cut_hi;
              while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (cpos[mid].x < xl) a0 = mid + 1; else a1 = mid;
              }
              lo = a0;
              a1 = hi;
              const float xh = xi + cut_hi;
              while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (cpos[mid].x <= xh) a0 = mid + 1; else a1 = mid;
              }
              hi = a0;
            }
            for (int q = lo; q < hi; q++) {
              const float4 c = cpos[q];
              const float dx = c.x - xi, dy = c.y - yi, dz = c.z - zi;
              const float cut = (rs + c.w) * cut_scale;
              const int j = cidx[q];
              const float d2 = dx * dx + dy * dy + dz * dz;
              if (j == i || !(d2 < cut * cut)) continue;
              const float sn = (ri + c.w) * kNear;
              if (nn + nf >= a.cap) {
                over = true;
              } else if (d2 < sn * sn) {
                {
                  const int sl = a.cap - 1 - nn;
                  a.nb.idx[(long)sl * N + i] = j;
                  const uint32_t idn = cid[q];
                  int qo = -1;
#pragma unroll
                  for (int k = 0; k < kCarry; k++)
                    if (oid[k] == idn) qo = k;
                  for (int k = kCarry; k < n_old && qo < 0; k++)
                    if (spring_partner(a.carry[(long)k * N + po].w) == idn) qo = k;
                  if (qo >= 0) {
                    a.nb.hist[(long)sl * N + i] = a.carry[(long)qo * N + po];
                    newbits |= 1ull << sl;
                  }
                }
                nn++;
              } else {
                a.nb.idx[(long)nf * N + i] = j;
                nf++;
              }
            }
          }
        }
        row = re;
      }
      if (mine) {
        if (over) atomicOr(a.status, ST_OVERFLOW);
        a.nb.cnt[i] = (nn << 16) | nf;
        a.nb.mask[i] = newbits | ((uint64_t)wallbits << kWallBit);
      }
    }
  }
}

template <typename T>
void launch_build_nbr(const NbrBuild<T> &a, int grid, hipStream_t s) {
  k_build_nbr<T><<<grid, kBuildThreads, 0, s>>>(a);
}

// ------------------------------------------------------------------ pairs
template <typename T>
__global__ void k_pairs(Dyn<T> d, Props<T> p, Nbr<T> nb, int n, int cap_slots, uint32_t *out, long cap,
                        unsigned long long *count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PosRec a = load_pos(d.pos, i);
  const int cw = nb.cnt[i], c_near = cw >> 16, c_far = cw & 0xffff;
  for (int v = 0; v < c_near + c_far; v++) {
    const int s = v < c_near ? cap_slots - 1 - v : v - c_near;
    const int j = nb.idx[(long)s * n + i];
    const PosRec b = load_pos(d.pos, j);
    if (b.id <= a.id) continue;
    const double d2 = dist2_exact(b.x - a.x, b.y - a.y, b.z - a.z);
    const double sr = (double)a.r + (double)b.r;
    if (d2 < sq_exact(sr)) {
      const unsigned long long k = atomicAdd(count, 1ull);
      if ((long)k < cap) {
        out[2 * k] = a.id;
        out[2 * k + 1] = b.id;
      }
    }
  }
}
template <typename T>
void launch_pairs(const Dyn<T> &d, const Props<T> &p, const Nbr<T> &nb, int n, int cap_slots, uint32_t *out, long cap,
                  unsigned long long *count, hipStream_t s) {
  k_pairs<T><<<(n + 255) / 256, 256, 0, s>>>(d, p, nb, n, cap_slots, out, cap, count);
}

#define INST(T)                                                                                                   \
  template void launch_bin<T>(const Dyn<T> &, const Props<T> &, const BedDev *, int, int32_t *, int32_t *,       \
                              int32_t *, uint32_t *, hipStream_t, const uint32_t *);                              \
  template void launch_permute<T>(const int32_t *, int, const Dyn<T> &, const Props<T> &, const Dyn<T> &,        \
                                  const Props<T> &, float4 *, unsigned *, hipStream_t, const uint32_t *);        \
  template void launch_carry<T>(const Nbr<T> &, int, Spring<T> *, uint32_t *, hipStream_t, const uint32_t *);    \
  template void launch_build_nbr<T>(const NbrBuild<T> &, int, hipStream_t);                                      \
  template void launch_pairs<T>(const Dyn<T> &, const Props<T> &, const Nbr<T> &, int, int, uint32_t *, long,         \
                                unsigned long long *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace demrx
