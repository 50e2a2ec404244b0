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

// Exclusive scan: tiles, then the tile sums (one block), then the offsets.
// With `clear` the input is zeroed as it is read (a counter array that must
// start its next use at zero).  (A single-pass variant that lets the last
// tile's block scan the tile sums needs a device-scope fence per block,
// which writes back the XCD's L2 each time: slower here than a launch.)
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int32_t *in, int32_t *out, int32_t *bsum, long m,
                                                              int clear, const uint32_t *gate) {
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
  if (clear) {
#pragma unroll
    for (int k = 0; k < kScanItems; k++)
      if (base + k < m) in[base + k] = 0;
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

void launch_scan(int32_t *in, int32_t *out, long m, int32_t *scratch, hipStream_t s, const uint32_t *gate,
                 bool clear) {
  const int nb = (int)((m + kScanTile - 1) / kScanTile);
  k_scan_tiles<<<nb, kScanThreads, 0, s>>>(in, out, scratch, m, clear ? 1 : 0, gate);
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
// it and moves to that rank.  The members' x and id come from the cell-ordered
// copies of the scatter, one contiguous run per cell; each block first stages
// its window of those copies (its own positions and kRankHalo on either side)
// in LDS, and reads from there whenever its parcel's cell lies inside it.
constexpr int kRankBlock = 256, kRankHalo = 64;

__global__ void __launch_bounds__(kRankBlock) k_cellrank(const int32_t *start, const int32_t *perm, CellOrd co, int n,
                                                         int32_t *perm_out, const uint32_t *gate) {
  if (gated_off(gate)) return;
  __shared__ double sx[kRankBlock + 2 * kRankHalo];
  __shared__ uint32_t sid[kRankBlock + 2 * kRankHalo];
  const int w0 = (int)blockIdx.x * kRankBlock - kRankHalo;  // first position of the window
  for (int t = threadIdx.x; t < kRankBlock + 2 * kRankHalo; t += kRankBlock) {
    const int q = w0 + t;
    if (q >= 0 && q < n) {
      sx[t] = co.x[q];
      sid[t] = co.id[q];
    }
  }
  __syncthreads();
  const int p = (int)blockIdx.x * kRankBlock + (int)threadIdx.x;
  if (p >= n) return;
  const int c = co.key[p];
  const int s = start[c], e = start[c + 1];
  const double x = sx[p - w0];
  const uint32_t id = sid[p - w0];
  int rank = 0;
  if (s >= w0 && e <= w0 + kRankBlock + 2 * kRankHalo) {
    for (int q = s - w0; q < e - w0; q++) {
      const double xq = sx[q];
      rank += (xq < x || (xq == x && sid[q] < id)) ? 1 : 0;
    }
  } else {
#pragma unroll 4
    for (int q = s; q < e; q++) {
      const double xq = co.x[q];
      rank += (xq < x || (xq == x && co.id[q] < id)) ? 1 : 0;
    }
  }
  perm_out[s + rank] = perm[p];
}
void launch_cellrank(const int32_t *start, const int32_t *perm, const CellOrd &co, int n, int32_t *perm_out,
                     hipStream_t s, const uint32_t *gate) {
  k_cellrank<<<(n + kRankBlock - 1) / kRankBlock, kRankBlock, 0, s>>>(start, perm, co, n, perm_out, gate);
}

// Permutation into the spare buffers (the other step buffer and the spare
// properties), then a copy back: the parcels keep the buffers they live in,
// so no buffer parity depends on whether a rebuild ran.
template <typename T>
__global__ void k_permute(const int32_t *perm, int n, Dyn<T> din, Props<T> pin, Dyn<T> dout, Props<T> pout,
                          float4 *xref, unsigned *dslot, Nbr<T> nb, Spring<T> *carry, uint64_t *carry_mask,
                          const uint32_t *gate) {
  if (gated_off(gate)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 2 * kSlots) {  // displacement and speed maxima restart at the rebuild
    dslot[j * kSlotPad] = 0u;
    dslot[j * kSlotPad + 1] = 0u;
  }
  const bool live = j < n;
  const int i = live ? perm[j] : 0;
  if (live) {
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
  // the contact springs of the old lists move to the new position in their
  // own slots (carry[s * N + j]) with the old contact mask; the wave visits
  // the union of its lanes' contact slots, so each visit reads and writes
  // one row of consecutive parcels
  const long N = n;
  const uint64_t m = live ? nb.mask[i] : 0ull;
  if (live) carry_mask[j] = m;
  const uint64_t b = m & ((1ull << kWallBit) - 1ull);
  uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo |= __shfl_xor(lo, o, 64);
    hi |= __shfl_xor(hi, o, 64);
  }
  uint64_t u = ((uint64_t)__builtin_amdgcn_readfirstlane(hi) << 32) | __builtin_amdgcn_readfirstlane(lo);
  while (u) {
    const int sl = __ffsll((unsigned long long)u) - 1;
    u &= u - 1;
    if ((b >> sl) & 1ull) carry[(long)sl * N + j] = nb.hist[(long)sl * N + i];
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
                    const Props<T> &pspare, float4 *xref, unsigned *dslot, const Nbr<T> &nb, Spring<T> *carry,
                    uint64_t *carry_mask, hipStream_t s, const uint32_t *gate) {
  const int g = (std::max(n, 2 * kSlots) + 255) / 256;
  k_permute<T><<<g, 256, 0, s>>>(perm, n, d, p, spare, pspare, xref, dslot, nb, carry, carry_mask, gate);
  k_copy_back<T><<<(n + 255) / 256, 256, 0, s>>>(n, spare, pspare, d, p, gate);
}

// Decide whether the lists must be rebuilt before the next `horizon` steps:
// D, the largest displacement of any parcel since the last rebuild (exact,
// from the FP32 reference positions), and V, the largest speed, both of the
// last step.  The lists hold every pair that can touch while D < skin/2, so
// they are rebuilt when D + grow V, with grow = 2 x horizon x dt (speeds may
// double within the horizon), could reach skin/2.  The step kernel's own
// exact check stays as the safety net.  One block of 64 threads.
__global__ void k_rebuild_check(const unsigned *dslot, int par_last, float lim, float grow, int force, uint32_t *flag,
                                unsigned long long *count, int32_t *zero2) {
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
    flag[0] = rb ? 1u : 0u;
    flag[1] = rb ? 0u : 1u;
    if (rb) *count += 1ull;
    zero2[0] = 0;  // item count and build queue of the chain behind the check
    zero2[1] = 0;
  }
}

void launch_rebuild_check(const unsigned *dslot, int par_last, double skin, double dt, int horizon, int force,
                          uint32_t *flag, unsigned long long *count, int32_t *zero2, hipStream_t s) {
  const float lim = 0.5f * (float)skin - 1e-7f;
  k_rebuild_check<<<1, 64, 0, s>>>(dslot, par_last, lim, (float)(2.0 * horizon * dt), force, flag, count, zero2);
}

__global__ void k_cell_identity(int32_t *order, int n, const int32_t *start, int32_t *start_d, long n_start,
                                const uint32_t *gate) {
  if (gated_off(gate)) return;
  const long m = n > n_start ? (long)n : n_start;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < m; k += (long)gridDim.x * blockDim.x) {
    if (k < n) order[k] = (int32_t)k;
    if (k < n_start) start_d[k] = start[k];
  }
}

void launch_cell_identity(int32_t *order, int n, const int32_t *start, int32_t *start_d, long n_start, hipStream_t s,
                          const uint32_t *gate) {
  k_cell_identity<<<grid_for(n > n_start ? (long)n : n_start, 256), 256, 0, s>>>(order, n, start, start_d, n_start,
                                                                                   gate);
}

// ------------------------------------------------------------------ work items
// The work items that hold parcels, in key order, in two launches: each
// block counts its items holding parcels, then each block adds up the counts
// of the blocks before it and writes its items there (wave ballots give the
// order inside the block).  The build's queue counter starts at zero: the
// rebuild check clears it.
__device__ __forceinline__ bool item_has_parcels(const Item *items, int t, int item_x, const BedDev *beds,
                                                 const int32_t *start) {
  const Item it = items[t];
  const BedDev &B = beds[it.bed];
  const int xe = min(it.x0 + item_x, B.nd[0]);
  return start[dem_key(B, xe - 1, it.iy, it.iz) + 1] > start[dem_key(B, it.x0, it.iy, it.iz)];
}

__global__ void __launch_bounds__(256) k_item_counts(const Item *items, int n_items, int item_x, const BedDev *beds,
                                                     const int32_t *start, int32_t *bcount, const uint32_t *gate) {
  if (gated_off(gate)) return;
  __shared__ int wsum[4];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool f = t < n_items && item_has_parcels(items, t, item_x, beds, start);
  const uint64_t bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) bcount[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(256) k_items(const Item *items, int n_items, int item_x, const BedDev *beds,
                                               const int32_t *start, const int32_t *bcount, int32_t *list,
                                               int32_t *count, const uint32_t *gate) {
  if (gated_off(gate)) return;
  __shared__ int wsum[4], part[256];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // this block's offset: the counts of the blocks before it
  int o = 0;
  for (int q = threadIdx.x; q < (int)blockIdx.x; q += blockDim.x) o += bcount[q];
  part[threadIdx.x] = o;
  const bool f = t < n_items && item_has_parcels(items, t, item_x, beds, start);
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const uint64_t bal = __ballot(f);
  if (lane == 0) wsum[w] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int base = 0;
    for (int q = 0; q < (int)blockDim.x; q++) base += part[q];
    part[0] = base;
    if (blockIdx.x == gridDim.x - 1) *count = base + wsum[0] + wsum[1] + wsum[2] + wsum[3];
  }
  __syncthreads();
  int off = part[0];
  for (int q = 0; q < w; q++) off += wsum[q];
  if (f) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = t;
}

void launch_items(const Item *items, int n_items, int item_x, const BedDev *beds, const int32_t *start,
                  int32_t *bcount, int32_t *list, int32_t *count, hipStream_t s, const uint32_t *gate) {
  const int nb = (n_items + 255) / 256;
  k_item_counts<<<nb, 256, 0, s>>>(items, n_items, item_x, beds, start, bcount, gate);
  k_items<<<nb, 256, 0, s>>>(items, n_items, item_x, beds, start, bcount, list, count, gate);
}

// ------------------------------------------------------------------ neighbour build
// Work item: `item_x` consecutive DEM cells of one row of a bed, whose
// parcels are the block's centre parcels (one per thread, in passes of
// kThreads).  The nine rows of the item's 3x3 (y, z) stencil, each spanning
// the cells x0-1 .. x0+item_x, are staged in LDS as FP32 positions (relative
// to a corner near the item) with the radius.  The cells of a bed row have
// consecutive keys (one key tile per bed plane), so a stencil row is one run
// of the sorted order; a run longer than the tile is cut into segments, and
// as many consecutive segments as fit are staged at a time.  Every segment
// is sorted by x, so each thread bisects for the first candidate with
// x_j >= x_i - w and scans up to the first with x_j > x_i + w, where
// w = r_i + skin + r_max, keeping the candidates closer than
// r_i + r_j + skin (a conservative FP32 test; the exact contact test runs
// every step).
//
// The list has two regions so that the step visits contacts in lockstep rows:
// candidates that touch now (FP32 test with a 1e-4 margin, a superset of the
// exact contacts) fill slots cap-1, cap-2, ... downwards, the others fill
// slots 0, 1, ... upwards; cnt packs (near << 16) | far.  After the scan the
// tangential springs of partners in contact before the rebuild (moved to
// the new positions by the permutation) are carried over to the near slots
// by matching original ids,
// which every spring record carries; keeping that match out of the scan
// keeps the scan's per-candidate work small.
constexpr float kNear = 1.0f + 1e-4f;
constexpr int kCarry = 8;     // old contacts held in registers; more are matched by a loop
constexpr int kMaxSeg = 64;   // staged segments per item

template <typename T, int kThreads, int kTile>
__global__ void __launch_bounds__(kThreads) k_build_nbr(NbrBuild<T> a) {
  if (gated_off(a.gate)) return;
  __shared__ float4 cpos[kTile];
  // segments: global start, length, stencil row; staged offset of each
  // segment of the current pass
  __shared__ int sg_start[kMaxSeg], sg_len[kMaxSeg], sg_row[kMaxSeg], sg_off[kMaxSeg + 1];
  __shared__ int row_s[9], row_e[9];
  __shared__ int n_seg, cen0, cen1, w_next;
  const int n_list = *a.list_count;
  const long N = a.n;
  const int cap = a.cap;
  const float cut_scale = 1.0f + 1e-5f;
  const int tid = threadIdx.x;
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
    const int xc = min(a.item_x, B.nd[0] - it.x0);
    // the nine stencil rows' runs, one thread each, then their segments
    if (tid < 9) {
      const int r = tid;
      const int iy2 = it.iy + (r % 3) - 1, iz2 = it.iz + (r / 3) - 1;
      int s0 = 0, s1 = 0;
      if (iy2 >= 0 && iy2 < B.nd[1] && iz2 >= 0 && iz2 < B.nd[2]) {
        const int xl = max(it.x0 - 1, 0), xh = min(it.x0 + xc, B.nd[0] - 1);
        s0 = a.start[dem_key(B, xl, iy2, iz2)];
        s1 = a.start[dem_key(B, xh, iy2, iz2) + 1];
        if (r == 4) {
          cen0 = a.start[dem_key(B, it.x0, iy2, iz2)];
          cen1 = a.start[dem_key(B, it.x0 + xc - 1, iy2, iz2) + 1];
        }
      }
      row_s[r] = s0;
      row_e[r] = s1;
    }
    __syncthreads();
    if (tid == 0) {
      int ns = 0;
      for (int r = 0; r < 9; r++) {
        int s0 = row_s[r];
        const int s1 = row_e[r];
        while (s0 < s1) {
          if (ns == kMaxSeg) {
            atomicOr(a.status, ST_OVERFLOW);
            break;
          }
          const int ln = min(s1 - s0, kTile);
          sg_start[ns] = s0;
          sg_len[ns] = ln;
          sg_row[ns] = r;
          ns++;
          s0 += ln;
        }
      }
      n_seg = ns;
    }
    __syncthreads();
    const int ns = n_seg, c0 = cen0, c1 = cen1;
    // FP32 coordinates relative to the corner of the aligned run of kItemXMax
    // cells holding the item (and to the item's own cell in y and z): the
    // same values, hence the same lists, for every item width
    const double xr = B.origin[0] + (it.x0 / kItemXMax) * kItemXMax * B.hd, yr = B.origin[1] + it.iy * B.hd,
                 zr = B.origin[2] + it.iz * B.hd;
    for (int cb = c0; cb < c1; cb += kThreads) {
      const int i = cb + tid;
      const bool mine = i < c1;
      float xi = 0.f, yi = 0.f, zi = 0.f, rs = 0.f, ri = 0.f, cut_hi = 0.f;
      int nn = 0, nf = 0;  // near / far candidates written
      bool over = false;
      int32_t *pnear = a.nb.idx + (long)(cap - 1) * N + i, *pfar = a.nb.idx + i;  // next near / far slot
      if (mine) {
        const PosRec pi = load_pos(a.d.pos, i);
        xi = (float)(pi.x - xr);
        yi = (float)(pi.y - yr);
        zi = (float)(pi.z - zr);
        ri = pi.r;
        rs = pi.r + (float)a.skin;
        // widest candidate distance along x for this centre
        cut_hi = (rs + (float)B.rmax) * cut_scale + 1e-9f;
      }
      int sg = 0;
      while (sg < ns) {
        // as many consecutive segments as fit in the tile (each fits alone)
        int se = sg, tot = 0;
        while (se < ns && tot + sg_len[se] <= kTile) tot += sg_len[se++];
        __syncthreads();  // the previous pass's readers are done with the tile
        if (tid == 0) {
          int o = 0;
          for (int q = sg; q < se; q++) {
            sg_off[q] = o;
            o += sg_len[q];
          }
          sg_off[se] = o;
        }
        __syncthreads();
        for (int t = tid; t < tot; t += kThreads) {
          int q = sg;
          while (q + 1 < se && sg_off[q + 1] <= t) q++;
          const PosRec pj = load_pos(a.d.pos, sg_start[q] + (t - sg_off[q]));
          cpos[t] = make_float4((float)(pj.x - xr), (float)(pj.y - yr), (float)(pj.z - zr), pj.r);
        }
        __syncthreads();
        if (mine) {
          for (int q = sg; q < se; q++) {
            const int b0 = sg_off[q], b1 = sg_off[q + 1];
            const int jb = sg_start[q] - b0;  // staged slot t holds parcel jb + t
            const int self = (i >= sg_start[q] && i < sg_start[q] + sg_len[q]) ? i - jb : -1;
            // the segment is sorted by x: bisect the window |x_j - x_i| <= cut_hi
            int lo = b0, hi = b1;
            {
              int a0 = b0, a1 = b1;
              const float xl = xi - cut_hi;
              while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (cpos[mid].x < xl) a0 = mid + 1; else a1 = mid;
              }
              lo = a0;
              a1 = b1;
              const float xh = xi + cut_hi;
              while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (cpos[mid].x <= xh) a0 = mid + 1; else a1 = mid;
              }
              hi = a0;
            }
            // four candidates per trip, all read before any is tested; the
            // list rows are written through running pointers
            for (int t = lo; t < hi; t += 4) {
              float4 c[4];
#pragma unroll
              for (int k = 0; k < 4; k++) c[k] = cpos[min(t + k, kTile - 1)];
#pragma unroll
              for (int k = 0; k < 4; k++) {
                const float dx = c[k].x - xi, dy = c[k].y - yi, dz = c[k].z - zi;
                const float cut = (rs + c[k].w) * cut_scale;
                const float d2 = dx * dx + dy * dy + dz * dz;
                if (t + k < hi && d2 < cut * cut && t + k != self) {
                  const float sn = (ri + c[k].w) * kNear;
                  if (nn + nf >= cap) {
                    over = true;
                  } else if (d2 < sn * sn) {
                    *pnear = jb + t + k;
                    pnear -= N;
                    nn++;
                  } else {
                    *pfar = jb + t + k;
                    pfar += N;
                    nf++;
                  }
                }
              }
            }
          }
        }
        sg = se;
      }
      if (mine) {
        // springs of the old contacts that are near candidates again (the
        // permutation left them at the new position, in their old slots)
        const uint64_t om = a.carry_mask[i];
        uint64_t rest = om & ((1ull << kWallBit) - 1ull);
        uint64_t newbits = 0;
        if (rest && nn > 0) {
          // partner ids and slots of the first kCarry old contacts; the rest
          // are matched by a loop over their bits
          uint32_t oid[kCarry];
          int osl[kCarry];
#pragma unroll
          for (int k = 0; k < kCarry; k++) {
            osl[k] = rest ? __ffsll((unsigned long long)rest) - 1 : 0;
            oid[k] = rest ? spring_partner(a.carry[(long)osl[k] * N + i].w) : 0xffffffffu;
            rest &= rest ? rest - 1 : 0ull;
          }
          for (int k0 = 0; k0 < nn; k0 += 4) {
            int jj[4];
            uint32_t idn[4];
#pragma unroll
            for (int u = 0; u < 4; u++) jj[u] = k0 + u < nn ? a.nb.idx[(long)(cap - 1 - k0 - u) * N + i] : -1;
#pragma unroll
            for (int u = 0; u < 4; u++) idn[u] = jj[u] >= 0 ? a.d.pos[jj[u]].id : 0xffffffffu;
#pragma unroll
            for (int u = 0; u < 4; u++) {
              if (jj[u] < 0) continue;
              int qs = -1;
#pragma unroll
              for (int k = 0; k < kCarry; k++)
                if (oid[k] == idn[u]) qs = osl[k];
              for (uint64_t r = rest; r && qs < 0; r &= r - 1) {
                const int sl2 = __ffsll((unsigned long long)r) - 1;
                if (spring_partner(a.carry[(long)sl2 * N + i].w) == idn[u]) qs = sl2;
              }
              if (qs >= 0) {
                const int sl = cap - 1 - k0 - u;
                a.nb.hist[(long)sl * N + i] = a.carry[(long)qs * N + i];
                newbits |= 1ull << sl;
              }
            }
          }
        }
        if (over) atomicOr(a.status, ST_OVERFLOW);
        a.nb.cnt[i] = (nn << 16) | nf;
        a.nb.mask[i] = newbits | (om & ~((1ull << kWallBit) - 1ull));
      }
    }
  }
}

// block size and LDS tile (candidates) of each build variant
struct BuildShape {
  int threads, tile;
};
constexpr BuildShape kBuildShapes[kBuildVariants] = {{512, 2048}, {256, 1024}, {256, 2048}, {1024, 4096}};

template <typename T, int V>
static void launch_build_v(const NbrBuild<T> &a, int grid, hipStream_t s) {
  constexpr BuildShape sh = kBuildShapes[V];
  k_build_nbr<T, sh.threads, sh.tile><<<grid, sh.threads, 0, s>>>(a);
}
template <typename T, int V>
static int build_blocks_v() {
  constexpr BuildShape sh = kBuildShapes[V];
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_build_nbr<T, sh.threads, sh.tile>, sh.threads, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int build_threads(int variant) { return kBuildShapes[variant].threads; }
int build_tile(int variant) { return kBuildShapes[variant].tile; }

template <typename T>
int build_blocks_per_cu(int variant) {
  switch (variant) {
    case 0: return build_blocks_v<T, 0>();
    case 1: return build_blocks_v<T, 1>();
    case 2: return build_blocks_v<T, 2>();
    default: return build_blocks_v<T, 3>();
  }
}

template <typename T>
void launch_build_nbr(const NbrBuild<T> &a, int variant, int grid, hipStream_t s) {
  switch (variant) {
    case 0: launch_build_v<T, 0>(a, grid, s); break;
    case 1: launch_build_v<T, 1>(a, grid, s); break;
    case 2: launch_build_v<T, 2>(a, grid, s); break;
    default: launch_build_v<T, 3>(a, grid, s); break;
  }
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

// ------------------------------------------------------------------ contact history
// Export: one record per pair in contact at the last step, taken from the side
// with the lower original id (both sides hold the same spring, in the
// orientation with the normal from the lower to the higher id), and every
// parcel's wall springs by original id.
template <typename T>
__global__ void k_contacts_export(const PosRec *pos, Nbr<T> nb, const T *wh, int n, int cap_slots, uint32_t *ids,
                                  double *xi, long cap, unsigned long long *count, uint8_t *wall_on,
                                  double *wall_xi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long N = n;
  const PosRec a = load_pos(pos, i);
  const uint64_t m = nb.mask[i];
  const int cw = nb.cnt[i], c_near = cw >> 16, c_far = cw & 0xffff;
  for (int v = 0; v < c_near + c_far; v++) {
    const int s = v < c_near ? cap_slots - 1 - v : v - c_near;
    if (!((m >> s) & 1ull)) continue;
    const int j = nb.idx[(long)s * N + i];
    const uint32_t bid = pos[j].id;
    if (bid <= a.id) continue;
    const Spring<T> h = nb.hist[(long)s * N + i];
    const unsigned long long k = atomicAdd(count, 1ull);
    if ((long)k < cap) {
      ids[2 * k] = a.id;
      ids[2 * k + 1] = bid;
      xi[3 * k] = (double)h.x;
      xi[3 * k + 1] = (double)h.y;
      xi[3 * k + 2] = (double)h.z;
    }
  }
  for (int w = 0; w < kMaxWalls; w++) {
    const bool on = (m >> (kWallBit + w)) & 1ull;
    wall_on[(long)a.id * kMaxWalls + w] = on ? 1 : 0;
#pragma unroll
    for (int c = 0; c < 3; c++)
      wall_xi[((long)a.id * kMaxWalls + w) * 3 + c] = on ? (double)wh[(long)(w * 3 + c) * N + a.id] : 0.0;
  }
}

__global__ void k_inverse_ids(const PosRec *pos, int n, int32_t *inv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) inv[pos[p].id] = p;
}

// Import: each pair's spring goes into both partners' current lists (slots
// 0, 1, ... in arrival order, the partner's id in the fourth component, the
// orientation unchanged) with the contact bits of those slots set, as a step
// leaves them; the next rebuild carries them to the pairs' near slots by
// id, so the slot order does not matter.
template <typename T>
__global__ void k_contacts_import(const uint32_t *ids, const double *xi, long np, const int32_t *inv, int n,
                                  int cap_slots, Spring<T> *hist, uint32_t *cnt, uint32_t *status) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const long N = n;
  const uint32_t ia = ids[2 * q], ib = ids[2 * q + 1];
  const int pa = inv[ia], pb = inv[ib];
  const T x = T(xi[3 * q]), y = T(xi[3 * q + 1]), z = T(xi[3 * q + 2]);
  const uint32_t ka = atomicAdd(cnt + pa, 1u), kb = atomicAdd(cnt + pb, 1u);
  if ((int)ka < cap_slots) hist[(long)ka * N + pa] = Spring<T>{x, y, z, spring_tag<T>(ib)};
  if ((int)kb < cap_slots) hist[(long)kb * N + pb] = Spring<T>{x, y, z, spring_tag<T>(ia)};
  if ((int)ka >= cap_slots || (int)kb >= cap_slots) atomicOr(status, ST_OVERFLOW);
}

template <typename T>
__global__ void k_walls_import(const PosRec *pos, int n, int cap_slots, const uint8_t *wall_on, const double *wall_xi,
                               T *wh, const uint32_t *cnt, uint64_t *mask) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const long N = n;
  const uint32_t id = pos[p].id;
  uint64_t bits = 0;
  for (int w = 0; w < kMaxWalls; w++) {
    const bool on = wall_on[(long)id * kMaxWalls + w] != 0;
    if (on) bits |= 1ull << w;
#pragma unroll
    for (int c = 0; c < 3; c++)
      wh[(long)(w * 3 + c) * N + id] = on ? T(wall_xi[((long)id * kMaxWalls + w) * 3 + c]) : T(0);
  }
  const uint32_t k = min(cnt[p], (uint32_t)cap_slots);
  mask[p] = (bits << kWallBit) | ((1ull << k) - 1ull);
}

template <typename T>
void launch_contacts_export(const PosRec *pos, const Nbr<T> &nb, const T *wh, int n, int cap_slots, uint32_t *ids,
                            double *xi, long cap, unsigned long long *count, uint8_t *wall_on, double *wall_xi,
                            hipStream_t s) {
  k_contacts_export<T><<<(n + 255) / 256, 256, 0, s>>>(pos, nb, wh, n, cap_slots, ids, xi, cap, count, wall_on,
                                                       wall_xi);
}
template <typename T>
void launch_contacts_import(const PosRec *pos, int n, int cap_slots, const uint32_t *ids, const double *xi, long np,
                            const uint8_t *wall_on, const double *wall_xi, int32_t *inv, uint32_t *cnt,
                            const Nbr<T> &nb, T *wh, uint32_t *status, hipStream_t s) {
  k_inverse_ids<<<(n + 255) / 256, 256, 0, s>>>(pos, n, inv);
  launch_fill_u32(cnt, 0u, n, s);
  if (np > 0)
    k_contacts_import<T><<<(unsigned)((np + 255) / 256), 256, 0, s>>>(ids, xi, np, inv, n, cap_slots, nb.hist, cnt,
                                                                     status);
  k_walls_import<T><<<(n + 255) / 256, 256, 0, s>>>(pos, n, cap_slots, wall_on, wall_xi, wh, cnt, nb.mask);
}

#define INST(T)                                                                                                   \
  template void launch_bin<T>(const Dyn<T> &, const Props<T> &, const BedDev *, int, int32_t *, int32_t *,       \
                              int32_t *, uint32_t *, hipStream_t, const uint32_t *);                              \
  template void launch_permute<T>(const int32_t *, int, const Dyn<T> &, const Props<T> &, const Dyn<T> &,        \
                                  const Props<T> &, float4 *, unsigned *, const Nbr<T> &, Spring<T> *,           \
                                  uint64_t *, hipStream_t, const uint32_t *);                                    \
  template void launch_build_nbr<T>(const NbrBuild<T> &, int, int, hipStream_t);                 \
  template int build_blocks_per_cu<T>(int);                                                                       \
  template void launch_contacts_export<T>(const PosRec *, const Nbr<T> &, const T *, int, int, uint32_t *, double *, \
                                          long, unsigned long long *, uint8_t *, double *, hipStream_t);           \
  template void launch_contacts_import<T>(const PosRec *, int, int, const uint32_t *, const double *, long,          \
                                          const uint8_t *, const double *, int32_t *, uint32_t *, const Nbr<T> &,  \
                                          T *, uint32_t *, hipStream_t);                                      \
  template void launch_pairs<T>(const Dyn<T> &, const Props<T> &, const Nbr<T> &, int, int, uint32_t *, long,         \
                                unsigned long long *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace demrx
