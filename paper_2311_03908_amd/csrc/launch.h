// Host-side launchers of the demrx kernels (one definition per kernel file).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "thermo.h"

namespace demrx {

// ---------------------------------------------------------------- k_build.hip
struct Item {  // a run of up to item_x DEM cells along x in one (y, z) row of a bed
  int bed, x0, iy, iz;
};
// item widths (DEM cells along x) the neighbour build can run with
constexpr int kItemWidths[3] = {8, 16, 32};
constexpr int kItemXMax = 32;
// per-step maxima and counts are gathered in kSlots padded slots (128 bytes
// apart) by per-wave atomics, and summed by their readers
constexpr int kSlots = 64, kSlotPad = 32, kSlotPad64 = 16;

// Launchers of the rebuild chain take `gate` (a device word; null: always
// run): with *gate == 0 their kernels return at once.
void launch_fill_i32(int32_t *p, int32_t v, long n, hipStream_t s, const uint32_t *gate = nullptr);
void launch_fill_u32(uint32_t *p, uint32_t v, long n, hipStream_t s);
// exclusive prefix sum of m ints; scratch needs scan_scratch_ints(m) ints;
// with clear, in is zeroed
long scan_scratch_ints(long m);
void launch_scan(int32_t *in, int32_t *out, long m, int32_t *scratch, hipStream_t s, const uint32_t *gate = nullptr,
                 bool clear = false);

template <typename T>
void launch_bin(const Dyn<T> &d, const Props<T> &p, const BedDev *beds, int n, int32_t *key, int32_t *slot,
                int32_t *count, uint32_t *status, hipStream_t s, const uint32_t *gate = nullptr);
// x, original id and DEM cell of the parcels in the scatter's cell order
struct CellOrd {
  double *x;
  uint32_t *id;
  int32_t *key;
};
void launch_scatter(const int32_t *key, const int32_t *slot, const int32_t *start, const PosRec *pos, int n,
                    int32_t *perm, const CellOrd &co, hipStream_t s, const uint32_t *gate = nullptr);
void launch_cellrank(const int32_t *start, const int32_t *perm, const CellOrd &co, int n, int32_t *perm_out,
                     hipStream_t s, const uint32_t *gate = nullptr);
// permute (d, p) by perm through the spare buffers and copy back, so the
// parcels stay in d and p; resets the displacement maxima and xref; moves
// the contact springs of the current lists nb to the new positions in their
// own slots (carry[s * N + j]) with the old contact masks (carry_mask[j])
template <typename T>
void launch_permute(const int32_t *perm, int n, const Dyn<T> &d, const Props<T> &p, const Dyn<T> &spare,
                    const Props<T> &pspare, float4 *xref, unsigned *dslot, const Nbr<T> &nb, Spring<T> *carry,
                    uint64_t *carry_mask, hipStream_t s, const uint32_t *gate);
// flag[0] = 1 when the lists could go stale within `horizon` steps (or
// force), else 0; flag[1] = its complement; zero2[0..1] (the work-item count
// and the build queue of the chain behind the check) set to 0
void launch_rebuild_check(const unsigned *dslot, int par_last, double skin, double dt, int horizon, int force,
                          uint32_t *flag, unsigned long long *count, int32_t *zero2, hipStream_t s);
// the cell order of parcels that a rebuild has just sorted: order[k] = k and
// start_d = start (n_start offsets); gated like the rebuild chain
void launch_cell_identity(int32_t *order, int n, const int32_t *start, int32_t *start_d, long n_start, hipStream_t s,
                          const uint32_t *gate);
// the work items holding parcels, in key order (bcount: one int per 256 items)
void launch_items(const Item *items, int n_items, int item_x, const BedDev *beds, const int32_t *start,
                  int32_t *bcount, int32_t *list, int32_t *count, hipStream_t s, const uint32_t *gate);

template <typename T>
struct NbrBuild {
  Dyn<T> d;             // sorted state (after the permutation)
  Props<T> p;           // sorted properties
  Nbr<T> nb;            // the lists written
  const Spring<T> *carry;       // springs of the old lists (launch_permute), by new position and old slot
  const uint64_t *carry_mask;   // old contact masks by new position
  const uint32_t *gate;
  const BedDev *beds;
  const int32_t *start;
  const Item *items;
  const int32_t *list, *list_count;
  int32_t *queue;  // work-item counter, zero at launch
  int n, cap;
  int item_x;      // DEM cells per work item (the width the items were made with)
  double skin;
  uint32_t *status;
};
// build variants: block size and LDS tile (candidate records staged at a time)
constexpr int kBuildVariants = 4;
int build_threads(int variant);
int build_tile(int variant);
template <typename T>
int build_blocks_per_cu(int variant);  // resident blocks per CU (occupancy query)
template <typename T>
void launch_build_nbr(const NbrBuild<T> &a, int variant, int grid, hipStream_t s);

template <typename T>
void launch_pairs(const Dyn<T> &d, const Props<T> &p, const Nbr<T> &nb, int n, int cap_slots, uint32_t *out, long cap,
                  unsigned long long *count, hipStream_t s);

// contact history for checkpoints: export (pairs in contact, a < b, and
// wall springs by original id) and import into the current lists, for the
// next rebuild to carry (inv, cnt: n ints of scratch)
template <typename T>
void launch_contacts_export(const PosRec *pos, const Nbr<T> &nb, const T *wh, int n, int cap_slots, uint32_t *ids,
                            double *xi, long cap, unsigned long long *count, uint8_t *wall_on, double *wall_xi,
                            hipStream_t s);
template <typename T>
void launch_contacts_import(const PosRec *pos, int n, int cap_slots, const uint32_t *ids, const double *xi, long np,
                            const uint8_t *wall_on, const double *wall_xi, int32_t *inv, uint32_t *cnt,
                            const Nbr<T> &nb, T *wh, uint32_t *status, hipStream_t s);

// ---------------------------------------------------------------- k_step.hip
template <typename T>
struct StepArgs {
  Dyn<T> in, out;
  Props<T> pr;
  Nbr<T> nb;
  const T *gtab;
  const BedDev *beds;
  const OreDev *ores;
  Phys ph;
  BedDev bed0;                   // copy of beds[0] (the records never change after init)
  uint32_t *status;
  const double *Tg;              // gas temperature per cell (energy equation)
  const float4 *xref;            // positions at the last rebuild (FP32)
  unsigned *dslot;               // [2][kSlots] padded: max squared displacement (+0), speed (+1); this step: par
  unsigned long long *cslot;     // [kSlots] padded: pp and wall contacts (mode 0 with count)
  int n, par, mode;              // mode 0: integrate; 1: write forces; 2: timing dry run
  int count;                     // 1: add this step's contacts to counters
  int xcd;                       // >1: XCD chunk of consecutive blocks (see xcd_block)
  double *Fout, *Tout;
  Spring<T> *hist_w;             // where the springs and masks are written: nb.hist and
  uint64_t *mask_w;              // nb.mask, or the rebuild's spare buffers in mode 2
};
template <typename T>
void launch_step(const StepArgs<T> &a, int block, hipStream_t s);


struct GasArgs {
  const double *ug, *vg, *wg, *p, *dpdx, *dpdy, *dpdz, *T, *xH2, *xH2O, *xN2;
};
template <typename T>
void launch_gas_table(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds,
                      const ThermoTab *thermo, int n_gas, const int2 *zr, T *gtab, uint32_t *status, hipStream_t s);
// per bed, the gas-cell layers [x, y] that parcels of the occupied list can
// reach within `reach` metres (zr: n_beds entries)
void launch_occ_zrange(const int32_t *list, const int32_t *count, const BedDev *beds, int n_beds, double reach,
                       int2 *zr, hipStream_t s);

// ---------------------------------------------------------------- k_couple.hip
// The beds' records as the coupling kernels read them: a single bed's record
// travels in the kernel arguments (scalar loads, no wait on vector memory);
// with several beds each is read from the device array.
struct BedSel {
  const BedDev *beds;
  int n_beds;
  BedDev one;  // copy of beds[0] (the records never change after init)
};
// f(record of bed index()); index() is evaluated only with several beds
template <typename I, typename F>
__device__ __forceinline__ void on_bed(const BedSel &s, I &&index, F &&f) {
  if (s.n_beds == 1)
    f(s.one);
  else
    f(s.beds[index()]);
}
struct DepositOut {
  double *eps_ctx;  // context voidage (null: not written; the occupied list only)
  double *eps, *np, *sumK, *sumKu, *sumKv, *sumKw, *sumKs;
};
void launch_occupied(const int32_t *start, const int32_t *cell_bed, const BedSel &bs, int n_gas, bool sums,
                     const DepositOut &o, int32_t *flags, int32_t *offs, int32_t *scratch, int32_t *list,
                     int32_t *count, hipStream_t s);
template <typename T>
void launch_deposit(const Dyn<T> &d, const Props<T> &p, const GasArgs &g, const int32_t *start,
                    const int32_t *order, const int32_t *cell_bed, const BedSel &bs, const OreDev *ores,
                    const Phys &ph, const int32_t *list, const int32_t *list_count, int max_list, bool sums, const DepositOut &o,
                    hipStream_t s);

template <typename T>
struct ReactArgs {
  Dyn<T> d;
  Props<T> p;
  GasArgs g;
  const double *eps;
  BedSel bs;
  const OreDev *ores;
  const ThermoTab *thermo;  // energy equation on (null: isothermal at the gas temperature)
  const double *theta;  // 6 values overriding every bed's, or null
  const double *rtab;   // per-cell quantities (launch_react_table) of the occupied cells, or null
  double dt;
  int n;
  int update_mass;
  double *pm;    // [4][N] per-parcel mdotH2, mdotH2O, EQ, ES (+ [4][N] hA, hA Tp, Qrm, Hr with energy)
  double *pw;    // [2][N] per-parcel w f_ov, w
  double *fov;   // original order (may be null)
  unsigned long long *clamps;
  uint32_t *status;
};
template <typename T>
void launch_react(const ReactArgs<T> &a, hipStream_t s);
// per occupied gas cell: H2 fraction, equilibria, rate constants, density,
// viscosity, molecular and each ore's pore diffusivity (kReactRow doubles a
// cell; up to kReactRow - 10 ores)
constexpr int kReactRow = 16;
void launch_react_table(const GasArgs &g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores,
                        int n_ores, const double *theta, const int32_t *list, const int32_t *list_count, int max_list,
                        double *tab, hipStream_t s);
void launch_gas_species(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                        double dt, const double *sumEQ, const double *sumES, double xin1, double xin2, double *o1,
                        double *o2, double *o3, uint32_t *status, hipStream_t s);
void launch_gas_momentum(const GasArgs &g, const double *eps, const int32_t *cell_bed, const BedDev *beds, int n_gas,
                         double dt, const double grav[3], const double *sK, const double *sKu, const double *sKv,
                         const double *sKw, double *uo, double *vo, double *wo, uint32_t *status, hipStream_t s);
struct CellSumOut {
  double *o[8];  // per-cell sums of the pm rows (null: not written)
  int rows;      // 4, or 8 with the energy equation
};
// cell sums over the occupied cells of launch_occupied (flags, list, count)
void launch_cellsum(const double *pm, int n, const int32_t *start, const int32_t *order, const int32_t *cell_bed,
                    const BedSel &bs, int n_gas, const int32_t *flags, const int32_t *list,
                    const int32_t *list_count, int max_list, const CellSumOut &o, hipStream_t s);
constexpr int kBedChunk = 4096;  // parcels per partial sum of the bed means
// bed means; with table set, the chunk table is built first from the beds'
// parcel ranges (which no rebuild changes: the sort is bed-major and parcels
// keep their bed), otherwise the table of an earlier call is used; a null
// pw builds the table only
void launch_bedsum(const double *pw, int n, const int32_t *start, const BedDev *beds, int n_beds, int4 *chunks,
                   int max_chunks, double *partial, double *bed_fov, bool table, hipStream_t s);

template <typename T>
void launch_init(const dem_parcels &in, int n, const Phys &ph, int n_ores, const ThermoTab *thermo, const Dyn<T> &d,
                 const Props<T> &p, uint32_t *status, hipStream_t s);
template <typename T>
void launch_export(const Dyn<T> &d, const Props<T> &p, int n, const dem_parcels &out, hipStream_t s);
template <typename T>
void launch_import(const dem_parcels &in, int n, const ThermoTab *thermo, const Dyn<T> &d, const Props<T> &p,
                   hipStream_t s);

// ---------------------------------------------------------------- k_adjoint.hip
struct AdjArgs {
  int n;                     // parcels (state in original-id order)
  int n_sub, dyn_every, ckpt_every;
  int k_base;                // interval held by record slot 0
  int s_begin, s_end;        // substeps run by a forward launch
  double dt;                 // reaction substep
  const int32_t *rec_cell;   // [slot][N] gas cell of every parcel
  const double *rec_F;       // [slot][N] film resistance
  const double *ctab;        // per gas cell reaction table (kCtab doubles)
  const double *dtab;        // per (gas cell, ore): tau / (D xi_l) of the three layers
  int n_ores;
  const double *dp, *k3;     // real diameter and k^3 by id
  const int32_t *ore, *kind; // ore index and f_ov kind by id
  void *state;               // [4][N] (float or double)
  void *ckpt;                // [n_ckpt][4][N] or null
  void *seg;                 // [ckpt_every + 1][4][N]
  double *part;              // [blocks][8]: J numerator, sum w, dJ/dtheta numerators
  double inv_W;
};
int adjoint_blocks(int n);
void launch_adj_cells(const GasArgs &g, const int32_t *cell_bed, const BedDev *beds, const OreDev *ores, int n_ores,
                      int n_gas, const double *theta, double *ctab, double *dtab, hipStream_t s);
template <typename T, typename S>
void launch_adj_static(const Dyn<T> &d, const Props<T> &p, const OreDev *ores, int n, double *dp, double *k3,
                       int32_t *ore, int32_t *kind, S *state, hipStream_t s);
template <typename T>
void launch_adj_record(const Dyn<T> &d, const Props<T> &p, const GasArgs &g, const double *eps, const BedDev *beds,
                       int n, int32_t *rec_cell, double *rec_F, hipStream_t s);
void launch_adjoint_forward(const AdjArgs &a, int fp32, hipStream_t s);
void launch_adjoint_backward(const AdjArgs &a, int fp32, hipStream_t s);

}  // namespace demrx
