// Internal declarations shared by the host API (pf_api.cpp) and the kernels
// (pf_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pf {

// One work tile: consecutive whole bus rows of one grid (see pf_kernels.hip).
struct TileDesc {
    int32_t r0, nrows;  // first row (global bus), number of rows
    int32_t i0, n;      // first record, number of records (shunt records included)
    int32_t ne;         // branch-end records (n - nrows)
    int32_t s0, ns;     // first Ybus slot, number of slots
    int32_t sh;         // one-row tiles: position of the bus-shunt record in the row (else 0)
    int64_t jp, jq;     // offsets of the tile's P rows and Q rows in one state's J values
};

static_assert(sizeof(TileDesc) == 48, "tile descriptors are uploaded as raw bytes");

// Ybus slots an element-wise tile may hold (its LDS copy of the J rows),
// for NT branch ends per tile: rows carry ~1.4 slots per branch end.
constexpr int kEwSlots(int NT) { return NT + NT / 2; }

// Element-wise lane word: LDS targets o11, o12 (11 bits each, at most
// 2 kEwSlots(512) = 1536) and the tile row (9 bits, < 512).
constexpr int32_t ew_pack(int32_t o11, int32_t o12, int32_t row) { return o11 | (o12 << 11) | (row << 22); }

// Ybus lane word: LDS targets o11, o12 (11 bits each, at most 2 * 512 + 1),
// the tile row (9 bits) and the diagonal flag (the sign bit).
constexpr int32_t yb_pack(int32_t o11, int32_t o12, int32_t row, bool diag) {
    return (int32_t)((uint32_t)o11 | ((uint32_t)o12 << 11) | ((uint32_t)row << 22) | (diag ? 0x80000000u : 0u));
}

// Device view of a handle, passed to kernels by value.
//
// Records ("items") are the unit of the element-wise method: one per branch
// end (at bus i, pointing to the remote bus j) and one per bus for its shunt
// (j == i), sorted by (bus, neighbour, branch).  Slots are Ybus nonzeros;
// without parallel branches item e and slot e coincide.  A record keeps the
// coupling admittance of its branch end; the own-end admittances of all
// records of a bus (and its shunt) share the factor v_i^2 in every
// evaluation and are summed once per bus (dA + j dC).
struct DevGrid {
    int32_t nb;           // buses over all grids
    int64_t nnz_y;        // Ybus nonzeros over all grids
    int64_t nnz_j;        // 4 nnz_y
    int32_t ntiles;       // element-wise tiles
    int32_t nytiles;      // Ybus tiles
    const int32_t *yrow;  // [nb+1] slot row pointer (global slot numbering)
    const int32_t *irow;  // [nb+1] item row pointer
    const int32_t *ycol;  // [nnz_y] global bus index of the column
    const int32_t *nbr;   // [nitems] remote bus (== own bus for the shunt record)
    const int32_t *slot;  // [nitems] global slot of the item
    const double *G, *B;  // [nitems] coupling admittance Re / Im of this end (0 for the shunt record)
    const double *Gr, *Br;  // [nitems] coupling admittance of the other end (adjoint)
    const double *dA, *dC;    // [nb+1] sum of own-end admittances + shunt (Re / Im); [nb] = 0
    const double *yre, *yim;  // [nnz_y] Ybus values
    const TileDesc *tiles;    // [ntiles] element-wise tiles
    const TileDesc *ytiles;   // [nytiles] Ybus tiles

    // Lane tables of the packed tiles, [ntiles * tile_items] (element-wise)
    // and [nytiles * tile_items] (Ybus), entry t * tile_items + k for thread
    // k of tile t.  Entries of idle lanes and of long-row tiles are inert.
    const int32_t *lane_j;      // element-wise branch end: remote bus
    const int32_t *lane_pk;     // ew_pack(o11, o12, row)
    const int32_t *lane_run;    // with parallel branches: records of the slot (first record of a slot), else 0
    const double2 *lane_gb;     // {G, B}
    const double2 *lane_grbr;   // {Gr, Br}
    const int2 *row_ew;         // [nb+1] {ra | rz << 16, d11 | d12 << 16}; [nb] inert
    const int32_t *ylane_j;     // Ybus nonzero: column bus
    const int32_t *ylane_pk;    // yb_pack(o11, o12, row, diag)
    const double2 *ylane_y;     // {Re Y, Im Y}
    const int2 *row_yb;         // [nb+1] {ya | yz << 16, dls}; [nb] inert
    const double2 *ylane_yt;    // Ybus lane: {Re, Im} of the transposed entry Y_ji (CSC Jacobian)
    const int32_t *yt_slot;     // [nnz_y] slot of the transposed entry (long rows, CSC Jacobian)
};

// Gather sources of the lane tables: record (element-wise) and slot (Ybus)
// of every lane, -1 for inert lanes.
struct DevLaneFill {
    int64_t nlanes, nylanes;  // element-wise, Ybus
    int32_t nb;
    const int32_t *lane_rec, *ylane_slot;
    const int32_t *ydslot;  // [nb] global slot of each bus's diagonal
    const int32_t *ylane_tslot;  // transposed slot of each Ybus lane, -1 inert
    const double *G, *B, *Gr, *Br, *yre, *yim;
    double2 *lane_gb, *lane_grbr, *ylane_y, *ylane_yt;
};

// Setup data, only read by the setup kernels.
struct DevSetup {
    int64_t nitems;
    int64_t nnz_y;
    const int32_t *item_br;    // [nitems] 2*branch + end (0 = from end, 1 = to end); -1 for a shunt record
    const int32_t *nbr;        // [nitems]
    const int32_t *slot_row;   // [nnz_y]
    const int32_t *slot_item;  // [nnz_y+1]
    const int32_t *irow;       // [nb+1]
    const int32_t *ycol;       // [nnz_y]
    const double *r, *x, *b, *tap, *shift;  // [nl]
    const double *gs, *bs;                  // [nb]
    int32_t nb;
    double *G, *B, *Gr, *Br;                // [nitems] outputs
    double *dA, *dC;                        // [nb] outputs
    double *yre, *yim;                      // [nnz_y] outputs
};

// Two-phase element-wise evaluation, the paper's own structure (Section
// IV.C): phase 1 evaluates every branch (both ends) and writes each end's
// P, Q and eight partials to scratch at the end's record position; phase 2
// sums each bus row in record order into P, Q and the row's J entries.
struct DevTwoPhase {
    int32_t nb, nl;
    int64_t nrec;                           // records: the scratch stride
    const int32_t *br_from, *br_to;         // [nl] global bus numbers
    const int32_t *br_rec;                  // [2 nl] record of the from end, of the to end
    const double *r, *x, *b, *tap, *shift;  // [nl]
    const double *gs, *bs;                  // [nb]
    const int32_t *irow, *item_br, *slot, *yrow, *ydslot;
    const int2 *jpq;                        // [nb] offsets of row i's P and Q parts in one state's J
    double *scr;                            // [10][nrec]
    const double *bc;                       // [6][nl] precomputed G, B, A_from, C_from, A_to, C_to
};

enum Kind { K_EW_S = 0, K_EW_SJ = 1, K_YB_S = 2, K_YB_SJ = 3, K_EW_VJP = 4, K_EW_SJ_CSC = 5, K_YB_SJ_CSC = 6 };

// Phasor source of the Ybus kernels: formed on the fly from (vm, va), or
// read from stored split / interleaved phasors (the values of the public
// PF_PHASOR_SPLIT and PF_PHASOR_INTERLEAVED).
enum { PH_FLY = 0, PH_SPLIT = 1, PH_INTERLEAVED = 2 };

// Order of the (tile, state chunk) work items over the workgroups (see
// work_item in pf_kernels.hip).
enum { WO_TILE = 0, WO_STATE = 1, WO_GROUPED = 2 };

struct Launch {
    int kind;
    int tile_items;        // workgroup size = records per tile
    int states_per_block;
    int order;             // WO_*
    int nstate;
    bool has_parallel;
    const double *vm, *va, *lp, *lq;
    double *p, *q, *jval, *gvm, *gva;
    int phasor;        // Ybus kinds: 0 on the fly from vm, va; 1 split, 2 interleaved stored phasors in ph
    const double *ph;  // stored phasors (layout of launch_phasor)
};

hipError_t launch_eval(const DevGrid &g, const Launch &L, hipStream_t stream);
// Workgroups of the evaluation kernel for (kind, tile_items, has_parallel)
// that one compute unit holds at once (0 if unknown).
int resident_blocks_per_cu(int kind, int tile_items, bool has_parallel);
hipError_t launch_setup_items(const DevSetup &s, hipStream_t stream);
// Fill the element-wise (ew) or Ybus (!ew) lane values from the record /
// slot arrays.
hipError_t launch_lane_fill(const DevLaneFill &f, bool ew, hipStream_t stream);
hipError_t launch_ybus_assemble(const DevSetup &s, hipStream_t stream);
// V = v e^{j theta} and U = e^{j theta} of n (state, bus) entries into ph:
// layout 1 = four planes [Re V | Im V | Re U | Im U] of n doubles, layout 2 =
// n pairs {Re V, Im V} then n pairs {Re U, Im U}.
hipError_t launch_phasor(int32_t layout, int64_t n, const double *vm, const double *va, double *ph, hipStream_t stream);
// Branch flows (and, if jac is not NULL, their 16 partials) of every branch
// at every state.
hipError_t launch_flows(const DevTwoPhase &d, int32_t nstate, const double *vm, const double *va, double *pf,
                        double *qf, double *pt, double *qt, double *jac, hipStream_t stream);
// Copy-add with atomic adds: three launches for all states (zero J, bus
// shunt terms, per-branch adds); jval 16-byte aligned.
hipError_t launch_copy_add(const DevTwoPhase &d, int32_t nstate, int64_t nnz_j, const double *vm, const double *va,
                           double *p, double *q, double *jval, bool pre, hipStream_t stream);
// out[s * out_nnz + map[k]] = jval[s * nnz_j + k] for every state s and
// entry k with 0 <= map[k] < out_nnz (other entries are skipped).
hipError_t launch_jscatter(int32_t nstate, int64_t nnz_j, const double *jval, const int32_t *map, int64_t out_nnz,
                           double *out, hipStream_t stream);
// Streaming copy of n doubles (16-byte aligned buffers), the bandwidth probe.
hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream);
// Precomputed branch constants (d.bc's layout) into bc.
hipError_t launch_branch_consts(const DevTwoPhase &d, double *bc, hipStream_t stream);
// The library's static scratch: a file-scope device array of
// kStaticScratchBytes (one copy per device, held until the process ends),
// used by the allocation-free two-phase entry point.  It holds ten doubles
// per record for at most kStaticScratchRecords records.
constexpr int64_t kStaticScratchBytes = int64_t(32) << 20;
constexpr int64_t kStaticScratchRecords = kStaticScratchBytes / (10 * (int64_t)sizeof(double));
// Device address of that array on `device`, which must be the current
// device.  Resolved with hipGetSymbolAddress on the first call for a device
// and cached; later calls make no HIP call.
hipError_t static_scratch(int device, double **out);
// States [0, nstate) one after another, two launches each.
hipError_t launch_two_phase(const DevTwoPhase &d, int32_t nstate, int64_t nnz_j, const double *vm, const double *va,
                            double *p, double *q, double *jval, bool pre, hipStream_t stream);

}  // namespace pf
