// Internal declarations shared by the host API (pf_api.cpp) and the kernels
// (pf_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pf {

// Device view of a handle, passed to kernels by value.
//
// Records ("items") are the unit of the element-wise method: one per branch
// end (at bus i, pointing to the remote bus j) and one per bus for its shunt
// (j == i), sorted by (bus, neighbour, branch).  Slots are Ybus nonzeros;
// without parallel branches item e and slot e coincide.
struct DevGrid {
    int32_t nb;           // buses over all grids
    int64_t nnz_y;        // Ybus nonzeros over all grids
    int64_t nnz_j;        // 4 nnz_y
    int32_t ntiles;
    const int32_t *yrow;  // [nb+1] slot row pointer (global slot numbering)
    const int32_t *irow;  // [nb+1] item row pointer
    const int32_t *ycol;  // [nnz_y] global bus index of the column
    const int32_t *nbr;   // [nitems] remote bus (== own bus for the shunt record)
    const int32_t *slot;  // [nitems] global slot of the item
    const double *A, *C;  // [nitems] own-end admittance Re / Im (shunt: g, b)
    const double *G, *B;  // [nitems] coupling admittance Re / Im of this end
    const double *Gr, *Br;  // [nitems] coupling admittance of the other end (adjoint)
    const double *yre, *yim;  // [nnz_y] Ybus values
    const int64_t *yoff;      // [ngrids+1] first slot of each grid
    const int32_t *tile_row;  // [ntiles+1] first row of each tile
    const int32_t *tile_grid;  // [ntiles] grid of each tile
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
    double *A, *C, *G, *B, *Gr, *Br;        // [nitems] outputs
    double *yre, *yim;                      // [nnz_y] outputs
};

enum Kind { K_EW_S = 0, K_EW_SJ = 1, K_YB_S = 2, K_YB_SJ = 3, K_EW_VJP = 4 };

struct Launch {
    int kind;
    int tile_items;        // workgroup size = records per tile
    int states_per_block;
    int nstate;
    bool has_parallel;
    const double *vm, *va, *lp, *lq;
    double *p, *q, *jval, *gvm, *gva;
};

hipError_t launch_eval(const DevGrid &g, const Launch &L, hipStream_t stream);
hipError_t launch_setup_items(const DevSetup &s, hipStream_t stream);
hipError_t launch_ybus_assemble(const DevSetup &s, hipStream_t stream);

}  // namespace pf
