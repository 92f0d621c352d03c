/*
 * pf.h -- C ABI of the MI355X (gfx950) power-injection and Jacobian library.
 *
 * The library computes, for given bus voltage magnitudes v and angles theta,
 * the complex nodal power injections S = P + jQ and the values of the sparse
 * polar power-flow Jacobian
 *     J = [ dP/dtheta  dP/dv ]
 *         [ dQ/dtheta  dQ/dv ]
 * by the two methods of "Bus Admittance Matrix Revisited: Is It Outdated on
 * Modern Computers?" (arXiv 2302.10736):
 *   - the element-wise method (Section II.B, eqs. (5)-(7); Section IV.C):
 *     every branch end is evaluated on its own, then reduced onto buses and
 *     into precomputed Jacobian slots;
 *   - the Ybus method (Section II.A, eqs. (1)-(4); Section IV.B): a complex
 *     CSR admittance matrix, S = V conj(Ybus V), and the two-pass Jacobian.
 * It also offers the adjoint (vector-Jacobian product) of the injections.
 *
 * Conventions shared by every call
 * --------------------------------
 * Branch model (Section II.B): branch l runs from bus h = fbus[l] to bus
 *   k = tbus[l]; series admittance y_hk = 1/(r + jx); line charging b is
 *   split as y_h = y_k = j b/2; an off-nominal ratio m e^{j phi} (m = tap,
 *   phi = shift in radians) sits on the h side; tap == 0 means m = 1.
 *   Parallel branches between one bus pair are allowed.
 * Bus shunts: g_i + j b_i adds v_i^2 (g_i - j b_i) to S_i (the paper's
 *   eq. (7) has no shunt term; with it, the element-wise sum equals eq. (1)
 *   with the shunt on the admittance diagonal).
 * Sign: S_i is the complex power injected into the network at bus i.
 * Ybus pattern: every diagonal (i, i), kept even when its value is zero,
 *   plus (h, k) and (k, h) for each branch; parallel branches share an
 *   entry; columns ascend within a row (Section IV.B.2 keeps such zeros).
 * Jacobian pattern (eq. (2), size 2nb x 2nb): rows [P_0..P_{nb-1},
 *   Q_0..Q_{nb-1}], columns [theta_0..theta_{nb-1}, v_0..v_{nb-1}], each of
 *   the four blocks carrying the Ybus pattern, stored in CSR.  For Ybus
 *   entry p (0-based position in the Ybus CSR) in row i:
 *       J11 at yrow[i] + p,          J12 at yrow[i+1] + p,
 *       J21 at 2 nnzY + yrow[i] + p,  J22 at 2 nnzY + yrow[i+1] + p,
 *   which is the closed form of the index arrays of Algorithm 2.
 * Multiple grids: one handle may hold G independent grids (block-diagonal
 *   concatenation).  Bus-indexed arrays of all grids are concatenated
 *   (grid g owns [bus_off[g], bus_off[g+1])); each grid keeps its own Ybus
 *   and J patterns with grid-local rows and columns; grid g's Ybus values
 *   start at y_off[g] and its J values at 4 y_off[g] (pf_grid_offsets).
 * States: nstate >= 0 independent voltage states per call.  State arrays are
 *   row-major [nstate][nb_total]; J values are [nstate][nnz_j_total].
 * Memory: grid arrays given to pf_build_pattern are host memory, copied
 *   during the call.  Every state, adjoint seed and output pointer of the
 *   evaluation calls is a DEVICE pointer on the handle's device, owned by the
 *   caller, 8-byte aligned (16-byte for jval); outputs must not overlap
 *   inputs.  `stream` is a hipStream_t (NULL = default stream).
 * Evaluation calls enqueue work on `stream` and return: they allocate
 *   nothing, never synchronise and never read device data back, so they may
 *   be captured in a HIP graph.
 * Streams: the fused evaluation calls only read the handle's device data,
 *   so one handle may serve several streams at once, with two exceptions
 *   the caller orders: pf_ybus rewrites the handle's Ybus values and Ybus
 *   lane tables on its own stream, so Ybus evaluations (and replays of
 *   graphs holding them) on other streams must be ordered after it (an
 *   event and hipStreamWaitEvent, or a synchronisation); and every
 *   PF_METHOD_ELEMENTWISE_TWO_PHASE call on a handle uses that handle's one
 *   scratch buffer, so such calls on one handle must not overlap.
 * Results are deterministic: every sum runs in a fixed order set by the
 *   pattern (bus, then neighbour, then branch), independent of launch shape
 *   (the copy-add baseline, PF_METHOD_ELEMENTWISE_ATOMIC, excepted).
 * Errors: every call returns a pf_status.  On a validation error nothing is
 *   written and nothing is launched; pf_last_error() describes it.  Faults of
 *   earlier asynchronous work surface as PF_EHIP on a later call.  No call
 *   aborts or throws.
 */
#ifndef PF_H
#define PF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_grid pf_grid; /* opaque; owns host and device copies of the grid data */

typedef enum pf_status {
    PF_OK = 0,
    PF_EINVAL = 1, /* invalid argument (index range, self loop, non-finite, tap < 0, r = x = 0, NULL) */
    PF_ENOMEM = 2, /* host or device allocation failed */
    PF_EHIP = 3,   /* HIP runtime error (including faults of earlier work) or no usable GPU */
    PF_ESTATE = 4, /* call not valid in the handle's state (e.g. Ybus values not assembled) */
    PF_EUNSUP = 5  /* valid but unsupported input (see pf_last_error) */
} pf_status;

typedef enum pf_method {
    PF_METHOD_ELEMENTWISE = 0, /* eqs. (5)-(7): per branch end, then reduction */
    PF_METHOD_YBUS = 1,        /* eqs. (1), (3), (4): complex CSR SpMV, two-pass Jacobian */
    /* Element-wise in the paper's two steps (Section IV.C): every branch
     * evaluated once (both ends) into scratch, then a separate per-bus
     * reduction into P, Q and J.  A baseline for the fused method above;
     * pf_jacobian_values only.  Its scratch (10 doubles per record) belongs
     * to the handle, allocated by pf_build_pattern; states run one after
     * another, two launches each. */
    PF_METHOD_ELEMENTWISE_TWO_PHASE = 2,
    /* Element-wise with the paper's copy-add reduction (Section IV.C.2) done
     * by atomic adds: J set to zero and P, Q and the diagonal entries to the
     * bus-shunt terms, then one thread per branch adds both ends' values.
     * Another baseline; pf_jacobian_values only, three launches for all
     * states.  The additions run in no fixed order: results agree with the
     * other methods to rounding, not bit for bit, and may differ between
     * runs.  jval must be 16-byte aligned. */
    PF_METHOD_ELEMENTWISE_ATOMIC = 3
} pf_method;

enum {
    PF_BUILD_HOST_ONLY = 1u /* build and validate the pattern and the launch schedule (tiles
                               and lane tables) on the host only: no device memory, no GPU
                               needed; evaluation calls return PF_ESTATE */
};

/* Build a handle: validate the grid, build the Ybus pattern, the Jacobian
 * pattern (eq. (2)), the bus-sorted branch-end records and the launch
 * schedule, copy everything to the current HIP device and compute the
 * per-record branch constants there.  Setup work; not part of the timed
 * evaluation (the paper pre-builds the pattern once, Section IV.B.3).  The
 * handle's device memory also holds the two-phase baseline's scratch (80
 * bytes per record, nb + 2 nl records).
 *   nb, nl        total buses (>= 1) and branches (>= 0) over all grids
 *   fbus, tbus    int32[nl], 0-based, grid-local bus indices; fbus != tbus
 *   r, x, b_charging, tap, shift   f64[nl]: p.u. series resistance and
 *                 reactance (not both 0), total charging susceptance,
 *                 off-nominal ratio (>= 0, 0 means 1), phase shift (rad)
 *   gs, bs        f64[nb] bus shunt conductance / susceptance; NULL = 0
 *   ngrids        >= 1; bus_off, br_off int32[ngrids+1] (NULL when 1):
 *                 grid g owns buses [bus_off[g], bus_off[g+1]) and branches
 *                 [br_off[g], br_off[g+1]); offsets start at 0, end at
 *                 nb / nl, and every grid has at least one bus
 *   flags         0 or PF_BUILD_HOST_ONLY
 *   out           receives the handle (set to NULL on error)
 * Errors: PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_EUNSUP (more than 2^31 - 1
 * records or Jacobian entries). */
int pf_build_pattern(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus,
                     const double *r, const double *x, const double *b_charging,
                     const double *tap, const double *shift, const double *gs,
                     const double *bs, int32_t ngrids, const int32_t *bus_off,
                     const int32_t *br_off, uint32_t flags, pf_grid **out);

/* Release a handle and its device memory.  NULL is allowed.  The caller
 * must make sure no enqueued work still uses the handle. */
void pf_grid_free(pf_grid *g);

/* Totals over all grids: buses, Ybus nonzeros, Jacobian nonzeros (4 nnz_y),
 * number of grids.  Any output pointer may be NULL. */
int pf_grid_sizes(const pf_grid *g, int64_t *nb, int64_t *nnz_y, int64_t *nnz_j, int32_t *ngrids);
int pf_pattern_sizes(const pf_grid *g, int64_t *nnz_y, int64_t *nnz_j);

/* Per-grid offsets of the Ybus values (y_off) and of the J values
 * (j_off = 4 y_off), int64[ngrids+1] host buffers. */
int pf_grid_offsets(const pf_grid *g, int64_t *y_off, int64_t *j_off);

/* Copy the patterns to caller-allocated HOST buffers, grid after grid, each
 * with grid-local rows and columns:
 *   y_rowptr int32[nb_total + ngrids], y_col int32[nnz_y],
 *   j_rowptr int32[2 nb_total + ngrids], j_col int32[nnz_j].
 * Any pointer may be NULL to skip that array.  Works on host-only handles. */
int pf_pattern_export(const pf_grid *g, int32_t *y_rowptr, int32_t *y_col, int32_t *j_rowptr,
                      int32_t *j_col);

/* Assemble the Ybus values (Section II.A, with branch entries matching
 * eqs. (5)-(6): Y_hh += (y_h + y_hk)/m^2, Y_hk += -y_hk e^{j phi}/m,
 * Y_kh += -y_hk e^{-j phi}/m, Y_kk += y_k + y_hk, Y_ii += g_i + j b_i) into
 * the handle; parallel branches are summed in pattern order.  Must precede
 * pf_injections_ybus and pf_jacobian_values(PF_METHOD_YBUS).  When y_re /
 * y_im are non-NULL the values are also copied to those DEVICE buffers
 * (f64[nnz_y], grid g at y_off[g]).  Enqueued on `stream`. */
int pf_ybus(pf_grid *g, double *y_re, double *y_im, void *stream);

/* Injections by the element-wise method (eqs. (5)-(7) plus bus shunts).
 * vm, va: f64[nstate][nb] device; p, q: f64[nstate][nb] device outputs. */
int pf_injections_elementwise(const pf_grid *g, int32_t nstate, const double *vm,
                              const double *va, double *p, double *q, void *stream);

/* Injections by the Ybus method (Section IV.B.1: U = e^{j theta},
 * V = v U, I = Ybus V, S = V conj(I)).  PF_ESTATE before pf_ybus. */
int pf_injections_ybus(const pf_grid *g, int32_t nstate, const double *vm, const double *va,
                       double *p, double *q, void *stream);

/* Injections and Jacobian values in one pass.
 *   method  PF_METHOD_ELEMENTWISE: the 16 partial derivatives per branch
 *           (Section II.B), reduced into the J slots (Section IV.C.2);
 *           PF_METHOD_YBUS: eqs. (3)-(4) by the row-wise two-pass scheme
 *           (Section IV.B.2), written in place into J (Section IV.B.3;
 *           PF_ESTATE before pf_ybus).
 *           PF_METHOD_ELEMENTWISE or PF_METHOD_YBUS | PF_JAC_CSC: jval in
 *           column-major (CSC) order, the storage sparse direct solvers take
 *           (the paper keeps J in CSC, Section IV.A).  The pattern is
 *           structurally symmetric, so the CSC column pointers and row
 *           indices are the exported j_rowptr and j_col: value k of column c
 *           is J(j_col[k], c); the values equal the CSR values transposed,
 *           bit for bit.  One launch, as for CSR; PF_EUNSUP with the
 *           two-phase and copy-add baselines.
 *   p, q    f64[nstate][nb] device outputs, or NULL to skip
 *   jval    f64[nstate][nnz_j] device output in the exported CSR order
 *           (CSC with PF_JAC_CSC). */
enum { PF_JAC_CSC = 0x100 };
/* OR-ed into PF_METHOD_ELEMENTWISE_TWO_PHASE or PF_METHOD_ELEMENTWISE_ATOMIC:
 * the branch kernel reads per-branch constants precomputed at build time
 * (coupling y_hk/m and both ends' own-end admittances, six doubles, the
 * paper's precomputation, Section IV.C.1) instead of deriving them from
 * r, x, b, tap on the fly.  Same values; PF_EUNSUP with the other methods
 * (the fused element-wise kernel always reads precomputed per-record
 * constants). */
enum { PF_EW_PRECOMPUTED = 0x200 };
int pf_jacobian_values(const pf_grid *g, int32_t method, int32_t nstate, const double *vm,
                       const double *va, double *p, double *q, double *jval, void *stream);

/* For callers that cannot allocate device memory or use a handle's own
 * buffers at call time (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): pf_jacobian_values with
 * PF_METHOD_ELEMENTWISE_TWO_PHASE (optionally | PF_EW_PRECOMPUTED), same
 * arguments, layouts and results bit for bit, whose scratch is the library's
 * static device array instead of the handle's buffer.  The array is 32 MiB
 * per device (ten doubles per record: grids of at most 419,430 records,
 * nb + 2 nl over all grids of the handle; larger grids get PF_EUNSUP), is
 * resolved once per device when a handle is built and stays allocated until
 * the process ends.  The call allocates nothing.  Every call on a device
 * shares that device's array and reads only what it wrote itself earlier in
 * the same call (nothing needs to start at zero), so calls that overlap on
 * one device (other streams, other threads, other handles) race and must be
 * ordered by the caller.  Errors: as pf_jacobian_values, plus PF_EINVAL for
 * another method and PF_EUNSUP for a grid beyond the limit. */
int pf_jacobian_two_phase_static(const pf_grid *g, int32_t method, int32_t nstate, const double *vm,
                                 const double *va, double *p, double *q, double *jval, void *stream);

/* Adjoint of the injections: for seeds lam_p, lam_q (f64[nstate][nb]),
 *   g_va = J11^T lam_p + J21^T lam_q,   g_vm = J12^T lam_p + J22^T lam_q,
 * i.e. the gradient of sum_i (lam_p_i P_i + lam_q_i Q_i) with respect to
 * (va, vm), without forming J.  Outputs f64[nstate][nb] device. */
int pf_injections_vjp(const pf_grid *g, int32_t nstate, const double *vm, const double *va,
                      const double *lam_p, const double *lam_q, double *g_vm, double *g_va,
                      void *stream);

/* Ybus method from stored phasors: the paper's two separate steps of the
 * injection computation (Section IV.B.1 and Table I: phasor calculation,
 * then the sparse product), with the phasors kept in one of the two storage
 * layouts it compares.  Ablation of the fused pf_injections_ybus /
 * pf_jacobian_values(PF_METHOD_YBUS), which form the phasors on the fly;
 * all three give bit-identical results.
 *   layout  PF_PHASOR_SPLIT: real and imaginary parts in separate arrays,
 *           ph = [Re V | Im V | Re U | Im U], four f64[nstate][nb] planes;
 *           PF_PHASOR_INTERLEAVED: {re, im} pairs, ph = nstate*nb pairs of
 *           V followed by nstate*nb pairs of U (16-byte aligned).
 *   ph      f64[4 nstate nb] device buffer, caller-owned.
 * pf_phasors writes V = v e^{j theta} and U = e^{j theta}.
 * pf_ybus_from_phasors reads them (U only when jval is non-NULL) and writes
 * p, q (f64[nstate][nb]; required when jval is NULL, else both may be NULL)
 * and jval (f64[nstate][nnz_j], CSR order, may be NULL).  One launch each.
 * Errors: PF_EINVAL for an unknown layout, a NULL buffer, unaligned
 * interleaved phasors or nothing to write; PF_ESTATE before pf_ybus
 * (pf_ybus_from_phasors) or on a host-only handle. */
enum { PF_PHASOR_SPLIT = 1, PF_PHASOR_INTERLEAVED = 2 };
int pf_phasors(const pf_grid *g, int32_t layout, int32_t nstate, const double *vm, const double *va,
               double *ph, void *stream);
int pf_ybus_from_phasors(const pf_grid *g, int32_t layout, int32_t nstate, const double *ph, double *p,
                         double *q, double *jval, void *stream);

/* Branch flows, eqs. (5)-(6): for every branch l (input order, grid after
 * grid) the power entering the branch at its from end, S_hk = pf + j qf,
 * and at its to end, S_kh = pt + j qt; f64[nstate][nl] device (nl over all
 * grids).  jac (device, may be NULL): the 16 partial derivatives per branch,
 * f64[nstate][16][nl], row 4 f + v holding d(Pf, Qf, Pt, Qt)[f] /
 * d(theta_from, theta_to, v_from, v_to)[v] (the derivatives line-flow limits
 * need; Section II.B).  One launch. */
int pf_branch_flows(const pf_grid *g, int32_t nstate, const double *vm, const double *va, double *pf,
                    double *qf, double *pt, double *qt, double *jac, void *stream);

/* Jacobian values in another sparsity pattern (Algorithm 2, Section
 * IV.B.3: indices into the target pattern found once by matching row and
 * column, then an in-place copy by those indices).  For targets whose
 * pattern holds J's entries and more, e.g. the extra couplings of series
 * devices such as a TCSC.
 * pf_jacobian_map (host): target pattern of size n x n, n = 2 nb, one grid
 *   per handle; layout PF_LAYOUT_CSR (ptr = row pointers, idx = column
 *   indices) or PF_LAYOUT_CSC (ptr = column pointers, idx = row indices);
 *   host arrays int32 ptr[n+1], idx[ptr[n]].  Writes map int32[nnz_j] (host):
 *   for J entry k in the exported CSR order its position in the target.
 *   PF_EINVAL if the target lacks an entry of J (the message names it) or
 *   is malformed; PF_EUNSUP for a multi-grid handle.  Works on host-only
 *   handles.
 * pf_jacobian_scatter (device): out[s * out_nnz + map[k]] =
 *   jval[s * nnz_j + k] for every state s and entry k; jval f64[nstate][nnz_j],
 *   map int32[nnz_j], out f64[nstate][out_nnz], all device; target entries
 *   that J does not cover are left as they are; map values outside
 *   [0, out_nnz) are skipped.  One launch. */
enum { PF_LAYOUT_CSR = 0, PF_LAYOUT_CSC = 1 };
int pf_jacobian_map(const pf_grid *g, int32_t layout, int32_t n, const int32_t *ptr, const int32_t *idx,
                    int32_t *map);
int pf_jacobian_scatter(const pf_grid *g, int32_t nstate, const double *jval, const int32_t *map, int64_t out_nnz,
                        double *out, void *stream);

/* Launch schedule.
 *   tile_items        workgroup size (64, 128, 256 or 512): branch ends per
 *                     element-wise work tile, Ybus nonzeros per Ybus tile
 *   states_per_block  voltage states one workgroup evaluates in turn, with
 *                     the tile's constants held in registers (>= 1; 0 =
 *                     automatic: at most 2 for Jacobian launches, at most 8
 *                     for injections, fewer when the tiles alone do not
 *                     fill the GPU; the adjoint splits each tile's states
 *                     into as many chunks as fill one round of resident
 *                     workgroups)
 *   order             order of the (tile, state chunk) work items over the
 *                     workgroups: PF_ORDER_TILE_MAJOR (the state chunks of
 *                     one tile are adjacent), PF_ORDER_STATE_MAJOR (the tiles
 *                     of one state chunk are adjacent, so concurrent
 *                     workgroups write neighbouring parts of J),
 *                     PF_ORDER_GROUPED (each of the 8 XCDs owns an eighth
 *                     of the tiles and walks them chunk by chunk: the tiles'
 *                     tables stay in its L2 while neighbouring workgroups
 *                     write neighbouring parts of J) or PF_ORDER_AUTO
 *                     (Jacobian launches: state-major while the tile tables
 *                     fit in 2 MB, which then stay in every XCD's L2,
 *                     grouped above that; injections and the adjoint:
 *                     tile-major, so the state chunks of one tile share
 *                     an L2)
 * The initial schedule is tile_items 256 (with several grids per handle:
 * the smallest of 64, 128, 256 that holds the mean branch ends per grid,
 * since tiles never span grids), states_per_block 0, PF_ORDER_AUTO.
 * Changing the schedule never changes results.  Rebuilds the tile list on
 * the host and device; not for use while work on the handle is in flight.
 * Graphs recorded before the call must be recorded again. */
enum { PF_ORDER_AUTO = 0, PF_ORDER_TILE_MAJOR = 1, PF_ORDER_STATE_MAJOR = 2, PF_ORDER_GROUPED = 3 };
int pf_set_schedule(pf_grid *g, int32_t tile_items, int32_t states_per_block, int32_t order);
/* ntiles: element-wise work tiles of the current schedule. */
int pf_get_schedule(const pf_grid *g, int32_t *tile_items, int32_t *states_per_block, int32_t *order,
                    int32_t *ntiles);

/* Recorded evaluation sequences (HIP graphs).
 * The evaluation calls above only enqueue kernels (no allocation, no host
 * synchronisation, no memory set), so a fixed sequence of them on fixed
 * buffers can be recorded once and replayed with a single launch; loops that
 * evaluate one grid many times (Newton iterations, repeated scenario sweeps)
 * then pay the host cost of a call once.
 *
 * pf_graph_create records `nops` operations in order:
 *   PF_OP_INJECTIONS  pf_injections_elementwise / pf_injections_ybus by
 *                     `method`; P = out_a, Q = out_b
 *   PF_OP_JACOBIAN    pf_jacobian_values(method); P = out_a, Q = out_b
 *                     (both may be NULL), J = jval
 *   PF_OP_VJP         pf_injections_vjp; lam_p, lam_q in, g_vm = out_a,
 *                     g_va = out_b
 * with the checks, layouts and error codes of those calls; unused pointers
 * are ignored.  On error *out stays NULL and nothing is recorded.  The graph
 * refers to the grid's device tables and to the given buffers (caller-owned,
 * device memory): free the graph before the grid, keep the buffers alive
 * while it is in use.  pf_ybus may run between launches (Ybus values are
 * refreshed in place); after pf_set_schedule, pf_graph_launch returns
 * PF_ESTATE and the graph must be recorded again.  pf_graph_launch enqueues
 * the whole sequence on `stream`; replays on one stream run in order, replays
 * on different streams may overlap and then race on shared outputs. */
typedef struct pf_graph pf_graph;
enum { PF_OP_INJECTIONS = 0, PF_OP_JACOBIAN = 1, PF_OP_VJP = 2 };
typedef struct {
    int32_t op;      /* PF_OP_* */
    int32_t method;  /* PF_METHOD_* (PF_OP_INJECTIONS, PF_OP_JACOBIAN) */
    int32_t nstate;
    const double *vm, *va;
    const double *lam_p, *lam_q; /* PF_OP_VJP */
    double *out_a, *out_b;
    double *jval; /* PF_OP_JACOBIAN */
} pf_op;
int pf_graph_create(const pf_grid *g, const pf_op *ops, int32_t nops, pf_graph **out);
int pf_graph_launch(const pf_graph *gr, void *stream);
void pf_graph_free(pf_graph *gr);

/* Schedule autotuner.  Times candidate launch schedules (pf_set_schedule)
 * for one operation and leaves the fastest set on the handle; results never
 * depend on the schedule, so tuning changes speed only.
 *   op      the operation, as for pf_graph_create, on the caller's DEVICE
 *           buffers (its outputs are overwritten); nstate >= 1
 *   ncand, cand  int32[3 ncand] host array of (tile_items, states_per_block,
 *           order) triples, or ncand = 0 for the default set: tile_items in
 *           {64, 128, 256, 512} x states_per_block in {0, 1, 2, 4, 8, 16, 32,
 *           64} up to nstate x the three work orders (one state: the four tile
 *           sizes, one state per workgroup)
 *   reps    calls per timing in [1, 1000]: each candidate records `reps`
 *           copies of the op in a graph, replays it untimed for 10 ms, then
 *           takes the median of three replays timed by HIP events on a
 *           private stream
 *   best    int32[3] out: the chosen triple; best_us (may be NULL): its
 *           device time per call in microseconds; tried (may be NULL): the
 *           number of candidates timed
 * Synchronises with its private stream; not for use while other work on
 * the handle is in flight (it changes the schedule, so graphs recorded
 * before must be recorded again).  On an error the handle keeps the
 * schedule it had.  Errors: those of pf_set_schedule and pf_graph_create,
 * PF_EINVAL for bad arguments, PF_ESTATE on a host-only handle. */
int pf_autotune(pf_grid *g, const pf_op *op, int32_t ncand, const int32_t *cand, int32_t reps, int32_t *best,
                double *best_us, int32_t *tried);

/* Description of the last error on the calling thread ("" if none).  The
 * string stays valid until the next pf_* call on that thread. */
const char *pf_last_error(void);

/* Library version string. */
const char *pf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
