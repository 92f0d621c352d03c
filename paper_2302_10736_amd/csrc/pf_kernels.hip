// HIP kernels for gfx950 (MI355X): nodal power injections, polar Jacobian
// values and their adjoint, by the element-wise method (Section II.B,
// eqs. (5)-(7); Section IV.C) and by the Ybus method (Section II.A,
// eqs. (1)-(4); Section IV.B).
//
// Work decomposition (both fused methods)
// ---------------------------------------
// Records are sorted by (bus, neighbour, branch).  A tile is a run of whole
// bus rows holding at most NT branch ends (element-wise; bus shunts live in
// the per-bus constants and take no lane) or NT Ybus nonzeros (NT =
// workgroup size); one thread owns one of them, and thread r < rows also
// owns row r of the tile.  Per voltage state a workgroup
//   1. evaluates every branch end (or nonzero) of the tile, writing the
//      off-diagonal Jacobian entries into an LDS copy of the tile's
//      Jacobian rows;
//   2. reduces each row sequentially, in record order, by its row thread,
//      which writes P_i, Q_i and the four diagonal Jacobian entries;
//   3. writes the tile's Jacobian rows with contiguous 16-byte streaming
//      stores: a tile's rows are two contiguous ranges of the CSR value
//      array (the P rows and the Q rows).
// No atomics; every sum has a fixed order set by the pattern, so results do
// not depend on the tile size or on the states per workgroup.  LDS buffers
// alternate between consecutive states (two barriers per state), and the
// gathers of the next state are issued before the current one is reduced.
// A row with more than NT records is a tile of its own, walked in pieces of
// NT records: the piece's 16-term chunks are summed in parallel and folded
// in order by one thread, so its sums keep the packed path's order.  The
// work items (tile, chunk of states) map to workgroups XCD by XCD in one of
// three orders (tile-major, state-major, grouped; see work_item).  The
// baselines further
// down (the two-phase and copy-add methods, branch flows) use one thread
// per branch instead.
//
// Element-wise records
// --------------------
// A branch-end record at bus i (remote bus j) holds the coupling admittance
// G + jB of its end: -y_hk e^{j phi}/m at the from end, -y_hk e^{-j phi}/m at
// the to end (the phase shift folded in), zero for the bus-shunt record.
// With t = theta_i - theta_j, alpha = G cos t + B sin t and
// beta = G sin t - B cos t, eqs. (5) and (6) split into real and imaginary
// parts read, for every record,
//   P_e = v_i^2 A_e + v_i v_j alpha,   Q_e = -v_i^2 C_e + v_i v_j beta,
// where A_e + jC_e is the record's own-end admittance ((y_h + y_hk)/m^2 at
// the from end, y_k + y_hk at the to end, g + jb for the shunt).  The own-end
// term of every record at bus i carries the same factor v_i^2, so the bus sum
// of eq. (7) is
//   P_i = v_i^2 dA_i + v_i a_i,   Q_i = -v_i^2 dC_i + v_i b_i,
// with the state-free bus constants dA + j dC = sum of A_e + jC_e (setup) and
// the per-state row sums a_i = sum_e v_j alpha_e, b_i = sum_e v_j beta_e.
// The 16 partials of a branch (Section II.B) are its two ends' remote partials
//   dP_e/dtheta_j =  v_i v_j beta,   dP_e/dv_j = v_i alpha,
//   dQ_e/dtheta_j = -v_i v_j alpha,  dQ_e/dv_j = v_i beta,
// written straight into J (one record per off-diagonal slot, or a fixed-order
// slot sum with parallel branches), and its own partials, whose bus sums are
//   dP_i/dtheta_i = -v_i b_i,          dP_i/dv_i = 2 v_i dA_i + a_i,
//   dQ_i/dtheta_i =  v_i a_i,          dQ_i/dv_i = b_i - 2 v_i dC_i.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "pf_internal.h"
#include "pf_math.h"

namespace pf {

// Series coefficients in constant memory: with external linkage the compiler
// reads them with scalar loads instead of folding them into vector-register
// immediates, so each polynomial step is one FMA with a scalar operand.
__constant__ SinCosCoef g_sincos = kSinCosTaylor;

namespace {

constexpr int kXcds = 8;

// sincos_rad, with its reduction and quadrant fix-up skipped when every lane
// of the wave has quadrant count 0 (angle differences within about pi/4, the
// usual case in power-flow states).  Same bits either way (pf_math.h), so a
// record's result does not depend on which lanes share its wave.
__device__ __forceinline__ void sincos_dev(double x, double *s, double *c) {
    if (__builtin_amdgcn_ballot_w64(sincos_quadrant(x) != 0.0) == 0) {
        sincos_series(x, s, c, g_sincos);
        return;
    }
    sincos_rad(x, s, c, g_sincos);
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of work items so that neighbouring tiles, and all state
// chunks of one tile, share one L2.
__device__ __forceinline__ int work_index(int nblocks) {
    const int b = blockIdx.x;
    const int per = nblocks / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Tiles per XCD in the grouped order.
__host__ __device__ __forceinline__ int grouped_tiles(int ntiles) { return (ntiles + kXcds - 1) / kXcds; }

// The work item of this workgroup: tile t and state chunk c, or false for a
// workgroup past the end.
//   WO_TILE:    item w (work_index), tile w / nchunk, chunk w % nchunk: the
//               state chunks of a tile are adjacent, on one XCD.
//   WO_STATE:   tile w % ntiles, chunk w / ntiles: the tiles of a chunk are
//               adjacent.
//   WO_GROUPED: XCD x owns tiles [x tx, x tx + tx), tx = ceil(ntiles / 8),
//               and walks them chunk by chunk (all its tiles for chunk 0,
//               then for chunk 1, ...): each tile's tables stay in that
//               XCD's L2 across chunks while consecutive workgroups write
//               neighbouring rows of one state's outputs.  The grid has
//               8 tx nchunk workgroups.
__device__ __forceinline__ bool work_item(int ntiles, int nchunk, int order, int &t, int &c) {
    if (nchunk == 1) {  // one chunk: every order maps tile = work_index (and the grids agree)
        t = work_index(gridDim.x);
        c = 0;
        return t < ntiles;
    }
    if (order == WO_GROUPED) {
        const int tx = grouped_tiles(ntiles);
        const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
        const int ntx = min(tx, ntiles - x * tx);  // tiles of XCD x (<= 0: none)
        if (ntx <= 0 || i >= ntx * nchunk) return false;
        t = x * tx + i % ntx;
        c = i / ntx;
        return true;
    }
    const int w = work_index(gridDim.x);
    if (w >= ntiles * nchunk) return false;
    if (order == WO_STATE) {
        t = w % ntiles;
        c = w / ntiles;
    } else {
        t = w / nchunk;
        c = w - t * nchunk;
    }
    return true;
}

// LDS-only workgroup barrier: orders LDS accesses across the barrier without
// waiting for outstanding global loads (prefetches) or stores.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

using Tile = TileDesc;

__device__ __forceinline__ Tile tile_of(const DevGrid &g, int t) { return g.tiles[t]; }

// LDS copy of one state's J rows of a packed tile with at most NS Ybus
// slots: the P rows in [0, 2 NS), the Q rows from kQ<NS> on, and one pad
// position (kPad<NS>, and kQ<NS> + kPad<NS> on the Q side) that absorbs the
// writes of lanes with nothing to write.  The Q offset keeps both halves
// 16-byte aligned.
template <int NS>
constexpr int kQ = 2 * NS + 2;
template <int NS>
constexpr int kPad = 2 * NS;
template <int NS>
constexpr int kJStage = 4 * NS + 4;

// Two 16-bit fields of a lane-table word.
__device__ __forceinline__ int lo16(int v) { return v & 0xffff; }
__device__ __forceinline__ int hi16(int v) { return (int)((unsigned)v >> 16); }

struct Cx {
    double re, im;
};
// Complex product with one rounding per product term and one fused step.
__device__ __forceinline__ Cx cmul(Cx a, Cx b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ Cx cconj(Cx a) { return {a.re, -a.im}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }

// Results are written once and never read back by the kernel that writes
// them.  Streaming (nontemporal) stores pass them on towards memory at once
// instead of leaving them dirty in L2, where the write-back at the end of the
// kernel would only start after the last workgroup has finished.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_out(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_out2(dvec2 *p, dvec2 v) { __builtin_nontemporal_store(v, p); }

// A row output (P, Q or an adjoint gradient) of the packed tiles: a plain
// store with PLAIN, else a streaming one.  The row ranges of neighbouring
// tiles share the 128-byte lines at their ends.  When a launch has few
// state chunks per tile, those tiles write the shared lines at about the
// same time: plain stores let L2 join the two parts of each line before it
// goes to memory, where streaming stores write two partial lines.  With
// many chunks per tile the lines would wait in L2 too long, and streaming
// stores are faster.
template <bool PLAIN>
__device__ __forceinline__ void st_row(double *p, double v) {
    if constexpr (PLAIN)
        *p = v;
    else
        __builtin_nontemporal_store(v, p);
}

// Copy a staged tile of J rows (LDS, slot capacity NS) to global memory
// with 16-byte stores.
template <int NT, int NS>
__device__ __forceinline__ void write_jrows(const Tile &c, const double *s_J, double *Js) {
    const dvec2 *src = reinterpret_cast<const dvec2 *>(s_J);
    dvec2 *dp = reinterpret_cast<dvec2 *>(Js + c.jp);
    dvec2 *dq = reinterpret_cast<dvec2 *>(Js + c.jq);
    for (int q = threadIdx.x; q < c.ns; q += NT) {
        st_out2(dp + q, src[q]);
        st_out2(dq + q, src[kQ<NS> / 2 + q]);
    }
}

// Fields of a Ybus lane word (yb_pack): LDS targets as ew_o11 / ew_o12,
// then the tile row and the diagonal flag.
__device__ __forceinline__ int yb_row(int v) { return (v >> 22) & 0x1ff; }
__device__ __forceinline__ bool yb_diag(int v) { return v < 0; }

// Fields of an element-wise lane word (ew_pack).
__device__ __forceinline__ int ew_o11(int v) { return v & 0x7ff; }
__device__ __forceinline__ int ew_o12(int v) { return (v >> 11) & 0x7ff; }
__device__ __forceinline__ int ew_row(int v) { return (int)((unsigned)v >> 22); }

// Walk states [sb, se) (never empty) with the per-state inputs of each state
// loaded one state ahead; `ra` holds state sb's inputs on entry.  Two
// register sets alternate (states are taken in pairs), so the loop never
// copies registers that are still being loaded: a copy would make the wave
// wait for every outstanding memory operation, including the previous
// state's stores.  The loop body has no branch: the memory counter counts
// loads and stores in issue order, and a load or store behind a branch makes
// the compiler wait for every outstanding operation where the paths join,
// prefetch included.  So every pair runs both of its states; when the count
// is odd, the last pair evaluates the last state twice and writes the same
// values to the same places again.  `proc(s, parity, in)` gets the parity of
// the state's position for the double-buffered LDS.
template <class In, bool ONE, class Load, class Proc>
__device__ __forceinline__ void pipelined_states(int sb, int se, In &ra, Load &&load, Proc &&proc) {
    if constexpr (ONE) {  // one state per workgroup: nothing to overlap, half the registers
        proc(sb, 0, ra);
        return;
    }
    In rb{};
    for (int s = sb; s < se; s += 2) {
        const int s1 = min(s + 1, se - 1);
        load(s1, rb);
        proc(s, 0, ra);
        load(min(s + 2, se - 1), ra);
        proc(s1, 1, rb);
    }
}

// Row sums of two LDS arrays over records [a, z), strictly left to right,
// continuing the running sums u and v.  Records are read four at a time so
// one LDS round trip serves four terms; the last zero to three records of
// the range are added one by one.
__device__ __forceinline__ void row_sum2_acc(const double *x, const double *y, int a, int z, double &u, double &v) {
    int q = a;
    for (; q + 3 < z; q += 4) {
        const double x0 = x[q], x1 = x[q + 1], x2 = x[q + 2], x3 = x[q + 3];
        const double y0 = y[q], y1 = y[q + 1], y2 = y[q + 2], y3 = y[q + 3];
        u += x0;
        v += y0;
        u += x1;
        v += y1;
        u += x2;
        v += y2;
        u += x3;
        v += y3;
    }
    if (q < z) {
        u += x[q];
        v += y[q];
    }
    if (q + 1 < z) {
        u += x[q + 1];
        v += y[q + 1];
    }
    if (q + 2 < z) {
        u += x[q + 2];
        v += y[q + 2];
    }
}

// Bus sums in an order set by the pattern alone: a row's terms (its branch
// ends, or its Ybus nonzeros) are taken in consecutive chunks of kSumChunk
// from the start of the row, each chunk is summed left to right from zero,
// and the chunk sums are added left to right (the first one taken as it
// is).  Rows of at most kSumChunk terms, nearly all of them, are a plain
// left-to-right sum.  Rows longer than a tile sum their chunks in parallel
// (chunk_sums, fold_chunks) and still produce the bits of the packed path,
// whatever the tile size.
constexpr int kSumChunk = 16;

__device__ __forceinline__ void row_sum2(const double *x, const double *y, int a, int z, double &sx, double &sy) {
    double u = 0.0, v = 0.0;
    const int e = min(z, a + kSumChunk);
    row_sum2_acc(x, y, a, e, u, v);
    for (int c = e; c < z; c += kSumChunk) {  // rows longer than one chunk
        double cu = 0.0, cv = 0.0;
        row_sum2_acc(x, y, c, min(z, c + kSumChunk), cu, cv);
        u += cu;
        v += cv;
    }
    sx = u;
    sy = v;
}

// Long rows, one piece of m <= NT terms starting at a multiple of kSumChunk
// in the row: thread q sums chunk q of the piece into csx[q], csy[q].
__device__ __forceinline__ void chunk_sums(const double *x, const double *y, int m, double *csx, double *csy) {
    const int q = threadIdx.x;
    if (q * kSumChunk < m) {
        double u = 0.0, v = 0.0;
        row_sum2_acc(x, y, q * kSumChunk, min(m, (q + 1) * kSumChunk), u, v);
        csx[q] = u;
        csy[q] = v;
    }
}

// Long rows, one thread: adds the piece's chunk sums in order to the running
// row sums (the row's first chunk is taken as it is).
__device__ __forceinline__ void fold_chunks(const double *csx, const double *csy, int m, bool first_piece, double &u,
                                            double &v) {
    const int nc = (m + kSumChunk - 1) / kSumChunk;
    int q = 0;
    if (first_piece && nc > 0) {
        u = csx[0];
        v = csy[0];
        q = 1;
    }
    row_sum2_acc(csx, csy, q, nc, u, v);  // left to right, four chunk sums per LDS round trip
}

// One element-wise record (see the file header): its row-sum terms and the
// four values of its off-diagonal J slot in staging order (P rows: theta
// part, v part; Q rows: theta part, v part).
struct EwRec {
    double a, b;  // v_j alpha, v_j beta (row sums)
    double o[4];  // CSR: dP_i/dtheta_j, dP_i/dv_j, dQ_i/dtheta_j, dQ_i/dv_j
};

__device__ __forceinline__ EwRec ew_record(double vi, double ti, double vj, double tj, double G, double B) {
    double sn, cs;
    sincos_dev(ti - tj, &sn, &cs);
    const double al = fma(G, cs, B * sn);
    const double be = fma(G, sn, -(B * cs));
    EwRec r;
    r.a = vj * al;
    r.b = vj * be;
    r.o[0] = vi * r.b;
    r.o[1] = vi * al;
    r.o[2] = -(vi * r.a);
    r.o[3] = vi * be;
    return r;
}

// The record for J in column-major (CSC) order.  The pattern is structurally
// symmetric, so column theta_i (v_i) of J occupies the positions of row P_i
// (Q_i) and lists rows P_k, then Q_k, for the same sorted k; the record's slot
// therefore receives the partials of the opposite end of the branch (bus j
// towards i: coupling Gr + jBr, angle -t) with respect to bus i:
//   dP_j/dtheta_i = v_j v_i beta',  dQ_j/dtheta_i = -v_j v_i alpha',
//   dP_j/dv_i     = v_j alpha',     dQ_j/dv_i     = v_j beta',
// alpha' = Gr cos t - Br sin t, beta' = -Gr sin t - Br cos t.  sin is odd and
// cos even bit for bit (sincos_rad), and the products round as the opposite
// record's CSR evaluation rounds them, so CSC values are the CSR values
// transposed exactly.
__device__ __forceinline__ EwRec ew_record_csc(double vi, double ti, double vj, double tj, double G, double B,
                                               double Gr, double Br) {
    double sn, cs;
    sincos_dev(ti - tj, &sn, &cs);
    const double al = fma(G, cs, B * sn);
    const double be = fma(G, sn, -(B * cs));
    const double al2 = fma(Gr, cs, -(Br * sn));
    const double be2 = fma(-Gr, sn, -(Br * cs));
    EwRec r;
    r.a = vj * al;
    r.b = vj * be;
    r.o[0] = vj * (vi * be2);
    r.o[1] = -(vj * (vi * al2));
    r.o[2] = vj * al2;
    r.o[3] = vj * be2;
    return r;
}

struct EwRow {
    double p, q, j11, j12, j21, j22;
};

__device__ __forceinline__ EwRow ew_row(double vi, double dA, double dC, double as, double bs) {
    EwRow o;
    o.p = vi * fma(vi, dA, as);
    o.q = vi * fma(-vi, dC, bs);
    o.j11 = -(vi * bs);
    o.j12 = fma(2.0 * vi, dA, as);
    o.j21 = vi * as;
    o.j22 = fma(-2.0 * vi, dC, bs);
    return o;
}

// ===================================================================
// Element-wise injections (WITH_J = false) and injections + Jacobian values.
// The body is shared by k_ew and k_ew_csc: CSC = true writes J in
// column-major order (WITH_J only) with the same tiles and staging, each
// record's slot filled by ew_record_csc and the diagonal entries
// dQ_i/dtheta_i and dP_i/dv_i trading places.
template <int NT, bool PAR, bool WITH_J, bool ONE, bool CSC, bool PLAIN>
__device__ __forceinline__ void ew_eval(const DevGrid &g, int nstate, int spb, int nchunk, int order,
                                        const double *__restrict__ vm, const double *__restrict__ va,
                                        double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    static_assert(WITH_J || !CSC, "the CSC order concerns J values");
    constexpr int NR = (WITH_J && PAR) ? NT : 1;  // remote partials kept for slot sums
    constexpr int NBUF = ONE ? 1 : 2;             // LDS buffers alternate between states
    constexpr int NS = kEwSlots(NT);              // Ybus slots per tile
    __shared__ int s_ls[NT];   // long rows: local slot of each branch end of a piece
    __shared__ int s_cls[2];    // long rows: slot carried into the next piece (-1: none), by piece parity
    __shared__ double s_carry[8];  // long rows: its partial sums, written [4, 8), read [0, 4)
    __shared__ double s_ab[NBUF][2][NT];
    __shared__ __align__(16) double s_J[NBUF][WITH_J ? kJStage<NS> : 2];
    __shared__ double s_rem[NBUF][4][NR];

    int t, c0;
    if (!work_item(g.ntiles, nchunk, order, t, c0)) return;
    const int sb = c0 * spb;
    const int se = min(nstate, sb + spb);
    const int k = threadIdx.x;
    // lane table entries do not depend on the tile descriptor: both load at once
    const size_t lane = (size_t)t * NT + k;
    const int j = g.lane_j[lane];
    const int pk = g.lane_pk[lane];
    const double2 gb = g.lane_gb[lane];
    double2 grbr = make_double2(0.0, 0.0);
    if constexpr (CSC) grbr = g.lane_grbr[lane];
    const Tile c = tile_of(g, t);
    const size_t nb = (size_t)g.nb;

    if (c.ne > NT) {
        // ---- one row with more than NT branch ends, walked in pieces of NT
        // branch ends (position p of the row's branch ends is record
        // i0 + p, one further from the bus-shunt record on, c.sh).  Each
        // thread evaluates one branch end of the piece; threads q < NT /
        // kSumChunk sum the piece's chunks and one thread (in the second wave
        // when there is one) folds them into the row sums in the order of
        // row_sum2, each piece's fold running beside the next piece's chunk
        // sums (two buffers of chunk sums).  Without parallel branches every
        // Ybus slot holds one record, whose lane writes the slot's four J
        // values as they are; with them, the first branch end of each slot
        // in the piece sums its slot's records in order and writes the four
        // values (a slot that the piece end cuts hands its partial sums to
        // the next piece through LDS, so every slot sum runs in record
        // order).  The folding thread writes the diagonal slot last, from the
        // row sums, and keeps its running sums in LDS, off the registers of
        // the packed path.  The (state, piece) items are walked with their loads two
        // stages ahead: while an item is summed, the remote states of the
        // next item and the records of the one after it are in flight.
        __shared__ double s_cs[2][2][NT / kSumChunk];  // chunk sums of the last two pieces, by piece parity
        constexpr int FT = NT >= 128 ? 64 : 0;  // the folding thread, off wave 0 when the tile has two waves
        __shared__ double s_rs[4];  // the folding thread's running row sums of the current state; dA, dC of the row
        const int i = c.r0;
        const int d = c.ns;  // slots in the row
        const int npc = (c.ne + NT - 1) / NT;  // pieces per state
        const int nit = (se - sb) * npc;
        const int sh = c.i0 + c.sh;  // the bus-shunt record: the diagonal slot
        const int ld = WITH_J ? (PAR ? g.slot[sh] : sh) - c.s0 : 0;
        auto rec = [&](int p) { return c.i0 + p + (p >= c.sh ? 1 : 0); };
        struct Rec {
            int je;   // remote bus
            int ls;   // the lane's slot, tile-relative
            int nls;  // slot of the next piece's first record (-1: last piece)
            double G, B, Gr, Br;
        };
        struct Gat {
            double vi, ti, vj, tj;
        };
        // Every lane loads valid entries: lanes past the piece end repeat its
        // last record (their values are never used).
        auto load_rec = [&](int it, Rec &r) {
            const int base = (it % npc) * NT;
            const int m = min(NT, c.ne - base);
            const int e = rec(base + min(k, m - 1));
            r.je = g.nbr[e];
            r.G = g.G[e];
            r.B = g.B[e];
            if constexpr (CSC) {
                r.Gr = g.Gr[e];
                r.Br = g.Br[e];
            }
            if constexpr (WITH_J) {
                const int en = rec(min(base + m, c.ne - 1));
                r.ls = (PAR ? g.slot[e] : e) - c.s0;
                const int nls = (PAR ? g.slot[en] : en) - c.s0;
                r.nls = base + m < c.ne ? nls : -1;
            }
        };
        auto load_gat = [&](int it, int je, Gat &x) {
            const size_t so = (size_t)(sb + it / npc) * nb;
            x.vj = vm[so + je];
            x.tj = va[so + je];
            x.vi = vm[so + i];
            x.ti = va[so + i];
        };
        Rec rc, rn;
        Gat gt;
        load_rec(0, rc);
        load_rec(min(1, nit - 1), rn);
        load_gat(0, rc.je, gt);
        if (k == 0) {
            s_rs[2] = g.dA[i];
            s_rs[3] = g.dC[i];
        }
        for (int it = 0; it < nit; ++it) {
            const int s = sb + it / npc, piece = it % npc, base = piece * NT;
            const int m = min(NT, c.ne - base);
            double *Js = WITH_J ? J + (size_t)s * (size_t)g.nnz_j : nullptr;
            if (WITH_J && k == 0 && piece == 0) s_cls[1] = -1;  // nothing carried into the first piece
            int ls = -1;
            if (WITH_J && k == 0) s_cls[piece & 1] = -1;  // read last in the previous piece
            if (k < m) {
                EwRec r;
                if constexpr (CSC)
                    r = ew_record_csc(gt.vi, gt.ti, gt.vj, gt.tj, rc.G, rc.B, rc.Gr, rc.Br);
                else
                    r = ew_record(gt.vi, gt.ti, gt.vj, gt.tj, rc.G, rc.B);
                s_ab[0][0][k] = r.a;
                s_ab[0][1][k] = r.b;
                if constexpr (WITH_J && !PAR) {  // one record per slot: its J values as they are
                    const int lsk = rc.ls;
                    st_out(Js + c.jp + lsk, r.o[0]);
                    st_out(Js + c.jp + d + lsk, r.o[1]);
                    st_out(Js + c.jq + lsk, r.o[2]);
                    st_out(Js + c.jq + d + lsk, r.o[3]);
                }
                if constexpr (WITH_J && PAR) {
                    s_J[0][0 * NT + k] = r.o[0];
                    s_J[0][1 * NT + k] = r.o[1];
                    s_J[0][2 * NT + k] = r.o[2];
                    s_J[0][3 * NT + k] = r.o[3];
                    ls = rc.ls;
                    s_ls[k] = ls;
                }
            }
            const int nls = rc.nls;
            const double vi = gt.vi;
            // the next item's remote states, then the records of the one after
            load_gat(min(it + 1, nit - 1), rn.je, gt);
            rc = rn;
            load_rec(min(it + 2, nit - 1), rn);
            lds_barrier();
            chunk_sums(s_ab[0][0], s_ab[0][1], m, s_cs[piece & 1][0], s_cs[piece & 1][1]);
            if (k == FT && piece > 0) {  // the previous (full) piece's chunk sums, while this piece's are summed
                double as = s_rs[0], bs = s_rs[1];
                fold_chunks(s_cs[(piece + 1) & 1][0], s_cs[(piece + 1) & 1][1], NT, piece == 1, as, bs);
                s_rs[0] = as;
                s_rs[1] = bs;
            }
            if constexpr (WITH_J && PAR) {
                const int prev_cls = s_cls[(piece + 1) & 1];  // slot carried in from the previous piece
                const bool cont = k == 0 && ls == prev_cls;
                const bool head = k < m && (k == 0 || ls != s_ls[k - 1]);
                if (head) {
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                    if (cont) {
                        a0 = s_carry[0];
                        a1 = s_carry[1];
                        a2 = s_carry[2];
                        a3 = s_carry[3];
                    }
                    int q = k;
                    for (; q < m && s_ls[q] == ls; ++q) {
                        a0 += s_J[0][0 * NT + q];
                        a1 += s_J[0][1 * NT + q];
                        a2 += s_J[0][2 * NT + q];
                        a3 += s_J[0][3 * NT + q];
                    }
                    if (q == m && nls == ls) {
                        s_carry[4] = a0;  // the slot goes on in the next piece
                        s_carry[5] = a1;
                        s_carry[6] = a2;
                        s_carry[7] = a3;
                        s_cls[piece & 1] = ls;
                    } else {
                        st_out(Js + c.jp + ls, a0);
                        st_out(Js + c.jp + d + ls, a1);
                        st_out(Js + c.jq + ls, a2);
                        st_out(Js + c.jq + d + ls, a3);
                    }
                }
            }
            lds_barrier();
            if (k == 0) {
                if constexpr (WITH_J && PAR) {  // the carried partial sums move to the slots read by the next piece
                    if (s_cls[piece & 1] >= 0) {
                        s_carry[0] = s_carry[4];
                        s_carry[1] = s_carry[5];
                        s_carry[2] = s_carry[6];
                        s_carry[3] = s_carry[7];
                    }
                }
            }
            if (piece == npc - 1) {  // the state's last piece: its own chunk sums, then the row results
                if (k == FT) {
                    double as = s_rs[0], bs = s_rs[1];
                    fold_chunks(s_cs[piece & 1][0], s_cs[piece & 1][1], m, false, as, bs);
                    const EwRow o = ew_row(vi, s_rs[2], s_rs[3], as, bs);
                    if (P) {
                        st_out(P + (size_t)s * nb + i, o.p);
                        st_out(Q + (size_t)s * nb + i, o.q);
                    }
                    if constexpr (WITH_J) {
                        st_out(Js + c.jp + ld, o.j11);
                        st_out(Js + c.jp + d + ld, CSC ? o.j21 : o.j12);
                        st_out(Js + c.jq + ld, CSC ? o.j12 : o.j21);
                        st_out(Js + c.jq + d + ld, o.j22);
                    }
                }
                lds_barrier();
            }
        }
        return;
    }

    // ---- packed tile: whole rows, at most NT branch ends.  Lane k holds
    // the tile's k-th branch end (inert past c.ne; shunt records take no
    // lane); its table entry gives the remote bus, the tile row and the LDS
    // targets (o11, o12) of its remote partials (the pad for idle lanes and,
    // with parallel branches, every record but the first of its slot, which
    // also gets the slot's record count).  Thread k < rows also owns row k.
    const int rowl = ew_row(pk);
    const int o11 = ew_o11(pk), o12 = ew_o12(pk);
    const int run = PAR ? g.lane_run[lane] : 0;
    const bool rowt = k < c.nrows;
    const int ir = c.r0 + (rowt ? k : 0);
    const int li = c.r0 + rowl;
    struct In {
        double vi, ti, vj, tj, vr;
    };
    auto load = [&](int s, In &x) {
        const double *vms = vm + (size_t)s * nb;
        const double *vas = va + (size_t)s * nb;
        x.vi = vms[li];
        x.ti = vas[li];
        x.vj = vms[j];
        x.tj = vas[j];
        x.vr = vms[ir];
    };
    // The first state's gathers go out before the row loads, and every load
    // is unconditional (each lane's indices are valid), so the waits before
    // the record phase cover the gathers only.
    In first;
    load(sb, first);
    const int irr = rowt ? ir : g.nb;  // lanes without a row read the inert entry
    const int2 rw = g.row_ew[irr];
    const double dA = g.dA[irr], dC = g.dC[irr];
    const int ra = lo16(rw.x), rz = hi16(rw.x), d11 = lo16(rw.y), d12 = hi16(rw.y);
    // Every lane evaluates a record and a row (inert lanes with zero
    // admittances, valid buses and empty row ranges), so each loaded value is
    // consumed on the straight-line path and the loads of the next state stay
    // in flight.  Stores come last: no load is waited for after a store.
    auto proc = [&](int s, int p, const In &x) {
        EwRec r;
        if constexpr (CSC)
            r = ew_record_csc(x.vi, x.ti, x.vj, x.tj, gb.x, gb.y, grbr.x, grbr.y);
        else
            r = ew_record(x.vi, x.ti, x.vj, x.tj, gb.x, gb.y);
        s_ab[p][0][k] = r.a;
        s_ab[p][1][k] = r.b;
        if constexpr (WITH_J) {
            if constexpr (PAR) {
                s_rem[p][0][k] = r.o[0];
                s_rem[p][1][k] = r.o[1];
                s_rem[p][2][k] = r.o[2];
                s_rem[p][3][k] = r.o[3];
            } else {
                s_J[p][o11] = r.o[0];
                s_J[p][o12] = r.o[1];
                s_J[p][kQ<NS> + o11] = r.o[2];
                s_J[p][kQ<NS> + o12] = r.o[3];
            }
        }
        lds_barrier();
        double as, bs;
        row_sum2(s_ab[p][0], s_ab[p][1], ra, rz, as, bs);
        const EwRow o = ew_row(x.vr, dA, dC, as, bs);
        if constexpr (WITH_J) {
            s_J[p][d11] = o.j11;
            s_J[p][d12] = CSC ? o.j21 : o.j12;
            s_J[p][kQ<NS> + d11] = CSC ? o.j12 : o.j21;
            s_J[p][kQ<NS> + d12] = o.j22;
            if constexpr (PAR) {  // the first record of a slot sums the slot, in record order
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int q = k; q < k + run; ++q) {
                    a0 += s_rem[p][0][q];
                    a1 += s_rem[p][1][q];
                    a2 += s_rem[p][2][q];
                    a3 += s_rem[p][3][q];
                }
                s_J[p][o11] = a0;
                s_J[p][o12] = a1;
                s_J[p][kQ<NS> + o11] = a2;
                s_J[p][kQ<NS> + o12] = a3;
            }
        }
        if (P && rowt) {
            st_row<PLAIN>(P + (size_t)s * nb + ir, o.p);
            st_row<PLAIN>(Q + (size_t)s * nb + ir, o.q);
        }
        if constexpr (WITH_J) {
            lds_barrier();
            write_jrows<NT, NS>(c, s_J[p], J + (size_t)s * (size_t)g.nnz_j);
        }
    };
    pipelined_states<In, ONE>(sb, se, first, load, proc);
}

// PLAIN: plain stores for the rows of P and Q (see st_row).  The
// injections of several states per workgroup are held to 80 registers
// (their natural count is a few above), so that six waves fit per SIMD
// instead of five.
template <int NT, bool PAR, bool WITH_J, bool ONE, bool PLAIN = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((!ONE && !WITH_J) ? 6 : 1, 8)))
    k_ew(DevGrid g, int nstate, int spb, int nchunk, int order, const double *__restrict__ vm, const double *__restrict__ va,
         double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    ew_eval<NT, PAR, WITH_J, ONE, false, PLAIN>(g, nstate, spb, nchunk, order, vm, va, P, Q, J);
}

// Injections and J values in CSC order.
template <int NT, bool PAR, bool ONE>
__global__ void __launch_bounds__(NT)
    k_ew_csc(DevGrid g, int nstate, int spb, int nchunk, int order, const double *__restrict__ vm,
             const double *__restrict__ va, double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    ew_eval<NT, PAR, true, ONE, true, false>(g, nstate, spb, nchunk, order, vm, va, P, Q, J);
}

// ===================================================================
// Stored phasors (Section IV.B.1 step 1): V = v e^{j theta}, U = e^{j theta}
// for n = nstate * nb (state, bus) entries.  PH_SPLIT: four planes of n
// doubles [Re V | Im V | Re U | Im U]; PH_INTERLEAVED: n pairs {Re V, Im V}
// followed by n pairs {Re U, Im U} (PH_* in pf_internal.h).

template <int PH>
__global__ void k_phasor(int64_t n, const double *__restrict__ vm, const double *__restrict__ va, double *__restrict__ ph) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sn, cs;
    sincos_dev(va[i], &sn, &cs);
    const double v = vm[i];
    if constexpr (PH == PH_SPLIT) {
        st_out(ph + i, v * cs);
        st_out(ph + n + i, v * sn);
        st_out(ph + 2 * n + i, cs);
        st_out(ph + 3 * n + i, sn);
    } else {
        dvec2 *p2 = reinterpret_cast<dvec2 *>(ph);
        st_out2(p2 + i, dvec2{v * cs, v * sn});
        st_out2(p2 + n + i, dvec2{cs, sn});
    }
}

// Per-state inputs of one Ybus nonzero: (v, theta) for PH_FLY, else the
// stored V (and U when the Jacobian needs it).
struct YbIn {
    double a, b, c, d;
};

template <int PH, bool WANT_U>
__device__ __forceinline__ void yb_load(const double *vm, const double *va, const double *ph, size_t n, size_t idx,
                                        YbIn &x) {
    if constexpr (PH == PH_FLY) {
        x.a = vm[idx];
        x.b = va[idx];
    } else if constexpr (PH == PH_SPLIT) {
        x.a = ph[idx];
        x.b = ph[n + idx];
        if constexpr (WANT_U) {
            x.c = ph[2 * n + idx];
            x.d = ph[3 * n + idx];
        } else {
            x.c = x.d = 0.0;
        }
    } else {
        const double2 *p2 = reinterpret_cast<const double2 *>(ph);
        const double2 v = p2[idx];
        x.a = v.x;
        x.b = v.y;
        if constexpr (WANT_U) {
            const double2 u = p2[n + idx];
            x.c = u.x;
            x.d = u.y;
        } else {
            x.c = x.d = 0.0;
        }
    }
}

// V and U of loaded inputs.
template <int PH>
__device__ __forceinline__ void yb_phasor(const YbIn &x, Cx &V, Cx &U) {
    if constexpr (PH == PH_FLY) {
        double sn, cs;
        sincos_dev(x.b, &sn, &cs);
        U = {cs, sn};
        V = {x.a * cs, x.a * sn};
    } else {
        V = {x.a, x.b};
        U = {x.c, x.d};
    }
}

// ===================================================================
// Ybus method: I = Ybus V, S = V conj(I) (eq. (1)) and, with WITH_J, the
// two-pass Jacobian of eqs. (3)-(4) done row-wise on the CSR matrix:
// pass 1 forms Y_ij V_j and the row sums I_i, pass 2 turns each nonzero into
//   dS_i/dtheta_j = j V_i (delta_ij conj(I_i) - conj(Y_ij V_j))
//   dS_i/dv_j     = V_i conj(Y_ij U_j) + delta_ij conj(I_i) U_i
// and writes the four real parts in place into J (Section IV.B.3).
// With PH = PH_FLY, U = e^{j theta} and V = v U are formed on the fly from
// (vm, va); the stored-phasor variants (Section V.A.1, Table I) read V and U
// written beforehand by k_phasor, either as separate real / imaginary planes
// (PH_SPLIT) or as interleaved {re, im} pairs (PH_INTERLEAVED).  k_phasor
// computes the same products as the on-the-fly path, so all three give
// bit-identical results.  A row's own V_i and U_i reach the other threads of
// the row through LDS.
// The single-state instantiation is held to 6 waves per SIMD (<= 80 VGPRs),
// so a 100k-bus grid's workgroups are all resident at once.
//
// CSC = true (WITH_J, phasors on the fly) writes J in column-major order,
// as k_ew_csc does: the nonzero (i, j) of row i receives the partials of
// S_j with respect to bus i's angle and magnitude,
//   dS_j/dtheta_i = j V_j (-conj(Y_ji V_i)),  dS_j/dv_i = V_j conj(Y_ji U_i),
// from the transposed entry Y_ji, with the products rounded as the CSR
// evaluation of row j rounds them (CSC values = CSR values transposed, bit
// for bit), and the diagonal entries dQ_i/dtheta_i and dP_i/dv_i trade
// places.
template <int NT, bool WITH_J, bool ONE, int PH, bool CSC>
__device__ __forceinline__ void yb_eval(const DevGrid &g, int nstate, int spb, int nchunk, int order,
                                        const double *__restrict__ vm, const double *__restrict__ va,
                                        const double *__restrict__ ph, double *__restrict__ P,
                                        double *__restrict__ Q, double *__restrict__ J) {
    static_assert(!CSC || (WITH_J && PH == PH_FLY), "the CSC order concerns J values");
    constexpr int NBUF = ONE ? 1 : 2;
    __shared__ double s_yv[NBUF][2][NT];  // Y_ij V_j
    __shared__ double s_vu[NBUF][4][NT];  // per row: V_i, U_i (re, im)
    __shared__ double s_yd[WITH_J ? 2 : 1][WITH_J ? NT : 1];  // per row: Y_ii (state-free, written once)
    __shared__ __align__(16) double s_J[NBUF][WITH_J ? kJStage<NT> : 2];

    int t, c0;
    if (!work_item(g.nytiles, nchunk, order, t, c0)) return;
    const int sb = c0 * spb;
    const int se = min(nstate, sb + spb);
    const int k = threadIdx.x;
    const size_t lane = (size_t)t * NT + k;
    const int j = g.ylane_j[lane];
    const int pk = g.ylane_pk[lane];
    const double2 yl = g.ylane_y[lane];
    double2 ylt = make_double2(0.0, 0.0);
    if constexpr (CSC) ylt = g.ylane_yt[lane];
    const Tile c = g.ytiles[t];
    const size_t nb = (size_t)g.nb;

    if (c.ns > NT) {
        // ---- one long row: pass 1 sums I_i in pieces of NT nonzeros (chunk sums in parallel,
        // folded in row_sum2's order by one thread, each piece's fold overlapping the next piece's
        // chunk sums), pass 2 writes J.
        __shared__ double s_cs[2][2][NT / kSumChunk];  // chunk sums of the last two pieces, by piece parity
        constexpr int FT = NT >= 128 ? 64 : 0;  // the folding thread, off wave 0 when the tile has two waves
        const int i = c.r0;
        const int d = c.ns;
        const size_t n = (size_t)nstate * nb;
        for (int s = sb; s < se; ++s) {
            const size_t so = (size_t)s * nb;
            Cx I = {0.0, 0.0};
            for (int base = 0; base < d; base += NT) {
                const int m = min(NT, d - base);
                if (k < m) {
                    const int p = c.s0 + base + k;
                    const int jc = g.ycol[p];
                    YbIn x;
                    yb_load<PH, false>(vm, va, ph, n, so + jc, x);
                    Cx Vj, Uj;
                    yb_phasor<PH>(x, Vj, Uj);
                    const Cx yv = cmul({g.yre[p], g.yim[p]}, Vj);
                    s_yv[0][0][k] = yv.re;
                    s_yv[0][1][k] = yv.im;
                }
                const int pc = base / NT;  // piece
                lds_barrier();
                chunk_sums(s_yv[0][0], s_yv[0][1], m, s_cs[pc & 1][0], s_cs[pc & 1][1]);
                if (k == FT && pc > 0)  // the previous (full) piece's chunk sums, while this piece's are summed
                    fold_chunks(s_cs[(pc + 1) & 1][0], s_cs[(pc + 1) & 1][1], NT, pc == 1, I.re, I.im);
                lds_barrier();
                if (k == FT && base + NT >= d) {  // the last piece: its own chunk sums, then I_i for every thread
                    fold_chunks(s_cs[pc & 1][0], s_cs[pc & 1][1], m, false, I.re, I.im);
                    s_vu[0][0][0] = I.re;
                    s_vu[0][1][0] = I.im;
                }
            }
            lds_barrier();
            YbIn xi;
            yb_load<PH, true>(vm, va, ph, n, so + i, xi);
            Cx Vi, Ui;
            yb_phasor<PH>(xi, Vi, Ui);
            const Cx Ic = {s_vu[0][0][0], -s_vu[0][1][0]};  // conj(I_i)
            if (k == 0 && P) {
                const Cx S = cmul(Vi, Ic);
                st_out(P + (size_t)s * nb + i, S.re);
                st_out(Q + (size_t)s * nb + i, S.im);
            }
            if constexpr (WITH_J) {
                double *Js = J + (size_t)s * (size_t)g.nnz_j;
                for (int lp = k; lp < d; lp += NT) {
                    const int p = c.s0 + lp;
                    const int jc = g.ycol[p];
                    YbIn xj;
                    yb_load<PH, true>(vm, va, ph, n, so + jc, xj);
                    Cx Vj, Uj;
                    yb_phasor<PH>(xj, Vj, Uj);
                    const Cx Y = {g.yre[p], g.yim[p]};
                    const Cx yv = cmul(Y, Vj);
                    const bool dg = jc == i;
                    const Cx x = {(dg ? Ic.re : 0.0) - yv.re, (dg ? Ic.im : 0.0) + yv.im};  // delta conj(I) - conj(YV)
                    const Cx dst = cmul({-Vi.im, Vi.re}, x);                                  // j V_i x
                    Cx dsv = cmul(Vi, cconj(cmul(Y, Uj)));
                    if (dg) dsv = cadd(dsv, cmul(Ic, Ui));
                    if constexpr (CSC) {
                        double a0 = dst.re, a1 = dst.im, a2 = dsv.re, a3 = dsv.im;  // the diagonal
                        if (!dg) {  // partials of S_jc with respect to bus i, from Y_(jc, i)
                            const int pt = g.yt_slot[p];
                            const Cx YT = {g.yre[pt], g.yim[pt]};
                            const Cx yt = cmul(YT, Vi);
                            const Cx so = cmul({-Vj.im, Vj.re}, {-yt.re, yt.im});
                            const Cx vo = cmul(Vj, cconj(cmul(YT, Ui)));
                            a0 = so.re;
                            a1 = so.im;
                            a2 = vo.re;
                            a3 = vo.im;
                        }
                        st_out(Js + c.jp + lp, a0);
                        st_out(Js + c.jp + d + lp, a1);
                        st_out(Js + c.jq + lp, a2);
                        st_out(Js + c.jq + d + lp, a3);
                    } else {
                        st_out(Js + c.jp + lp, dst.re);
                        st_out(Js + c.jp + d + lp, dsv.re);
                        st_out(Js + c.jq + lp, dst.im);
                        st_out(Js + c.jq + d + lp, dsv.im);
                    }
                }
            }
            lds_barrier();
        }
        return;
    }

    // ---- packed tile: lane k holds nonzero c.s0 + k (inert past c.ns) with
    // its column bus, tile row, diagonal flag and LDS targets (the pad for
    // the diagonal nonzero, whose entries the row thread writes).
    const int row = yb_row(pk);
    const bool diag = yb_diag(pk);
    const int o11 = ew_o11(pk), o12 = ew_o12(pk);
    const Cx Y = {yl.x, yl.y};
    if constexpr (WITH_J) {
        if (diag) {  // the row's Ybus diagonal, for its diagonal J entries (ordered by the first barrier)
            s_yd[0][row] = Y.re;
            s_yd[1][row] = Y.im;
        }
    }
    const bool rowt = k < c.nrows;
    const int ir = c.r0 + (rowt ? k : 0);
    const size_t n = (size_t)nstate * nb;
    using In = YbIn;
    auto load = [&](int s, In &x) { yb_load<PH, WITH_J>(vm, va, ph, n, (size_t)s * nb + j, x); };
    In first;  // first state's gathers before the row loads, as in k_ew
    load(sb, first);
    const int irr = rowt ? ir : g.nb;
    const int2 rw = g.row_yb[irr];
    const int ra = lo16(rw.x), rz = hi16(rw.x), dd11 = ra + rw.y, dd12 = rz + rw.y;
    // As in k_ew: every lane computes, only stores depend on the lane's role
    // (inert lanes have Y = 0 and a valid bus).
    auto proc = [&](int s, int p, const In &x) {
        Cx Vj, Uj;
        yb_phasor<PH>(x, Vj, Uj);
        const Cx yv = cmul(Y, Vj);
        s_yv[p][0][k] = yv.re;
        s_yv[p][1][k] = yv.im;
        if (diag) {  // the diagonal nonzero carries the row's own phasor
            s_vu[p][0][row] = Vj.re;
            s_vu[p][1][row] = Vj.im;
            if constexpr (WITH_J || PH == PH_FLY) {
                s_vu[p][2][row] = Uj.re;
                s_vu[p][3][row] = Uj.im;
            }
        }
        lds_barrier();
        Cx I;
        row_sum2(s_yv[p][0], s_yv[p][1], ra, rz, I.re, I.im);
        const int kr = rowt ? k : 0;
        const Cx Vk = {s_vu[p][0][kr], s_vu[p][1][kr]};
        const Cx Ic = {I.re, -I.im};
        const Cx S = cmul(Vk, Ic);
        if constexpr (WITH_J) {
            // diagonal entry of row k (Y_ii V_i recomputed from Y_ii and V_i)
            const Cx Ui = {s_vu[p][2][kr], s_vu[p][3][kr]};
            const Cx Yd = {s_yd[0][kr], s_yd[1][kr]};
            const Cx yu = cmul(Yd, Ui);
            const Cx yvi = cmul(Yd, Vk);
            const Cx x2 = {Ic.re - yvi.re, Ic.im + yvi.im};
            const Cx dst = cmul({-Vk.im, Vk.re}, x2);
            const Cx dsv = cadd(cmul(Vk, cconj(yu)), cmul(Ic, Ui));
            s_J[p][dd11] = dst.re;
            s_J[p][dd12] = CSC ? dst.im : dsv.re;
            s_J[p][kQ<NT> + dd11] = CSC ? dsv.re : dst.im;
            s_J[p][kQ<NT> + dd12] = dsv.im;
            // off-diagonal entry of this nonzero
            const Cx Vi = {s_vu[p][0][row], s_vu[p][1][row]};
            if constexpr (CSC) {
                const Cx Uo = {s_vu[p][2][row], s_vu[p][3][row]};
                const Cx YT = {ylt.x, ylt.y};
                const Cx yt = cmul(YT, Vi);
                const Cx so = cmul({-Vj.im, Vj.re}, {-yt.re, yt.im});  // j V_j (-conj(Y_ji V_i))
                const Cx vo = cmul(Vj, cconj(cmul(YT, Uo)));
                s_J[p][o11] = so.re;
                s_J[p][o12] = so.im;
                s_J[p][kQ<NT> + o11] = vo.re;
                s_J[p][kQ<NT> + o12] = vo.im;
            } else {
                const Cx dso = cmul({-Vi.im, Vi.re}, {-yv.re, yv.im});  // j V_i (-conj(Y_ij V_j))
                const Cx dvo = cmul(Vi, cconj(cmul(Y, Uj)));
                s_J[p][o11] = dso.re;
                s_J[p][o12] = dvo.re;
                s_J[p][kQ<NT> + o11] = dso.im;
                s_J[p][kQ<NT> + o12] = dvo.im;
            }
        }
        if (P && rowt) {  // stores last (see k_ew)
            st_out(P + (size_t)s * nb + ir, S.re);
            st_out(Q + (size_t)s * nb + ir, S.im);
        }
        if constexpr (WITH_J) {
            lds_barrier();
            write_jrows<NT, NT>(c, s_J[p], J + (size_t)s * (size_t)g.nnz_j);
        }
    };
    pipelined_states<In, ONE>(sb, se, first, load, proc);
}

template <int NT, bool WITH_J, bool ONE, int PH>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ONE ? 6 : 1, 8)))
    k_ybus(DevGrid g, int nstate, int spb, int nchunk, int order, const double *__restrict__ vm, const double *__restrict__ va,
           const double *__restrict__ ph, double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    yb_eval<NT, WITH_J, ONE, PH, false>(g, nstate, spb, nchunk, order, vm, va, ph, P, Q, J);
}

// Injections and J values in CSC order by the Ybus method.
template <int NT, bool ONE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ONE ? 6 : 1, 8)))
    k_ybus_csc(DevGrid g, int nstate, int spb, int nchunk, int order, const double *__restrict__ vm,
               const double *__restrict__ va, double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    yb_eval<NT, true, ONE, PH_FLY, true>(g, nstate, spb, nchunk, order, vm, va, nullptr, P, Q, J);
}

// ===================================================================
// Adjoint of the element-wise injections.  Column i of J collects the own
// partials of every record at bus i (rows P_i, Q_i) and the remote partials
// of the opposite end of each incident branch (rows P_j, Q_j).  Record e (at
// i, towards j) therefore contributes to bus i
//   g_va += v_i v_j (lQ_i alpha - lP_i beta + lP_j beta' - lQ_j alpha')
//   g_vm += v_j (lP_i alpha + lQ_i beta + lP_j alpha' + lQ_j beta')
// where alpha', beta' use the other end's coupling (Gr, Br) at angle -t:
//   alpha' = Gr cos t - Br sin t,  beta' = -Gr sin t - Br cos t,
// and the own-end terms add 2 v_i (lP_i dA_i - lQ_i dC_i) to g_vm once per
// bus.  Sums per bus run in record order; J is never formed.
struct VjpIn {
    double vi, ti, vj, tj, lpi, lqi, lpj, lqj;
};

__device__ __forceinline__ void vjp_record(const VjpIn &x, double G, double B, double Gr, double Br, double &ga,
                                           double &gv) {
    double sn, cs;
    sincos_dev(x.ti - x.tj, &sn, &cs);
    const double al = fma(G, cs, B * sn), be = fma(G, sn, -(B * cs));
    const double al2 = fma(Gr, cs, -(Br * sn)), be2 = fma(-Gr, sn, -(Br * cs));
    const double ta = fma(-x.lqj, al2, fma(x.lpj, be2, fma(-x.lpi, be, x.lqi * al)));
    const double tv = fma(x.lqj, be2, fma(x.lpj, al2, fma(x.lqi, be, x.lpi * al)));
    ga = (x.vi * x.vj) * ta;
    gv = x.vj * tv;
}

// g_vm of bus i: the record sum plus the own-end term 2 v_i (lP_i dA_i - lQ_i dC_i).
__device__ __forceinline__ double vjp_own(double sum, double vi, double lpi, double lqi, double dA, double dC) {
    return fma(2.0 * vi, fma(lpi, dA, -(lqi * dC)), sum);
}

// PLAIN: plain stores for the gradient rows (see st_row).
template <int NT, bool ONE, bool PLAIN = false>
__global__ void __launch_bounds__(NT)
    k_ew_vjp(DevGrid g, int nstate, int spb, int nchunk, int order, const double *__restrict__ vm,
             const double *__restrict__ va, const double *__restrict__ lp, const double *__restrict__ lq,
             double *__restrict__ gvm, double *__restrict__ gva) {
    __shared__ double s_val[ONE ? 1 : 2][2][NT];

    int t, c0;
    if (!work_item(g.ntiles, nchunk, order, t, c0)) return;
    const int sb = c0 * spb;
    const int se = min(nstate, sb + spb);
    const int k = threadIdx.x;
    const size_t lane = (size_t)t * NT + k;
    const int j = g.lane_j[lane];
    const int rowl = ew_row(g.lane_pk[lane]);
    const double2 gb = g.lane_gb[lane], grb = g.lane_grbr[lane];
    const Tile c = tile_of(g, t);
    const size_t nb = (size_t)g.nb;

    auto fetch = [&](size_t so, int i, int jj) {
        VjpIn x;
        x.vi = vm[so + i];
        x.ti = va[so + i];
        x.vj = vm[so + jj];
        x.tj = va[so + jj];
        x.lpi = lp[so + i];
        x.lqi = lq[so + i];
        x.lpj = lp[so + jj];
        x.lqj = lq[so + jj];
        return x;
    };

    if (c.ne > NT) {
        // one row with more than NT branch ends, in pieces of NT branch ends
        // (the bus-shunt record, position c.sh, contributes nothing and is
        // skipped); chunk sums in parallel, folded in row_sum2's order by one
        // thread, each piece's fold beside the next piece's chunk sums.  The
        // remote bus of the next (state, piece) item is loaded one item
        // ahead, so each item's gathers go out at once.
        __shared__ double s_cs[2][2][NT / kSumChunk];  // chunk sums of the last two pieces, by piece parity
        constexpr int FT = NT >= 128 ? 64 : 0;  // the folding thread, off wave 0 when the tile has two waves
        __shared__ double s_rs[4];  // the folding thread's running sums of the current state; dA, dC of the row
        const int i = c.r0;
        const int npc = (c.ne + NT - 1) / NT;  // pieces per state
        const int nit = (se - sb) * npc;
        // lanes past the piece end repeat its last record (values unused)
        auto rec_of = [&](int it) {
            const int base = (it % npc) * NT;
            const int pos = base + min(k, min(NT, c.ne - base) - 1);
            return c.i0 + pos + (pos >= c.sh ? 1 : 0);
        };
        int jn = g.nbr[rec_of(0)];
        if (k == 0) {
            s_rs[2] = g.dA[i];
            s_rs[3] = g.dC[i];
        }
        for (int it = 0; it < nit; ++it) {
            const int s = sb + it / npc, piece = it % npc;
            const int m = min(NT, c.ne - piece * NT);
            const int e = rec_of(it);
            const VjpIn x = fetch((size_t)s * nb, i, jn);
            const double G = g.G[e], B = g.B[e], Gr = g.Gr[e], Br = g.Br[e];
            jn = g.nbr[rec_of(min(it + 1, nit - 1))];
            if (k < m) {
                double ga, gv;
                vjp_record(x, G, B, Gr, Br, ga, gv);
                s_val[0][0][k] = ga;
                s_val[0][1][k] = gv;
            }
            lds_barrier();
            chunk_sums(s_val[0][0], s_val[0][1], m, s_cs[piece & 1][0], s_cs[piece & 1][1]);
            if (k == FT && piece > 0) {  // the previous (full) piece's chunk sums, while this piece's are summed
                double acc_a = s_rs[0], acc_v = s_rs[1];
                fold_chunks(s_cs[(piece + 1) & 1][0], s_cs[(piece + 1) & 1][1], NT, piece == 1, acc_a, acc_v);
                s_rs[0] = acc_a;
                s_rs[1] = acc_v;
            }
            lds_barrier();
            if (k == FT && piece == npc - 1) {  // the state's last piece: its own chunk sums, then the gradients
                double acc_a = s_rs[0], acc_v = s_rs[1];
                fold_chunks(s_cs[piece & 1][0], s_cs[piece & 1][1], m, false, acc_a, acc_v);
                {
                    const size_t so = (size_t)s * nb;
                    st_out(gva + so + i, acc_a);
                    st_out(gvm + so + i, vjp_own(acc_v, x.vi, x.lpi, x.lqi, s_rs[2], s_rs[3]));
                }
            }
        }
        return;
    }

    // ---- packed tile (lane tables as in k_ew); row threads hand their bus's
    // values to the row's lanes through LDS
    __shared__ double s_own[ONE ? 1 : 2][4][NT];
    const bool rowt = k < c.nrows;
    const int ir = c.r0 + (rowt ? k : 0);
    struct In {
        double vj, tj, lpj, lqj, vr, tr, lpr, lqr;
    };
    // Only waves that hold a row load the row values (uniform per wave, so
    // the other waves skip four loads per state; their values are unused).
    const bool anyrow = (k & ~63) < c.nrows;
    // The row values go out first: waiting for them (before the barrier of
    // the state ahead, below) then leaves the remote gathers in flight.
    auto load = [&](int s, In &in) {
        const size_t so = (size_t)s * nb;
        if (anyrow) {
            in.vr = vm[so + ir];
            in.tr = va[so + ir];
            in.lpr = lp[so + ir];
            in.lqr = lq[so + ir];
        } else {
            in.vr = in.tr = in.lpr = in.lqr = 0.0;
        }
        in.vj = vm[so + j];
        in.tj = va[so + j];
        in.lpj = lp[so + j];
        in.lqj = lq[so + j];
    };
    In first;
    load(sb, first);
    const int irr = rowt ? ir : g.nb;
    const int2 rw = g.row_ew[irr];
    const double dA = g.dA[irr], dC = g.dC[irr];
    const int ra = lo16(rw.x), rz = hi16(rw.x);
    // A state's own-bus values reach its lanes through LDS buffer p (the
    // state's parity).  With several states per workgroup the row threads
    // write the next state's values into the other buffer before this
    // state's barrier, so each state takes one barrier.  Buffer p of either
    // array is rewritten only after the barrier that follows its last read.
    auto put_own = [&](int p, const In &in) {
        if (rowt) {
            s_own[p][0][k] = in.vr;
            s_own[p][1][k] = in.tr;
            s_own[p][2][k] = in.lpr;
            s_own[p][3][k] = in.lqr;
        }
    };
    auto record = [&](int p, const In &in) {
        VjpIn x;
        x.vi = s_own[p][0][rowl];
        x.ti = s_own[p][1][rowl];
        x.lpi = s_own[p][2][rowl];
        x.lqi = s_own[p][3][rowl];
        x.vj = in.vj;
        x.tj = in.tj;
        x.lpj = in.lpj;
        x.lqj = in.lqj;
        double ga, gv;
        vjp_record(x, gb.x, gb.y, grb.x, grb.y, ga, gv);
        s_val[p][0][k] = ga;
        s_val[p][1][k] = gv;
    };
    auto finish = [&](int s, int p, const In &in) {
        double a, v;
        row_sum2(s_val[p][0], s_val[p][1], ra, rz, a, v);
        const double gm = vjp_own(v, in.vr, in.lpr, in.lqr, dA, dC);
        if (rowt) {
            const size_t so = (size_t)s * nb;
            st_row<PLAIN>(gva + so + ir, a);
            st_row<PLAIN>(gvm + so + ir, gm);
        }
    };
    put_own(0, first);
    lds_barrier();
    if constexpr (ONE) {
        record(0, first);
        lds_barrier();
        finish(sb, 0, first);
    } else {
        // two states per trip, the next state's loads in flight while a
        // state is evaluated; an odd count repeats the last state
        In rb{};
        for (int s = sb; s < se; s += 2) {
            const int s1 = min(s + 1, se - 1);
            load(s1, rb);
            record(0, first);
            put_own(1, rb);
            lds_barrier();
            finish(s, 0, first);
            load(min(s + 2, se - 1), first);
            record(1, rb);
            put_own(0, first);
            lds_barrier();
            finish(s1, 1, rb);
        }
    }
}

// ===================================================================
// Setup: record coupling admittances from the branch parameters.
__device__ __forceinline__ void branch_admittances(const DevSetup &s, int l, double &gsr, double &bsr, double &m,
                                                   double &bh, double &sp, double &cp) {
    const double r = s.r[l], x = s.x[l];
    const double den = r * r + x * x;
    gsr = r / den;  // y_hk = 1/(r + jx)
    bsr = -x / den;
    m = s.tap[l] == 0.0 ? 1.0 : s.tap[l];
    bh = 0.5 * s.b[l];
    sincos_dev(s.shift[l], &sp, &cp);
}

__global__ void k_items_init(DevSetup s) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= s.nitems) return;
    const int br = s.item_br[e];
    if (br < 0) {  // bus shunt record: no coupling
        s.G[e] = 0.0;
        s.B[e] = 0.0;
        s.Gr[e] = 0.0;
        s.Br[e] = 0.0;
        return;
    }
    double gsr, bsr, m, bh, sp, cp;
    branch_admittances(s, br >> 1, gsr, bsr, m, bh, sp, cp);
    // -y_hk e^{+j phi}/m (from end) and -y_hk e^{-j phi}/m (to end)
    const double gf = -(gsr * cp - bsr * sp) / m, bf = -(gsr * sp + bsr * cp) / m;
    const double gt = -(gsr * cp + bsr * sp) / m, bt = -(bsr * cp - gsr * sp) / m;
    const bool to_end = (br & 1) != 0;
    s.G[e] = to_end ? gt : gf;
    s.B[e] = to_end ? bt : bf;
    s.Gr[e] = to_end ? gf : gt;
    s.Br[e] = to_end ? bf : bt;
}

// Setup: per bus, the sum in record order of the own-end admittances
// ((y_h + y_hk)/m^2 at a from end, y_k + y_hk at a to end) and the shunt.
__global__ void k_bus_diag(DevSetup s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > s.nb) return;
    if (i == s.nb) {  // the inert entry read by lanes without a row
        s.dA[i] = 0.0;
        s.dC[i] = 0.0;
        return;
    }
    double re = 0.0, im = 0.0;
    for (int e = s.irow[i]; e < s.irow[i + 1]; ++e) {
        const int br = s.item_br[e];
        if (br < 0) {
            re += s.gs[i];
            im += s.bs[i];
            continue;
        }
        double gsr, bsr, m, bh, sp, cp;
        branch_admittances(s, br >> 1, gsr, bsr, m, bh, sp, cp);
        const double f = (br & 1) ? 1.0 : 1.0 / (m * m);
        re += gsr * f;
        im += (bsr + bh) * f;
    }
    s.dA[i] = re;
    s.dC[i] = im;
}

// Setup: Ybus values.  The diagonal is the bus constant above; an
// off-diagonal slot sums the coupling admittances of its records (more than
// one for parallel branches) in record order.
__global__ void k_ybus_assemble(DevSetup s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.nnz_y) return;
    const int i = s.slot_row[p];
    double re = 0.0, im = 0.0;
    if (s.ycol[p] == i) {
        re = s.dA[i];
        im = s.dC[i];
    } else {
        for (int e = s.slot_item[p]; e < s.slot_item[p + 1]; ++e) {
            re += s.G[e];
            im += s.B[e];
        }
    }
    s.yre[p] = re;
    s.yim[p] = im;
}

// ===================================================================
// Two-phase element-wise evaluation (see DevTwoPhase).  Per branch end at
// bus i with remote bus j, with the series admittance g_s + j b_s = 1/(r + jx),
// tap m and shift phi on the from side, eqs. (5)-(6) in real form read
//   d = theta_i - theta_j - phi_e,  w = v_i v_j,
//   alpha = G cos d + B sin d,  beta = G sin d - B cos d,  G = g_s/m, B = b_s/m,
//   P = v_i^2 A - w alpha,  Q = -v_i^2 C - w beta,
// with A = g_s/m^2, C = (b/2 + b_s)/m^2, phi_e = phi at the from end and
// A = g_s, C = b/2 + b_s, phi_e = -phi at the to end; the partials follow from
// d alpha/d d = -beta and d beta/d d = alpha.
// P, Q of one branch end and its partials with respect to the end's own
// bus i and the remote bus j.
struct EndVals {
    double p, q, dpti, dpvi, dqti, dqvi, dptj, dpvj, dqtj, dqvj;
};

__device__ __forceinline__ EndVals branch_end(double vi, double vj, double d, double A, double C, double G, double B) {
    double sn, cs;
    sincos_dev(d, &sn, &cs);
    const double al = fma(G, cs, B * sn), be = fma(G, sn, -(B * cs));
    const double w = vi * vj;
    EndVals o;
    o.p = fma(vi * vi, A, -(w * al));
    o.q = fma(-(vi * vi), C, -(w * be));
    o.dpti = w * be;
    o.dpvi = fma(2.0 * vi, A, -(vj * al));
    o.dqti = -(w * al);
    o.dqvi = fma(-2.0 * vi, C, -(vj * be));
    o.dptj = -(w * be);
    o.dpvj = -(vi * al);
    o.dqtj = w * al;
    o.dqvj = -(vi * be);
    return o;
}

// The constants of branch l's two ends from its parameters (r, x, b, tap,
// shift): coupling G + jB = y_hk / m and the own-end terms A + jC of the
// from end ((y_h + y_hk)/m^2) and of the to end (y_k + y_hk), with
// y_hk = 1/(r + jx) and y_h = y_k = jb/2.
struct BranchConsts {
    double G, B, Af, Cf, At, Ct;
};

__device__ __forceinline__ BranchConsts branch_consts(double r, double x, double b, double tap) {
    const double den = fma(r, r, x * x);
    const double gsr = r / den, bsr = -x / den;
    const double m = tap == 0.0 ? 1.0 : tap;
    const double bh = 0.5 * b;
    return {gsr / m, bsr / m, gsr / (m * m), (bh + bsr) / (m * m), gsr, bh + bsr};
}

// Precomputed branch constants, [6][nl]: the planes of BranchConsts (the
// paper's precomputation of the per-branch constants, Section IV.C.1).
__global__ void k_branch_consts(DevTwoPhase d, double *__restrict__ bc) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.nl) return;
    const BranchConsts c = branch_consts(d.r[l], d.x[l], d.b[l], d.tap[l]);
    const size_t n = (size_t)d.nl;
    bc[0 * n + l] = c.G;
    bc[1 * n + l] = c.B;
    bc[2 * n + l] = c.Af;
    bc[3 * n + l] = c.Cf;
    bc[4 * n + l] = c.At;
    bc[5 * n + l] = c.Ct;
}

// Both ends of branch l (from end first) at one state.  PRE reads the
// precomputed constants (56 bytes per branch with the shift) instead of
// deriving them from the parameters (40 bytes); the values are the same.
template <bool PRE = false>
__device__ __forceinline__ void branch_ends(const DevTwoPhase &d, int l, const double *vm, const double *va,
                                            EndVals &f, EndVals &t) {
    const int h = d.br_from[l], k = d.br_to[l];
    BranchConsts c;
    if constexpr (PRE) {
        const size_t n = (size_t)d.nl;
        c = {d.bc[l], d.bc[n + l], d.bc[2 * n + l], d.bc[3 * n + l], d.bc[4 * n + l], d.bc[5 * n + l]};
    } else {
        c = branch_consts(d.r[l], d.x[l], d.b[l], d.tap[l]);
    }
    const double phi = d.shift[l];
    const double vh = vm[h], th = va[h], vk = vm[k], tk = va[k];
    f = branch_end(vh, vk, th - tk - phi, c.Af, c.Cf, c.G, c.B);
    t = branch_end(vk, vh, tk - th + phi, c.At, c.Ct, c.G, c.B);
}

// Plain stores: the reduction kernel reads the scratch right after, from cache.
__device__ __forceinline__ void tp_store(double *sc, int64_t stride, int e, const EndVals &o) {
    sc[0 * stride + e] = o.p;
    sc[1 * stride + e] = o.q;
    sc[2 * stride + e] = o.dpti;
    sc[3 * stride + e] = o.dpvi;
    sc[4 * stride + e] = o.dqti;
    sc[5 * stride + e] = o.dqvi;
    sc[6 * stride + e] = o.dptj;
    sc[7 * stride + e] = o.dpvj;
    sc[8 * stride + e] = o.dqtj;
    sc[9 * stride + e] = o.dqvj;
}

template <bool PRE>
__global__ void k_tp_branch(DevTwoPhase d, const double *__restrict__ vm, const double *__restrict__ va) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.nl) return;
    EndVals f, t;
    branch_ends<PRE>(d, l, vm, va, f, t);
    tp_store(d.scr, d.nrec, d.br_rec[2 * l], f);
    tp_store(d.scr, d.nrec, d.br_rec[2 * l + 1], t);
}

// Branch flows and (WITH_J) their 16 partials: one thread per (branch,
// state); every output array is written with consecutive branches in
// consecutive lanes.
template <bool WITH_J>
__global__ void k_flows(DevTwoPhase d, int nstate, const double *__restrict__ vm, const double *__restrict__ va,
                        double *__restrict__ pf, double *__restrict__ qf, double *__restrict__ pt,
                        double *__restrict__ qt, double *__restrict__ jac) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.nl) return;
    for (int s = blockIdx.y; s < nstate; s += gridDim.y) {
        const size_t sb = (size_t)s * d.nb, sl = (size_t)s * d.nl;
        EndVals f, t;
        branch_ends(d, l, vm + sb, va + sb, f, t);
        st_out(pf + sl + l, f.p);
        st_out(qf + sl + l, f.q);
        st_out(pt + sl + l, t.p);
        st_out(qt + sl + l, t.q);
        if constexpr (WITH_J) {
            // rows d(Pf, Qf, Pt, Qt) / d(theta_from, theta_to, v_from, v_to)
            const double v[16] = {f.dpti, f.dptj, f.dpvi, f.dpvj, f.dqti, f.dqtj, f.dqvi, f.dqvj,
                                  t.dptj, t.dpti, t.dpvj, t.dpvi, t.dqtj, t.dqti, t.dqvj, t.dqvi};
            double *js = jac + (size_t)s * 16 * d.nl;
#pragma unroll
            for (int q = 0; q < 16; ++q) st_out(js + (size_t)q * d.nl + l, v[q]);
        }
    }
}

__global__ void k_tp_reduce(DevTwoPhase d, const double *__restrict__ vm, double *__restrict__ P,
                            double *__restrict__ Q, double *__restrict__ J) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.nb) return;
    const int64_t st = d.nrec;
    const double *sc = d.scr;
    const double v = vm[i];
    const int y0 = d.yrow[i], deg = d.yrow[i + 1] - y0;
    const int64_t jp = d.jpq[i].x, jq = d.jpq[i].y;
    double p = 0.0, q = 0.0, o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int cur = -1;
    auto flush = [&]() {
        if (cur < 0) return;
        st_out(J + jp + cur, a0);
        st_out(J + jp + deg + cur, a1);
        st_out(J + jq + cur, a2);
        st_out(J + jq + deg + cur, a3);
    };
    for (int e = d.irow[i]; e < d.irow[i + 1]; ++e) {
        if (d.item_br[e] < 0) {  // the bus shunt, at its sorted place
            const double gg = d.gs[i], bb = d.bs[i];
            p = fma(v * v, gg, p);
            q = fma(-(v * v), bb, q);
            o1 = fma(2.0 * v, gg, o1);
            o3 = fma(-2.0 * v, bb, o3);
            continue;
        }
        p += sc[0 * st + e];
        q += sc[1 * st + e];
        o0 += sc[2 * st + e];
        o1 += sc[3 * st + e];
        o2 += sc[4 * st + e];
        o3 += sc[5 * st + e];
        const int ls = d.slot[e] - y0;
        if (ls != cur) {  // parallel branches share a slot and are adjacent
            flush();
            cur = ls;
            a0 = a1 = a2 = a3 = 0.0;
        }
        a0 += sc[6 * st + e];
        a1 += sc[7 * st + e];
        a2 += sc[8 * st + e];
        a3 += sc[9 * st + e];
    }
    flush();
    const int dp = d.ydslot[i] - y0;
    st_out(J + jp + dp, o0);
    st_out(J + jp + deg + dp, o1);
    st_out(J + jq + dp, o2);
    st_out(J + jq + deg + dp, o3);
    if (P) {
        st_out(P + i, p);
        st_out(Q + i, q);
    }
}

// ===================================================================
// Copy-add on the GPU: the reduction the paper calls copy-add (Section
// IV.C.2, the J elements added into the pre-built pattern), with atomic adds
// in place of its sequential adds.  The outputs are first set to the bus
// shunt terms (P, Q and the diagonal dP/dv, dQ/dv entries) and to zero (the
// rest of J); then one thread per branch adds both ends' power and eight
// partials into P, Q and the J slots.  The additions happen in no fixed
// order, so results match the other methods to rounding only.
__global__ void k_ca_zero(int64_t n2, double2 *__restrict__ J) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        st_out2(reinterpret_cast<dvec2 *>(J + i), dvec2{0.0, 0.0});
}

__global__ void k_ca_bus(DevTwoPhase d, int nstate, int64_t nnz_j, const double *__restrict__ vm,
                         double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.nb) return;
    const double gg = d.gs[i], bb = d.bs[i];
    const int y0 = d.yrow[i], deg = d.yrow[i + 1] - y0, dp = d.ydslot[i] - y0;
    const int64_t jp = d.jpq[i].x, jq = d.jpq[i].y;
    for (int s = blockIdx.y; s < nstate; s += gridDim.y) {
        const double v = vm[(size_t)s * d.nb + i];
        if (P) {
            st_out(P + (size_t)s * d.nb + i, (v * v) * gg);
            st_out(Q + (size_t)s * d.nb + i, -((v * v) * bb));
        }
        double *Js = J + (size_t)s * (size_t)nnz_j;
        st_out(Js + jp + deg + dp, (2.0 * v) * gg);
        st_out(Js + jq + deg + dp, -((2.0 * v) * bb));
    }
}

// Adds one branch end (record e at bus i) into P, Q and row i's J slots.
__device__ __forceinline__ void ca_add_end(const DevTwoPhase &d, int e, int i, const EndVals &o, double *P, double *Q,
                                           double *Js) {
    const int y0 = d.yrow[i], deg = d.yrow[i + 1] - y0;
    const int so = d.slot[e] - y0, dp = d.ydslot[i] - y0;
    const int64_t jp = d.jpq[i].x, jq = d.jpq[i].y;
    if (P) {
        unsafeAtomicAdd(P + i, o.p);
        unsafeAtomicAdd(Q + i, o.q);
    }
    unsafeAtomicAdd(Js + jp + dp, o.dpti);
    unsafeAtomicAdd(Js + jp + deg + dp, o.dpvi);
    unsafeAtomicAdd(Js + jq + dp, o.dqti);
    unsafeAtomicAdd(Js + jq + deg + dp, o.dqvi);
    unsafeAtomicAdd(Js + jp + so, o.dptj);
    unsafeAtomicAdd(Js + jp + deg + so, o.dpvj);
    unsafeAtomicAdd(Js + jq + so, o.dqtj);
    unsafeAtomicAdd(Js + jq + deg + so, o.dqvj);
}

template <bool PRE>
__global__ void k_ca_branch(DevTwoPhase d, int nstate, int64_t nnz_j, const double *__restrict__ vm,
                            const double *__restrict__ va, double *P, double *Q, double *J) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.nl) return;
    const int h = d.br_from[l], k = d.br_to[l];
    const int ef = d.br_rec[2 * l], et = d.br_rec[2 * l + 1];
    for (int s = blockIdx.y; s < nstate; s += gridDim.y) {
        const size_t sb = (size_t)s * d.nb;
        EndVals f, t;
        branch_ends<PRE>(d, l, vm + sb, va + sb, f, t);
        double *Js = J + (size_t)s * (size_t)nnz_j;
        ca_add_end(d, ef, h, f, P ? P + sb : nullptr, Q ? Q + sb : nullptr, Js);
        ca_add_end(d, et, k, t, P ? P + sb : nullptr, Q ? Q + sb : nullptr, Js);
    }
}

// Jacobian values into another pattern (Algorithm 2's in-place copy by
// precomputed indices): one thread per J entry reads its target position
// once and copies the entry of every state.  Positions outside the target
// are skipped, so a wrong map cannot write out of bounds.
__global__ void k_jscatter(int32_t nstate, int64_t nnz_j, const double *__restrict__ jval,
                           const int32_t *__restrict__ map, int64_t out_nnz, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz_j) return;
    const int32_t m = map[k];
    if (m < 0 || m >= out_nnz) return;
    for (int32_t s = blockIdx.y; s < nstate; s += gridDim.y)
        st_out(out + (size_t)s * (size_t)out_nnz + m, jval[(size_t)s * (size_t)nnz_j + k]);
}

// Lane values: copies of the record constants (element-wise) or Ybus values
// in lane order; inert lanes get zeros.
__global__ void k_lane_fill(DevLaneFill f, bool ew) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ew) {
        if (l >= f.nlanes) return;
        const int e = f.lane_rec[l];
        f.lane_gb[l] = e >= 0 ? make_double2(f.G[e], f.B[e]) : make_double2(0.0, 0.0);
        f.lane_grbr[l] = e >= 0 ? make_double2(f.Gr[e], f.Br[e]) : make_double2(0.0, 0.0);
    } else {
        if (l < f.nylanes) {
            const int q = f.ylane_slot[l], qt = f.ylane_tslot[l];
            f.ylane_y[l] = q >= 0 ? make_double2(f.yre[q], f.yim[q]) : make_double2(0.0, 0.0);
            f.ylane_yt[l] = qt >= 0 ? make_double2(f.yre[qt], f.yim[qt]) : make_double2(0.0, 0.0);
        }
    }
}

template <int NT, bool ONE, bool WITH_J>
void launch_ybus_ph(const DevGrid &g, const Launch &L, dim3 grid, dim3 block, int spb, int nchunk, hipStream_t st) {
    double *J = WITH_J ? L.jval : nullptr;
    switch (L.phasor) {
        case PH_SPLIT:
            hipLaunchKernelGGL((k_ybus<NT, WITH_J, ONE, PH_SPLIT>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order,
                               L.vm, L.va, L.ph, L.p, L.q, J);
            break;
        case PH_INTERLEAVED:
            hipLaunchKernelGGL((k_ybus<NT, WITH_J, ONE, PH_INTERLEAVED>), grid, block, 0, st, g, L.nstate, spb, nchunk,
                               L.order, L.vm, L.va, L.ph, L.p, L.q, J);
            break;
        default:
            hipLaunchKernelGGL((k_ybus<NT, WITH_J, ONE, PH_FLY>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order,
                               L.vm, L.va, L.ph, L.p, L.q, J);
            break;
    }
}

template <int NT, bool ONE>
hipError_t launch_ybus(const DevGrid &g, const Launch &L, dim3 grid, dim3 block, int spb, int nchunk, hipStream_t st) {
    if (L.phasor != PH_FLY && L.phasor != PH_SPLIT && L.phasor != PH_INTERLEAVED) return hipErrorInvalidValue;
    if (L.kind == K_YB_SJ_CSC) {
        if (L.phasor != PH_FLY) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_ybus_csc<NT, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                           L.p, L.q, L.jval);
    } else if (L.kind == K_YB_SJ)
        launch_ybus_ph<NT, ONE, true>(g, L, grid, block, spb, nchunk, st);
    else
        launch_ybus_ph<NT, ONE, false>(g, L, grid, block, spb, nchunk, st);
    return hipGetLastError();
}

template <int NT, bool ONE>
hipError_t launch_nt(const DevGrid &g, const Launch &L, hipStream_t st) {
    const int spb = L.states_per_block;
    const int nchunk = (L.nstate + spb - 1) / spb;
    const bool yb = L.kind == K_YB_S || L.kind == K_YB_SJ || L.kind == K_YB_SJ_CSC;
    const int64_t ntl = yb ? g.nytiles : g.ntiles;
    const int64_t blocks = L.order == WO_GROUPED ? (int64_t)kXcds * grouped_tiles((int)ntl) * nchunk
                                                 : (ntl * nchunk + kXcds - 1) / kXcds * kXcds;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks), block(NT);
    // Plain row stores for the injections and the adjoint when a tile has at
    // most eight state chunks (see st_row).
    const bool plain = !ONE && nchunk <= 8;
    switch (L.kind) {
        case K_EW_S:
            if (L.has_parallel && plain)
                hipLaunchKernelGGL((k_ew<NT, true, false, ONE, !ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order,
                                   L.vm, L.va, L.p, L.q, nullptr);
            else if (L.has_parallel)
                hipLaunchKernelGGL((k_ew<NT, true, false, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                                   L.p, L.q, nullptr);
            else if (plain)
                hipLaunchKernelGGL((k_ew<NT, false, false, ONE, !ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order,
                                   L.vm, L.va, L.p, L.q, nullptr);
            else
                hipLaunchKernelGGL((k_ew<NT, false, false, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                                   L.p, L.q, nullptr);
            break;
        case K_EW_SJ:
            if (L.has_parallel)
                hipLaunchKernelGGL((k_ew<NT, true, true, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                                   L.p, L.q, L.jval);
            else
                hipLaunchKernelGGL((k_ew<NT, false, true, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                                   L.p, L.q, L.jval);
            break;
        case K_EW_SJ_CSC:
            if (L.has_parallel)
                hipLaunchKernelGGL((k_ew_csc<NT, true, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm,
                                   L.va, L.p, L.q, L.jval);
            else
                hipLaunchKernelGGL((k_ew_csc<NT, false, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm,
                                   L.va, L.p, L.q, L.jval);
            break;
        case K_YB_S:
        case K_YB_SJ:
        case K_YB_SJ_CSC:
            return launch_ybus<NT, ONE>(g, L, grid, block, spb, nchunk, st);
        case K_EW_VJP:
            if (plain)
                hipLaunchKernelGGL((k_ew_vjp<NT, ONE, !ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va,
                                   L.lp, L.lq, L.gvm, L.gva);
            else
                hipLaunchKernelGGL((k_ew_vjp<NT, ONE>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.order, L.vm, L.va, L.lp,
                                   L.lq, L.gvm, L.gva);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NT, bool ONE>
int occupancy_nt(int kind, bool par) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    auto q = [&](const void *f) { e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, NT, 0); };
    switch (kind) {
        case K_EW_S:
            q(par ? reinterpret_cast<const void *>(&k_ew<NT, true, false, ONE>)
                  : reinterpret_cast<const void *>(&k_ew<NT, false, false, ONE>));
            break;
        case K_EW_SJ:
            q(par ? reinterpret_cast<const void *>(&k_ew<NT, true, true, ONE>)
                  : reinterpret_cast<const void *>(&k_ew<NT, false, true, ONE>));
            break;
        case K_EW_SJ_CSC:
            q(par ? reinterpret_cast<const void *>(&k_ew_csc<NT, true, ONE>)
                  : reinterpret_cast<const void *>(&k_ew_csc<NT, false, ONE>));
            break;
        case K_YB_S:
            q(reinterpret_cast<const void *>(&k_ybus<NT, false, ONE, PH_FLY>));
            break;
        case K_YB_SJ:
            q(reinterpret_cast<const void *>(&k_ybus<NT, true, ONE, PH_FLY>));
            break;
        case K_YB_SJ_CSC:
            q(reinterpret_cast<const void *>(&k_ybus_csc<NT, ONE>));
            break;
        case K_EW_VJP:
            q(reinterpret_cast<const void *>(&k_ew_vjp<NT, ONE>));
            break;
        default:
            break;
    }
    return e == hipSuccess ? n : 0;
}

template <bool ONE>
hipError_t launch_one(const DevGrid &g, const Launch &L, hipStream_t stream) {
    switch (L.tile_items) {
        case 64:
            return launch_nt<64, ONE>(g, L, stream);
        case 128:
            return launch_nt<128, ONE>(g, L, stream);
        case 256:
            return launch_nt<256, ONE>(g, L, stream);
        case 512:
            return launch_nt<512, ONE>(g, L, stream);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

// One state per workgroup runs the instantiation without the state loop.
hipError_t launch_eval(const DevGrid &g, const Launch &L, hipStream_t stream) {
    return L.states_per_block == 1 ? launch_one<true>(g, L, stream) : launch_one<false>(g, L, stream);
}

int resident_blocks_per_cu(int kind, int tile_items, bool has_parallel) {
    // One value per (kind, tile size, parallel flag): a property of the
    // compiled kernel and the device, so concurrent first calls agree.
    static std::atomic<int> cache[7][4][2] = {};
    if (kind < 0 || kind > 6) return 0;
    const int ti = tile_items == 64 ? 0 : tile_items == 128 ? 1 : tile_items == 256 ? 2 : tile_items == 512 ? 3 : -1;
    if (ti < 0) return 0;
    std::atomic<int> &slot = cache[kind][ti][has_parallel ? 1 : 0];
    int v = slot.load();
    if (v > 0) return v;
    switch (tile_items) {
        case 64:
            v = occupancy_nt<64, false>(kind, has_parallel);
            break;
        case 128:
            v = occupancy_nt<128, false>(kind, has_parallel);
            break;
        case 256:
            v = occupancy_nt<256, false>(kind, has_parallel);
            break;
        default:
            v = occupancy_nt<512, false>(kind, has_parallel);
            break;
    }
    slot.store(v);
    return v;
}

hipError_t launch_setup_items(const DevSetup &s, hipStream_t stream) {
    if (s.nitems > 0) {
        const int64_t blocks = (s.nitems + 255) / 256;
        hipLaunchKernelGGL(k_items_init, dim3((unsigned)blocks), dim3(256), 0, stream, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (s.nb > 0) {
        const int64_t blocks = ((int64_t)s.nb + 1 + 255) / 256;
        hipLaunchKernelGGL(k_bus_diag, dim3((unsigned)blocks), dim3(256), 0, stream, s);
    }
    return hipGetLastError();
}

hipError_t launch_lane_fill(const DevLaneFill &f, bool ew, hipStream_t stream) {
    const int64_t n = ew ? f.nlanes : f.nylanes;
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_lane_fill, dim3((unsigned)blocks), dim3(256), 0, stream, f, ew);
    return hipGetLastError();
}

// Scratch of the allocation-free two-phase entry point (k_tp_branch writes
// ten values per record into it, k_tp_reduce reads them back).  In host code
// `scratch` names a host-side stand-in, not device memory: kernels only ever
// receive the device address that static_scratch() resolves.
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

hipError_t static_scratch(int device, double **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_two_phase(const DevTwoPhase &d, int32_t nstate, int64_t nnz_j, const double *vm, const double *va,
                            double *p, double *q, double *jval, bool pre, hipStream_t stream) {
    const unsigned gb = (unsigned)((d.nl + 255) / 256), gr = (unsigned)((d.nb + 255) / 256);
    for (int32_t s = 0; s < nstate; ++s) {
        const size_t so = (size_t)s * d.nb;
        if (d.nl > 0) {
            if (pre)
                hipLaunchKernelGGL(k_tp_branch<true>, dim3(gb), dim3(256), 0, stream, d, vm + so, va + so);
            else
                hipLaunchKernelGGL(k_tp_branch<false>, dim3(gb), dim3(256), 0, stream, d, vm + so, va + so);
        }
        hipLaunchKernelGGL(k_tp_reduce, dim3(gr), dim3(256), 0, stream, d, vm + so, p ? p + so : nullptr,
                           q ? q + so : nullptr, jval + (size_t)s * (size_t)nnz_j);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_copy_add(const DevTwoPhase &d, int32_t nstate, int64_t nnz_j, const double *vm, const double *va,
                           double *p, double *q, double *jval, bool pre, hipStream_t stream) {
    if (nstate == 0) return hipSuccess;
    const unsigned ys = (unsigned)std::min<int32_t>(nstate, 65535);
    const int64_t n2 = (int64_t)nstate * nnz_j / 2;  // nnz_j = 4 nnz_y is even
    if (n2 > 0) {
        const int64_t blocks = std::min<int64_t>((n2 + 255) / 256, 65536);
        hipLaunchKernelGGL(k_ca_zero, dim3((unsigned)blocks), dim3(256), 0, stream, n2, reinterpret_cast<double2 *>(jval));
    }
    if (d.nb > 0)
        hipLaunchKernelGGL(k_ca_bus, dim3((unsigned)((d.nb + 255) / 256), ys), dim3(256), 0, stream, d, nstate, nnz_j, vm, p,
                           q, jval);
    if (d.nl > 0) {
        const dim3 grid((unsigned)((d.nl + 255) / 256), ys);
        if (pre)
            hipLaunchKernelGGL(k_ca_branch<true>, grid, dim3(256), 0, stream, d, nstate, nnz_j, vm, va, p, q, jval);
        else
            hipLaunchKernelGGL(k_ca_branch<false>, grid, dim3(256), 0, stream, d, nstate, nnz_j, vm, va, p, q, jval);
    }
    return hipGetLastError();
}

hipError_t launch_flows(const DevTwoPhase &d, int32_t nstate, const double *vm, const double *va, double *pf,
                        double *qf, double *pt, double *qt, double *jac, hipStream_t stream) {
    if (d.nl == 0 || nstate == 0) return hipSuccess;
    const dim3 grid((unsigned)((d.nl + 255) / 256), (unsigned)std::min<int32_t>(nstate, 65535));
    if (jac)
        hipLaunchKernelGGL(k_flows<true>, grid, dim3(256), 0, stream, d, nstate, vm, va, pf, qf, pt, qt, jac);
    else
        hipLaunchKernelGGL(k_flows<false>, grid, dim3(256), 0, stream, d, nstate, vm, va, pf, qf, pt, qt, jac);
    return hipGetLastError();
}

hipError_t launch_phasor(int32_t layout, int64_t n, const double *vm, const double *va, double *ph, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    if (layout == PH_SPLIT)
        hipLaunchKernelGGL(k_phasor<PH_SPLIT>, dim3((unsigned)blocks), dim3(256), 0, stream, n, vm, va, ph);
    else if (layout == PH_INTERLEAVED)
        hipLaunchKernelGGL(k_phasor<PH_INTERLEAVED>, dim3((unsigned)blocks), dim3(256), 0, stream, n, vm, va, ph);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_jscatter(int32_t nstate, int64_t nnz_j, const double *jval, const int32_t *map, int64_t out_nnz,
                           double *out, hipStream_t stream) {
    if (nstate == 0 || nnz_j == 0) return hipSuccess;
    const int64_t blocks = (nnz_j + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks, (unsigned)std::min<int32_t>(nstate, 65535));
    hipLaunchKernelGGL(k_jscatter, grid, dim3(256), 0, stream, nstate, nnz_j, jval, map, out_nnz, out);
    return hipGetLastError();
}

hipError_t launch_branch_consts(const DevTwoPhase &d, double *bc, hipStream_t stream) {
    if (d.nl == 0) return hipSuccess;
    hipLaunchKernelGGL(k_branch_consts, dim3((unsigned)((d.nl + 255) / 256)), dim3(256), 0, stream, d, bc);
    return hipGetLastError();
}

hipError_t launch_ybus_assemble(const DevSetup &s, hipStream_t stream) {
    if (s.nnz_y == 0) return hipSuccess;
    const int64_t blocks = (s.nnz_y + 255) / 256;
    hipLaunchKernelGGL(k_ybus_assemble, dim3((unsigned)blocks), dim3(256), 0, stream, s);
    return hipGetLastError();
}

}  // namespace pf
