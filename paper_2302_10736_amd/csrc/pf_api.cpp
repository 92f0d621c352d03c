// Host side of the C ABI declared in include/pf.h: input validation, the
// Ybus / Jacobian patterns, the bus-sorted branch-end records, the tile
// schedule, device upload and the launch of the evaluation kernels.
//
// Setup follows the paper's advice to build the sparsity pattern once and
// reuse it (Section IV.B.3, Algorithm 2; Section IV.C.2): nothing here runs
// in the evaluation calls except argument checks and one kernel launch.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "../../include/pf_testing.h"
#include "pf_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(PF_EHIP, std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

// Every device allocation of the library goes through here, so that a test
// can make the next n of them fail (pf_debug_fail_allocs).
std::atomic<int> g_fail_allocs{0};

hipError_t dev_alloc(void **p, size_t bytes) {
    int n = g_fail_allocs.load();
    while (n > 0) {
        if (g_fail_allocs.compare_exchange_weak(n, n - 1)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc(p, bytes);
}

// Device arrays are carved from one allocation; each array starts on a
// 256-byte boundary.
struct Arena {
    size_t off = 0;
    template <class T>
    size_t take(size_t n) {
        size_t o = (off + 255) & ~size_t(255);
        off = o + n * sizeof(T);
        return o;
    }
};

}  // namespace

struct pf_grid {
    int32_t nb = 0, nl = 0, ngrids = 1;
    int64_t nnz_y = 0, nitems = 0;
    bool has_parallel = false;
    bool host_only = false;
    bool ybus_valid = false;
    int device = -1;

    std::vector<int32_t> bus_off, br_off;  // [G+1]
    std::vector<int64_t> y_off;            // [G+1]
    std::vector<int32_t> yrow, ycol;       // global numbering
    std::vector<int32_t> irow, nbr, slot, item_br;
    std::vector<int32_t> slot_row, slot_item;

    int32_t tile_items = 256, states_per_block = 0, order = PF_ORDER_AUTO;
    std::vector<pf::TileDesc> tiles, ytiles;  // element-wise and Ybus work tiles
    int32_t num_cus = 0;
    pf::DevLaneFill lanes{};  // gather sources and targets of the lane values
    pf::DevTwoPhase tp{};     // two-phase element-wise tables and scratch (inside dmem)

    void *dmem = nullptr;   // grid data
    void *dtile = nullptr;  // schedule
    uint64_t sched_gen = 0;  // bumped by every schedule change (recorded graphs check it)
    pf::DevGrid dev{};
    pf::DevSetup setup{};  // device view used by the setup kernels
};

namespace {

bool finite_all(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// Row-aligned tiles inside each grid, built greedily.
//   Element-wise tiles (g->tiles): at most NT branch ends (one lane each), NT
//   rows and kEwSlots(NT) Ybus slots (the LDS copy of the tile's J rows).  A
//   row with more than NT branch ends is a tile of its own, walked in chunks.
//   Ybus tiles (g->ytiles): at most NT slots (one lane each); a row with more
//   than NT slots is a tile of its own.
// Shunt records take no lane: their only content is the diagonal slot, whose
// J entries the row thread writes.
void build_tiles(pf_grid *g, int NT) {
    const int NS = pf::kEwSlots(NT);
    g->tiles.clear();
    g->ytiles.clear();
    for (int32_t gi = 0; gi < g->ngrids; ++gi) {
        const int32_t rb = g->bus_off[gi], re = g->bus_off[gi + 1];
        auto desc = [&](int32_t a, int32_t z) {
            pf::TileDesc d;
            d.r0 = a;
            d.nrows = z - a;
            d.i0 = g->irow[a];
            d.n = g->irow[z] - d.i0;
            d.ne = d.n - (z - a);  // one shunt record per row
            d.s0 = g->yrow[a];
            d.ns = g->yrow[z] - d.s0;
            d.sh = 0;
            if (z == a + 1)  // one row: where its bus-shunt record sits among its records
                for (int32_t e = g->irow[a]; e < g->irow[z]; ++e)
                    if (g->item_br[e] < 0) d.sh = e - d.i0;
            // Grid gi's J values start at 4 y_off[gi]; its P rows hold
            // 2 nnz_y(gi) values, so row i's P part starts at
            // 2 y_off[gi] + 2 yrow[i] and its Q part at 2 y_off[gi+1] + 2 yrow[i].
            d.jp = 2 * g->y_off[gi] + 2 * (int64_t)d.s0;
            d.jq = 2 * g->y_off[gi + 1] + 2 * (int64_t)d.s0;
            return d;
        };
        // element-wise
        int32_t start = rb;
        int64_t ce = 0, cs = 0;
        auto close = [&](std::vector<pf::TileDesc> &out, int32_t upto) {
            if (upto > start) out.push_back(desc(start, upto));
            start = upto;
            ce = cs = 0;
        };
        for (int32_t r = rb; r < re; ++r) {
            const int64_t ne = g->irow[r + 1] - g->irow[r] - 1, ns = g->yrow[r + 1] - g->yrow[r];
            if (ne > NT) {
                close(g->tiles, r);
                close(g->tiles, r + 1);
                continue;
            }
            if (ce + ne > NT || cs + ns > NS || r - start + 1 > NT) close(g->tiles, r);
            ce += ne;
            cs += ns;
        }
        close(g->tiles, re);
        // Ybus
        start = rb;
        for (int32_t r = rb; r < re; ++r) {
            const int64_t ns = g->yrow[r + 1] - g->yrow[r];
            if (ns > NT) {
                close(g->ytiles, r);
                close(g->ytiles, r + 1);
                continue;
            }
            if (cs + ns > NT) close(g->ytiles, r);
            cs += ns;
        }
        close(g->ytiles, re);
    }
}

// Lane tables of the packed tiles (tile size NT).  Positions inside the LDS
// copy of a tile's J rows (slot capacity NS): the P rows take [0, 2 NS), the
// Q rows start at 2 NS + 2, and position 2 NS (Q: 4 NS + 2) is a pad that
// absorbs the writes of lanes with nothing to write.  For row r of a tile
// with local slot range [ya, yz) and local slot ls, dP/dtheta sits at
// ya + ls and dP/dv at yz + ls (eq. (2): J11 and J12 entries of one
// row are adjacent, as are J21 and J22).
struct HostLanes {
    std::vector<int32_t> lane_j, lane_rec, lane_pk, lane_run;
    std::vector<int32_t> ylane_j, ylane_slot, ylane_pk;
    std::vector<int32_t> row_ew, row_yb;                 // pairs per bus, + one inert entry at nb
    std::vector<int32_t> ydslot;                         // [nb] global Ybus slot of each diagonal
    std::vector<int32_t> yt_slot;                        // [nnz_y] slot of the transposed entry
    std::vector<int32_t> ylane_tslot;                    // transposed slot of each Ybus lane, -1 inert
};

HostLanes build_lanes(const pf_grid *g) {
    const int NT = g->tile_items;
    const int32_t epad = 2 * pf::kEwSlots(NT), ypad = 2 * NT;
    const size_t nle = g->tiles.size() * (size_t)NT, nly = g->ytiles.size() * (size_t)NT;
    HostLanes h;
    h.lane_j.assign(nle, 0);
    h.lane_rec.assign(nle, -1);
    h.lane_pk.assign(nle, pf::ew_pack(epad, epad, 0));
    h.lane_run.assign(g->has_parallel ? nle : 1, 0);
    h.ylane_j.assign(nly, 0);
    h.ylane_slot.assign(nly, -1);
    h.ylane_pk.assign(nly, pf::yb_pack(ypad, ypad, 0, false));
    // Entry nb is what lanes without a row read: empty ranges, pad targets.
    h.row_ew.assign(2 * ((size_t)g->nb + 1), 0);
    h.row_yb.assign(2 * ((size_t)g->nb + 1), 0);
    h.row_ew[2 * (size_t)g->nb + 1] = epad | (epad << 16);
    h.row_yb[2 * (size_t)g->nb + 1] = ypad;
    h.ydslot.assign(g->nb, 0);
    auto diag_slot = [&](int32_t i) {
        for (int32_t q = g->yrow[i]; q < g->yrow[i + 1]; ++q)
            if (g->ycol[q] == i) return q;
        return g->yrow[i];  // every bus has its diagonal slot
    };
    for (int32_t i = 0; i < g->nb; ++i) h.ydslot[i] = diag_slot(i);
    // (j, i) for every slot (i, j): the pattern is symmetric and columns ascend within a row
    h.yt_slot.assign(g->nnz_y, 0);
    for (int32_t i = 0; i < g->nb; ++i)
        for (int32_t q = g->yrow[i]; q < g->yrow[i + 1]; ++q) {
            const int32_t j = g->ycol[q];
            const int32_t *a = g->ycol.data() + g->yrow[j], *z = g->ycol.data() + g->yrow[j + 1];
            h.yt_slot[q] = (int32_t)(std::lower_bound(a, z, i) - g->ycol.data());
        }
    h.ylane_tslot.assign(nly, -1);
    for (size_t t = 0; t < g->tiles.size(); ++t) {
        const pf::TileDesc &c = g->tiles[t];
        const size_t base = t * NT;
        for (int k = 0; k < NT; ++k) h.lane_j[base + k] = c.r0;
        if (c.ne > NT) continue;  // long row: walked without lane tables
        int32_t lane = 0;
        for (int32_t row = 0; row < c.nrows; ++row) {
            const int32_t i = c.r0 + row;
            const int32_t ya = g->yrow[i] - c.s0, yz = g->yrow[i + 1] - c.s0;
            const int32_t dls = h.ydslot[i] - c.s0;
            const int32_t ra = lane;
            for (int32_t e = g->irow[i]; e < g->irow[i + 1]; ++e) {
                if (g->item_br[e] < 0) continue;  // the shunt record
                const size_t L = base + lane++;
                const int32_t ls = g->slot[e] - c.s0;
                // first branch end of its slot (parallel branches share a slot)
                const bool head = e == g->irow[i] || g->slot[e - 1] != g->slot[e] || g->item_br[e - 1] < 0;
                int32_t run = 0;
                if (head)
                    while (e + run < g->irow[i + 1] && g->slot[e + run] == g->slot[e]) ++run;
                h.lane_j[L] = g->nbr[e];
                h.lane_rec[L] = e;
                h.lane_pk[L] = head ? pf::ew_pack(ya + ls, yz + ls, row) : pf::ew_pack(epad, epad, row);
                if (g->has_parallel) h.lane_run[L] = run;
            }
            h.row_ew[2 * i] = ra | (lane << 16);
            h.row_ew[2 * i + 1] = (ya + dls) | ((yz + dls) << 16);
        }
    }
    for (size_t t = 0; t < g->ytiles.size(); ++t) {
        const pf::TileDesc &c = g->ytiles[t];
        const size_t base = t * NT;
        for (int k = 0; k < NT; ++k) h.ylane_j[base + k] = c.r0;
        if (c.ns > NT) continue;
        for (int32_t row = 0; row < c.nrows; ++row) {
            const int32_t i = c.r0 + row;
            const int32_t ya = g->yrow[i] - c.s0, yz = g->yrow[i + 1] - c.s0;
            h.row_yb[2 * i] = ya | (yz << 16);
            h.row_yb[2 * i + 1] = h.ydslot[i] - c.s0;
            for (int32_t q = g->yrow[i]; q < g->yrow[i + 1]; ++q) {
                const size_t L = base + (q - c.s0);
                const int32_t ls = q - c.s0;
                const bool dg = g->ycol[q] == i;
                h.ylane_j[L] = g->ycol[q];
                h.ylane_slot[L] = q;
                h.ylane_tslot[L] = h.yt_slot[q];
                h.ylane_pk[L] = dg ? pf::yb_pack(ypad, ypad, row, true) : pf::yb_pack(ya + ls, yz + ls, row, false);
            }
        }
    }
    return h;
}

// Upload the schedule (tiles and lane tables) of g->tiles / g->ytiles /
// g->tile_items into a fresh device allocation.  The handle switches to it
// only when every step succeeded; on failure the new allocation is released
// and the handle keeps its previous device schedule untouched.
int upload_tiles(pf_grid *g) {
    if (g->host_only) {  // the lane tables are still built: the whole schedule is validated on the host
        (void)build_lanes(g);
        return PF_OK;
    }
    const HostLanes h = build_lanes(g);
    const size_t nt = g->tiles.size(), nyt = g->ytiles.size();
    const size_t nle = nt * (size_t)g->tile_items, nly = nyt * (size_t)g->tile_items;
    const size_t nrun = h.lane_run.size();
    Arena ar;
    const size_t o_t = ar.take<pf::TileDesc>(nt), o_yt = ar.take<pf::TileDesc>(nyt);
    const size_t o_lj = ar.take<int32_t>(nle), o_lrec = ar.take<int32_t>(nle), o_lpk = ar.take<int32_t>(nle);
    const size_t o_lrun = ar.take<int32_t>(nrun);
    const size_t o_lgb = ar.take<double2>(nle), o_lgr = ar.take<double2>(nle), o_rew = ar.take<int2>(g->nb + 1);
    const size_t o_yj = ar.take<int32_t>(nly), o_yslot = ar.take<int32_t>(nly), o_ypk = ar.take<int32_t>(nly);
    const size_t o_yy = ar.take<double2>(nly), o_ryb = ar.take<int2>(g->nb + 1);
    const size_t o_yds = ar.take<int32_t>(g->nb);
    const size_t o_yts = ar.take<int32_t>(g->nnz_y), o_ylt = ar.take<int32_t>(nly), o_yyt = ar.take<double2>(nly);
    void *mem = nullptr;
    hipError_t e = dev_alloc(&mem, ar.off);
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(PF_ENOMEM, "device allocation of the schedule failed")
                                        : hip_fail(e, "hipMalloc(schedule)");
    char *base = static_cast<char *>(mem);
    hipError_t ee = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (ee == hipSuccess && bytes) ee = hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice);
    };
    up(o_t, g->tiles.data(), nt * sizeof(pf::TileDesc));
    up(o_yt, g->ytiles.data(), nyt * sizeof(pf::TileDesc));
    up(o_lj, h.lane_j.data(), nle * 4);
    up(o_lrec, h.lane_rec.data(), nle * 4);
    up(o_lpk, h.lane_pk.data(), nle * 4);
    up(o_lrun, h.lane_run.data(), nrun * 4);
    up(o_rew, h.row_ew.data(), ((size_t)g->nb + 1) * 8);
    up(o_yj, h.ylane_j.data(), nly * 4);
    up(o_yslot, h.ylane_slot.data(), nly * 4);
    up(o_ypk, h.ylane_pk.data(), nly * 4);
    up(o_ryb, h.row_yb.data(), ((size_t)g->nb + 1) * 8);
    up(o_yds, h.ydslot.data(), (size_t)g->nb * 4);
    up(o_yts, h.yt_slot.data(), (size_t)g->nnz_y * 4);
    up(o_ylt, h.ylane_tslot.data(), nly * 4);
    if (ee != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(ee, "hipMemcpy(schedule)");
    }
    pf::DevGrid d = g->dev;
    d.tiles = reinterpret_cast<const pf::TileDesc *>(base + o_t);
    d.ntiles = (int32_t)nt;
    d.ytiles = reinterpret_cast<const pf::TileDesc *>(base + o_yt);
    d.nytiles = (int32_t)nyt;
    d.lane_j = reinterpret_cast<const int32_t *>(base + o_lj);
    d.lane_pk = reinterpret_cast<const int32_t *>(base + o_lpk);
    d.lane_run = reinterpret_cast<const int32_t *>(base + o_lrun);
    d.lane_gb = reinterpret_cast<const double2 *>(base + o_lgb);
    d.lane_grbr = reinterpret_cast<const double2 *>(base + o_lgr);
    d.row_ew = reinterpret_cast<const int2 *>(base + o_rew);
    d.ylane_j = reinterpret_cast<const int32_t *>(base + o_yj);
    d.ylane_pk = reinterpret_cast<const int32_t *>(base + o_ypk);
    d.ylane_y = reinterpret_cast<const double2 *>(base + o_yy);
    d.row_yb = reinterpret_cast<const int2 *>(base + o_ryb);
    d.yt_slot = reinterpret_cast<const int32_t *>(base + o_yts);
    d.ylane_yt = reinterpret_cast<const double2 *>(base + o_yyt);
    pf::DevLaneFill f = g->lanes;
    f.nlanes = (int64_t)nle;
    f.nylanes = (int64_t)nly;
    f.lane_rec = reinterpret_cast<const int32_t *>(base + o_lrec);
    f.ylane_slot = reinterpret_cast<const int32_t *>(base + o_yslot);
    f.G = d.G;
    f.B = d.B;
    f.Gr = d.Gr;
    f.Br = d.Br;
    f.yre = d.yre;
    f.yim = d.yim;
    f.lane_gb = reinterpret_cast<double2 *>(base + o_lgb);
    f.lane_grbr = reinterpret_cast<double2 *>(base + o_lgr);
    f.ylane_y = reinterpret_cast<double2 *>(base + o_yy);
    f.ylane_tslot = reinterpret_cast<const int32_t *>(base + o_ylt);
    f.ylane_yt = reinterpret_cast<double2 *>(base + o_yyt);
    f.nb = g->nb;
    f.ydslot = reinterpret_cast<const int32_t *>(base + o_yds);
    // Record constants exist once the setup kernels ran; Ybus values once
    // pf_ybus ran.  Until then the Ybus lanes stay unfilled and the Ybus
    // evaluation calls refuse to run.
    e = pf::launch_lane_fill(f, true, nullptr);
    if (e == hipSuccess && g->ybus_valid) e = pf::launch_lane_fill(f, false, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "lane table kernel");
    }
    void *old = g->dtile;
    g->dtile = mem;
    g->dev = d;
    g->lanes = f;
    if (old) (void)hipFree(old);
    return PF_OK;
}

int validate(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus, const double *r,
             const double *x, const double *b, const double *tap, const double *shift, const double *gs,
             const double *bs, int32_t ngrids, const int32_t *bus_off, const int32_t *br_off,
             uint32_t flags) {
    if (flags & ~uint32_t(PF_BUILD_HOST_ONLY)) return fail(PF_EINVAL, "unknown flag bits");
    if (nb <= 0) return fail(PF_EINVAL, "nb must be >= 1");
    if (nl < 0) return fail(PF_EINVAL, "nl must be >= 0");
    if (ngrids <= 0) return fail(PF_EINVAL, "ngrids must be >= 1");
    if (ngrids > nb) return fail(PF_EINVAL, "every grid needs at least one bus (ngrids > nb)");
    if (nl > 0 && (!fbus || !tbus || !r || !x || !b || !tap || !shift))
        return fail(PF_EINVAL, "branch arrays must not be NULL when nl > 0");
    if (ngrids > 1 && (!bus_off || !br_off)) return fail(PF_EINVAL, "bus_off and br_off are required when ngrids > 1");
    if (ngrids > 1) {
        if (bus_off[0] != 0 || bus_off[ngrids] != nb) return fail(PF_EINVAL, "bus_off must run from 0 to nb");
        if (br_off[0] != 0 || br_off[ngrids] != nl) return fail(PF_EINVAL, "br_off must run from 0 to nl");
        for (int32_t k = 0; k < ngrids; ++k) {
            if (bus_off[k + 1] <= bus_off[k]) return fail(PF_EINVAL, "bus_off must be strictly increasing");
            if (br_off[k + 1] < br_off[k]) return fail(PF_EINVAL, "br_off must be non-decreasing");
        }
    }
    int32_t gk = 0;
    for (int32_t l = 0; l < nl; ++l) {
        if (ngrids > 1)
            while (l >= br_off[gk + 1]) ++gk;
        int32_t nbg = ngrids > 1 ? bus_off[gk + 1] - bus_off[gk] : nb;
        if (fbus[l] < 0 || fbus[l] >= nbg || tbus[l] < 0 || tbus[l] >= nbg)
            return fail(PF_EINVAL, "branch " + std::to_string(l) + ": bus index out of range");
        if (fbus[l] == tbus[l]) return fail(PF_EINVAL, "branch " + std::to_string(l) + ": from == to");
        if (!std::isfinite(r[l]) || !std::isfinite(x[l]) || !std::isfinite(b[l]) || !std::isfinite(tap[l]) ||
            !std::isfinite(shift[l]))
            return fail(PF_EINVAL, "branch " + std::to_string(l) + ": non-finite parameter");
        if (tap[l] < 0) return fail(PF_EINVAL, "branch " + std::to_string(l) + ": tap < 0");
        if (r[l] == 0.0 && x[l] == 0.0) return fail(PF_EINVAL, "branch " + std::to_string(l) + ": r = x = 0");
    }
    if (gs && !finite_all(gs, nb)) return fail(PF_EINVAL, "non-finite bus shunt conductance");
    if (bs && !finite_all(bs, nb)) return fail(PF_EINVAL, "non-finite bus shunt susceptance");
    if ((int64_t)nb + 2 * (int64_t)nl > INT32_MAX) return fail(PF_EUNSUP, "more than 2^31-1 records");
    if (4 * ((int64_t)nb + 2 * (int64_t)nl) > INT32_MAX) return fail(PF_EUNSUP, "Jacobian larger than 2^31-1 entries");
    return PF_OK;
}

}  // namespace

extern "C" {

const char *pf_last_error(void) { return g_err.c_str(); }

const char *pf_version(void) { return "pf-mi355x 0.1 (gfx950, FP64)"; }

int pf_build_pattern(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus, const double *r,
                     const double *x, const double *b, const double *tap, const double *shift, const double *gs,
                     const double *bs, int32_t ngrids, const int32_t *bus_off, const int32_t *br_off,
                     uint32_t flags, pf_grid **out) {
    g_err.clear();
    if (!out) return fail(PF_EINVAL, "out must not be NULL");
    *out = nullptr;
    int st = validate(nb, nl, fbus, tbus, r, x, b, tap, shift, gs, bs, ngrids, bus_off, br_off, flags);
    if (st) return st;

    pf_grid *g = new (std::nothrow) pf_grid;
    if (!g) return fail(PF_ENOMEM, "host allocation failed");
    try {
        g->nb = nb;
        g->nl = nl;
        g->ngrids = ngrids;
        g->host_only = (flags & PF_BUILD_HOST_ONLY) != 0;
        g->bus_off.assign(ngrids + 1, 0);
        g->br_off.assign(ngrids + 1, 0);
        if (ngrids > 1) {
            std::copy(bus_off, bus_off + ngrids + 1, g->bus_off.begin());
            std::copy(br_off, br_off + ngrids + 1, g->br_off.begin());
        } else {
            g->bus_off[1] = nb;
            g->br_off[1] = nl;
        }
        // Global bus numbers of both branch ends.
        std::vector<int32_t> gf(nl), gt(nl);
        for (int32_t k = 0; k < ngrids; ++k)
            for (int32_t l = g->br_off[k]; l < g->br_off[k + 1]; ++l) {
                gf[l] = fbus[l] + g->bus_off[k];
                gt[l] = tbus[l] + g->bus_off[k];
            }
        // Records per bus: one shunt record + one per incident branch end.
        const int64_t ni = (int64_t)nb + 2 * (int64_t)nl;
        g->nitems = ni;
        g->irow.assign(nb + 1, 0);
        for (int32_t i = 0; i < nb; ++i) g->irow[i + 1] = 1;
        for (int32_t l = 0; l < nl; ++l) {
            g->irow[gf[l] + 1]++;
            g->irow[gt[l] + 1]++;
        }
        for (int32_t i = 0; i < nb; ++i) g->irow[i + 1] += g->irow[i];
        // Sort key inside a bus: (neighbour, branch, end); the shunt record
        // has neighbour == own bus and sorts before nothing else with it.
        std::vector<int64_t> key(ni);
        std::vector<int32_t> fill(g->irow.begin(), g->irow.end() - 1);
        g->nbr.assign(ni, 0);
        g->item_br.assign(ni, 0);
        for (int32_t i = 0; i < nb; ++i) {
            int32_t e = fill[i]++;
            key[e] = ((int64_t)i << 32) | 0;  // shunt record first among equal neighbours
            g->nbr[e] = i;
            g->item_br[e] = -1;
        }
        for (int32_t l = 0; l < nl; ++l) {
            int32_t e = fill[gf[l]]++;
            key[e] = ((int64_t)gt[l] << 32) | (uint32_t)(2 * l + 1);
            g->nbr[e] = gt[l];
            g->item_br[e] = 2 * l;  // from end
            e = fill[gt[l]]++;
            key[e] = ((int64_t)gf[l] << 32) | (uint32_t)(2 * l + 2);
            g->nbr[e] = gf[l];
            g->item_br[e] = 2 * l + 1;  // to end
        }
        std::vector<int32_t> perm;
        for (int32_t i = 0; i < nb; ++i) {
            int32_t a = g->irow[i], z = g->irow[i + 1];
            perm.resize(z - a);
            for (int32_t t = 0; t < z - a; ++t) perm[t] = a + t;
            std::sort(perm.begin(), perm.end(), [&](int32_t u, int32_t v) { return key[u] < key[v]; });
            std::vector<int32_t> nb2(z - a), br2(z - a);
            for (int32_t t = 0; t < z - a; ++t) {
                nb2[t] = g->nbr[perm[t]];
                br2[t] = g->item_br[perm[t]];
            }
            std::copy(nb2.begin(), nb2.end(), g->nbr.begin() + a);
            std::copy(br2.begin(), br2.end(), g->item_br.begin() + a);
        }
        // Slots: distinct neighbours of each bus (parallel branches merge).
        g->slot.assign(ni, 0);
        g->yrow.assign(nb + 1, 0);
        g->ycol.clear();
        g->ycol.reserve(ni);
        g->slot_row.clear();
        g->slot_item.clear();
        for (int32_t i = 0; i < nb; ++i) {
            for (int32_t e = g->irow[i]; e < g->irow[i + 1]; ++e) {
                if (e == g->irow[i] || g->nbr[e] != g->nbr[e - 1]) {
                    g->ycol.push_back(g->nbr[e]);
                    g->slot_row.push_back(i);
                    g->slot_item.push_back(e);
                }
                g->slot[e] = (int32_t)g->ycol.size() - 1;
            }
            g->yrow[i + 1] = (int32_t)g->ycol.size();
        }
        g->nnz_y = (int64_t)g->ycol.size();
        g->slot_item.push_back((int32_t)ni);
        g->has_parallel = g->nnz_y != ni;
        g->y_off.assign(ngrids + 1, 0);
        for (int32_t k = 0; k <= ngrids; ++k) g->y_off[k] = g->yrow[g->bus_off[k]];
        if ((int64_t)g->nnz_y * 4 > INT32_MAX) {
            delete g;
            return fail(PF_EUNSUP, "Jacobian larger than 2^31-1 entries");
        }
        // Tiles never span grids, so a grid with fewer branch ends than a tile
        // leaves lanes idle: with many small grids, start from the smallest
        // tile that holds an average grid's branch ends.
        if (ngrids > 1) {
            const int64_t mean_ends = (2 * (int64_t)nl + ngrids - 1) / ngrids;
            g->tile_items = mean_ends <= 64 ? 64 : mean_ends <= 128 ? 128 : 256;
        }
        build_tiles(g, g->tile_items);

        if (g->host_only) {
            (void)upload_tiles(g);  // host-only: builds the lane tables, touches no device
            *out = g;
            return PF_OK;
        }

        // ---------------------------------------------------------- device
        hipError_t e = hipGetDevice(&g->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&g->num_cus, hipDeviceAttributeMultiprocessorCount, g->device);
        if (e != hipSuccess) {
            delete g;
            return hip_fail(e, "hipGetDevice");
        }
        // Set-up of the library's static scratch on this device (the address
        // is resolved once per device and cached; a failure is reported by
        // the entry point that uses it, pf_jacobian_two_phase_static).
        {
            double *scr = nullptr;
            (void)pf::static_scratch(g->device, &scr);
        }
        Arena ar;
        size_t o_yrow = ar.take<int32_t>(nb + 1), o_irow = ar.take<int32_t>(nb + 1);
        size_t o_ycol = ar.take<int32_t>(g->nnz_y), o_nbr = ar.take<int32_t>(ni), o_slot = ar.take<int32_t>(ni);
        size_t o_G = ar.take<double>(ni), o_B = ar.take<double>(ni), o_Gr = ar.take<double>(ni),
               o_Br = ar.take<double>(ni), o_dA = ar.take<double>(nb + 1),
               o_dC = ar.take<double>(nb + 1);
        size_t o_yre = ar.take<double>(g->nnz_y), o_yim = ar.take<double>(g->nnz_y);
        // setup-only arrays
        size_t o_ibr = ar.take<int32_t>(ni), o_srow = ar.take<int32_t>(g->nnz_y),
               o_sitem = ar.take<int32_t>(g->nnz_y + 1);
        size_t o_r = ar.take<double>(nl), o_x = ar.take<double>(nl), o_b = ar.take<double>(nl),
               o_tap = ar.take<double>(nl), o_sh = ar.take<double>(nl);
        size_t o_gs = ar.take<double>(nb), o_bs = ar.take<double>(nb);
        // two-phase tables
        size_t o_bf = ar.take<int32_t>(nl), o_bt = ar.take<int32_t>(nl), o_brec = ar.take<int32_t>(2 * (size_t)nl),
               o_jpq = ar.take<int2>(nb), o_bc = ar.take<double>(6 * (size_t)nl);
        // two-phase scratch: ten values per record, owned by the handle
        size_t o_scr = ar.take<double>(10 * (size_t)ni);
        e = dev_alloc(&g->dmem, ar.off);
        if (e != hipSuccess) {
            g->dmem = nullptr;
            delete g;
            return e == hipErrorOutOfMemory ? fail(PF_ENOMEM, "device allocation failed")
                                            : hip_fail(e, "hipMalloc(grid)");
        }
        char *base = static_cast<char *>(g->dmem);
        auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
            if (!bytes) return hipSuccess;
            return hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice);
        };
        std::vector<double> zeros;
        const double *gsp = gs, *bsp = bs;
        if (!gs || !bs) zeros.assign(nb, 0.0);
        if (!gsp) gsp = zeros.data();
        if (!bsp) bsp = zeros.data();
        hipError_t ee = hipSuccess;
        auto chk = [&](hipError_t x2) {
            if (ee == hipSuccess) ee = x2;
        };
        chk(up(o_yrow, g->yrow.data(), (nb + 1) * 4));
        chk(up(o_irow, g->irow.data(), (nb + 1) * 4));
        chk(up(o_ycol, g->ycol.data(), g->nnz_y * 4));
        chk(up(o_nbr, g->nbr.data(), ni * 4));
        chk(up(o_slot, g->slot.data(), ni * 4));
        chk(up(o_ibr, g->item_br.data(), ni * 4));
        chk(up(o_srow, g->slot_row.data(), g->nnz_y * 4));
        chk(up(o_sitem, g->slot_item.data(), (g->nnz_y + 1) * 4));
        chk(up(o_r, r, nl * 8));
        chk(up(o_x, x, nl * 8));
        chk(up(o_b, b, nl * 8));
        chk(up(o_tap, tap, nl * 8));
        chk(up(o_sh, shift, nl * 8));
        chk(up(o_gs, gsp, nb * 8));
        chk(up(o_bs, bsp, nb * 8));
        {
            std::vector<int32_t> brec(2 * (size_t)nl, 0);
            for (int64_t e2 = 0; e2 < ni; ++e2)
                if (g->item_br[e2] >= 0) brec[g->item_br[e2]] = (int32_t)e2;
            std::vector<int32_t> jpq(2 * (size_t)nb);
            for (int32_t k = 0; k < ngrids; ++k)
                for (int32_t i = g->bus_off[k]; i < g->bus_off[k + 1]; ++i) {
                    jpq[2 * (size_t)i] = (int32_t)(2 * g->y_off[k] + 2 * (int64_t)g->yrow[i]);
                    jpq[2 * (size_t)i + 1] = (int32_t)(2 * g->y_off[k + 1] + 2 * (int64_t)g->yrow[i]);
                }
            chk(up(o_bf, gf.data(), (size_t)nl * 4));
            chk(up(o_bt, gt.data(), (size_t)nl * 4));
            chk(up(o_brec, brec.data(), 2 * (size_t)nl * 4));
            chk(up(o_jpq, jpq.data(), (size_t)nb * 8));
        }
        if (ee != hipSuccess) {
            int rc = hip_fail(ee, "hipMemcpy(grid)");
            pf_grid_free(g);
            return rc;
        }
        auto I32 = [&](size_t o) { return reinterpret_cast<int32_t *>(base + o); };
        auto F64 = [&](size_t o) { return reinterpret_cast<double *>(base + o); };
        pf::DevGrid &d = g->dev;
        d.nb = nb;
        d.nnz_y = g->nnz_y;
        d.nnz_j = 4 * g->nnz_y;
        d.yrow = I32(o_yrow);
        d.irow = I32(o_irow);
        d.ycol = I32(o_ycol);
        d.nbr = I32(o_nbr);
        d.slot = I32(o_slot);
        d.dA = F64(o_dA);
        d.dC = F64(o_dC);
        d.G = F64(o_G);
        d.B = F64(o_B);
        d.Gr = F64(o_Gr);
        d.Br = F64(o_Br);
        d.yre = F64(o_yre);
        d.yim = F64(o_yim);

        pf::DevSetup s{};
        s.nitems = ni;
        s.nnz_y = g->nnz_y;
        s.item_br = I32(o_ibr);
        s.nbr = I32(o_nbr);
        s.slot_row = I32(o_srow);
        s.slot_item = I32(o_sitem);
        s.irow = I32(o_irow);
        s.ycol = I32(o_ycol);
        s.r = F64(o_r);
        s.x = F64(o_x);
        s.b = F64(o_b);
        s.tap = F64(o_tap);
        s.shift = F64(o_sh);
        s.gs = F64(o_gs);
        s.bs = F64(o_bs);
        s.nb = nb;
        s.dA = F64(o_dA);
        s.dC = F64(o_dC);
        s.G = F64(o_G);
        s.B = F64(o_B);
        s.Gr = F64(o_Gr);
        s.Br = F64(o_Br);
        s.yre = F64(o_yre);
        s.yim = F64(o_yim);
        g->setup = s;
        pf::DevTwoPhase &tp = g->tp;
        tp.nb = nb;
        tp.nl = nl;
        tp.nrec = ni;
        tp.br_from = I32(o_bf);
        tp.br_to = I32(o_bt);
        tp.br_rec = I32(o_brec);
        tp.r = s.r;
        tp.x = s.x;
        tp.b = s.b;
        tp.tap = s.tap;
        tp.shift = s.shift;
        tp.gs = s.gs;
        tp.bs = s.bs;
        tp.irow = d.irow;
        tp.item_br = s.item_br;
        tp.slot = d.slot;
        tp.yrow = d.yrow;
        tp.jpq = reinterpret_cast<const int2 *>(base + o_jpq);
        tp.bc = F64(o_bc);
        tp.scr = F64(o_scr);
        e = pf::launch_setup_items(s, nullptr);
        if (e == hipSuccess) e = pf::launch_branch_consts(tp, F64(o_bc), nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            int rc = hip_fail(e, "record constants kernel");
            pf_grid_free(g);
            return rc;
        }
        st = upload_tiles(g);
        if (st) {
            pf_grid_free(g);
            return st;
        }
        *out = g;
        return PF_OK;
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(PF_ENOMEM, "host allocation failed");
    }
}

void pf_grid_free(pf_grid *g) {
    if (!g) return;
    if (g->dmem) (void)hipFree(g->dmem);
    if (g->dtile) (void)hipFree(g->dtile);
    delete g;
}

int pf_grid_sizes(const pf_grid *g, int64_t *nb, int64_t *nnz_y, int64_t *nnz_j, int32_t *ngrids) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (nb) *nb = g->nb;
    if (nnz_y) *nnz_y = g->nnz_y;
    if (nnz_j) *nnz_j = 4 * g->nnz_y;
    if (ngrids) *ngrids = g->ngrids;
    return PF_OK;
}

int pf_pattern_sizes(const pf_grid *g, int64_t *nnz_y, int64_t *nnz_j) {
    return pf_grid_sizes(g, nullptr, nnz_y, nnz_j, nullptr);
}

int pf_grid_offsets(const pf_grid *g, int64_t *y_off, int64_t *j_off) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    for (int32_t k = 0; k <= g->ngrids; ++k) {
        if (y_off) y_off[k] = g->y_off[k];
        if (j_off) j_off[k] = 4 * g->y_off[k];
    }
    return PF_OK;
}

int pf_pattern_export(const pf_grid *g, int32_t *y_rowptr, int32_t *y_col, int32_t *j_rowptr, int32_t *j_col) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    int64_t yr = 0, yc = 0, jr = 0, jc = 0;
    for (int32_t k = 0; k < g->ngrids; ++k) {
        const int32_t b0 = g->bus_off[k], b1 = g->bus_off[k + 1], nbg = b1 - b0;
        const int32_t s0 = g->yrow[b0];
        const int32_t nnzg = g->yrow[b1] - s0;
        for (int32_t i = b0; i <= b1; ++i) {
            if (y_rowptr) y_rowptr[yr] = g->yrow[i] - s0;
            ++yr;
        }
        for (int32_t p = s0; p < g->yrow[b1]; ++p) {
            if (y_col) y_col[yc] = g->ycol[p] - b0;
            ++yc;
        }
        // J rows: P rows then Q rows; row i holds theta columns then v columns.
        for (int32_t half = 0; half < 2; ++half) {
            for (int32_t i = b0; i < b1; ++i) {
                int32_t a = g->yrow[i] - s0, z = g->yrow[i + 1] - s0;
                if (j_rowptr) j_rowptr[jr] = half * 2 * nnzg + 2 * a;
                ++jr;
                if (j_col) {
                    for (int32_t p = a; p < z; ++p) j_col[jc++] = g->ycol[p + s0] - b0;
                    for (int32_t p = a; p < z; ++p) j_col[jc++] = g->ycol[p + s0] - b0 + nbg;
                }
            }
        }
        if (j_rowptr) j_rowptr[jr] = 4 * nnzg;
        ++jr;
    }
    return PF_OK;
}

int pf_jacobian_map(const pf_grid *g, int32_t layout, int32_t n, const int32_t *ptr, const int32_t *idx,
                    int32_t *map) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (g->ngrids != 1) return fail(PF_EUNSUP, "pf_jacobian_map takes a handle with one grid");
    if (layout != PF_LAYOUT_CSR && layout != PF_LAYOUT_CSC) return fail(PF_EINVAL, "unknown layout");
    const int32_t nb = g->nb;
    if ((int64_t)n != 2 * (int64_t)nb) return fail(PF_EINVAL, "the target pattern must be 2 nb x 2 nb");
    if (!ptr || !idx || !map) return fail(PF_EINVAL, "NULL pointer");
    if (ptr[0] != 0) return fail(PF_EINVAL, "ptr[0] must be 0");
    for (int32_t r = 0; r < n; ++r)
        if (ptr[r + 1] < ptr[r]) return fail(PF_EINVAL, "ptr must not decrease");
    bool sorted = true;
    for (int32_t r = 0; r < n; ++r)
        for (int32_t q = ptr[r]; q < ptr[r + 1]; ++q) {
            if (idx[q] < 0 || idx[q] >= n) return fail(PF_EINVAL, "index out of range in the target pattern");
            if (q > ptr[r] && idx[q] <= idx[q - 1]) sorted = false;
        }
    // Position of (major, minor) in the target: major = row (CSR) or column
    // (CSC); binary search when every segment ascends, else a linear scan.
    auto find = [&](int32_t major, int32_t minor) -> int32_t {
        int32_t a = ptr[major], z = ptr[major + 1];
        if (sorted) {
            while (a < z) {
                const int32_t m = a + (z - a) / 2;
                if (idx[m] < minor)
                    a = m + 1;
                else
                    z = m;
            }
            return (a < ptr[major + 1] && idx[a] == minor) ? a : -1;
        }
        for (int32_t q = a; q < z; ++q)
            if (idx[q] == minor) return q;
        return -1;
    };
    // Our entries in the exported CSR order: P rows then Q rows, each row's
    // theta columns then its v columns.
    int64_t k = 0;
    for (int32_t half = 0; half < 2; ++half)
        for (int32_t i = 0; i < nb; ++i) {
            const int32_t r = half * nb + i;
            for (int32_t part = 0; part < 2; ++part)
                for (int32_t p = g->yrow[i]; p < g->yrow[i + 1]; ++p) {
                    const int32_t c = g->ycol[p] + part * nb;
                    const int32_t pos = layout == PF_LAYOUT_CSR ? find(r, c) : find(c, r);
                    if (pos < 0) {
                        char msg[96];
                        std::snprintf(msg, sizeof msg, "the target pattern lacks J entry (%d, %d)", r, c);
                        return fail(PF_EINVAL, msg);
                    }
                    map[k++] = pos;
                }
        }
    return PF_OK;
}

int pf_set_schedule(pf_grid *g, int32_t tile_items, int32_t states_per_block, int32_t order) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (tile_items != 64 && tile_items != 128 && tile_items != 256 && tile_items != 512)
        return fail(PF_EINVAL, "tile_items must be 64, 128, 256 or 512");
    if (states_per_block < 0) return fail(PF_EINVAL, "states_per_block must be >= 0");
    if (order != PF_ORDER_AUTO && order != PF_ORDER_TILE_MAJOR && order != PF_ORDER_STATE_MAJOR &&
        order != PF_ORDER_GROUPED)
        return fail(PF_EINVAL, "unknown order");
    if (tile_items != g->tile_items) {
        // new tiles on the host and device; on failure the old ones stay
        std::vector<pf::TileDesc> old_t, old_yt;
        try {
            old_t = g->tiles;
            old_yt = g->ytiles;
        } catch (const std::bad_alloc &) {
            return fail(PF_ENOMEM, "host allocation failed");
        }
        const int32_t old_items = g->tile_items;
        int st = PF_OK;
        try {
            g->tile_items = tile_items;
            build_tiles(g, tile_items);
            st = upload_tiles(g);
        } catch (const std::bad_alloc &) {
            st = fail(PF_ENOMEM, "host allocation failed");
        }
        if (st != PF_OK) {
            g->tiles.swap(old_t);
            g->ytiles.swap(old_yt);
            g->tile_items = old_items;
            return st;
        }
    }
    g->states_per_block = states_per_block;
    g->order = order;
    ++g->sched_gen;
    return PF_OK;
}

int pf_get_schedule(const pf_grid *g, int32_t *tile_items, int32_t *states_per_block, int32_t *order,
                    int32_t *ntiles) {
    g_err.clear();
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (tile_items) *tile_items = g->tile_items;
    if (states_per_block) *states_per_block = g->states_per_block;
    if (order) *order = g->order;
    if (ntiles) *ntiles = (int32_t)g->tiles.size();
    return PF_OK;
}

}  // extern "C"

namespace {

int check_eval(const pf_grid *g, int32_t nstate) {
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (g->host_only) return fail(PF_ESTATE, "handle was built with PF_BUILD_HOST_ONLY");
    if (nstate < 0) return fail(PF_EINVAL, "nstate must be >= 0");
    if ((int64_t)nstate * 4 * g->nnz_y > INT64_MAX / 16) return fail(PF_EUNSUP, "batch too large");
    return PF_OK;
}

bool is_jacobian(int kind) {
    return kind == pf::K_EW_SJ || kind == pf::K_YB_SJ || kind == pf::K_EW_SJ_CSC || kind == pf::K_YB_SJ_CSC;
}

// Bytes of tile tables a launch walks per state: about 24 per lane and 24
// per bus.
int64_t table_bytes(const pf_grid *g, int kind) {
    const bool yb = kind == pf::K_YB_S || kind == pf::K_YB_SJ || kind == pf::K_YB_SJ_CSC;
    const int64_t nt = std::max<int64_t>(1, (int64_t)(yb ? g->ytiles : g->tiles).size());
    return 24 * nt * (int64_t)g->tile_items + 24 * (int64_t)g->nb;
}

// Work order of a launch (pf::WO_*).  Automatic: for Jacobian launches
// state-major while the tables fit in one XCD's L2 (2 MB of its 4 MB), so
// the tiles of a state write neighbouring parts of J together, else grouped
// (each XCD walks its own eighth of the tiles state by state: their tables
// stay in its L2 while neighbouring workgroups still write neighbouring J
// rows); tile-major for injections and the adjoint (the state chunks of one
// tile run on one XCD, so its tables come from that XCD's L2 after the
// first chunk).
int work_order(const pf_grid *g, int kind) {
    switch (g->order) {
        case PF_ORDER_TILE_MAJOR:
            return pf::WO_TILE;
        case PF_ORDER_STATE_MAJOR:
            return pf::WO_STATE;
        case PF_ORDER_GROUPED:
            return pf::WO_GROUPED;
        default:
            if (!is_jacobian(kind)) return pf::WO_TILE;
            return table_bytes(g, kind) <= ((int64_t)2 << 20) ? pf::WO_STATE : pf::WO_GROUPED;
    }
}

// States per workgroup.  A workgroup keeps its tile's record constants in
// registers and walks its states one after another, so fewer, longer
// workgroups read the constants fewer times, while more, shorter workgroups
// keep more of every state's output stream in flight.  The automatic choice
// takes at most 2 states per workgroup for Jacobian launches (their time is
// the J stream: 8 nnzJ bytes per state against a few bytes of constants),
// 1 when the tables a workgroup's XCD walks stay in its 4 MB L2 between
// states (an eighth of them in the grouped order, all otherwise), and at
// most 8 for injections (small per-state outputs, so reusing the constants
// pays); fewer when the tiles alone would leave part of one round of
// resident workgroups empty (it then splits each tile's states into about
// resident capacity / tiles chunks).  The adjoint takes exactly that split,
// however many states it gives a workgroup: its record constants (both
// ends' couplings) are the heaviest, and one round of workgroups that each
// walk their share of the states measured fastest.
int auto_states_per_block(const pf_grid *g, int kind, int32_t nstate) {
    if (g->states_per_block > 0) return std::min<int32_t>(g->states_per_block, std::max(nstate, 1));
    if (nstate <= 1) return 1;
    const bool yb = kind == pf::K_YB_S || kind == pf::K_YB_SJ || kind == pf::K_YB_SJ_CSC;
    const int64_t nt = std::max<int64_t>(1, (int64_t)(yb ? g->ytiles : g->tiles).size());
    int per_cu = pf::resident_blocks_per_cu(kind, g->tile_items, g->has_parallel);
    if (per_cu <= 0) per_cu = 4;
    const int64_t capacity = (int64_t)std::max(g->num_cus, 1) * per_cu;
    int64_t chunks = std::max<int64_t>(1, capacity / nt);
    chunks = std::min<int64_t>(chunks, nstate);
    const int fill = (int)((nstate + chunks - 1) / chunks);
    if (is_jacobian(kind)) {
        // One state per workgroup (the lean single-state kernel) when the
        // tile tables an XCD walks stay in its L2 across states (an eighth
        // of them in the grouped order); else two.
        int64_t tb = table_bytes(g, kind);
        if (work_order(g, kind) == pf::WO_GROUPED) tb /= 8;
        return std::min(fill, tb <= ((int64_t)2 << 20) ? 1 : 2);
    }
    if (kind == pf::K_EW_VJP) return fill;
    return std::min(fill, 8);
}

// The two-phase baseline with the given scratch (ten doubles per record).
int run_two_phase(const pf_grid *g, int32_t nstate, const double *vm, const double *va, double *p, double *q,
                  double *jval, bool pre, double *scr, void *stream) {
    if (nstate == 0) return PF_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    pf::DevTwoPhase d = g->tp;
    d.ydslot = g->lanes.ydslot;
    d.scr = scr;
    e = pf::launch_two_phase(d, nstate, 4 * g->nnz_y, vm, va, p, q, jval, pre, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

int run(const pf_grid *g, pf::Launch &L, void *stream) {
    L.tile_items = g->tile_items;
    L.has_parallel = g->has_parallel;
    L.states_per_block = auto_states_per_block(g, L.kind, L.nstate);
    L.order = work_order(g, L.kind);
    if (L.nstate == 0) return PF_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    e = pf::launch_eval(g->dev, L, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_ybus(pf_grid *g, double *y_re, double *y_im, void *stream) {
    g_err.clear();
    int st = check_eval(g, 1);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pf::DevSetup &d = g->setup;
    hipError_t e = pf::launch_ybus_assemble(d, s);
    if (e == hipSuccess) e = pf::launch_lane_fill(g->lanes, false, s);
    if (e != hipSuccess) return hip_fail(e, "Ybus assembly launch");
    if (y_re) {
        e = hipMemcpyAsync(y_re, g->dev.yre, g->nnz_y * sizeof(double), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy of Ybus real parts");
    }
    if (y_im) {
        e = hipMemcpyAsync(y_im, g->dev.yim, g->nnz_y * sizeof(double), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy of Ybus imaginary parts");
    }
    g->ybus_valid = true;
    return PF_OK;
}

int pf_injections_elementwise(const pf_grid *g, int32_t nstate, const double *vm, const double *va, double *p,
                              double *q, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (nstate > 0 && (!vm || !va || !p || !q)) return fail(PF_EINVAL, "NULL state or output pointer");
    pf::Launch L{};
    L.kind = pf::K_EW_S;
    L.nstate = nstate;
    L.vm = vm;
    L.va = va;
    L.p = p;
    L.q = q;
    return run(g, L, stream);
}

int pf_injections_ybus(const pf_grid *g, int32_t nstate, const double *vm, const double *va, double *p, double *q,
                       void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (!g->ybus_valid) return fail(PF_ESTATE, "pf_ybus has not been called on this handle");
    if (nstate > 0 && (!vm || !va || !p || !q)) return fail(PF_EINVAL, "NULL state or output pointer");
    pf::Launch L{};
    L.kind = pf::K_YB_S;
    L.nstate = nstate;
    L.vm = vm;
    L.va = va;
    L.p = p;
    L.q = q;
    return run(g, L, stream);
}

int pf_jacobian_values(const pf_grid *g, int32_t method, int32_t nstate, const double *vm, const double *va,
                       double *p, double *q, double *jval, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    const bool csc = (method & PF_JAC_CSC) != 0;
    const bool pre = (method & PF_EW_PRECOMPUTED) != 0;
    method &= ~(PF_JAC_CSC | PF_EW_PRECOMPUTED);
    if (method != PF_METHOD_ELEMENTWISE && method != PF_METHOD_YBUS && method != PF_METHOD_ELEMENTWISE_TWO_PHASE &&
        method != PF_METHOD_ELEMENTWISE_ATOMIC)
        return fail(PF_EINVAL, "unknown method");
    if (csc && method != PF_METHOD_ELEMENTWISE && method != PF_METHOD_YBUS)
        return fail(PF_EUNSUP, "the CSC order is available with PF_METHOD_ELEMENTWISE and PF_METHOD_YBUS");
    if (pre && method != PF_METHOD_ELEMENTWISE_TWO_PHASE && method != PF_METHOD_ELEMENTWISE_ATOMIC)
        return fail(PF_EUNSUP, "PF_EW_PRECOMPUTED applies to the two-phase and copy-add methods");
    if (method == PF_METHOD_YBUS && !g->ybus_valid)
        return fail(PF_ESTATE, "pf_ybus has not been called on this handle");
    if (nstate > 0 && (!vm || !va || !jval)) return fail(PF_EINVAL, "NULL state or Jacobian pointer");
    if ((p == nullptr) != (q == nullptr)) return fail(PF_EINVAL, "p and q must both be given or both be NULL");
    if (reinterpret_cast<uintptr_t>(jval) % 16) return fail(PF_EINVAL, "jval must be 16-byte aligned");
    if (method == PF_METHOD_ELEMENTWISE_ATOMIC) {
        if (nstate == 0) return PF_OK;
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
        pf::DevTwoPhase d = g->tp;
        d.ydslot = g->lanes.ydslot;
        e = pf::launch_copy_add(d, nstate, 4 * g->nnz_y, vm, va, p, q, jval, pre, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return PF_OK;
    }
    if (method == PF_METHOD_ELEMENTWISE_TWO_PHASE)
        return run_two_phase(g, nstate, vm, va, p, q, jval, pre, g->tp.scr, stream);
    pf::Launch L{};
    L.kind = method == PF_METHOD_ELEMENTWISE ? (csc ? pf::K_EW_SJ_CSC : pf::K_EW_SJ)
                                             : (csc ? pf::K_YB_SJ_CSC : pf::K_YB_SJ);
    L.nstate = nstate;
    L.vm = vm;
    L.va = va;
    L.p = p;
    L.q = q;
    L.jval = jval;
    return run(g, L, stream);
}

int pf_jacobian_two_phase_static(const pf_grid *g, int32_t method, int32_t nstate, const double *vm,
                                 const double *va, double *p, double *q, double *jval, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if ((method & ~PF_EW_PRECOMPUTED) != PF_METHOD_ELEMENTWISE_TWO_PHASE)
        return fail(PF_EINVAL, "method must be PF_METHOD_ELEMENTWISE_TWO_PHASE, optionally | PF_EW_PRECOMPUTED");
    const bool pre = (method & PF_EW_PRECOMPUTED) != 0;
    if (g->nitems > pf::kStaticScratchRecords)
        return fail(PF_EUNSUP, "the grid has " + std::to_string(g->nitems) + " records (nb + 2 nl); the static scratch "
                               "holds at most " + std::to_string(pf::kStaticScratchRecords) +
                               " (use pf_jacobian_values)");
    if (nstate > 0 && (!vm || !va || !jval)) return fail(PF_EINVAL, "NULL state or Jacobian pointer");
    if ((p == nullptr) != (q == nullptr)) return fail(PF_EINVAL, "p and q must both be given or both be NULL");
    if (reinterpret_cast<uintptr_t>(jval) % 16) return fail(PF_EINVAL, "jval must be 16-byte aligned");
    if (nstate == 0) return PF_OK;
    double *scr = nullptr;
    const hipError_t e = pf::static_scratch(g->device, &scr);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    return run_two_phase(g, nstate, vm, va, p, q, jval, pre, scr, stream);
}

static_assert(PF_PHASOR_SPLIT == pf::PH_SPLIT && PF_PHASOR_INTERLEAVED == pf::PH_INTERLEAVED,
              "public phasor layouts name the kernels' phasor sources");

int pf_phasors(const pf_grid *g, int32_t layout, int32_t nstate, const double *vm, const double *va, double *ph,
               void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (layout != PF_PHASOR_SPLIT && layout != PF_PHASOR_INTERLEAVED) return fail(PF_EINVAL, "unknown phasor layout");
    if (nstate == 0) return PF_OK;
    if (!vm || !va || !ph) return fail(PF_EINVAL, "NULL state or phasor pointer");
    if (layout == PF_PHASOR_INTERLEAVED && reinterpret_cast<uintptr_t>(ph) % 16)
        return fail(PF_EINVAL, "interleaved phasors must be 16-byte aligned");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    e = pf::launch_phasor(layout, (int64_t)nstate * g->nb, vm, va, ph, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

int pf_ybus_from_phasors(const pf_grid *g, int32_t layout, int32_t nstate, const double *ph, double *p, double *q,
                         double *jval, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (layout != PF_PHASOR_SPLIT && layout != PF_PHASOR_INTERLEAVED) return fail(PF_EINVAL, "unknown phasor layout");
    if (!g->ybus_valid) return fail(PF_ESTATE, "pf_ybus has not been called on this handle");
    if ((p == nullptr) != (q == nullptr)) return fail(PF_EINVAL, "p and q must both be given or both be NULL");
    if (nstate > 0 && !ph) return fail(PF_EINVAL, "NULL phasor pointer");
    if (nstate > 0 && !jval && !p) return fail(PF_EINVAL, "nothing to write: p, q and jval are NULL");
    if (layout == PF_PHASOR_INTERLEAVED && reinterpret_cast<uintptr_t>(ph) % 16)
        return fail(PF_EINVAL, "interleaved phasors must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(jval) % 16) return fail(PF_EINVAL, "jval must be 16-byte aligned");
    pf::Launch L{};
    L.kind = jval ? pf::K_YB_SJ : pf::K_YB_S;
    L.nstate = nstate;
    L.phasor = layout;
    L.ph = ph;
    L.p = p;
    L.q = q;
    L.jval = jval;
    return run(g, L, stream);
}

int pf_jacobian_scatter(const pf_grid *g, int32_t nstate, const double *jval, const int32_t *map, int64_t out_nnz,
                        double *out, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (out_nnz < 0 || out_nnz > INT32_MAX) return fail(PF_EINVAL, "out_nnz must lie in [0, 2^31 - 1]");
    if (nstate == 0 || 4 * g->nnz_y == 0) return PF_OK;
    if (!jval || !map || !out) return fail(PF_EINVAL, "NULL pointer");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    e = pf::launch_jscatter(nstate, 4 * g->nnz_y, jval, map, out_nnz, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

int pf_debug_fail_allocs(int32_t n) {
    g_err.clear();
    if (n < 0) return fail(PF_EINVAL, "n must be >= 0");
    g_fail_allocs.store(n);
    return PF_OK;
}

int pf_stream_copy(const double *src, double *dst, int64_t n, void *stream) {
    g_err.clear();
    if (n < 0) return fail(PF_EINVAL, "n must be >= 0");
    if (n == 0) return PF_OK;
    if (!src || !dst) return fail(PF_EINVAL, "NULL buffer");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u)
        return fail(PF_EINVAL, "buffers must be 16-byte aligned");
    if (src < dst + n && dst < src + n) return fail(PF_EINVAL, "buffers overlap");
    const hipError_t e = pf::launch_stream_copy(src, dst, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

int pf_branch_flows(const pf_grid *g, int32_t nstate, const double *vm, const double *va, double *pf, double *qf,
                    double *pt, double *qt, double *jac, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (nstate == 0 || g->nl == 0) return PF_OK;  // nothing to write
    if (!vm || !va || !pf || !qf || !pt || !qt) return fail(PF_EINVAL, "NULL state or output pointer");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    e = pf::launch_flows(g->tp, nstate, vm, va, pf, qf, pt, qt, jac, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PF_OK;
}

int pf_injections_vjp(const pf_grid *g, int32_t nstate, const double *vm, const double *va, const double *lam_p,
                      const double *lam_q, double *g_vm, double *g_va, void *stream) {
    g_err.clear();
    int st = check_eval(g, nstate);
    if (st) return st;
    if (nstate > 0 && (!vm || !va || !lam_p || !lam_q || !g_vm || !g_va))
        return fail(PF_EINVAL, "NULL state, seed or output pointer");
    pf::Launch L{};
    L.kind = pf::K_EW_VJP;
    L.nstate = nstate;
    L.vm = vm;
    L.va = va;
    L.lp = lam_p;
    L.lq = lam_q;
    L.gvm = g_vm;
    L.gva = g_va;
    return run(g, L, stream);
}

}  // extern "C"

// ---------------------------------------------------------------- graphs

struct pf_graph {
    const pf_grid *g = nullptr;
    uint64_t gen = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int op_kind(const pf_op &o) {
    switch (o.op) {
        case PF_OP_INJECTIONS:
            return o.method == PF_METHOD_YBUS ? pf::K_YB_S : pf::K_EW_S;
        case PF_OP_JACOBIAN:
            if (o.method & PF_JAC_CSC)
                return (o.method & ~PF_JAC_CSC) == PF_METHOD_YBUS ? pf::K_YB_SJ_CSC : pf::K_EW_SJ_CSC;
            return o.method == PF_METHOD_YBUS ? pf::K_YB_SJ : pf::K_EW_SJ;
        default:
            return pf::K_EW_VJP;
    }
}

int record_op(const pf_grid *g, const pf_op &o, void *stream) {
    switch (o.op) {
        case PF_OP_INJECTIONS:
            if (o.method == PF_METHOD_ELEMENTWISE)
                return pf_injections_elementwise(g, o.nstate, o.vm, o.va, o.out_a, o.out_b, stream);
            if (o.method == PF_METHOD_YBUS) return pf_injections_ybus(g, o.nstate, o.vm, o.va, o.out_a, o.out_b, stream);
            return fail(PF_EINVAL, "unknown method");
        case PF_OP_JACOBIAN:
            return pf_jacobian_values(g, o.method, o.nstate, o.vm, o.va, o.out_a, o.out_b, o.jval, stream);
        case PF_OP_VJP:
            return pf_injections_vjp(g, o.nstate, o.vm, o.va, o.lam_p, o.lam_q, o.out_a, o.out_b, stream);
        default:
            return fail(PF_EINVAL, "unknown op");
    }
}

}  // namespace

extern "C" {

int pf_graph_create(const pf_grid *g, const pf_op *ops, int32_t nops, pf_graph **out) {
    g_err.clear();
    if (!out) return fail(PF_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!g) return fail(PF_EINVAL, "NULL handle");
    if (!ops || nops <= 0) return fail(PF_EINVAL, "need at least one op");
    if (g->host_only) return fail(PF_ESTATE, "handle was built with PF_BUILD_HOST_ONLY");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    // Resolve every launch shape before recording, so that nothing but
    // kernel launches happens while the stream is captured.
    for (int32_t k = 0; k < nops; ++k)
        if (ops[k].nstate > 0) auto_states_per_block(g, op_kind(ops[k]), ops[k].nstate);
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    int st = PF_OK;
    for (int32_t k = 0; k < nops && st == PF_OK; ++k) st = record_op(g, ops[k], s);
    std::string err = g_err;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    (void)hipStreamDestroy(s);
    if (st != PF_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != PF_OK) return fail(st, err);
        return hip_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    pf_graph *gr = new (std::nothrow) pf_graph;
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(PF_ENOMEM, "host allocation failed");
    }
    gr->g = g;
    gr->gen = g->sched_gen;
    gr->graph = graph;
    gr->exec = exec;
    *out = gr;
    return PF_OK;
}

int pf_graph_launch(const pf_graph *gr, void *stream) {
    g_err.clear();
    if (!gr) return fail(PF_EINVAL, "NULL graph");
    if (gr->gen != gr->g->sched_gen) return fail(PF_ESTATE, "the grid's schedule changed since the graph was recorded");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != gr->g->device) return fail(PF_EINVAL, "current HIP device differs from the handle's device");
    e = hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return PF_OK;
}

void pf_graph_free(pf_graph *gr) {
    if (!gr) return;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner

namespace {

// Time per call (microseconds) of `op` under the handle's current schedule:
// a graph of `reps` copies of the op replayed untimed for warm_ms, then the
// median over `samples` replays timed by HIP events on stream `st`.
int time_op(const pf_grid *g, const pf_op &op, int32_t reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
            double *us) {
    std::vector<pf_op> ops(reps, op);
    pf_graph *gr = nullptr;
    int rc = pf_graph_create(g, ops.data(), reps, &gr);
    if (rc) return rc;
    constexpr double warm_ms = 10.0;
    constexpr int samples = 3;
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = hipSuccess;
    do {
        rc = pf_graph_launch(gr, st);
        if (rc) break;
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
    } while (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() < warm_ms);
    double t[samples];
    for (int k = 0; k < samples && !rc && e == hipSuccess; ++k) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) rc = pf_graph_launch(gr, st);
        if (!rc && e == hipSuccess) e = hipEventRecord(e1, st);
        if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[k] = 1e3 * (double)ms / reps;
    }
    pf_graph_free(gr);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotuner timing");
    std::sort(t, t + samples);
    *us = t[samples / 2];
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_autotune(pf_grid *g, const pf_op *op, int32_t ncand, const int32_t *cand, int32_t reps, int32_t *best,
                double *best_us, int32_t *tried) {
    g_err.clear();
    if (!g || !op || !best) return fail(PF_EINVAL, "NULL handle, op or output");
    if (g->host_only) return fail(PF_ESTATE, "handle was built with PF_BUILD_HOST_ONLY");
    if (ncand < 0 || (ncand > 0 && !cand)) return fail(PF_EINVAL, "ncand < 0, or candidates missing");
    if (reps < 1 || reps > 1000) return fail(PF_EINVAL, "reps must lie in [1, 1000]");
    if (op->nstate < 1) return fail(PF_EINVAL, "the op needs at least one state");
    std::vector<int32_t> c;
    try {
        if (ncand > 0) {
            c.assign(cand, cand + 3 * (size_t)ncand);
        } else {
            const int32_t tiles[4] = {64, 128, 256, 512};
            const int32_t spbs[8] = {0, 1, 2, 4, 8, 16, 32, 64};
            for (int32_t t : tiles) {
                if (op->nstate == 1) {
                    c.insert(c.end(), {t, 1, PF_ORDER_TILE_MAJOR});
                    continue;
                }
                for (int32_t s : spbs)
                    if (s <= op->nstate)
                        for (int32_t o : {PF_ORDER_TILE_MAJOR, PF_ORDER_STATE_MAJOR, PF_ORDER_GROUPED})
                            c.insert(c.end(), {t, s, o});
            }
        }
    } catch (const std::bad_alloc &) {
        return fail(PF_ENOMEM, "host allocation failed");
    }
    const int32_t n = (int32_t)(c.size() / 3);
    const int32_t orig[3] = {g->tile_items, g->states_per_block, g->order};
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = e == hipSuccess ? PF_OK : hip_fail(e, "autotuner stream or events");
    int32_t bi = -1;
    double bt = 0.0;
    for (int32_t k = 0; k < n && rc == PF_OK; ++k) {
        rc = pf_set_schedule(g, c[3 * k], c[3 * k + 1], c[3 * k + 2]);
        double us = 0.0;
        if (rc == PF_OK) rc = time_op(g, *op, reps, st, e0, e1, &us);
        if (rc == PF_OK && (bi < 0 || us < bt)) {
            bi = k;
            bt = us;
        }
    }
    std::string err = g_err;
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (rc != PF_OK || bi < 0) {
        (void)pf_set_schedule(g, orig[0], orig[1], orig[2]);  // back to where the handle started
        return rc != PF_OK ? fail(rc, err) : fail(PF_EINVAL, "no candidate schedules");
    }
    rc = pf_set_schedule(g, c[3 * bi], c[3 * bi + 1], c[3 * bi + 2]);
    if (rc) return rc;
    best[0] = c[3 * bi];
    best[1] = c[3 * bi + 1];
    best[2] = c[3 * bi + 2];
    if (best_us) *best_us = bt;
    if (tried) *tried = n;
    return PF_OK;
}

}  // extern "C"
