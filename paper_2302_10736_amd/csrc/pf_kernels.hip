// HIP kernels for gfx950 (MI355X): nodal power injections, polar Jacobian
// values and their adjoint, by the element-wise method (Section II.B,
// eqs. (5)-(7); Section IV.C) and by the Ybus method (Section II.A,
// eqs. (1)-(4); Section IV.B).
//
// Work decomposition (both methods)
// ---------------------------------
// Records are sorted by (bus, neighbour, branch).  A tile is a run of whole
// bus rows holding at most NT records (NT = workgroup size); one thread
// owns one record.  Per voltage state a workgroup
//   1. evaluates every record of the tile (one branch end, or the bus shunt,
//      for the element-wise method; one Ybus nonzero for the Ybus method),
//   2. reduces the records of each row in LDS, sequentially in record order,
//      by the thread that owns the row's diagonal record,
//   3. assembles the tile's Jacobian rows in LDS and writes them out with
//      contiguous 16-byte stores: a tile's rows are contiguous in the CSR
//      value array, once for the P rows and once for the Q rows.
// There are no atomics; every sum has a fixed order set by the pattern, so
// results do not depend on the tile size or the number of states per
// workgroup.  A row with more than NT records forms a tile of its own,
// walked in chunks with the same sequential order.
//
// Record constants (from the branch data, computed once at setup):
//   A + jC  own-end admittance: Re/Im of (y_h + y_hk)/m^2 at the from end,
//           of (y_k + y_hk) at the to end, of (g + jb) for a bus shunt;
//   G + jB  coupling admittance of this end: -y_hk e^{j phi}/m at the from
//           end, -y_hk e^{-j phi}/m at the to end, 0 for a bus shunt;
//   Gr, Br  coupling admittance of the other end of the same branch.
// With t = theta_i - theta_j, w = v_i v_j, alpha = G cos t + B sin t,
// beta = G sin t - B cos t, one record contributes
//   P = v_i^2 A + w alpha,   Q = -v_i^2 C + w beta,
// i.e. eq. (5) (from end) or eq. (6) (to end) split into real and imaginary
// parts, and its eight partial derivatives
//   dP/dtheta_i = -w beta    dP/dtheta_j =  w beta
//   dP/dv_i = 2 v_i A + v_j alpha    dP/dv_j = v_i alpha
//   dQ/dtheta_i =  w alpha   dQ/dtheta_j = -w alpha
//   dQ/dv_i = -2 v_i C + v_j beta    dQ/dv_j = v_i beta
// (the 16 partials of one branch are the 8 + 8 of its two ends).

#include <hip/hip_runtime.h>

#include "pf_internal.h"

namespace pf {
namespace {

constexpr int kXcds = 8;

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of work items so that neighbouring tiles, and all state
// chunks of one tile, share one L2.
__device__ __forceinline__ int work_index(int nblocks) {
    const int b = blockIdx.x;
    const int per = nblocks / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

struct Tile {
    int r0, nrows;  // first row, number of rows
    int i0, n;      // first record, number of records
    int s0, ns;     // first slot, number of slots
    int64_t jp, jq;  // offsets of the tile's P rows and Q rows in one state's J values
};

__device__ __forceinline__ Tile tile_of(const DevGrid &g, int t) {
    Tile c;
    c.r0 = g.tile_row[t];
    const int r1 = g.tile_row[t + 1];
    c.nrows = r1 - c.r0;
    c.i0 = g.irow[c.r0];
    c.n = g.irow[r1] - c.i0;
    c.s0 = g.yrow[c.r0];
    c.ns = g.yrow[r1] - c.s0;
    const int gi = g.tile_grid[t];
    // Grid gi's J values start at 4 yoff[gi]; its P rows hold 2 nnz_y(gi)
    // values, so row i's P part starts at 2 yoff[gi] + 2 yrow[i] and its Q
    // part at 2 yoff[gi+1] + 2 yrow[i].
    c.jp = 2 * g.yoff[gi] + 2 * (int64_t)c.s0;
    c.jq = 2 * g.yoff[gi + 1] + 2 * (int64_t)c.s0;
    return c;
}

// Local row pointers of a packed tile (records and slots) into LDS.
template <int NT>
__device__ __forceinline__ void stage_rows(const DevGrid &g, const Tile &c, int *s_irow, int *s_yrow) {
    for (int q = threadIdx.x; q <= c.nrows; q += NT) {
        s_irow[q] = g.irow[c.r0 + q] - c.i0;
        s_yrow[q] = g.yrow[c.r0 + q] - c.s0;
    }
}

// Largest q in [0, nrows) with rowptr[q] <= k.
__device__ __forceinline__ int row_of(int k, const int *rowptr, int nrows) {
    int lo = 0, hi = nrows - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rowptr[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cconj(Cx a) { return {a.re, -a.im}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }

// Copy a staged tile of J rows (LDS) to global memory with 16-byte stores.
template <int NT>
__device__ __forceinline__ void write_jrows(const Tile &c, const double *s_J, double *Js) {
    const double2 *src = reinterpret_cast<const double2 *>(s_J);
    double2 *dp = reinterpret_cast<double2 *>(Js + c.jp);
    double2 *dq = reinterpret_cast<double2 *>(Js + c.jq);
    for (int q = threadIdx.x; q < c.ns; q += NT) {
        dp[q] = src[q];
        dq[q] = src[NT + q];
    }
}

// One element-wise record: power and the eight partials (see file header).
struct EwOut {
    double p, q;               // record's contribution to P_i, Q_i
    double dpt, dpv, dqt, dqv;  // own-bus partials (diagonal slot)
    double rpt, rpv, rqt, rqv;  // remote-bus partials (slot (i, j))
};

__device__ __forceinline__ EwOut ew_record(double vi, double ti, double vj, double tj, double A, double C, double G,
                                           double B) {
    double sn, cs;
    sincos(ti - tj, &sn, &cs);
    const double w = vi * vj;
    const double al = G * cs + B * sn;
    const double be = G * sn - B * cs;
    EwOut o;
    o.p = vi * vi * A + w * al;
    o.q = w * be - vi * vi * C;
    o.dpt = -(w * be);
    o.dpv = 2.0 * vi * A + vj * al;
    o.dqt = w * al;
    o.dqv = vj * be - 2.0 * vi * C;
    o.rpt = w * be;
    o.rpv = vi * al;
    o.rqt = -(w * al);
    o.rqv = vi * be;
    return o;
}

// ===================================================================
// Element-wise injections and Jacobian values.
template <int NT, bool PAR, bool WITH_J>
__global__ void __launch_bounds__(NT)
    k_ew(DevGrid g, int nstate, int spb, int nchunk, const double *__restrict__ vm, const double *__restrict__ va,
         double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    __shared__ int s_irow[NT + 1];
    __shared__ int s_yrow[NT + 1];
    constexpr int NV = WITH_J ? 6 : 2;        // values per record kept for the row sums
    constexpr int NR = (WITH_J && PAR) ? NT : 1;  // remote partials kept for slot sums
    __shared__ double s_val[NV][NT];
    __shared__ double s_pq[2][NT];
    __shared__ __align__(16) double s_J[WITH_J ? 4 * NT : 2];
    __shared__ double s_rem[4][NR];
    __shared__ int s_slot[NR];
    __shared__ int s_diag;

    const int W = g.ntiles * nchunk;
    const int w = work_index(gridDim.x);
    if (w >= W) return;
    const int t = w / nchunk;
    const int sb = (w - t * nchunk) * spb;
    const int se = min(nstate, sb + spb);
    const Tile c = tile_of(g, t);
    const int k = threadIdx.x;
    const size_t nb = (size_t)g.nb;

    if (c.n > NT) {
        // ---- one long row, walked in chunks of NT records by thread 0's sequential sums
        const int i = c.r0;
        const int d = c.ns;  // slots in the row
        if (k == 0) s_diag = -1;  // set by the shunt record's thread below; same in every state
        __syncthreads();
        for (int s = sb; s < se; ++s) {
            const size_t so = (size_t)s * nb;
            double *Js = WITH_J ? J + (size_t)s * (size_t)g.nnz_j : nullptr;
            double acc[6] = {0, 0, 0, 0, 0, 0};
            double racc[4] = {0, 0, 0, 0};
            int cur = -1;
            for (int base = 0; base < c.n; base += NT) {
                const bool live = base + k < c.n;
                if (live) {
                    const int e = c.i0 + base + k;
                    const int j = g.nbr[e];
                    const EwOut o = ew_record(vm[so + i], va[so + i], vm[so + j], va[so + j], g.A[e], g.C[e],
                                              g.G[e], g.B[e]);
                    s_val[0][k] = o.p;
                    s_val[1][k] = o.q;
                    if constexpr (WITH_J) {
                        s_val[2][k] = o.dpt;
                        s_val[3][k] = o.dpv;
                        s_val[4][k] = o.dqt;
                        s_val[5][k] = o.dqv;
                        // long rows reuse the J stage as remote-partial storage
                        s_J[0 * NT + k] = o.rpt;
                        s_J[1 * NT + k] = o.rpv;
                        s_J[2 * NT + k] = o.rqt;
                        s_J[3 * NT + k] = o.rqv;
                        const int ls = (PAR ? g.slot[e] : e) - c.s0;
                        s_irow[k] = ls;
                        if (j == i) s_diag = ls;
                    }
                }
                __syncthreads();
                if (k == 0) {
                    const int m = min(NT, c.n - base);
                    for (int q = 0; q < m; ++q) {
                        acc[0] += s_val[0][q];
                        acc[1] += s_val[1][q];
                        if constexpr (WITH_J) {
                            acc[2] += s_val[2][q];
                            acc[3] += s_val[3][q];
                            acc[4] += s_val[4][q];
                            acc[5] += s_val[5][q];
                            const int ls = s_irow[q];
                            if (ls != cur) {
                                if (cur >= 0 && cur != s_diag) {
                                    Js[c.jp + cur] = racc[0];
                                    Js[c.jp + d + cur] = racc[1];
                                    Js[c.jq + cur] = racc[2];
                                    Js[c.jq + d + cur] = racc[3];
                                }
                                cur = ls;
                                racc[0] = racc[1] = racc[2] = racc[3] = 0.0;
                            }
                            racc[0] += s_J[0 * NT + q];
                            racc[1] += s_J[1 * NT + q];
                            racc[2] += s_J[2 * NT + q];
                            racc[3] += s_J[3 * NT + q];
                        }
                    }
                }
                __syncthreads();
            }
            if (k == 0) {
                if (P) {
                    P[so + i] = acc[0];
                    Q[so + i] = acc[1];
                }
                if constexpr (WITH_J) {
                    if (cur >= 0 && cur != s_diag) {
                        Js[c.jp + cur] = racc[0];
                        Js[c.jp + d + cur] = racc[1];
                        Js[c.jq + cur] = racc[2];
                        Js[c.jq + d + cur] = racc[3];
                    }
                    const int ld = s_diag;
                    Js[c.jp + ld] = acc[2];
                    Js[c.jp + d + ld] = acc[3];
                    Js[c.jq + ld] = acc[4];
                    Js[c.jq + d + ld] = acc[5];
                }
            }
            __syncthreads();
        }
        return;
    }

    // ---- packed tile: whole rows, at most NT records
    stage_rows<NT>(g, c, s_irow, s_yrow);
    const bool live = k < c.n;
    int j = 0, ls = 0;
    double A = 0.0, C = 0.0, G = 0.0, B = 0.0;
    if (live) {
        const int e = c.i0 + k;
        j = g.nbr[e];
        A = g.A[e];
        C = g.C[e];
        G = g.G[e];
        B = g.B[e];
        ls = (PAR ? g.slot[e] : e) - c.s0;  // without parallel branches, slot == record
    }
    __syncthreads();
    const int row = live ? row_of(k, s_irow, c.nrows) : 0;
    const int i = c.r0 + row;
    const bool diag = live && j == i;
    const int o11 = s_yrow[row] + ls;      // J11 / J21 position inside the staged P / Q rows
    const int o12 = s_yrow[row + 1] + ls;  // J12 / J22
    if constexpr (WITH_J && PAR)
        if (live) s_slot[k] = ls;

    for (int s = sb; s < se; ++s) {
        const size_t so = (size_t)s * nb;
        if (live) {
            const EwOut o = ew_record(vm[so + i], va[so + i], vm[so + j], va[so + j], A, C, G, B);
            s_val[0][k] = o.p;
            s_val[1][k] = o.q;
            if constexpr (WITH_J) {
                s_val[2][k] = o.dpt;
                s_val[3][k] = o.dpv;
                s_val[4][k] = o.dqt;
                s_val[5][k] = o.dqv;
                if constexpr (PAR) {
                    s_rem[0][k] = o.rpt;
                    s_rem[1][k] = o.rpv;
                    s_rem[2][k] = o.rqt;
                    s_rem[3][k] = o.rqv;
                } else if (!diag) {
                    s_J[o11] = o.rpt;
                    s_J[o12] = o.rpv;
                    s_J[2 * NT + o11] = o.rqt;
                    s_J[2 * NT + o12] = o.rqv;
                }
            }
        }
        __syncthreads();
        if (diag) {
            const int a = s_irow[row], z = s_irow[row + 1];
            double sp = 0.0, sq = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
            for (int q = a; q < z; ++q) {
                sp += s_val[0][q];
                sq += s_val[1][q];
                if constexpr (WITH_J) {
                    d0 += s_val[2][q];
                    d1 += s_val[3][q];
                    d2 += s_val[4][q];
                    d3 += s_val[5][q];
                }
            }
            s_pq[0][row] = sp;
            s_pq[1][row] = sq;
            if constexpr (WITH_J) {
                s_J[o11] = d0;
                s_J[o12] = d1;
                s_J[2 * NT + o11] = d2;
                s_J[2 * NT + o12] = d3;
            }
        } else if (live) {
            if constexpr (WITH_J && PAR) {
              if (k == 0 || s_slot[k - 1] != ls) {  // first record of its slot sums the slot
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int q = k; q < c.n && s_slot[q] == ls; ++q) {
                    a0 += s_rem[0][q];
                    a1 += s_rem[1][q];
                    a2 += s_rem[2][q];
                    a3 += s_rem[3][q];
                }
                s_J[o11] = a0;
                s_J[o12] = a1;
                s_J[2 * NT + o11] = a2;
                s_J[2 * NT + o12] = a3;
              }
            }
        }
        __syncthreads();
        if (WITH_J) write_jrows<NT>(c, s_J, J + (size_t)s * (size_t)g.nnz_j);
        if (P) {
            for (int q = k; q < c.nrows; q += NT) {
                P[so + c.r0 + q] = s_pq[0][q];
                Q[so + c.r0 + q] = s_pq[1][q];
            }
        }
        __syncthreads();
    }
}

// ===================================================================
// Ybus method: I = Ybus V, S = V conj(I) (eq. (1)) and, with WITH_J, the
// two-pass Jacobian of eqs. (3)-(4) done row-wise on the CSR matrix:
// pass 1 forms I_i, pass 2 turns each nonzero into
//   dS_i/dtheta_j = j V_i (delta_ij conj(I_i) - conj(Y_ij V_j))
//   dS_i/dv_j     = V_i conj(Y_ij U_j) + delta_ij conj(I_i) U_i
// and writes the four real parts in place into J (Section IV.B.2).
// U = e^{j theta} and V = v U are formed on the fly from (vm, va).
template <int NT, bool WITH_J>
__global__ void __launch_bounds__(NT)
    k_ybus(DevGrid g, int nstate, int spb, int nchunk, const double *__restrict__ vm, const double *__restrict__ va,
           double *__restrict__ P, double *__restrict__ Q, double *__restrict__ J) {
    __shared__ int s_irow[NT + 1];
    __shared__ int s_yrow[NT + 1];
    __shared__ double s_yv[2][NT];
    __shared__ double s_row[4][NT];  // per row: I_i (re, im), V_i (re, im)
    __shared__ double s_u[2][NT];    // per row: U_i
    __shared__ __align__(16) double s_J[WITH_J ? 4 * NT : 1];

    const int W = g.ntiles * nchunk;
    const int w = work_index(gridDim.x);
    if (w >= W) return;
    const int t = w / nchunk;
    const int sb = (w - t * nchunk) * spb;
    const int se = min(nstate, sb + spb);
    const Tile c = tile_of(g, t);
    const int k = threadIdx.x;
    const size_t nb = (size_t)g.nb;

    if (c.n > NT) {
        // ---- one long row: pass 1 sums I_i in chunks (thread 0, in slot order), pass 2 writes J.
        const int i = c.r0;
        const int d = c.ns;
        for (int s = sb; s < se; ++s) {
            const size_t so = (size_t)s * nb;
            Cx I = {0.0, 0.0};
            for (int base = 0; base < d; base += NT) {
                if (base + k < d) {
                    const int p = c.s0 + base + k;
                    const int j = g.ycol[p];
                    double sn, cs;
                    sincos(va[so + j], &sn, &cs);
                    const double v = vm[so + j];
                    const Cx yv = cmul({g.yre[p], g.yim[p]}, {v * cs, v * sn});
                    s_yv[0][k] = yv.re;
                    s_yv[1][k] = yv.im;
                }
                __syncthreads();
                if (k == 0) {
                    const int m = min(NT, d - base);
                    for (int q = 0; q < m; ++q) {
                        I.re += s_yv[0][q];
                        I.im += s_yv[1][q];
                    }
                }
                __syncthreads();
            }
            double sn, cs;
            sincos(va[so + i], &sn, &cs);
            const Cx Ui = {cs, sn};
            const double vi = vm[so + i];
            const Cx Vi = {vi * cs, vi * sn};
            if (k == 0) {
                s_row[0][0] = I.re;
                s_row[1][0] = I.im;
                if (P) {
                    const Cx S = cmul(Vi, cconj(I));
                    P[so + i] = S.re;
                    Q[so + i] = S.im;
                }
            }
            __syncthreads();
            if constexpr (WITH_J) {
                const Cx Ic = {s_row[0][0], -s_row[1][0]};  // conj(I_i)
                double *Js = J + (size_t)s * (size_t)g.nnz_j;
                for (int lp = k; lp < d; lp += NT) {
                    const int p = c.s0 + lp;
                    const int j = g.ycol[p];
                    double snj, csj;
                    sincos(va[so + j], &snj, &csj);
                    const double v = vm[so + j];
                    const Cx Y = {g.yre[p], g.yim[p]};
                    const Cx Uj = {csj, snj};
                    const Cx yv = cmul(Y, {v * csj, v * snj});
                    const bool dg = j == i;
                    const Cx x = csub(dg ? Ic : Cx{0.0, 0.0}, cconj(yv));
                    const Cx dst = cmul({-Vi.im, Vi.re}, x);  // j V_i x
                    Cx dsv = cmul(Vi, cconj(cmul(Y, Uj)));
                    if (dg) dsv = cadd(dsv, cmul(Ic, Ui));
                    Js[c.jp + lp] = dst.re;
                    Js[c.jp + d + lp] = dsv.re;
                    Js[c.jq + lp] = dst.im;
                    Js[c.jq + d + lp] = dsv.im;
                }
            }
            __syncthreads();
        }
        return;
    }

    stage_rows<NT>(g, c, s_irow, s_yrow);
    const bool live = k < c.ns;
    int j = 0;
    Cx Y = {0.0, 0.0};
    if (live) {
        const int p = c.s0 + k;
        j = g.ycol[p];
        Y = {g.yre[p], g.yim[p]};
    }
    __syncthreads();
    const int row = live ? row_of(k, s_yrow, c.nrows) : 0;
    const int i = c.r0 + row;
    const bool diag = live && j == i;
    const int o11 = s_yrow[row] + k;
    const int o12 = s_yrow[row + 1] + k;

    for (int s = sb; s < se; ++s) {
        const size_t so = (size_t)s * nb;
        Cx Uj = {0.0, 0.0}, yv = {0.0, 0.0};
        if (live) {
            double sn, cs;
            sincos(va[so + j], &sn, &cs);
            const double v = vm[so + j];
            Uj = {cs, sn};
            yv = cmul(Y, {v * cs, v * sn});
            s_yv[0][k] = yv.re;
            s_yv[1][k] = yv.im;
            if (diag) {  // the diagonal nonzero carries the row's own phasor
                s_row[2][row] = v * cs;
                s_row[3][row] = v * sn;
                s_u[0][row] = cs;
                s_u[1][row] = sn;
            }
        }
        __syncthreads();
        if (diag) {
            const int a = s_yrow[row], z = s_yrow[row + 1];
            Cx I = {0.0, 0.0};
            for (int q = a; q < z; ++q) {
                I.re += s_yv[0][q];
                I.im += s_yv[1][q];
            }
            s_row[0][row] = I.re;
            s_row[1][row] = I.im;
        }
        __syncthreads();
        if (P) {
            for (int q = k; q < c.nrows; q += NT) {
                const Cx S = cmul({s_row[2][q], s_row[3][q]}, {s_row[0][q], -s_row[1][q]});
                P[so + c.r0 + q] = S.re;
                Q[so + c.r0 + q] = S.im;
            }
        }
        if constexpr (WITH_J) {
            if (live) {
                const Cx Vi = {s_row[2][row], s_row[3][row]};
                const Cx Ic = {s_row[0][row], -s_row[1][row]};
                const Cx x = csub(diag ? Ic : Cx{0.0, 0.0}, cconj(yv));
                const Cx dst = cmul({-Vi.im, Vi.re}, x);
                Cx dsv = cmul(Vi, cconj(cmul(Y, Uj)));
                if (diag) dsv = cadd(dsv, cmul(Ic, {s_u[0][row], s_u[1][row]}));
                s_J[o11] = dst.re;
                s_J[o12] = dsv.re;
                s_J[2 * NT + o11] = dst.im;
                s_J[2 * NT + o12] = dsv.im;
            }
            __syncthreads();
            write_jrows<NT>(c, s_J, J + (size_t)s * (size_t)g.nnz_j);
        }
        __syncthreads();
    }
}

// ===================================================================
// Adjoint of the element-wise injections.  Column i of J collects the own
// partials of every record at bus i (rows P_i, Q_i) and the remote partials
// of the opposite end of each incident branch (rows P_j, Q_j).  Record e (at
// i, towards j) therefore contributes to bus i
//   g_va += lP_i (-w beta) + lQ_i (w alpha) + lP_j (w beta') - lQ_j (w alpha')
//   g_vm += lP_i (2 v_i A + v_j alpha) + lQ_i (v_j beta - 2 v_i C)
//         + lP_j (v_j alpha') + lQ_j (v_j beta')
// where alpha', beta' use the other end's coupling (Gr, Br) at angle -t:
//   alpha' = Gr cos t - Br sin t,  beta' = -Gr sin t - Br cos t.
// Sums per bus run in record order; J is never formed.
template <int NT>
__global__ void __launch_bounds__(NT)
    k_ew_vjp(DevGrid g, int nstate, int spb, int nchunk, const double *__restrict__ vm,
             const double *__restrict__ va, const double *__restrict__ lp, const double *__restrict__ lq,
             double *__restrict__ gvm, double *__restrict__ gva) {
    __shared__ int s_irow[NT + 1];
    __shared__ int s_yrow[NT + 1];
    __shared__ double s_val[2][NT];
    __shared__ double s_out[2][NT];

    const int W = g.ntiles * nchunk;
    const int w = work_index(gridDim.x);
    if (w >= W) return;
    const int t = w / nchunk;
    const int sb = (w - t * nchunk) * spb;
    const int se = min(nstate, sb + spb);
    const Tile c = tile_of(g, t);
    const int k = threadIdx.x;
    const size_t nb = (size_t)g.nb;

    auto record = [&](int e, int i, size_t so, double &ga, double &gv) {
        const int j = g.nbr[e];
        const double vi = vm[so + i], ti = va[so + i], vj = vm[so + j], tj = va[so + j];
        const double lpi = lp[so + i], lqi = lq[so + i], lpj = lp[so + j], lqj = lq[so + j];
        const double A = g.A[e], C = g.C[e], G = g.G[e], B = g.B[e], Gr = g.Gr[e], Br = g.Br[e];
        double sn, cs;
        sincos(ti - tj, &sn, &cs);
        const double wv = vi * vj;
        const double al = G * cs + B * sn, be = G * sn - B * cs;
        const double al2 = Gr * cs - Br * sn, be2 = -(Gr * sn) - Br * cs;
        ga = wv * (lqi * al - lpi * be + lpj * be2 - lqj * al2);
        gv = lpi * (2.0 * vi * A + vj * al) + lqi * (vj * be - 2.0 * vi * C) + vj * (lpj * al2 + lqj * be2);
    };

    if (c.n > NT) {
        const int i = c.r0;
        for (int s = sb; s < se; ++s) {
            const size_t so = (size_t)s * nb;
            double acc_a = 0.0, acc_v = 0.0;
            for (int base = 0; base < c.n; base += NT) {
                if (base + k < c.n) {
                    double ga, gv;
                    record(c.i0 + base + k, i, so, ga, gv);
                    s_val[0][k] = ga;
                    s_val[1][k] = gv;
                }
                __syncthreads();
                if (k == 0) {
                    const int m = min(NT, c.n - base);
                    for (int q = 0; q < m; ++q) {
                        acc_a += s_val[0][q];
                        acc_v += s_val[1][q];
                    }
                }
                __syncthreads();
            }
            if (k == 0) {
                gva[so + i] = acc_a;
                gvm[so + i] = acc_v;
            }
        }
        return;
    }

    stage_rows<NT>(g, c, s_irow, s_yrow);
    __syncthreads();
    const bool live = k < c.n;
    const int row = live ? row_of(k, s_irow, c.nrows) : 0;
    const int i = c.r0 + row;
    const bool head = live && s_irow[row] == k;  // first record of the row sums it
    for (int s = sb; s < se; ++s) {
        const size_t so = (size_t)s * nb;
        if (live) {
            double ga, gv;
            record(c.i0 + k, i, so, ga, gv);
            s_val[0][k] = ga;
            s_val[1][k] = gv;
        }
        __syncthreads();
        if (head) {
            double a = 0.0, v = 0.0;
            for (int q = s_irow[row]; q < s_irow[row + 1]; ++q) {
                a += s_val[0][q];
                v += s_val[1][q];
            }
            s_out[0][row] = a;
            s_out[1][row] = v;
        }
        __syncthreads();
        for (int q = k; q < c.nrows; q += NT) {
            gva[so + c.r0 + q] = s_out[0][q];
            gvm[so + c.r0 + q] = s_out[1][q];
        }
        __syncthreads();
    }
}

// ===================================================================
// Setup: record constants from the branch parameters.
__global__ void k_items_init(DevSetup s) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= s.nitems) return;
    const int br = s.item_br[e];
    if (br < 0) {  // bus shunt record
        const int i = s.nbr[e];
        s.A[e] = s.gs[i];
        s.C[e] = s.bs[i];
        s.G[e] = 0.0;
        s.B[e] = 0.0;
        s.Gr[e] = 0.0;
        s.Br[e] = 0.0;
        return;
    }
    const int l = br >> 1;
    const bool to_end = (br & 1) != 0;
    const double r = s.r[l], x = s.x[l];
    const double den = r * r + x * x;
    const double gsr = r / den, bsr = -x / den;  // y_hk = 1/(r + jx)
    const double m = s.tap[l] == 0.0 ? 1.0 : s.tap[l];
    const double bh = 0.5 * s.b[l];
    double sp, cp;
    sincos(s.shift[l], &sp, &cp);
    // -y_hk e^{+j phi}/m (from end) and -y_hk e^{-j phi}/m (to end)
    const double gf = -(gsr * cp - bsr * sp) / m, bf = -(gsr * sp + bsr * cp) / m;
    const double gt = -(gsr * cp + bsr * sp) / m, bt = -(bsr * cp - gsr * sp) / m;
    if (!to_end) {
        s.A[e] = gsr / (m * m);
        s.C[e] = (bsr + bh) / (m * m);
        s.G[e] = gf;
        s.B[e] = bf;
        s.Gr[e] = gt;
        s.Br[e] = bt;
    } else {
        s.A[e] = gsr;
        s.C[e] = bsr + bh;
        s.G[e] = gt;
        s.B[e] = bt;
        s.Gr[e] = gf;
        s.Br[e] = bf;
    }
}

// Setup: Ybus values.  The diagonal sums the own-end admittances of all
// records of the row (shunt included); an off-diagonal slot sums the
// coupling admittances of its records (more than one for parallel branches).
__global__ void k_ybus_assemble(DevSetup s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.nnz_y) return;
    const int i = s.slot_row[p];
    double re = 0.0, im = 0.0;
    if (s.ycol[p] == i) {
        for (int e = s.irow[i]; e < s.irow[i + 1]; ++e) {
            re += s.A[e];
            im += s.C[e];
        }
    } else {
        for (int e = s.slot_item[p]; e < s.slot_item[p + 1]; ++e) {
            re += s.G[e];
            im += s.B[e];
        }
    }
    s.yre[p] = re;
    s.yim[p] = im;
}

template <int NT>
hipError_t launch_nt(const DevGrid &g, const Launch &L, hipStream_t st) {
    const int spb = L.states_per_block;
    const int nchunk = (L.nstate + spb - 1) / spb;
    const int64_t work = (int64_t)g.ntiles * nchunk;
    const int64_t blocks = (work + kXcds - 1) / kXcds * kXcds;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks), block(NT);
    switch (L.kind) {
        case K_EW_S:
            if (L.has_parallel)
                hipLaunchKernelGGL((k_ew<NT, true, false>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va,
                                   L.p, L.q, nullptr);
            else
                hipLaunchKernelGGL((k_ew<NT, false, false>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va,
                                   L.p, L.q, nullptr);
            break;
        case K_EW_SJ:
            if (L.has_parallel)
                hipLaunchKernelGGL((k_ew<NT, true, true>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va,
                                   L.p, L.q, L.jval);
            else
                hipLaunchKernelGGL((k_ew<NT, false, true>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va,
                                   L.p, L.q, L.jval);
            break;
        case K_YB_S:
            hipLaunchKernelGGL((k_ybus<NT, false>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va, L.p, L.q,
                               nullptr);
            break;
        case K_YB_SJ:
            hipLaunchKernelGGL((k_ybus<NT, true>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va, L.p, L.q,
                               L.jval);
            break;
        case K_EW_VJP:
            hipLaunchKernelGGL((k_ew_vjp<NT>), grid, block, 0, st, g, L.nstate, spb, nchunk, L.vm, L.va, L.lp, L.lq,
                               L.gvm, L.gva);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const DevGrid &g, const Launch &L, hipStream_t stream) {
    switch (L.tile_items) {
        case 64:
            return launch_nt<64>(g, L, stream);
        case 128:
            return launch_nt<128>(g, L, stream);
        case 256:
            return launch_nt<256>(g, L, stream);
        case 512:
            return launch_nt<512>(g, L, stream);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_setup_items(const DevSetup &s, hipStream_t stream) {
    if (s.nitems == 0) return hipSuccess;
    const int64_t blocks = (s.nitems + 255) / 256;
    hipLaunchKernelGGL(k_items_init, dim3((unsigned)blocks), dim3(256), 0, stream, s);
    return hipGetLastError();
}

hipError_t launch_ybus_assemble(const DevSetup &s, hipStream_t stream) {
    if (s.nnz_y == 0) return hipSuccess;
    const int64_t blocks = (s.nnz_y + 255) / 256;
    hipLaunchKernelGGL(k_ybus_assemble, dim3((unsigned)blocks), dim3(256), 0, stream, s);
    return hipGetLastError();
}

}  // namespace pf
