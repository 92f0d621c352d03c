/*
 * Plain FP64 CPU oracle for nodal power injections and the polar power-flow
 * Jacobian, after "Bus Admittance Matrix Revisited: Is It Outdated on Modern
 * Computers?" (arXiv 2302.10736).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may load
 * or call this code: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header or constant
 * with the GPU library.
 *
 * Every function is a direct, unoptimised transcription of the paper's
 * definitions: scalar loops, C99 complex arithmetic, one grid and one state
 * per call, built with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math).  Sparse placement is done by plain search inside a CSR row.
 *
 * Conventions (readings where the paper is silent):
 *  - branch l runs from bus h = fbus[l] to bus k = tbus[l] (0-based);
 *    series admittance y_hk = 1/(r + jx); terminal shunts
 *    y_h = y_k = j b/2 (pi model); off-nominal ratio m e^{j phi} on the h
 *    side; tap == 0 means m = 1; shift in radians;
 *  - a bus shunt g + jb at bus i adds v_i^2 (g - jb) to S_i, so that the
 *    element-wise sum of eq. (7) equals eq. (1) with the shunt on the
 *    admittance diagonal;
 *  - S is the complex power injected into the network, S = P + jQ.
 *
 * Parity pins (see tests): a two-bus closed form from circuit laws, the
 * power-balance identity, complex-step derivatives of a textbook polar
 * form, dense brute force, agreement between the two methods, and the
 * brute-force index search of Algorithm 2.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Branch admittances of the pi model with the transformer on the h side:
 * the Ybus entries for which eqs. (5) and (6) read
 *   S_hk = V_h conj(yff V_h + yft V_k),  S_kh = V_k conj(ytf V_h + ytt V_k).
 * Matching term by term (Section II.B):
 *   yff = (y_h + y_hk)/m^2,  yft = -y_hk e^{j phi}/m,
 *   ytf = -y_hk e^{-j phi}/m, ytt = y_k + y_hk.                           */
static void branch_admittances(double r, double x, double b, double tap, double shift,
                               cplx *yff, cplx *yft, cplx *ytf, cplx *ytt)
{
    double m = (tap == 0.0) ? 1.0 : tap;
    cplx yhk = 1.0 / (r + I * x);
    cplx ysh = I * (b / 2.0);
    *yff = (ysh + yhk) / (m * m);
    *yft = -yhk * cexp(I * shift) / m;
    *ytf = -yhk * cexp(-I * shift) / m;
    *ytt = ysh + yhk;
}

/* ---------------------------------------------------------------------- */
/* Ybus in CSR (Section IV.A.1; eq. (1)).  COO triplets (row, col, value):
 * one diagonal shunt entry per bus (kept even when zero, so every diagonal
 * is structurally present) and four per branch; sorted by (row, col,
 * sequence number); duplicates summed in that order.
 * yrow: int32[nb+1]; ycol, yre, yim: capacity nb + 4 nl.  Returns nnz.   */

typedef struct { int32_t row, col; int64_t seq; cplx val; } coo_t;

static int coo_cmp(const void *pa, const void *pb)
{
    const coo_t *a = pa, *b = pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    return (a->seq > b->seq) - (a->seq < b->seq);
}

int64_t orc_ybus(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus,
                 const double *r, const double *x, const double *b, const double *tap,
                 const double *shift, const double *gs, const double *bs,
                 int32_t *yrow, int32_t *ycol, double *yre, double *yim)
{
    int64_t n = (int64_t)nb + 4 * (int64_t)nl, c = 0;
    coo_t *e = malloc(sizeof(coo_t) * (size_t)(n ? n : 1));
    if (!e) return -1;
    for (int32_t i = 0; i < nb; ++i) {
        e[c].row = i; e[c].col = i; e[c].seq = c;
        e[c].val = (gs ? gs[i] : 0.0) + I * (bs ? bs[i] : 0.0);
        ++c;
    }
    for (int32_t l = 0; l < nl; ++l) {
        cplx yff, yft, ytf, ytt;
        int32_t h = fbus[l], k = tbus[l];
        branch_admittances(r[l], x[l], b[l], tap[l], shift[l], &yff, &yft, &ytf, &ytt);
        e[c].row = h; e[c].col = h; e[c].seq = c; e[c].val = yff; ++c;
        e[c].row = h; e[c].col = k; e[c].seq = c; e[c].val = yft; ++c;
        e[c].row = k; e[c].col = h; e[c].seq = c; e[c].val = ytf; ++c;
        e[c].row = k; e[c].col = k; e[c].seq = c; e[c].val = ytt; ++c;
    }
    qsort(e, (size_t)n, sizeof(coo_t), coo_cmp);
    int64_t nnz = 0;
    for (int32_t i = 0; i <= nb; ++i) yrow[i] = 0;
    for (int64_t q = 0; q < n; ++q) {
        if (nnz > 0 && ycol[nnz - 1] == e[q].col && q > 0 && e[q - 1].row == e[q].row) {
            cplx s = yre[nnz - 1] + I * yim[nnz - 1];
            s += e[q].val;
            yre[nnz - 1] = creal(s);
            yim[nnz - 1] = cimag(s);
        } else {
            ycol[nnz] = e[q].col;
            yre[nnz] = creal(e[q].val);
            yim[nnz] = cimag(e[q].val);
            yrow[e[q].row + 1]++;
            ++nnz;
        }
    }
    for (int32_t i = 0; i < nb; ++i) yrow[i + 1] += yrow[i];
    free(e);
    return nnz;
}

/* ---------------------------------------------------------------------- */
/* Injections by the Ybus method (Section IV.B.1, steps 1-3; eq. (1)):
 *   1) U = e^{j theta}, V = vm U;  2) I = Ybus V;  3) S = V conj(I).      */
void orc_inject_ybus(int32_t nb, const int32_t *yrow, const int32_t *ycol, const double *yre,
                     const double *yim, const double *vm, const double *va, double *p, double *q)
{
    cplx *V = malloc(sizeof(cplx) * (size_t)(nb ? nb : 1));
    for (int32_t i = 0; i < nb; ++i) V[i] = vm[i] * cexp(I * va[i]);
    for (int32_t i = 0; i < nb; ++i) {
        cplx cur = 0.0;
        for (int32_t t = yrow[i]; t < yrow[i + 1]; ++t) cur += (yre[t] + I * yim[t]) * V[ycol[t]];
        cplx s = V[i] * conj(cur);
        p[i] = creal(s);
        q[i] = cimag(s);
    }
    free(V);
}

/* ---------------------------------------------------------------------- */
/* Injections by the element-wise method: eqs. (5) and (6) per branch,
 * summed at the terminal buses in branch order (eq. (7)), then the bus
 * shunt term v_i^2 (g_i - j b_i).                                         */
void orc_inject_ew(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus,
                   const double *r, const double *x, const double *b, const double *tap,
                   const double *shift, const double *gs, const double *bs,
                   const double *vm, const double *va, double *p, double *q)
{
    cplx *S = calloc((size_t)(nb ? nb : 1), sizeof(cplx));
    for (int32_t l = 0; l < nl; ++l) {
        int32_t h = fbus[l], k = tbus[l];
        double m = (tap[l] == 0.0) ? 1.0 : tap[l];
        cplx yhk = 1.0 / (r[l] + I * x[l]);
        cplx yh = I * (b[l] / 2.0), yk = I * (b[l] / 2.0);
        double vh = vm[h], vk = vm[k];
        double delta = va[h] - va[k] - shift[l];
        cplx shk = vh * vh * conj(yh + yhk) / (m * m) - vh * vk * conj(yhk) / m * cexp(I * delta);
        cplx skh = -vh * vk * conj(yhk) / m * cexp(-I * delta) + vk * vk * conj(yk + yhk);
        S[h] += shk;
        S[k] += skh;
    }
    for (int32_t i = 0; i < nb; ++i) {
        cplx ysh = (gs ? gs[i] : 0.0) + I * (bs ? bs[i] : 0.0);
        S[i] += vm[i] * vm[i] * conj(ysh);
        p[i] = creal(S[i]);
        q[i] = cimag(S[i]);
    }
    free(S);
}

/* ---------------------------------------------------------------------- */
/* Jacobian pattern, eq. (2): a 2nb x 2nb matrix with rows
 * [P_0..P_{nb-1}, Q_0..Q_{nb-1}] and columns [theta_0.., v_0..]; each of
 * the four blocks carries the Ybus pattern (Section IV.B.2).  Row i of the
 * top half holds the Ybus columns of row i, then the same columns + nb.
 * jrow: int32[2nb+1]; jcol: int32[4 nnzY].                                 */
void orc_jac_pattern(int32_t nb, const int32_t *yrow, const int32_t *ycol, int32_t *jrow,
                     int32_t *jcol)
{
    int64_t c = 0;
    jrow[0] = 0;
    for (int32_t half = 0; half < 2; ++half) {
        for (int32_t i = 0; i < nb; ++i) {
            for (int32_t t = yrow[i]; t < yrow[i + 1]; ++t) jcol[c++] = ycol[t];
            for (int32_t t = yrow[i]; t < yrow[i + 1]; ++t) jcol[c++] = ycol[t] + nb;
            jrow[half * nb + i + 1] = (int32_t)c;
        }
    }
}

/* Add val at (row, col) of a CSR matrix, found by linear search of the row.
 * Returns 0, or -1 when (row, col) is not in the pattern.                 */
static int csr_add(const int32_t *jrow, const int32_t *jcol, double *jval, int32_t row,
                   int32_t col, double val)
{
    for (int32_t t = jrow[row]; t < jrow[row + 1]; ++t) {
        if (jcol[t] == col) {
            jval[t] += val;
            return 0;
        }
    }
    return -1;
}

/* ---------------------------------------------------------------------- */
/* Jacobian by the Ybus method: every entry of eqs. (3) and (4) on the Ybus
 * pattern,
 *   dS_i/dtheta_j = j V_i (delta_ij conj(I_i) - conj(Y_ij V_j)),
 *   dS_i/dv_j     = delta_ij conj(I_i) U_i + V_i conj(Y_ij U_j),
 * with J11 = Re dS/dtheta, J12 = Re dS/dv, J21 = Im dS/dtheta,
 * J22 = Im dS/dv (eq. (2)).  jval must be zeroed by the caller; returns
 * the number of entries that did not fit the pattern (0 when correct).   */
int64_t orc_jac_ybus(int32_t nb, const int32_t *yrow, const int32_t *ycol, const double *yre,
                     const double *yim, const double *vm, const double *va, const int32_t *jrow,
                     const int32_t *jcol, double *jval)
{
    cplx *U = malloc(sizeof(cplx) * (size_t)(nb ? nb : 1));
    cplx *V = malloc(sizeof(cplx) * (size_t)(nb ? nb : 1));
    cplx *Ib = malloc(sizeof(cplx) * (size_t)(nb ? nb : 1));
    int64_t miss = 0;
    for (int32_t i = 0; i < nb; ++i) {
        U[i] = cexp(I * va[i]);
        V[i] = vm[i] * U[i];
    }
    for (int32_t i = 0; i < nb; ++i) {
        Ib[i] = 0.0;
        for (int32_t t = yrow[i]; t < yrow[i + 1]; ++t) Ib[i] += (yre[t] + I * yim[t]) * V[ycol[t]];
    }
    for (int32_t i = 0; i < nb; ++i) {
        for (int32_t t = yrow[i]; t < yrow[i + 1]; ++t) {
            int32_t j = ycol[t];
            cplx Y = yre[t] + I * yim[t];
            cplx d = (i == j) ? conj(Ib[i]) : 0.0;
            cplx dst = I * V[i] * (d - conj(Y * V[j]));
            cplx dsv = V[i] * conj(Y * U[j]) + ((i == j) ? conj(Ib[i]) * U[i] : 0.0);
            miss += csr_add(jrow, jcol, jval, i, j, creal(dst)) != 0;
            miss += csr_add(jrow, jcol, jval, i, nb + j, creal(dsv)) != 0;
            miss += csr_add(jrow, jcol, jval, nb + i, j, cimag(dst)) != 0;
            miss += csr_add(jrow, jcol, jval, nb + i, nb + j, cimag(dsv)) != 0;
        }
    }
    free(U);
    free(V);
    free(Ib);
    return miss;
}

/* ---------------------------------------------------------------------- */
/* Jacobian by the element-wise method: the 16 partial derivatives of
 * P_h, Q_h, P_k, Q_k with respect to v_h, theta_h, v_k, theta_k for every
 * branch (Section II.B), obtained by differentiating eqs. (5) and (6):
 *   S_hk = v_h^2 a_h - v_h v_k c e^{j d},   S_kh = v_k^2 a_k - v_h v_k c e^{-j d}
 * with a_h = conj(y_h + y_hk)/m^2, a_k = conj(y_k + y_hk),
 * c = conj(y_hk)/m, d = theta_h - theta_k - phi.  Each partial is added at
 * its (row, column) of the eq. (2) pattern; then the bus shunt term
 * d/dv_i of v_i^2 conj(g_i + j b_i).  jval must be zeroed by the caller.   */
int64_t orc_jac_ew(int32_t nb, int32_t nl, const int32_t *fbus, const int32_t *tbus,
                   const double *r, const double *x, const double *b, const double *tap,
                   const double *shift, const double *gs, const double *bs, const double *vm,
                   const double *va, const int32_t *jrow, const int32_t *jcol, double *jval)
{
    int64_t miss = 0;
    for (int32_t l = 0; l < nl; ++l) {
        int32_t h = fbus[l], k = tbus[l];
        double m = (tap[l] == 0.0) ? 1.0 : tap[l];
        cplx yhk = 1.0 / (r[l] + I * x[l]);
        cplx ysh = I * (b[l] / 2.0);
        cplx ah = conj(ysh + yhk) / (m * m), ak = conj(ysh + yhk), c = conj(yhk) / m;
        double vh = vm[h], vk = vm[k];
        double d = va[h] - va[k] - shift[l];
        cplx ef = cexp(I * d), et = cexp(-I * d);
        /* d S_hk / d (theta_h, theta_k, v_h, v_k) */
        cplx f_th = -I * vh * vk * c * ef;
        cplx f_tk = I * vh * vk * c * ef;
        cplx f_vh = 2.0 * vh * ah - vk * c * ef;
        cplx f_vk = -vh * c * ef;
        /* d S_kh / d (theta_h, theta_k, v_h, v_k) */
        cplx t_th = I * vh * vk * c * et;
        cplx t_tk = -I * vh * vk * c * et;
        cplx t_vh = -vk * c * et;
        cplx t_vk = 2.0 * vk * ak - vh * c * et;
        int32_t rows[2] = {h, k};
        cplx ds[2][4] = {{f_th, f_tk, f_vh, f_vk}, {t_th, t_tk, t_vh, t_vk}};
        int32_t cols[4] = {h, k, nb + h, nb + k};
        for (int e = 0; e < 2; ++e) {
            for (int v = 0; v < 4; ++v) {
                miss += csr_add(jrow, jcol, jval, rows[e], cols[v], creal(ds[e][v])) != 0;
                miss += csr_add(jrow, jcol, jval, nb + rows[e], cols[v], cimag(ds[e][v])) != 0;
            }
        }
    }
    for (int32_t i = 0; i < nb; ++i) {
        cplx ysh = (gs ? gs[i] : 0.0) + I * (bs ? bs[i] : 0.0);
        cplx dsv = 2.0 * vm[i] * conj(ysh);
        miss += csr_add(jrow, jcol, jval, i, nb + i, creal(dsv)) != 0;
        miss += csr_add(jrow, jcol, jval, nb + i, nb + i, cimag(dsv)) != 0;
    }
    return miss;
}

/* ---------------------------------------------------------------------- */
/* Vector-Jacobian product g = J^T [lam_P; lam_Q] from a formed CSR J:
 * g_theta = J11^T lam_P + J21^T lam_Q and g_v = J12^T lam_P + J22^T lam_Q.
 * lam: f64[2nb] = [lam_P, lam_Q]; g: f64[2nb] = [g_theta, g_v], written.  */
void orc_vjp(int32_t nb, const int32_t *jrow, const int32_t *jcol, const double *jval,
             const double *lam, double *g)
{
    for (int32_t c = 0; c < 2 * nb; ++c) g[c] = 0.0;
    for (int32_t row = 0; row < 2 * nb; ++row)
        for (int32_t t = jrow[row]; t < jrow[row + 1]; ++t) g[jcol[t]] += jval[t] * lam[row];
}

/* Branch flows, eqs. (5)-(6): the power entering branch l at its h end,
 * S_hk = pf + j qf, and at its k end, S_kh = pt + j qt (branch order). */
void orc_branch_flows(int32_t nl, const int32_t *fbus, const int32_t *tbus, const double *r,
                      const double *x, const double *b, const double *tap, const double *shift,
                      const double *vm, const double *va, double *pf, double *qf, double *pt,
                      double *qt)
{
    for (int32_t l = 0; l < nl; ++l) {
        int32_t h = fbus[l], k = tbus[l];
        double m = (tap[l] == 0.0) ? 1.0 : tap[l];
        cplx yhk = 1.0 / (r[l] + I * x[l]);
        cplx yh = I * (b[l] / 2.0), yk = I * (b[l] / 2.0);
        double vh = vm[h], vk = vm[k];
        double delta = va[h] - va[k] - shift[l];
        cplx shk = vh * vh * conj(yh + yhk) / (m * m) - vh * vk * conj(yhk) / m * cexp(I * delta);
        cplx skh = -vh * vk * conj(yhk) / m * cexp(-I * delta) + vk * vk * conj(yk + yhk);
        pf[l] = creal(shk);
        qf[l] = cimag(shk);
        pt[l] = creal(skh);
        qt[l] = cimag(skh);
    }
}

/* The 16 partial derivatives of the branch flows, jac[16][nl]: row q of
 * 4 q..4 q + 3 holds d(Pf, Qf, Pt, Qt)[q] / d(theta_h, theta_k, v_h, v_k). */
void orc_branch_flow_jac(int32_t nl, const int32_t *fbus, const int32_t *tbus, const double *r,
                         const double *x, const double *b, const double *tap, const double *shift,
                         const double *vm, const double *va, double *jac)
{
    for (int32_t l = 0; l < nl; ++l) {
        int32_t h = fbus[l], k = tbus[l];
        double m = (tap[l] == 0.0) ? 1.0 : tap[l];
        cplx yhk = 1.0 / (r[l] + I * x[l]);
        cplx ysh = I * (b[l] / 2.0);
        cplx ah = conj(ysh + yhk) / (m * m), ak = conj(ysh + yhk), c = conj(yhk) / m;
        double vh = vm[h], vk = vm[k];
        double d = va[h] - va[k] - shift[l];
        cplx ef = cexp(I * d), et = cexp(-I * d);
        cplx f[4] = {-I * vh * vk * c * ef, I * vh * vk * c * ef, 2.0 * vh * ah - vk * c * ef, -vh * c * ef};
        cplx t[4] = {I * vh * vk * c * et, -I * vh * vk * c * et, -vk * c * et, 2.0 * vk * ak - vh * c * et};
        for (int v = 0; v < 4; ++v) {
            jac[(size_t)(0 + v) * nl + l] = creal(f[v]);
            jac[(size_t)(4 + v) * nl + l] = cimag(f[v]);
            jac[(size_t)(8 + v) * nl + l] = creal(t[v]);
            jac[(size_t)(12 + v) * nl + l] = cimag(t[v]);
        }
    }
}
