/*
 * Oracle: plain CPU FP64 reference of the hydrothermal finite-element method
 * (Sun et al., "An HPC-Based Hydrothermal Finite Element Simulator ...").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load.
 * It shares no code with the GPU library.
 *
 * What it computes (plain definitions, no blocking or fusion):
 *   - tensor-product Lagrange Q_p elements (p = 1, 2) with equispaced nodes on
 *     a box mesh (uniform or rectilinear) or, given the coordinates of every
 *     node, on general hexahedra of the box topology (isoparametric map with
 *     the same basis: x(xi) = sum_a x_a N_a(xi), gradients through the
 *     inverse Jacobian, volume element |det J|), Gauss-Legendre quadrature
 *     with (p+1) points per direction unless the caller asks for more;
 *   - element matrices of the bilinear form
 *         a(v,u) = m_c (v,u) + s_c (grad v, grad u) + (v, beta . grad u)
 *     where beta = adv_scale * q_h and q_h = -k_c (grad P_h + rho_w g e_z) is
 *     the Darcy flux evaluated from the nodal pressure at each quadrature
 *     point (Section 2, Eqs. 1-4 and the definition of q);
 *   - their assembly into a global CSR matrix, CSR products, load vectors for
 *     volume, gravity, face and line terms, the line mass matrix used by an
 *     injection well, and Jacobi-preconditioned CG / GMRES solvers with a
 *     long-double residual for iterative refinement;
 *   - plain-loop 3D convolutions (forward, backward-data, backward-weight)
 *     for the learned-preconditioner network.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 8
#define MAXNL 27

typedef struct {
    double x0[3];
    double L[3];
    int32_t n[3];
    int32_t p;
    /* Rectilinear (graded) meshes: cell-edge coordinates per axis, n[d] + 1
     * increasing values from x0[d] to x0[d] + L[d]; NULL = uniform spacing. */
    const double *edges[3];
    /* General hexahedra: coordinates of every node, [node][3] (node index
     * i + NX (j + NY k)); NULL = box geometry from x0, L and edges. */
    const double *xyz;
} orc_mesh;

typedef struct {
    const double *mass;   /* [C] coefficient of (v,u); NULL = 0            */
    const double *stiff;  /* [C] coefficient of (grad v, grad u); NULL = 0 */
    const double *kvel;   /* [C] k of the Darcy flux; NULL = no advection  */
    const double *P;      /* [N] nodal pressure for the Darcy flux         */
    double adv_scale;     /* multiplies q_h in the advective term          */
    double rho_g;         /* rho_w * g                                     */
    int32_t nq;           /* Gauss points per direction                    */
} orc_op;

/* ---------------------------------------------------------------- basics */
static int gauss01(int nq, double *x, double *w)
{
    /* Gauss-Legendre nodes/weights on [-1,1], mapped to [0,1]. */
    double t[MAXQ], c[MAXQ];
    switch (nq) {
    case 1: t[0] = 0.0; c[0] = 2.0; break;
    case 2: t[0] = -1.0 / sqrt(3.0); t[1] = -t[0]; c[0] = c[1] = 1.0; break;
    case 3: t[0] = -sqrt(0.6); t[1] = 0.0; t[2] = sqrt(0.6);
            c[0] = c[2] = 5.0 / 9.0; c[1] = 8.0 / 9.0; break;
    default: {
        /* Newton iteration on the Legendre polynomial for larger rules. */
        for (int i = 0; i < nq; i++) {
            double z = cos(M_PI * (i + 0.75) / (nq + 0.5)), pp = 0.0;
            for (int it = 0; it < 100; it++) {
                double p1 = 1.0, p2 = 0.0;
                for (int j = 0; j < nq; j++) {
                    double p3 = p2; p2 = p1;
                    p1 = ((2.0 * j + 1.0) * z * p2 - j * p3) / (j + 1.0);
                }
                pp = nq * (z * p1 - p2) / (z * z - 1.0);
                double dz = p1 / pp;
                z -= dz;
                if (fabs(dz) < 1e-16) break;
            }
            t[nq - 1 - i] = z;
            c[nq - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
        }
    }
    }
    for (int i = 0; i < nq; i++) { x[i] = 0.5 * (t[i] + 1.0); w[i] = 0.5 * c[i]; }
    return nq;
}

/* 1D Lagrange basis of degree p on the equispaced nodes a/p of [0,1]. */
static void lagrange(int p, double xi, double *N, double *dN)
{
    for (int a = 0; a <= p; a++) {
        double ta = (double)a / p, val = 1.0, der = 0.0;
        for (int b = 0; b <= p; b++) {
            if (b == a) continue;
            double tb = (double)b / p;
            double term = 1.0 / (ta - tb);
            /* product rule */
            der = der * (xi - tb) * term + val * term;
            val = val * (xi - tb) * term;
        }
        N[a] = val;
        dN[a] = der;
    }
}

static inline int64_t nodes_dim(const orc_mesh *m, int d) { return (int64_t)m->p * m->n[d] + 1; }

/* Lower coordinate and size of cell i along axis d. */
static inline double cell_lo(const orc_mesh *m, int d, int i)
{
    return m->edges[d] ? m->edges[d][i] : m->x0[d] + i * (m->L[d] / m->n[d]);
}
static inline double cell_h(const orc_mesh *m, int d, int i)
{
    return m->edges[d] ? m->edges[d][i + 1] - m->edges[d][i] : m->L[d] / m->n[d];
}

/* Nodes whose shape functions share a cell with node i along one axis. */
static void couple_range(int p, int n, int i, int *lo, int *hi)
{
    int cmin, cmax;
    if (i % p == 0) { cmin = i / p - 1; cmax = i / p; }
    else { cmin = cmax = i / p; }
    if (cmin < 0) cmin = 0;
    if (cmax > n - 1) cmax = n - 1;
    *lo = p * cmin;
    *hi = p * (cmax + 1);
}

int64_t orc_num_nodes(const orc_mesh *m)
{
    return nodes_dim(m, 0) * nodes_dim(m, 1) * nodes_dim(m, 2);
}

/* ------------------------------------------------------------- CSR layout */
int64_t orc_csr_rowptr(const orc_mesh *m, int64_t *rowptr)
{
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1), NZ = nodes_dim(m, 2);
    int64_t r = 0;
    rowptr[0] = 0;
    for (int64_t k = 0; k < NZ; k++) {
        int zl, zh; couple_range(m->p, m->n[2], (int)k, &zl, &zh);
        for (int64_t j = 0; j < NY; j++) {
            int yl, yh; couple_range(m->p, m->n[1], (int)j, &yl, &yh);
            for (int64_t i = 0; i < NX; i++) {
                int xl, xh; couple_range(m->p, m->n[0], (int)i, &xl, &xh);
                rowptr[r + 1] = rowptr[r] + (int64_t)(xh - xl + 1) * (yh - yl + 1) * (zh - zl + 1);
                r++;
            }
        }
    }
    return rowptr[r];
}

void orc_csr_cols(const orc_mesh *m, const int64_t *rowptr, int32_t *col)
{
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1), NZ = nodes_dim(m, 2);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < NZ; k++) {
        int zl, zh; couple_range(m->p, m->n[2], (int)k, &zl, &zh);
        for (int64_t j = 0; j < NY; j++) {
            int yl, yh; couple_range(m->p, m->n[1], (int)j, &yl, &yh);
            for (int64_t i = 0; i < NX; i++) {
                int xl, xh; couple_range(m->p, m->n[0], (int)i, &xl, &xh);
                int64_t pos = rowptr[i + NX * (j + NY * k)];
                for (int c = zl; c <= zh; c++)
                    for (int b = yl; b <= yh; b++)
                        for (int a = xl; a <= xh; a++)
                            col[pos++] = (int32_t)(a + NX * (b + NY * (int64_t)c));
            }
        }
    }
}

/* Position of column J in row I (both given as (i,j,k) triples). */
static inline int64_t csr_pos(const orc_mesh *m, const int64_t *rowptr, int64_t NX, int64_t NY,
                              int i, int j, int k, int a, int b, int c)
{
    int xl, xh, yl, yh, zl, zh;
    couple_range(m->p, m->n[0], i, &xl, &xh);
    couple_range(m->p, m->n[1], j, &yl, &yh);
    couple_range(m->p, m->n[2], k, &zl, &zh);
    int64_t wx = xh - xl + 1, wy = yh - yl + 1;
    return rowptr[i + NX * (j + NY * (int64_t)k)] + (int64_t)(c - zl) * wy * wx + (int64_t)(b - yl) * wx + (a - xl);
}

/* ------------------------------------------------------- element matrices */
/* Local node a = ax + (p+1)*(ay + (p+1)*az); global node of (cx,cy,cz,a). */
static inline int64_t gnode(const orc_mesh *m, int cx, int cy, int cz, int ax, int ay, int az)
{
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1);
    int p = m->p;
    return (int64_t)(p * cx + ax) + NX * ((int64_t)(p * cy + ay) + NY * (int64_t)(p * cz + az));
}

/* Shape functions N[a] and physical gradients G[a][d] of the nl local basis
 * functions of cell (cx,cy,cz) at the reference point whose 1D basis values
 * and derivatives along x, y, z are bx, dx, by, dy, bz, dz; returns the
 * volume element det J (> 0 for a valid cell).  Box cells map each axis
 * affinely (J = diag(h)); general hexahedra use the isoparametric map,
 * J_ij = d x_i / d xi_j = sum_a x_a,i dN_a/dxi_j, and grad N_a = J^-T
 * grad_xi N_a. */
static double cell_geometry(const orc_mesh *m, int cx, int cy, int cz, const double *bx, const double *dx,
                            const double *by, const double *dy, const double *bz, const double *dz,
                            double *N, double (*G)[3])
{
    int p = m->p, n1 = p + 1;
    double R[MAXNL][3];
    for (int az = 0; az < n1; az++)
        for (int ay = 0; ay < n1; ay++)
            for (int ax = 0; ax < n1; ax++) {
                int a = ax + n1 * (ay + n1 * az);
                N[a] = bx[ax] * by[ay] * bz[az];
                R[a][0] = dx[ax] * by[ay] * bz[az];
                R[a][1] = bx[ax] * dy[ay] * bz[az];
                R[a][2] = bx[ax] * by[ay] * dz[az];
            }
    int nl = n1 * n1 * n1;
    if (!m->xyz) {
        double h[3] = {cell_h(m, 0, cx), cell_h(m, 1, cy), cell_h(m, 2, cz)};
        for (int a = 0; a < nl; a++)
            for (int d = 0; d < 3; d++) G[a][d] = R[a][d] / h[d];
        return h[0] * h[1] * h[2];
    }
    double J[3][3] = {{0.0}};
    for (int az = 0; az < n1; az++)
        for (int ay = 0; ay < n1; ay++)
            for (int ax = 0; ax < n1; ax++) {
                int a = ax + n1 * (ay + n1 * az);
                const double *X = m->xyz + 3 * gnode(m, cx, cy, cz, ax, ay, az);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) J[i][j] += X[i] * R[a][j];
            }
    /* inverse by cofactors: Jinv = adj(J) / det J */
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    /* (J^-1)_{ji} = C_ij / det, so (J^-T grad_xi N)_i = sum_j C_ij R_j / det */
    for (int a = 0; a < nl; a++)
        for (int i = 0; i < 3; i++)
            G[a][i] = (C[i][0] * R[a][0] + C[i][1] * R[a][1] + C[i][2] * R[a][2]) / det;
    return det;
}

void orc_element_matrix(const orc_mesh *m, const orc_op *op, int cx, int cy, int cz, double *Ae)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1, nq = op->nq;
    int64_t c = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    double cm = op->mass ? op->mass[c] : 0.0;
    double cs = op->stiff ? op->stiff[c] : 0.0;
    double Pl[MAXNL];
    int adv = op->kvel != NULL && op->P != NULL;
    for (int az = 0; az < n1; az++)
        for (int ay = 0; ay < n1; ay++)
            for (int ax = 0; ax < n1; ax++)
                Pl[ax + n1 * (ay + n1 * az)] = adv ? op->P[gnode(m, cx, cy, cz, ax, ay, az)] : 0.0;
    memset(Ae, 0, sizeof(double) * nl * nl);
    for (int qz = 0; qz < nq; qz++)
        for (int qy = 0; qy < nq; qy++)
            for (int qx = 0; qx < nq; qx++) {
                double N[MAXNL], G[MAXNL][3];
                double detj = cell_geometry(m, cx, cy, cz, B[qx], D[qx], B[qy], D[qy], B[qz], D[qz], N, G);
                double w = gw[qx] * gw[qy] * gw[qz] * detj;
                double beta[3] = {0.0, 0.0, 0.0};
                if (adv) {
                    double gp[3] = {0.0, 0.0, 0.0};
                    for (int b = 0; b < nl; b++)
                        for (int d = 0; d < 3; d++) gp[d] += G[b][d] * Pl[b];
                    double k = op->kvel[c];
                    /* q_h = -k (grad P_h + rho_w g e_z), z up */
                    double q[3] = {-k * gp[0], -k * gp[1], -k * (gp[2] + op->rho_g)};
                    for (int d = 0; d < 3; d++) beta[d] = op->adv_scale * q[d];
                }
                for (int a = 0; a < nl; a++)
                    for (int b = 0; b < nl; b++) {
                        double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
                        double bg = beta[0] * G[b][0] + beta[1] * G[b][1] + beta[2] * G[b][2];
                        Ae[a * nl + b] += w * (cm * N[a] * N[b] + cs * gg + N[a] * bg);
                    }
            }
}

/* Assemble the global matrix (values only; pattern from orc_csr_*). */
void orc_assemble(const orc_mesh *m, const orc_op *op, const int64_t *rowptr, double *val)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1);
    memset(val, 0, sizeof(double) * rowptr[orc_num_nodes(m)]);
    /* Cells of equal index parity share no node: 8 colours, no races. */
    for (int color = 0; color < 8; color++) {
        int ox = color & 1, oy = (color >> 1) & 1, oz = (color >> 2) & 1;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
        for (int cz = oz; cz < m->n[2]; cz += 2)
            for (int cy = oy; cy < m->n[1]; cy += 2) {
                double Ae[MAXNL * MAXNL];
                for (int cx = ox; cx < m->n[0]; cx += 2) {
                    orc_element_matrix(m, op, cx, cy, cz, Ae);
                    for (int a = 0; a < nl; a++) {
                        int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
                        int I = p * cx + ax, J = p * cy + ay, K = p * cz + az;
                        for (int b = 0; b < nl; b++) {
                            int bx = b % n1, by = (b / n1) % n1, bz = b / (n1 * n1);
                            int64_t pos = csr_pos(m, rowptr, NX, NY, I, J, K,
                                                  p * cx + bx, p * cy + by, p * cz + bz);
                            val[pos] += Ae[a * nl + b];
                        }
                    }
                }
            }
    }
}

/* Rows of the assembled operator times x, computed from element matrices of
 * the cells around each requested node (for spot checks on large meshes).
 * Only columns with colmask[j] == 0 contribute when colmask != NULL. */
void orc_apply_rows(const orc_mesh *m, const orc_op *op, const double *x, const uint8_t *colmask,
                    const int64_t *rows, int64_t nrows, double *out)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t I = rows[r];
        int i = (int)(I % NX), j = (int)((I / NX) % NY), k = (int)(I / (NX * NY));
        double Ae[MAXNL * MAXNL];
        double acc = 0.0;
        int c0[3], c1[3], idx[3] = {i, j, k};
        for (int d = 0; d < 3; d++) {
            if (idx[d] % p == 0) { c0[d] = idx[d] / p - 1; c1[d] = idx[d] / p; }
            else { c0[d] = c1[d] = idx[d] / p; }
            if (c0[d] < 0) c0[d] = 0;
            if (c1[d] > m->n[d] - 1) c1[d] = m->n[d] - 1;
        }
        for (int cz = c0[2]; cz <= c1[2]; cz++)
            for (int cy = c0[1]; cy <= c1[1]; cy++)
                for (int cx = c0[0]; cx <= c1[0]; cx++) {
                    orc_element_matrix(m, op, cx, cy, cz, Ae);
                    int a = (i - p * cx) + n1 * ((j - p * cy) + n1 * (k - p * cz));
                    for (int b = 0; b < nl; b++) {
                        int bx = b % n1, by = (b / n1) % n1, bz = b / (n1 * n1);
                        int64_t J = gnode(m, cx, cy, cz, bx, by, bz);
                        if (colmask && colmask[J]) continue;
                        acc += Ae[a * nl + b] * x[J];
                    }
                }
        out[r] = acc;
    }
}

/* Same rows with every element entry and x entry taken in absolute value:
 * an upper bound of (|A| |x|)_I used to scale rounding-error tolerances. */
void orc_apply_rows_abs(const orc_mesh *m, const orc_op *op, const double *x, const uint8_t *colmask,
                        const int64_t *rows, int64_t nrows, double *out)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    int64_t NX = nodes_dim(m, 0), NY = nodes_dim(m, 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t I = rows[r];
        int i = (int)(I % NX), j = (int)((I / NX) % NY), k = (int)(I / (NX * NY));
        double Ae[MAXNL * MAXNL];
        double acc = 0.0;
        int c0[3], c1[3], idx[3] = {i, j, k};
        for (int d = 0; d < 3; d++) {
            if (idx[d] % p == 0) { c0[d] = idx[d] / p - 1; c1[d] = idx[d] / p; }
            else { c0[d] = c1[d] = idx[d] / p; }
            if (c0[d] < 0) c0[d] = 0;
            if (c1[d] > m->n[d] - 1) c1[d] = m->n[d] - 1;
        }
        for (int cz = c0[2]; cz <= c1[2]; cz++)
            for (int cy = c0[1]; cy <= c1[1]; cy++)
                for (int cx = c0[0]; cx <= c1[0]; cx++) {
                    orc_element_matrix(m, op, cx, cy, cz, Ae);
                    int a = (i - p * cx) + n1 * ((j - p * cy) + n1 * (k - p * cz));
                    for (int b = 0; b < nl; b++) {
                        int bx = b % n1, by = (b / n1) % n1, bz = b / (n1 * n1);
                        int64_t J = gnode(m, cx, cy, cz, bx, by, bz);
                        if (colmask && colmask[J]) continue;
                        acc += fabs(Ae[a * nl + b]) * fabs(x[J]);
                    }
                }
        out[r] = acc;
    }
}

/* --------------------------------------------------------- load vectors */
/* out_a += sum_cells int N_a f dV, with f given at the nq^3 Gauss points of
 * every cell (cell-major, then qx fastest). */
void orc_load_qp(const orc_mesh *m, int nq, const double *fq, double *out)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    int64_t nq3 = (int64_t)nq * nq * nq;
    for (int cz = 0; cz < m->n[2]; cz++)
        for (int cy = 0; cy < m->n[1]; cy++)
            for (int cx = 0; cx < m->n[0]; cx++) {
                int64_t c = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                double s[MAXNL] = {0.0};
                for (int qz = 0; qz < nq; qz++)
                    for (int qy = 0; qy < nq; qy++)
                        for (int qx = 0; qx < nq; qx++) {
                            double N[MAXNL], G[MAXNL][3];
                            double detj = cell_geometry(m, cx, cy, cz, B[qx], D[qx], B[qy], D[qy], B[qz], D[qz], N, G);
                            double w = gw[qx] * gw[qy] * gw[qz] * detj * fq[c * nq3 + qx + nq * (qy + nq * qz)];
                            for (int a = 0; a < nl; a++) s[a] += w * N[a];
                        }
                for (int az = 0; az < n1; az++)
                    for (int ay = 0; ay < n1; ay++)
                        for (int ax = 0; ax < n1; ax++)
                            out[gnode(m, cx, cy, cz, ax, ay, az)] += s[ax + n1 * (ay + n1 * az)];
            }
}

/* out_a += sum_cells g_c int dN_a/dz dV  (cellwise-constant g). */
void orc_load_gradz(const orc_mesh *m, const double *g, int nq, double *out)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    for (int cz = 0; cz < m->n[2]; cz++)
        for (int cy = 0; cy < m->n[1]; cy++)
            for (int cx = 0; cx < m->n[0]; cx++) {
                int64_t c = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                double s[MAXNL] = {0.0};
                for (int qz = 0; qz < nq; qz++)
                    for (int qy = 0; qy < nq; qy++)
                        for (int qx = 0; qx < nq; qx++) {
                            double N[MAXNL], G[MAXNL][3];
                            double detj = cell_geometry(m, cx, cy, cz, B[qx], D[qx], B[qy], D[qy], B[qz], D[qz], N, G);
                            double w = gw[qx] * gw[qy] * gw[qz] * detj;
                            for (int a = 0; a < nl; a++) s[a] += w * G[a][2];
                        }
                for (int az = 0; az < n1; az++)
                    for (int ay = 0; ay < n1; ay++)
                        for (int ax = 0; ax < n1; ax++)
                            out[gnode(m, cx, cy, cz, ax, ay, az)] += g[c] * s[ax + n1 * (ay + n1 * az)];
            }
}

/* out_a += value * int_face N_a dA over boundary face f (0..5 = x-,x+,y-,y+,z-,z+).
 * General hexahedra: dA = |dx/dxi_1 x dx/dxi_2| dxi_1 dxi_2 on the face. */
void orc_load_face(const orc_mesh *m, int face, double value, int nq, double *out)
{
    int p = m->p, n1 = p + 1;
    int dn = face / 2, side = face % 2;
    int d1 = (dn + 1) % 3, d2 = (dn + 2) % 3;
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    int cn = side ? m->n[dn] - 1 : 0;
    int an = side ? p : 0;
    for (int c2 = 0; c2 < m->n[d2]; c2++)
        for (int c1 = 0; c1 < m->n[d1]; c1++) {
            int cc[3];
            cc[dn] = cn; cc[d1] = c1; cc[d2] = c2;
            for (int a2 = 0; a2 < n1; a2++)
                for (int a1 = 0; a1 < n1; a1++) {
                    double s = 0.0;
                    for (int q2 = 0; q2 < nq; q2++)
                        for (int q1 = 0; q1 < nq; q1++) {
                            double da;
                            if (!m->xyz) {
                                da = cell_h(m, d1, c1) * cell_h(m, d2, c2);
                            } else {
                                /* tangents of the face's isoparametric map */
                                double t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
                                for (int b2 = 0; b2 < n1; b2++)
                                    for (int b1 = 0; b1 < n1; b1++) {
                                        int aa[3];
                                        aa[dn] = an; aa[d1] = b1; aa[d2] = b2;
                                        const double *X = m->xyz + 3 * gnode(m, cc[0], cc[1], cc[2], aa[0], aa[1], aa[2]);
                                        for (int i = 0; i < 3; i++) {
                                            t1[i] += X[i] * D[q1][b1] * B[q2][b2];
                                            t2[i] += X[i] * B[q1][b1] * D[q2][b2];
                                        }
                                    }
                                double nx = t1[1] * t2[2] - t1[2] * t2[1];
                                double ny = t1[2] * t2[0] - t1[0] * t2[2];
                                double nz = t1[0] * t2[1] - t1[1] * t2[0];
                                da = sqrt(nx * nx + ny * ny + nz * nz);
                            }
                            s += gw[q1] * gw[q2] * da * B[q1][a1] * B[q2][a2];
                        }
                    int aa[3];
                    aa[dn] = an; aa[d1] = a1; aa[d2] = a2;
                    out[gnode(m, cc[0], cc[1], cc[2], aa[0], aa[1], aa[2])] += value * s;
                }
        }
}

/* Cell and local coordinate of a point along axis d (closed box). */
static void locate(const orc_mesh *m, int d, double x, int *c, double *xi)
{
    if (m->edges[d]) {
        /* last cell whose lower edge is <= x, within 0 .. n-1 */
        int lo = 0, hi = m->n[d] - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (m->edges[d][mid] <= x) lo = mid; else hi = mid - 1;
        }
        *c = lo;
        *xi = (x - m->edges[d][lo]) / (m->edges[d][lo + 1] - m->edges[d][lo]);
        return;
    }
    double h = cell_h(m, d, 0);
    double s = (x - m->x0[d]) / h;
    int ci = (int)floor(s);
    if (ci < 0) ci = 0;
    if (ci > m->n[d] - 1) ci = m->n[d] - 1;
    *c = ci;
    *xi = s - ci;
}

/* out_a += value * int_{z0}^{z1} N_a(x, y, z) dz along a vertical line. */
void orc_load_line(const orc_mesh *m, double x, double y, double z0, double z1, double value,
                   int nq, double *out)
{
    int p = m->p, n1 = p + 1;
    int cx, cy; double xi, eta;
    locate(m, 0, x, &cx, &xi);
    locate(m, 1, y, &cy, &eta);
    double Bx[3], By[3], dd[3];
    lagrange(p, xi, Bx, dd);
    lagrange(p, eta, By, dd);
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    for (int cz = 0; cz < m->n[2]; cz++) {
        double hz = cell_h(m, 2, cz), zlo = cell_lo(m, 2, cz), zhi = zlo + hz;
        double a = z0 > zlo ? z0 : zlo, b = z1 < zhi ? z1 : zhi;
        if (!(b > a)) continue;
        for (int az = 0; az < n1; az++) {
            double s = 0.0;
            for (int q = 0; q < nq; q++) {
                double z = a + (b - a) * gx[q];
                double Bz[3], dz[3];
                lagrange(p, (z - zlo) / hz, Bz, dz);
                s += gw[q] * (b - a) * Bz[az];
            }
            for (int ay = 0; ay < n1; ay++)
                for (int ax = 0; ax < n1; ax++)
                    out[gnode(m, cx, cy, cz, ax, ay, az)] += value * Bx[ax] * By[ay] * s;
        }
    }
}

/* Triplets of coef * int_{z0}^{z1} N_a N_b dz along a vertical line.
 * Returns the number of triplets written (caller provides room for
 * nz * (p+1)^6 entries). */
int64_t orc_line_mass(const orc_mesh *m, double x, double y, double z0, double z1, double coef,
                      int nq, int64_t *ri, int64_t *ci, double *v)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    int cx, cy; double xi, eta;
    locate(m, 0, x, &cx, &xi);
    locate(m, 1, y, &cy, &eta);
    double Bx[3], By[3], dd[3];
    lagrange(p, xi, Bx, dd);
    lagrange(p, eta, By, dd);
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    int64_t cnt = 0;
    for (int cz = 0; cz < m->n[2]; cz++) {
        double hz = cell_h(m, 2, cz), zlo = cell_lo(m, 2, cz), zhi = zlo + hz;
        double a = z0 > zlo ? z0 : zlo, b = z1 < zhi ? z1 : zhi;
        if (!(b > a)) continue;
        double Mz[3][3] = {{0}};
        for (int q = 0; q < nq; q++) {
            double z = a + (b - a) * gx[q];
            double Bz[3], dz[3];
            lagrange(p, (z - zlo) / hz, Bz, dz);
            for (int s = 0; s < n1; s++)
                for (int t = 0; t < n1; t++) Mz[s][t] += gw[q] * (b - a) * Bz[s] * Bz[t];
        }
        for (int A = 0; A < nl; A++) {
            int ax = A % n1, ay = (A / n1) % n1, az = A / (n1 * n1);
            for (int Bi = 0; Bi < nl; Bi++) {
                int bx = Bi % n1, by = (Bi / n1) % n1, bz = Bi / (n1 * n1);
                ri[cnt] = gnode(m, cx, cy, cz, ax, ay, az);
                ci[cnt] = gnode(m, cx, cy, cz, bx, by, bz);
                v[cnt] = coef * Bx[ax] * By[ay] * Bx[bx] * By[by] * Mz[az][bz];
                cnt++;
            }
        }
    }
    return cnt;
}

/* Values of the FE function u at the nq^3 Gauss points of every cell. */
void orc_eval_qp(const orc_mesh *m, int nq, const double *u, double *out)
{
    int p = m->p, n1 = p + 1;
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    int64_t nq3 = (int64_t)nq * nq * nq;
#pragma omp parallel for collapse(2) schedule(static)
    for (int cz = 0; cz < m->n[2]; cz++)
        for (int cy = 0; cy < m->n[1]; cy++)
            for (int cx = 0; cx < m->n[0]; cx++) {
                int64_t c = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                for (int qz = 0; qz < nq; qz++)
                    for (int qy = 0; qy < nq; qy++)
                        for (int qx = 0; qx < nq; qx++) {
                            double s = 0.0;
                            for (int az = 0; az < n1; az++)
                                for (int ay = 0; ay < n1; ay++)
                                    for (int ax = 0; ax < n1; ax++)
                                        s += B[qx][ax] * B[qy][ay] * B[qz][az] *
                                             u[gnode(m, cx, cy, cz, ax, ay, az)];
                            out[c * nq3 + qx + nq * (qy + nq * qz)] = s;
                        }
            }
}

/* Darcy flux q_h = -k (grad P_h + rho_g e_z) at the nq^3 Gauss points of
 * every cell: out[(c*nq3 + q)*3 + d]. */
void orc_flux_qp(const orc_mesh *m, int nq, const double *kc, const double *P, double rho_g,
                 double *out)
{
    int p = m->p, n1 = p + 1, nl = n1 * n1 * n1;
    double gx[MAXQ], gw[MAXQ];
    gauss01(nq, gx, gw);
    double B[MAXQ][3], D[MAXQ][3];
    for (int q = 0; q < nq; q++) lagrange(p, gx[q], B[q], D[q]);
    int64_t nq3 = (int64_t)nq * nq * nq;
#pragma omp parallel for collapse(2) schedule(static)
    for (int cz = 0; cz < m->n[2]; cz++)
        for (int cy = 0; cy < m->n[1]; cy++)
            for (int cx = 0; cx < m->n[0]; cx++) {
                int64_t c = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                double Pl[MAXNL];
                for (int az = 0; az < n1; az++)
                    for (int ay = 0; ay < n1; ay++)
                        for (int ax = 0; ax < n1; ax++)
                            Pl[ax + n1 * (ay + n1 * az)] = P[gnode(m, cx, cy, cz, ax, ay, az)];
                for (int qz = 0; qz < nq; qz++)
                    for (int qy = 0; qy < nq; qy++)
                        for (int qx = 0; qx < nq; qx++) {
                            double N[MAXNL], G[MAXNL][3];
                            (void)cell_geometry(m, cx, cy, cz, B[qx], D[qx], B[qy], D[qy], B[qz], D[qz], N, G);
                            double g[3] = {0.0, 0.0, 0.0};
                            for (int a = 0; a < nl; a++)
                                for (int d = 0; d < 3; d++) g[d] += G[a][d] * Pl[a];
                            int64_t o = (c * nq3 + qx + nq * (qy + nq * qz)) * 3;
                            out[o + 0] = -kc[c] * g[0];
                            out[o + 1] = -kc[c] * g[1];
                            out[o + 2] = -kc[c] * (g[2] + rho_g);
                        }
            }
}

/* -------------------------------------------------------- linear algebra */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) s += val[e] * x[col[e]];
        y[i] = s;
    }
}

/* r = b - A x with the row sums accumulated in long double. */
void orc_residual_ld(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                     const double *b, const double *x, double *r)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        long double s = (long double)b[i];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
            s -= (long double)val[e] * (long double)x[col[e]];
        r[i] = (double)s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

static void diag_of(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, double *d)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        d[i] = 1.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++)
            if (col[e] == i) { d[i] = val[e]; break; }
    }
}

/* Jacobi-preconditioned conjugate gradients.  Stops when the true residual
 * satisfies ||b - A x|| <= rtol ||b|| (checked whenever the recursive one
 * does) or after maxit iterations.  Returns iterations; *relres gets the
 * final true relative residual. */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
            const double *b, double *x, double rtol, int maxit, double *relres)
{
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double));
    diag_of(n, rowptr, col, val, d);
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    orc_spmv(n, rowptr, col, val, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    int it = 0;
    double rn = sqrt(dot(n, r, r));
    while (rn > rtol * bn && it < maxit) {
        for (int64_t i = 0; i < n; i++) { z[i] = r[i] / d[i]; p[i] = z[i]; }
        double rz = dot(n, r, z);
        while (it < maxit) {
            orc_spmv(n, rowptr, col, val, p, q);
            double pq = dot(n, p, q);
            if (pq == 0.0) break;
            double alpha = rz / pq;
            for (int64_t i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            it++;
            rn = sqrt(dot(n, r, r));
            if (rn <= rtol * bn) break;
            for (int64_t i = 0; i < n; i++) z[i] = r[i] / d[i];
            double rz1 = dot(n, r, z);
            double beta = rz1 / rz;
            rz = rz1;
            for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
        /* true residual; restart from it if the recursion drifted */
        orc_spmv(n, rowptr, col, val, x, q);
        for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
        rn = sqrt(dot(n, r, r));
        if (rn <= rtol * bn) break;
        if (it >= maxit) break;
    }
    *relres = rn / bn;
    free(r); free(z); free(p); free(q); free(d);
    return it;
}

/* Restarted GMRES(m) with right Jacobi preconditioning and modified
 * Gram-Schmidt.  Same stopping rule as orc_pcg. */
int orc_gmres(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *b, double *x, int m, double rtol, int maxit, double *relres)
{
    double *V = malloc((size_t)(m + 1) * n * sizeof(double));
    double *w = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double));
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(m * sizeof(double)), *sn = malloc(m * sizeof(double));
    double *g = malloc((m + 1) * sizeof(double)), *y = malloc(m * sizeof(double));
    diag_of(n, rowptr, col, val, d);
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    int it = 0;
    double rn = 0.0;
    for (;;) {
        orc_spmv(n, rowptr, col, val, x, w);
        for (int64_t i = 0; i < n; i++) V[i] = b[i] - w[i];
        rn = sqrt(dot(n, V, V));
        if (rn <= rtol * bn || it >= maxit) break;
        for (int64_t i = 0; i < n; i++) V[i] /= rn;
        memset(g, 0, (m + 1) * sizeof(double));
        g[0] = rn;
        int j;
        for (j = 0; j < m && it < maxit; j++) {
            double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            for (int64_t i = 0; i < n; i++) z[i] = vj[i] / d[i];
            orc_spmv(n, rowptr, col, val, z, vn);
            for (int i = 0; i <= j; i++) {
                double h = dot(n, vn, V + (size_t)i * n);
                H[i * m + j] = h;
                for (int64_t t = 0; t < n; t++) vn[t] -= h * V[(size_t)i * n + t];
            }
            double hn = sqrt(dot(n, vn, vn));
            H[(j + 1) * m + j] = hn;
            if (hn > 0.0)
                for (int64_t t = 0; t < n; t++) vn[t] /= hn;
            for (int i = 0; i < j; i++) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double r = hypot(a, c);
            cs[j] = a / r; sn[j] = c / r;
            H[j * m + j] = r; H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            it++;
            if (fabs(g[j + 1]) <= rtol * bn * 0.5 || hn == 0.0) { j++; break; }
        }
        for (int i = j - 1; i >= 0; i--) {
            double s = g[i];
            for (int t = i + 1; t < j; t++) s -= H[i * m + t] * y[t];
            y[i] = s / H[i * m + i];
        }
        memset(w, 0, n * sizeof(double));
        for (int i = 0; i < j; i++)
            for (int64_t t = 0; t < n; t++) w[t] += y[i] * V[(size_t)i * n + t];
        for (int64_t t = 0; t < n; t++) x[t] += w[t] / d[t];
    }
    *relres = rn / bn;
    free(V); free(w); free(z); free(d); free(H); free(cs); free(sn); free(g); free(y);
    return it;
}

/* --------------------------------------------------- 3D convolutions */
/* Plain-loop 3D convolution, cross-correlation form with zero padding:
 *   y[n][co][z][y][x] = bias[co] + sum_{ci,dz,dy,dx} w[co][ci][dz][dy][dx]
 *                                       * x[n][ci][z*s+dz-pad][...]
 * Arrays are NCDHW, double precision. */
void orc_conv3d_fwd(const double *x, const double *w, const double *bias, double *y,
                    int N, int Ci, int Co, int D, int H, int W, int ks, int stride, int pad,
                    int Do, int Ho, int Wo)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int n = 0; n < N; n++)
        for (int co = 0; co < Co; co++)
            for (int oz = 0; oz < Do; oz++)
                for (int oy = 0; oy < Ho; oy++)
                    for (int ox = 0; ox < Wo; ox++) {
                        double s = bias ? bias[co] : 0.0;
                        for (int ci = 0; ci < Ci; ci++)
                            for (int dz = 0; dz < ks; dz++) {
                                int iz = oz * stride + dz - pad;
                                if (iz < 0 || iz >= D) continue;
                                for (int dy = 0; dy < ks; dy++) {
                                    int iy = oy * stride + dy - pad;
                                    if (iy < 0 || iy >= H) continue;
                                    for (int dx = 0; dx < ks; dx++) {
                                        int ix = ox * stride + dx - pad;
                                        if (ix < 0 || ix >= W) continue;
                                        s += w[((((int64_t)co * Ci + ci) * ks + dz) * ks + dy) * ks + dx] *
                                             x[((((int64_t)n * Ci + ci) * D + iz) * H + iy) * W + ix];
                                    }
                                }
                            }
                        y[((((int64_t)n * Co + co) * Do + oz) * Ho + oy) * Wo + ox] = s;
                    }
}

/* Gradient of sum(gy * conv(x,w)) with respect to x. */
void orc_conv3d_bwd_data(const double *gy, const double *w, double *gx, int N, int Ci, int Co,
                         int D, int H, int W, int ks, int stride, int pad, int Do, int Ho, int Wo)
{
    memset(gx, 0, sizeof(double) * (size_t)N * Ci * D * H * W);
#pragma omp parallel for collapse(2) schedule(static)
    for (int n = 0; n < N; n++)
        for (int ci = 0; ci < Ci; ci++)
            for (int co = 0; co < Co; co++)
                for (int oz = 0; oz < Do; oz++)
                    for (int oy = 0; oy < Ho; oy++)
                        for (int ox = 0; ox < Wo; ox++) {
                            double g = gy[((((int64_t)n * Co + co) * Do + oz) * Ho + oy) * Wo + ox];
                            for (int dz = 0; dz < ks; dz++) {
                                int iz = oz * stride + dz - pad;
                                if (iz < 0 || iz >= D) continue;
                                for (int dy = 0; dy < ks; dy++) {
                                    int iy = oy * stride + dy - pad;
                                    if (iy < 0 || iy >= H) continue;
                                    for (int dx = 0; dx < ks; dx++) {
                                        int ix = ox * stride + dx - pad;
                                        if (ix < 0 || ix >= W) continue;
                                        gx[((((int64_t)n * Ci + ci) * D + iz) * H + iy) * W + ix] +=
                                            g * w[((((int64_t)co * Ci + ci) * ks + dz) * ks + dy) * ks + dx];
                                    }
                                }
                            }
                        }
}

/* Gradient of sum(gy * conv(x,w)) with respect to w (and bias if gb). */
void orc_conv3d_bwd_weight(const double *x, const double *gy, double *gw, double *gb, int N,
                           int Ci, int Co, int D, int H, int W, int ks, int stride, int pad,
                           int Do, int Ho, int Wo)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int co = 0; co < Co; co++)
        for (int ci = 0; ci < Ci; ci++)
            for (int dz = 0; dz < ks; dz++)
                for (int dy = 0; dy < ks; dy++)
                    for (int dx = 0; dx < ks; dx++) {
                        double s = 0.0;
                        for (int n = 0; n < N; n++)
                            for (int oz = 0; oz < Do; oz++) {
                                int iz = oz * stride + dz - pad;
                                if (iz < 0 || iz >= D) continue;
                                for (int oy = 0; oy < Ho; oy++) {
                                    int iy = oy * stride + dy - pad;
                                    if (iy < 0 || iy >= H) continue;
                                    for (int ox = 0; ox < Wo; ox++) {
                                        int ix = ox * stride + dx - pad;
                                        if (ix < 0 || ix >= W) continue;
                                        s += gy[((((int64_t)n * Co + co) * Do + oz) * Ho + oy) * Wo + ox] *
                                             x[((((int64_t)n * Ci + ci) * D + iz) * H + iy) * W + ix];
                                    }
                                }
                            }
                        gw[((((int64_t)co * Ci + ci) * ks + dz) * ks + dy) * ks + dx] = s;
                    }
    if (gb) {
        for (int co = 0; co < Co; co++) {
            double s = 0.0;
            for (int n = 0; n < N; n++)
                for (int64_t e = 0; e < (int64_t)Do * Ho * Wo; e++)
                    s += gy[((int64_t)n * Co + co) * Do * Ho * Wo + e];
            gb[co] = s;
        }
    }
}

/* Thread count of the parallel loops (timing runs at one thread). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
