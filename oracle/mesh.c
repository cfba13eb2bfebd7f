/*
 * Oracle: grid geometry, Voronoi volumes, edge coefficients, link variables and
 * the Hermitian matrix K-hat.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper passages followed:
 *  - Sec. 3, Voronoi regions V_j and mass lumping F_2 ~ sum |V_j| (...): vol.
 *  - Corollary on simplex edge coefficients and the Remark giving
 *    alpha = 1/2 cot(theta) for triangles; alpha_jk is summed over all
 *    simplices adjacent to the edge.  2D grids: the Remark's cotangent,
 *    triangle by triangle; simplicial meshes (triangles and tetrahedra):
 *    the Corollary's system M alpha = b per simplex (for triangles a second
 *    route to the Remark's numbers), and the control volume of a node as
 *    the sum of its shares 1/(2 dim) alpha_e |e|^2 over each simplex's edges
 *    at it (the Voronoi region's part of a simplex that holds its
 *    circumcentre).
 *    3D (cube grid, degenerate Delaunay): alpha = |dual Voronoi facet| / |e|.
 *  - Link variable U_jk = exp(-i int_{x_k}^{x_j} e_jk . A(w) dw), integral taken
 *    along the straight edge; evaluated here by 3-point Gauss-Legendre, which is
 *    exact for the linear potentials A = M r.  The dipole potential of the
 *    experiments (Sec. 4.1), A_d(x) = m x (x - x0) / |x - x0|^3 scaled by mu,
 *    has a closed-form edge integral: with a = x_k - x0 and e = x_j - x_k,
 *    e . (m x (a + t e)) = m . (a x e) for every t, and
 *    int_0^1 q(t)^(-3/2) dt, q = A t^2 + B t + C (A = |e|^2, B = 2 a.e,
 *    C = |a|^2), is [(4 A t + 2 B) / ((4 A C - B^2) sqrt q)] from 0 to 1.
 *  - Discrete kinetic energy operator (edge form) and the Remark K = D^-1 K-hat:
 *    K-hat_jj = sum alpha, K-hat_jk = -alpha U_jk, K-hat_kj = -alpha conj(U_jk).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int64_t node_index(const orc_mesh *m, const int64_t *c)
{
    int64_t idx = 0, s = 1;
    for (int a = 0; a < m->dim; ++a) { idx += c[a] * s; s *= m->N[a]; }
    return idx;
}

static void node_coords(const orc_mesh *m, int64_t i, int64_t *c)
{
    for (int a = 0; a < 3; ++a) c[a] = 0;
    for (int a = 0; a < m->dim; ++a) { c[a] = i % m->N[a]; i /= m->N[a]; }
}

/* A(r) = amat r */
static void potential(const double *amat, const double *r, double *A)
{
    for (int a = 0; a < 3; ++a)
        A[a] = amat[3 * a + 0] * r[0] + amat[3 * a + 1] * r[1] + amat[3 * a + 2] * r[2];
}

/* line integral of e.A along the straight edge from xk to xj */
static double edge_integral(const double *amat, const double *xk, const double *xj)
{
    /* Gauss-Legendre, 3 points on [0,1] */
    static const double t[3] = {0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852};
    static const double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double e[3], s = 0.0;
    for (int a = 0; a < 3; ++a) e[a] = xj[a] - xk[a];
    for (int g = 0; g < 3; ++g) {
        double r[3], A[3];
        for (int a = 0; a < 3; ++a) r[a] = xk[a] + t[g] * e[a];
        potential(amat, r, A);
        s += w[g] * (e[0] * A[0] + e[1] * A[1] + e[2] * A[2]);
    }
    return s;
}

/* the same integral for mu A_d (dip = {mu, m[3], x0[3]}), closed form */
static double edge_integral_dipole(const double *dip, const double *xk, const double *xj)
{
    const double mu = dip[0], *mm = dip + 1, *x0 = dip + 4;
    double a[3], e[3];
    for (int c = 0; c < 3; ++c) { a[c] = xk[c] - x0[c]; e[c] = xj[c] - xk[c]; }
    const double axe[3] = {a[1] * e[2] - a[2] * e[1], a[2] * e[0] - a[0] * e[2], a[0] * e[1] - a[1] * e[0]};
    const double num = mm[0] * axe[0] + mm[1] * axe[1] + mm[2] * axe[2];
    const double A = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    const double B = 2.0 * (a[0] * e[0] + a[1] * e[1] + a[2] * e[2]);
    const double C = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    const double disc = 4.0 * A * C - B * B;
    if (!(disc > 0.0)) return 0.0;  /* the edge's line passes through x0: m . (a x e) = 0 */
    const double F1 = (4.0 * A + 2.0 * B) / (disc * sqrt(A + B + C));
    const double F0 = 2.0 * B / (disc * sqrt(C));
    return mu * num * (F1 - F0);
}

/* 1/2 cot of the angle at vertex p between the edges p->q and p->r
 * (Remark: alpha = 1/2 t / sqrt(1 - t^2), t the cosine of the angle). */
static double half_cot(const double *p, const double *q, const double *r)
{
    double u[2] = {q[0] - p[0], q[1] - p[1]}, v[2] = {r[0] - p[0], r[1] - p[1]};
    double nu = sqrt(u[0] * u[0] + u[1] * u[1]), nv = sqrt(v[0] * v[0] + v[1] * v[1]);
    double t = (u[0] * v[0] + u[1] * v[1]) / (nu * nv);
    return 0.5 * t / sqrt(1.0 - t * t);
}

typedef struct { int64_t j, k; double alpha; } edge_rec;

/* position of the axis edge (lo, hi) in the edge list built below (edges are
   listed axis by axis, each axis in ascending order of its lower node), or -1
   if (lo, hi) is not an axis edge */
static int64_t edge_slot(const orc_mesh *m, int64_t lo, int64_t hi)
{
    int64_t cl[3], ch[3];
    node_coords(m, lo, cl);
    node_coords(m, hi, ch);
    int ax = -1, ndiff = 0;
    for (int a = 0; a < m->dim; ++a)
        if (cl[a] != ch[a]) { ax = a; ++ndiff; }
    if (ndiff != 1 || ch[ax] != cl[ax] + 1) return -1;
    int64_t off = 0;
    for (int a = 0; a < ax; ++a) off += m->n / m->N[a] * (m->N[a] - 1);
    int64_t r = 0, s = 1;
    for (int a = 0; a < m->dim; ++a) {
        int64_t extent = (a == ax) ? m->N[a] - 1 : m->N[a];
        r += cl[a] * s;
        s *= extent;
    }
    return off + r;
}

static int mesh_build(int dim, const int64_t *N, const double *L, const double *amat, const double *dip,
                      orc_mesh **out);

/* edge list -> edge arrays, link variables and K-hat in CSR (shared by the
   grid and simplicial builders; the caller frees E) */
static void finish_mesh(orc_mesh *m, const edge_rec *E, int64_t ne, const double *amat, const double *dip)
{
    const int64_t n = m->n;
    m->ne = ne;
    m->ej = malloc((size_t)ne * sizeof(int64_t));
    m->ek = malloc((size_t)ne * sizeof(int64_t));
    m->alpha = malloc((size_t)ne * sizeof(double));
    m->U = malloc((size_t)ne * sizeof(cplx));
    for (int64_t q = 0; q < ne; ++q) {
        m->ej[q] = E[q].j;
        m->ek[q] = E[q].k;
        m->alpha[q] = E[q].alpha;
        double phi = dip ? edge_integral_dipole(dip, &m->x[3 * E[q].k], &m->x[3 * E[q].j])
                         : edge_integral(amat, &m->x[3 * E[q].k], &m->x[3 * E[q].j]);
        m->U[q] = cexp(-I * phi);
    }

    /* K-hat in CSR.  Row i: diagonal sum of alpha over incident edges; for the
       edge (j,k): K(j,k) = -alpha U_jk, K(k,j) = -alpha conj(U_jk). */
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t q = 0; q < ne; ++q) { cnt[m->ej[q]]++; cnt[m->ek[q]]++; }
    m->rp = malloc((size_t)(n + 1) * sizeof(int64_t));
    m->rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) m->rp[i + 1] = m->rp[i] + cnt[i] + 1;
    int64_t nnz = m->rp[n];
    m->ci = malloc((size_t)nnz * sizeof(int64_t));
    m->kv = malloc((size_t)nnz * sizeof(cplx));
    int64_t *fill = calloc((size_t)n, sizeof(int64_t));
    double *diag = calloc((size_t)n, sizeof(double));
    /* write (column, value) pairs, then sort each row by column */
    typedef struct { int64_t c; cplx v; } ent;
    ent *tmp = malloc((size_t)nnz * sizeof(ent));
    for (int64_t q = 0; q < ne; ++q) {
        int64_t j = m->ej[q], k = m->ek[q];
        double al = m->alpha[q];
        tmp[m->rp[j] + fill[j]].c = k;
        tmp[m->rp[j] + fill[j]].v = -al * m->U[q];
        fill[j]++;
        tmp[m->rp[k] + fill[k]].c = j;
        tmp[m->rp[k] + fill[k]].v = -al * conj(m->U[q]);
        fill[k]++;
        diag[j] += al;
        diag[k] += al;
    }
    for (int64_t i = 0; i < n; ++i) {
        tmp[m->rp[i] + fill[i]].c = i;
        tmp[m->rp[i] + fill[i]].v = diag[i];
        /* insertion sort on column */
        for (int64_t p = m->rp[i] + 1; p < m->rp[i + 1]; ++p) {
            ent e = tmp[p];
            int64_t q = p - 1;
            while (q >= m->rp[i] && tmp[q].c > e.c) { tmp[q + 1] = tmp[q]; --q; }
            tmp[q + 1] = e;
        }
    }
    for (int64_t p = 0; p < nnz; ++p) { m->ci[p] = tmp[p].c; m->kv[p] = tmp[p].v; }
    free(tmp);
    free(fill);
    free(diag);
    free(cnt);
}



int orc_mesh_build(int dim, const int64_t *N, const double *L, const double *amat,
                   orc_mesh **out)
{
    return mesh_build(dim, N, L, amat, NULL, out);
}

int orc_mesh_build_dipole(int dim, const int64_t *N, const double *L, double mu, const double *m,
                          const double *x0, orc_mesh **out)
{
    static const double zero[9] = {0};
    double dip[7] = {mu, m[0], m[1], m[2], x0[0], x0[1], x0[2]};
    return mesh_build(dim, N, L, zero, dip, out);
}

static int mesh_build(int dim, const int64_t *N, const double *L, const double *amat, const double *dip,
                      orc_mesh **out)
{
    if (dim != 2 && dim != 3) return ORC_ERR_ARG;
    orc_mesh *m = calloc(1, sizeof(*m));
    m->dim = dim;
    m->grid = 1;
    m->n = 1;
    for (int a = 0; a < 3; ++a) { m->N[a] = 1; m->L[a] = 0; m->h[a] = 0; }
    for (int a = 0; a < dim; ++a) {
        if (N[a] < 2) { free(m); return ORC_ERR_ARG; }
        m->N[a] = N[a];
        m->L[a] = L[a];
        m->h[a] = L[a] / (double)(N[a] - 1);
        m->n *= N[a];
    }
    memcpy(m->amat, amat, 9 * sizeof(double));
    const int64_t n = m->n;

    /* node coordinates, domain centred at the origin */
    m->x = calloc((size_t)n * 3, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        node_coords(m, i, c);
        for (int a = 0; a < dim; ++a) m->x[3 * i + a] = -0.5 * m->L[a] + (double)c[a] * m->h[a];
    }

    /* Voronoi region of a tensor-grid node, clipped to the domain: a box whose
       extent on each axis is half the spacing towards each existing neighbour */
    m->vol = malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        node_coords(m, i, c);
        double v = 1.0;
        for (int a = 0; a < dim; ++a) {
            double ext = 0.0;
            if (c[a] > 0) ext += 0.5 * m->h[a];
            if (c[a] < m->N[a] - 1) ext += 0.5 * m->h[a];
            v *= ext;
        }
        m->vol[i] = v;
    }

    /* axis edges: (j, k) with j = k + stride_a */
    int64_t ne_max = 0;
    for (int a = 0; a < dim; ++a) ne_max += n / m->N[a] * (m->N[a] - 1);
    edge_rec *E = calloc((size_t)ne_max, sizeof(edge_rec));
    int64_t ne = 0;
    int64_t stride[3] = {1, m->N[0], m->N[0] * m->N[1]};
    for (int a = 0; a < dim; ++a)
        for (int64_t k = 0; k < n; ++k) {
            int64_t c[3];
            node_coords(m, k, c);
            if (c[a] == m->N[a] - 1) continue;
            E[ne].j = k + stride[a];
            E[ne].k = k;
            E[ne].alpha = 0.0;
            ++ne;
        }

    if (dim == 2) {
        /* Delaunay triangulation of each grid cell by the diagonal (i,j)-(i+1,j+1);
           accumulate 1/2 cot(opposite angle) into every axis edge.  The diagonal's
           own coefficient is 1/2 cot(90 deg) = 0, so it carries no term. */
        for (int64_t cy = 0; cy + 1 < m->N[1]; ++cy)
            for (int64_t cx = 0; cx + 1 < m->N[0]; ++cx) {
                int64_t c00[3] = {cx, cy, 0}, c10[3] = {cx + 1, cy, 0};
                int64_t c01[3] = {cx, cy + 1, 0}, c11[3] = {cx + 1, cy + 1, 0};
                int64_t p00 = node_index(m, c00), p10 = node_index(m, c10);
                int64_t p01 = node_index(m, c01), p11 = node_index(m, c11);
                int64_t tri[2][3] = {{p00, p10, p11}, {p00, p01, p11}};
                for (int t = 0; t < 2; ++t)
                    for (int e = 0; e < 3; ++e) {
                        int64_t a0 = tri[t][e], a1 = tri[t][(e + 1) % 3], opp = tri[t][(e + 2) % 3];
                        double coef = half_cot(&m->x[3 * opp], &m->x[3 * a0], &m->x[3 * a1]);
                        int64_t lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
                        int64_t q = edge_slot(m, lo, hi);
                        if (q >= 0) E[q].alpha += coef;
                    }
            }
    } else {
        /* 3D: the dual Voronoi facet of an axis edge is the axis-normal box of
           half-spacings around the edge midpoint, clipped to the domain */
        for (int64_t q = 0; q < ne; ++q) {
            int64_t ck[3], cj[3];
            node_coords(m, E[q].k, ck);
            node_coords(m, E[q].j, cj);
            int ax = 0;
            for (int a = 0; a < 3; ++a) if (cj[a] != ck[a]) ax = a;
            double area = 1.0;
            for (int b = 0; b < 3; ++b) {
                if (b == ax) continue;
                double ext = 0.0;
                if (ck[b] > 0) ext += 0.5 * m->h[b];
                if (ck[b] < m->N[b] - 1) ext += 0.5 * m->h[b];
                area *= ext;
            }
            E[q].alpha = area / m->h[ax];
        }
    }

    finish_mesh(m, E, ne, amat, dip);
    free(E);
    *out = m;
    return ORC_OK;
}

/* ---------------------------------------------------------- simplicial --- */
/* M a = b for m x m (m <= 6), Gaussian elimination with partial pivoting;
   M and b are overwritten; 0 if singular */
static int solve_small(int m, double M[6][6], double b[6], double a[6])
{
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (!(fabs(M[piv][c]) > 0.0)) return 0;
        for (int k = 0; k < m; ++k) { double t = M[c][k]; M[c][k] = M[piv][k]; M[piv][k] = t; }
        double t = b[c]; b[c] = b[piv]; b[piv] = t;
        for (int r = c + 1; r < m; ++r) {
            double f = M[r][c] / M[c][c];
            for (int k = c; k < m; ++k) M[r][k] -= f * M[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int c = m - 1; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < m; ++k) s -= M[c][k] * a[k];
        a[c] = s / M[c][c];
    }
    return 1;
}

static int cmp_edge(const void *x, const void *y)
{
    const edge_rec *a = x, *b = y;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return 0;
}

/* index of the edge (hi, lo) in the sorted list */
static int64_t find_edge(const edge_rec *E, int64_t ne, int64_t hi, int64_t lo)
{
    int64_t a = 0, b = ne - 1;
    while (a <= b) {
        int64_t c = (a + b) / 2;
        if (E[c].j == hi && E[c].k == lo) return c;
        if (E[c].j < hi || (E[c].j == hi && E[c].k < lo)) a = c + 1;
        else b = c - 1;
    }
    return -1;
}

/* |S| of the simplex with vertex coordinates P[0..dim] (rows of 3) */
static double simplex_volume(int dim, const double P[4][3])
{
    double u[3], v[3], w[3];
    for (int c = 0; c < 3; ++c) { u[c] = P[1][c] - P[0][c]; v[c] = P[2][c] - P[0][c]; }
    if (dim == 2) return 0.5 * fabs(u[0] * v[1] - u[1] * v[0]);
    for (int c = 0; c < 3; ++c) w[c] = P[3][c] - P[0][c];
    return fabs(u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                u[2] * (v[0] * w[1] - v[1] * w[0])) / 6.0;
}

static int simplex_build(int dim, int64_t n, const double *x, int64_t ncell, const int64_t *cells,
                         const double *amat, const double *dip, orc_mesh **out)
{
    const int nv = dim + 1, ned = dim * (dim + 1) / 2;
    if ((dim != 2 && dim != 3) || n < dim + 1 || ncell < 1) return ORC_ERR_ARG;
    for (int64_t t = 0; t < nv * ncell; ++t)
        if (cells[t] < 0 || cells[t] >= n) return ORC_ERR_ARG;
    orc_mesh *m = calloc(1, sizeof(*m));
    m->dim = dim;
    m->grid = 0;
    m->n = n;
    m->N[0] = n;
    m->N[1] = m->N[2] = 1;
    for (int a = 0; a < 9; ++a) m->amat[a] = amat[a];
    m->x = calloc((size_t)n * 3, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < dim; ++c) m->x[3 * i + c] = x[dim * i + c];
    m->vol = calloc((size_t)n, sizeof(double));
    /* the local edges of a simplex: vertex pairs (a, b), a < b */
    int ea[6], eb[6], q = 0;
    for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b) { ea[q] = a; eb[q] = b; ++q; }
    /* the distinct edges, (j, k) with j > k, in ascending order */
    edge_rec *E = malloc((size_t)(ned * ncell) * sizeof(edge_rec));
    for (int64_t t = 0; t < ncell; ++t)
        for (int e = 0; e < ned; ++e) {
            int64_t a = cells[nv * t + ea[e]], b = cells[nv * t + eb[e]];
            E[ned * t + e].j = a > b ? a : b;
            E[ned * t + e].k = a > b ? b : a;
            E[ned * t + e].alpha = 0.0;
        }
    qsort(E, (size_t)(ned * ncell), sizeof(edge_rec), cmp_edge);
    int64_t ne = 0;
    for (int64_t r = 0; r < ned * ncell; ++r)
        if (ne == 0 || cmp_edge(&E[ne - 1], &E[r]) != 0) E[ne++] = E[r];
    /* per simplex: the Corollary's system M alpha = b for its edge
       coefficients, M_ij = <e_i, e_j>^2, b_i = |S| |e_i|^2; then each
       vertex's share 1/(2 dim) alpha_e |e|^2 of each of its edges */
    for (int64_t t = 0; t < ncell; ++t) {
        const int64_t *p = &cells[nv * t];
        double P[4][3] = {{0}};
        for (int a = 0; a < nv; ++a)
            for (int c = 0; c < 3; ++c) P[a][c] = m->x[3 * p[a] + c];
        const double vol = simplex_volume(dim, P);
        if (!(vol > 0.0)) { free(E); orc_mesh_free(m); return ORC_ERR_ARG; }
        double e[6][3], M[6][6], bb[6], al[6], l2[6];
        for (int i = 0; i < ned; ++i) {
            for (int c = 0; c < 3; ++c) e[i][c] = P[eb[i]][c] - P[ea[i]][c];
            l2[i] = e[i][0] * e[i][0] + e[i][1] * e[i][1] + e[i][2] * e[i][2];
            bb[i] = vol * l2[i];
        }
        for (int i = 0; i < ned; ++i)
            for (int j = 0; j < ned; ++j) {
                double d = e[i][0] * e[j][0] + e[i][1] * e[j][1] + e[i][2] * e[j][2];
                M[i][j] = d * d;
            }
        if (!solve_small(ned, M, bb, al)) { free(E); orc_mesh_free(m); return ORC_ERR_ARG; }
        for (int i = 0; i < ned; ++i) {
            int64_t a = p[ea[i]], c = p[eb[i]];
            int64_t r = find_edge(E, ne, a > c ? a : c, a > c ? c : a);
            E[r].alpha += al[i];
            m->vol[a] += al[i] * l2[i] / (2.0 * dim);
            m->vol[c] += al[i] * l2[i] / (2.0 * dim);
        }
    }
    finish_mesh(m, E, ne, amat, dip);
    free(E);
    *out = m;
    return ORC_OK;
}

int orc_mesh_build_tri(int64_t n, const double *xy, int64_t ntri, const int64_t *tri, const double *amat,
                       orc_mesh **out)
{
    return simplex_build(2, n, xy, ntri, tri, amat, NULL, out);
}

int orc_mesh_build_tri_dipole(int64_t n, const double *xy, int64_t ntri, const int64_t *tri, double mu,
                              const double *mm, const double *x0, orc_mesh **out)
{
    static const double zero[9] = {0};
    double dip[7] = {mu, mm[0], mm[1], mm[2], x0[0], x0[1], x0[2]};
    return simplex_build(2, n, xy, ntri, tri, zero, dip, out);
}

int orc_mesh_build_tet(int64_t n, const double *xyz, int64_t ntet, const int64_t *tet, const double *amat,
                       orc_mesh **out)
{
    return simplex_build(3, n, xyz, ntet, tet, amat, NULL, out);
}

int orc_mesh_build_tet_dipole(int64_t n, const double *xyz, int64_t ntet, const int64_t *tet, double mu,
                              const double *mm, const double *x0, orc_mesh **out)
{
    static const double zero[9] = {0};
    double dip[7] = {mu, mm[0], mm[1], mm[2], x0[0], x0[1], x0[2]};
    return simplex_build(3, n, xyz, ntet, tet, zero, dip, out);
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->x); free(m->vol); free(m->ej); free(m->ek); free(m->alpha); free(m->U);
    free(m->rp); free(m->ci); free(m->kv);
    free(m);
}
