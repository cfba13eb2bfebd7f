/*
 * Oracle: smoothed-aggregation AMG with one pre- and one post-smoothing step of
 * symmetric Gauss-Seidel (Sec. 4.1: the preconditioner R_k = AMG_k(H, D .),
 * H = K-hat + 2 D |psi|^2; the experiments use smoothed aggregation with 1+1
 * symmetric Gauss-Seidel steps).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper fixes only "smoothed aggregation, V-cycle, 1 pre + 1 post symmetric
 * Gauss-Seidel, Hermitian AMG_k".  Every other choice below is a stated reading
 * (Vanek-Mandel-Brezina smoothed aggregation with deterministic distance-2
 * maximal-independent-set aggregation):
 *   strength      : every structural off-diagonal entry (theta = 0)
 *   priorities    : the smaller index first (the greedy pass of standard
 *                   aggregation; hashed priorities gave sparser, irregular roots
 *                   and a V-cycle that weakens as the grid is refined)
 *   roots         : scan by ascending index; a node becomes a root iff no root
 *                   lies within graph distance 2
 *   phase A       : a non-root neighbour of a root joins that root
 *   phase B       : every other node joins the aggregate of its phase-A-assigned
 *                   neighbour whose root has the smallest index (phase-A state only)
 *   numbering     : aggregates ordered by ascending root index
 *   tentative P   : T(i, a) = 1 / sqrt(|a|)   (near-null-space vector 1)
 *   smoothing     : P = T - omega D^-1 A T, omega = (4/3) / rho~, rho~ the estimate of
 *                   rho(D^-1 A) after 20 power-iteration steps from the start
 *                   s_i = (h1_i - 1/2) + i (h2_i - 1/2), h = fmix32(i ^ salt) / 2^32
 *                   (salts 0x2545F491, 0x6C8E9CF5): y = D^-1 A x_{k-1},
 *                   rho_k = ||y|| / ||x_{k-1}||, x_k = y / ||y||
 *   restriction   : R = P^H
 *   Galerkin      : A_{l+1} = R A P, entries i <= j computed, A(j,i) = conj A(i,j),
 *                   diagonal real
 *   stopping      : stop at n_l <= max_coarse, at l = max_levels - 1, or when an
 *                   aggregation keeps more than 0.85 n_l nodes
 *   coarse solve  : dense Cholesky of the coarsest operator
 *   colours       : level 0 of a tensor grid: parity of the index sum; otherwise
 *                   greedy in ascending index order, smallest colour unused by
 *                   already coloured neighbours, followed by two iterated-greedy
 *                   passes (classes in reverse order)
 *   SGS sweep     : colours 0 .. C-1, then C-2 .. 0
 *   V-cycle       : x = SGS(0, b); r = b - A x; x += P V(R r); x = SGS(x, b)
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* MurmurHash3 fmix32 (Appleby, public domain description) */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* aggregation priority: the smaller index first */
static uint64_t mis_key(int64_t i, int l)
{
    (void)l;
    return ~(uint64_t)i;
}
#define ORC_RECOLOUR_PASSES 2

/* colour priority: the smaller index first (on the regular aggregates of a
 * grid the index order colours the coarse graphs with about half the colours
 * of a degree or hash order) */
static uint64_t color_key(int64_t i, int64_t deg, int l)
{
    (void)deg;
    (void)l;
    return ~(uint64_t)i;
}

typedef struct { uint64_t key; int64_t i; } keyed;

static int cmp_keyed_desc(const void *a, const void *b)
{
    uint64_t x = ((const keyed *)a)->key, y = ((const keyed *)b)->key;
    return (x < y) - (x > y);
}

static int64_t *order_by_key(int64_t n, int l, uint64_t (*kf)(int64_t, int))
{
    keyed *k = malloc((size_t)n * sizeof(keyed));
    for (int64_t i = 0; i < n; ++i) { k[i].key = kf(i, l); k[i].i = i; }
    qsort(k, (size_t)n, sizeof(keyed), cmp_keyed_desc);
    int64_t *ord = malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) ord[i] = k[i].i;
    free(k);
    return ord;
}

/* --------------------------------------------------------- aggregation --- */
static int aggregate(orc_level *L, int l)
{
    const int64_t n = L->n;
    int64_t *ord = order_by_key(n, l, mis_key);
    char *blocked = calloc((size_t)n, 1), *isroot = calloc((size_t)n, 1);
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = ord[t];
        if (blocked[i]) continue;
        isroot[i] = 1;
        blocked[i] = 1;
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            int64_t j = L->ci[p];
            blocked[j] = 1;
            for (int64_t q = L->rp[j]; q < L->rp[j + 1]; ++q) blocked[L->ci[q]] = 1;
        }
    }
    free(ord);
    free(blocked);

    int64_t *rootA = malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        rootA[i] = -1;
        if (isroot[i]) { rootA[i] = i; continue; }
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            int64_t j = L->ci[p];
            if (j != i && isroot[j] && (rootA[i] < 0 || mis_key(j, l) > mis_key(rootA[i], l)))
                rootA[i] = j;
        }
    }
    int64_t *root = malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        root[i] = rootA[i];
        if (rootA[i] >= 0) continue;
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            int64_t j = L->ci[p];
            if (j == i || rootA[j] < 0) continue;
            if (root[i] < 0 || mis_key(rootA[j], l) > mis_key(root[i], l)) root[i] = rootA[j];
        }
    }
    int64_t *id = malloc((size_t)n * sizeof(int64_t));
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) id[i] = isroot[i] ? nc++ : -1;
    int rc = ORC_OK;
    L->agg = malloc((size_t)n * sizeof(int64_t));
    L->root = malloc((size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (isroot[i]) L->root[id[i]] = i;
        if (root[i] < 0) { rc = ORC_ERR_AGGREGATION; L->agg[i] = -1; }
        else L->agg[i] = id[root[i]];
    }
    L->nc = nc;
    free(id); free(root); free(rootA); free(isroot);
    return rc;
}

/* ------------------------------------------------------------ colours --- */
static void colour_level(orc_level *L, int l, int grid_dim, const int64_t *grid_N)
{
    const int64_t n = L->n;
    L->color = malloc((size_t)n * sizeof(int32_t));
    if (l == 0 && grid_dim > 0) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t r = i, s = 0;
            for (int a = 0; a < grid_dim; ++a) { s += r % grid_N[a]; r /= grid_N[a]; }
            L->color[i] = (int32_t)(s % 2);
        }
        L->ncolors = n > 1 ? 2 : 1;
        return;
    }
    for (int64_t i = 0; i < n; ++i) L->color[i] = -1;
    keyed *kk = malloc((size_t)n * sizeof(keyed));
    for (int64_t i = 0; i < n; ++i) {
        int64_t deg = 0;
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) deg += L->ci[p] != i;
        kk[i].key = color_key(i, deg, l);
        kk[i].i = i;
    }
    qsort(kk, (size_t)n, sizeof(keyed), cmp_keyed_desc);
    int64_t *ord = malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) ord[i] = kk[i].i;
    free(kk);
    int maxc = 0;
    char *used = calloc((size_t)n + 2, 1);
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = ord[t];
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            int32_t c = L->color[L->ci[p]];
            if (L->ci[p] != i && c >= 0) used[c] = 1;
        }
        int32_t c = 0;
        while (used[c]) ++c;
        L->color[i] = c;
        if (c + 1 > maxc) maxc = c + 1;
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            int32_t cc = L->color[L->ci[p]];
            if (cc >= 0) used[cc] = 0;
        }
    }
    free(ord);
    /* iterated greedy (Culberson): greedy once more with the vertices taken a
     * colour class at a time, the classes in reverse order (a class is an
     * independent set, so the order inside it does not matter); this never
     * needs more colours than there are classes and often fewer */
    int32_t *nw = malloc((size_t)n * sizeof(int32_t));
    for (int pass = 0; pass < ORC_RECOLOUR_PASSES; ++pass) {
        for (int64_t i = 0; i < n; ++i) nw[i] = -1;
        int newmax = 0;
        for (int32_t cls = maxc - 1; cls >= 0; --cls)
            for (int64_t i = 0; i < n; ++i) {
                if (L->color[i] != cls) continue;
                for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
                    if (L->ci[p] != i && nw[L->ci[p]] >= 0) used[nw[L->ci[p]]] = 1;
                int32_t c = 0;
                while (used[c]) ++c;
                nw[i] = c;
                if (c + 1 > newmax) newmax = c + 1;
                for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
                    if (nw[L->ci[p]] >= 0) used[nw[L->ci[p]]] = 0;
            }
        memcpy(L->color, nw, (size_t)n * sizeof(int32_t));
        maxc = newmax;
    }
    free(nw);
    free(used);
    L->ncolors = maxc;
}

/* ------------------------------------------------------ prolongation --- */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static double diag_re(const orc_level *L, int64_t i)
{
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
        if (L->ci[p] == i) return creal(L->v[p]);
    return 0.0;
}

/* rho(D^-1 A) estimated by ORC_RHO_STEPS power-iteration steps from a fixed
 * counter-hash start vector (the estimate PyAMG's smoothed aggregation uses
 * in place of a bound; the Gershgorin bound over-states rho and under-smooths P) */
#define ORC_RHO_STEPS 20
static double rho_estimate(const orc_level *L)
{
    const int64_t n = L->n;
    cplx *x = malloc((size_t)n * sizeof(cplx)), *y = malloc((size_t)n * sizeof(cplx));
    for (int64_t i = 0; i < n; ++i) {
        const double a = (double)fmix32((uint32_t)i ^ 0x2545F491u) / 4294967296.0 - 0.5;
        const double b = (double)fmix32((uint32_t)i ^ 0x6C8E9CF5u) / 4294967296.0 - 0.5;
        x[i] = a + I * b;
    }
    double xn = 0.0;
    for (int64_t i = 0; i < n; ++i) xn += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    xn = sqrt(xn);
    double rho = 0.0;
    for (int k = 0; k < ORC_RHO_STEPS; ++k) {
        double yn = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            cplx s = 0.0;
            for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) s += L->v[p] * x[L->ci[p]];
            y[i] = s / diag_re(L, i);
            yn += creal(y[i]) * creal(y[i]) + cimag(y[i]) * cimag(y[i]);
        }
        yn = sqrt(yn);
        rho = yn / xn;
        for (int64_t i = 0; i < n; ++i) x[i] = y[i] / yn;
        xn = 1.0;
    }
    free(x);
    free(y);
    return rho;
}

static void build_p(orc_level *L)
{
    const int64_t n = L->n, nc = L->nc;
    int64_t *size = calloc((size_t)nc, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) size[L->agg[i]]++;

    L->omega = (4.0 / 3.0) / rho_estimate(L);

    /* pattern: row i has the aggregates of {i} and its neighbours */
    L->prp = malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t cap = L->rp[n];
    L->pci = malloc((size_t)cap * sizeof(int64_t));
    L->pv = malloc((size_t)cap * sizeof(cplx));
    int64_t nnz = 0, maxrow = 1;
    for (int64_t i = 0; i < n; ++i)
        if (L->rp[i + 1] - L->rp[i] > maxrow) maxrow = L->rp[i + 1] - L->rp[i];
    int64_t *buf = malloc((size_t)maxrow * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        L->prp[i] = nnz;
        int64_t m = 0;
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) buf[m++] = L->agg[L->ci[p]];
        qsort(buf, (size_t)m, sizeof(int64_t), cmp_i64);
        int64_t u = 0;
        for (int64_t t = 0; t < m; ++t)
            if (u == 0 || buf[t] != buf[u - 1]) buf[u++] = buf[t];
        double dii = diag_re(L, i);
        for (int64_t t = 0; t < u; ++t) {
            int64_t a = buf[t];
            double ta = 1.0 / sqrt((double)size[a]);
            cplx at = 0;
            for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
                if (L->agg[L->ci[p]] == a) at += L->v[p] * ta;
            cplx val = (L->agg[i] == a ? ta : 0.0) - (L->omega / dii) * at;
            L->pci[nnz] = a;
            L->pv[nnz] = val;
            ++nnz;
        }
    }
    L->prp[n] = nnz;
    free(buf);
    free(size);

    /* R = P^H by transposition; rows of R list fine indices in ascending order */
    L->rrp = calloc((size_t)nc + 1, sizeof(int64_t));
    for (int64_t p = 0; p < nnz; ++p) L->rrp[L->pci[p] + 1]++;
    for (int64_t a = 0; a < nc; ++a) L->rrp[a + 1] += L->rrp[a];
    L->rci = malloc((size_t)nnz * sizeof(int64_t));
    L->rv = malloc((size_t)nnz * sizeof(cplx));
    int64_t *fill = calloc((size_t)nc, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = L->prp[i]; p < L->prp[i + 1]; ++p) {
            int64_t a = L->pci[p], q = L->rrp[a] + fill[a]++;
            L->rci[q] = i;
            L->rv[q] = conj(L->pv[p]);
        }
    free(fill);
}

/* A_{l+1} = R A P, Hermitian by construction */
static void galerkin(const orc_level *L, orc_level *C)
{
    const int64_t nc = L->nc;
    C->n = nc;
    int64_t *mark = malloc((size_t)nc * sizeof(int64_t));
    for (int64_t a = 0; a < nc; ++a) mark[a] = -1;
    int64_t *list = malloc((size_t)nc * sizeof(int64_t));
    C->rp = malloc((size_t)(nc + 1) * sizeof(int64_t));
    /* symbolic: structural pattern of R A P */
    int64_t nnz = 0;
    for (int64_t ic = 0; ic < nc; ++ic) {
        int64_t m = 0;
        for (int64_t p = L->rrp[ic]; p < L->rrp[ic + 1]; ++p) {
            int64_t i = L->rci[p];
            for (int64_t q = L->rp[i]; q < L->rp[i + 1]; ++q) {
                int64_t j = L->ci[q];
                for (int64_t s = L->prp[j]; s < L->prp[j + 1]; ++s) {
                    int64_t jc = L->pci[s];
                    if (mark[jc] != ic) { mark[jc] = ic; list[m++] = jc; }
                }
            }
        }
        nnz += m;
    }
    C->nnz = nnz;
    C->ci = malloc((size_t)nnz * sizeof(int64_t));
    C->v = malloc((size_t)nnz * sizeof(cplx));
    for (int64_t a = 0; a < nc; ++a) mark[a] = -1;
    cplx *acc = calloc((size_t)nc, sizeof(cplx));
    nnz = 0;
    for (int64_t ic = 0; ic < nc; ++ic) {
        C->rp[ic] = nnz;
        int64_t m = 0;
        for (int64_t p = L->rrp[ic]; p < L->rrp[ic + 1]; ++p) {
            int64_t i = L->rci[p];
            for (int64_t q = L->rp[i]; q < L->rp[i + 1]; ++q) {
                int64_t j = L->ci[q];
                for (int64_t s = L->prp[j]; s < L->prp[j + 1]; ++s) {
                    int64_t jc = L->pci[s];
                    if (mark[jc] != ic) { mark[jc] = ic; list[m++] = jc; acc[jc] = 0; }
                    if (jc >= ic) acc[jc] += L->rv[p] * L->v[q] * L->pv[s];
                }
            }
        }
        qsort(list, (size_t)m, sizeof(int64_t), cmp_i64);
        for (int64_t t = 0; t < m; ++t) {
            int64_t jc = list[t];
            cplx val;
            if (jc > ic) val = acc[jc];
            else if (jc == ic) val = creal(acc[jc]);
            else {
                /* mirror the already computed upper-triangle entry (jc, ic) */
                val = 0;
                for (int64_t r = C->rp[jc]; r < C->rp[jc + 1]; ++r)
                    if (C->ci[r] == ic) { val = conj(C->v[r]); break; }
            }
            C->ci[nnz] = jc;
            C->v[nnz] = val;
            ++nnz;
        }
    }
    C->rp[nc] = nnz;
    free(acc);
    free(list);
    free(mark);
}

/* ------------------------------------------------------------ Cholesky --- */
static int cholesky(const orc_level *L, cplx **out)
{
    const int64_t n = L->n;
    cplx *A = calloc((size_t)(n * n), sizeof(cplx));
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
            A[i * n + L->ci[p]] = L->v[p];
            if (L->ci[p] == i && fabs(creal(L->v[p])) > dmax) dmax = fabs(creal(L->v[p]));
        }
    /* A = L L^H, L lower triangular with positive real diagonal */
    for (int64_t j = 0; j < n; ++j) {
        double d = creal(A[j * n + j]);
        for (int64_t k = 0; k < j; ++k) d -= creal(A[j * n + k] * conj(A[j * n + k]));
        if (!(d > 1e-12 * dmax)) { free(A); return ORC_ERR_SINGULAR; }
        double ljj = sqrt(d);
        A[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            cplx s = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * conj(A[j * n + k]);
            A[i * n + j] = s / ljj;
        }
        for (int64_t i = 0; i < j; ++i) A[i * n + j] = 0;
    }
    *out = A;
    return ORC_OK;
}

static void cholesky_solve(const cplx *Lf, int64_t n, const cplx *b, cplx *x)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= Lf[i * n + k] * x[k];
        x[i] = s / Lf[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        cplx s = x[i];
        for (int64_t k = i + 1; k < n; ++k) s -= conj(Lf[k * n + i]) * x[k];
        x[i] = s / Lf[i * n + i];
    }
}

/* ------------------------------------------------------------- build --- */
static void free_level(orc_level *L)
{
    free(L->rp); free(L->ci); free(L->v); free(L->agg); free(L->root);
    free(L->prp); free(L->pci); free(L->pv); free(L->rrp); free(L->rci); free(L->rv);
    free(L->color);
    memset(L, 0, sizeof(*L));
}

int orc_amg_build(int64_t n, const int64_t *rp, const int64_t *ci, const cplx *v,
                  int grid_dim, const int64_t *grid_N, int max_coarse, int max_levels,
                  orc_amg **out)
{
    if (max_levels < 1 || max_levels > ORC_MAX_LEVELS || n < 1) return ORC_ERR_ARG;
    orc_amg *a = calloc(1, sizeof(*a));
    a->grid_dim = grid_dim;
    for (int d = 0; d < grid_dim; ++d) a->grid_N[d] = grid_N[d];
    orc_level *L0 = &a->lev[0];
    L0->n = n;
    L0->nnz = rp[n];
    L0->rp = malloc((size_t)(n + 1) * sizeof(int64_t));
    L0->ci = malloc((size_t)rp[n] * sizeof(int64_t));
    L0->v = malloc((size_t)rp[n] * sizeof(cplx));
    memcpy(L0->rp, rp, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(L0->ci, ci, (size_t)rp[n] * sizeof(int64_t));
    memcpy(L0->v, v, (size_t)rp[n] * sizeof(cplx));
    int l = 0, rc = ORC_OK;
    for (;;) {
        orc_level *L = &a->lev[l];
        colour_level(L, l, grid_dim, grid_N);
        if (L->n <= max_coarse || l == max_levels - 1) break;
        rc = aggregate(L, l);
        if (rc != ORC_OK) break;
        if ((double)L->nc > 0.85 * (double)L->n) {
            free(L->agg); free(L->root);
            L->agg = NULL; L->root = NULL; L->nc = 0;
            break;
        }
        build_p(L);
        galerkin(L, &a->lev[l + 1]);
        ++l;
    }
    a->nlev = l + 1;
    if (rc == ORC_OK) rc = cholesky(&a->lev[l], &a->chol);
    if (rc != ORC_OK) { orc_amg_free(a); return rc; }
    *out = a;
    return ORC_OK;
}

void orc_amg_free(orc_amg *a)
{
    if (!a) return;
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) free_level(&a->lev[l]);
    free(a->chol);
    free(a);
}

/* ------------------------------------------------------------ V-cycle --- */
void orc_sgs(const orc_level *L, cplx *x, const cplx *b)
{
    const int C = L->ncolors;
    for (int t = 0; t < 2 * C - 1; ++t) {
        int c = t < C ? t : 2 * C - 2 - t;
        for (int64_t i = 0; i < L->n; ++i) {
            if (L->color[i] != c) continue;
            cplx s = b[i];
            double d = 0.0;
            for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
                if (L->ci[p] == i) d = creal(L->v[p]);
                else s -= L->v[p] * x[L->ci[p]];
            }
            x[i] = s / d;
        }
    }
}

static void vcycle(const orc_amg *a, int l, const cplx *b, cplx *x)
{
    const orc_level *L = &a->lev[l];
    if (l == a->nlev - 1) { cholesky_solve(a->chol, L->n, b, x); return; }
    for (int64_t i = 0; i < L->n; ++i) x[i] = 0;
    orc_sgs(L, x, b);
    cplx *r = malloc((size_t)L->n * sizeof(cplx));
    for (int64_t i = 0; i < L->n; ++i) {
        cplx s = b[i];
        for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) s -= L->v[p] * x[L->ci[p]];
        r[i] = s;
    }
    cplx *bc = malloc((size_t)L->nc * sizeof(cplx)), *xc = malloc((size_t)L->nc * sizeof(cplx));
    for (int64_t ic = 0; ic < L->nc; ++ic) {
        cplx s = 0;
        for (int64_t p = L->rrp[ic]; p < L->rrp[ic + 1]; ++p) s += L->rv[p] * r[L->rci[p]];
        bc[ic] = s;
    }
    vcycle(a, l + 1, bc, xc);
    for (int64_t i = 0; i < L->n; ++i)
        for (int64_t p = L->prp[i]; p < L->prp[i + 1]; ++p) x[i] += L->pv[p] * xc[L->pci[p]];
    orc_sgs(L, x, b);
    free(r); free(bc); free(xc);
}

void orc_amg_solve(const orc_amg *a, const cplx *b, cplx *x, int cycles)
{
    const orc_level *L = &a->lev[0];
    const int64_t n = L->n;
    vcycle(a, 0, b, x);
    if (cycles <= 1) return;
    cplx *r = malloc((size_t)n * sizeof(cplx)), *e = malloc((size_t)n * sizeof(cplx));
    for (int c = 1; c < cycles; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            cplx s = b[i];
            for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) s -= L->v[p] * x[L->ci[p]];
            r[i] = s;
        }
        vcycle(a, 0, r, e);
        for (int64_t i = 0; i < n; ++i) x[i] += e[i];
    }
    free(r); free(e);
}
