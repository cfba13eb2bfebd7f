// Setup of the smoothed-aggregation preconditioner R_k = AMG_k(H, D .) with
// H = K-hat + 2 D |psi|^2 (Sec. 4.1, eq. prec2; smoothed aggregation with
// 1 + 1 symmetric Gauss-Seidel steps).  The paper leaves the aggregation and
// smoothing parameters open; this library fixes them as follows:
//   strength     every structural off-diagonal entry (theta = 0), so the
//                integer part of the hierarchy depends only on the grid
//   priorities   the smaller index first (the greedy pass of standard
//                aggregation: regular, densely packed roots; hashed priorities
//                left a V-cycle that weakened as the grid was refined)
//   roots        distance-2 maximal independent set, computed in parallel
//                rounds: an undecided node becomes a root when it has the
//                smallest index among undecided nodes within distance 2 (this
//                equals the serial greedy choice in ascending index order)
//   assignment   neighbours of a root join it; the remaining nodes join the
//                aggregate of their assigned neighbour with the smallest root
//   numbering    aggregates in ascending root index
//   prolongator  P = T - omega D^-1 A T, T = 1/sqrt|a|, omega = (4/3) / rho~,
//                rho~ the estimate of rho(D^-1 A) after 20 power-iteration
//                steps from a counter-hash start; R = P^H; A_{l+1} = R A P
//                (upper triangle, mirrored; real diagonal)
//   colours      level 0: red-black parity of the grid; coarser: Jones-Plassmann
//                rounds with index priorities (equal to greedy colouring in
//                ascending index order: 4 colours on the regular coarse grids
//                where degree or hash orders needed 7-8), then two
//                iterated-greedy passes
//   coarsest     dense Cholesky
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>

#include "amg.h"
#include "stencil.h"

namespace glk {

// ------------------------------------------------------------ scan ----
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_tile(const int *__restrict__ in, int *__restrict__ out,
                                                      int *__restrict__ bsum, int n)
{
    __shared__ int sm[kBlock];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems], t = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        t += v[k];
    }
    sm[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int add = threadIdx.x >= (unsigned)o ? sm[threadIdx.x - o] : 0;
        __syncthreads();
        sm[threadIdx.x] += add;
        __syncthreads();
    }
    int ex = sm[threadIdx.x] - t;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = sm[kBlock - 1];
}

__global__ void k_scan_add(int *out, const int *boff, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] += boff[i / kScanTile];
}

// exclusive scan of in[0..n) into out; returns the total (synchronises s)
static int64_t scan_excl(const int *in, int *out, int n, hipStream_t s)
{
    if (n <= 0) return 0;
    const int nb = (n + kScanTile - 1) / kScanTile;
    DevBuf<int> bsum(nb), boff(nb);
    k_scan_tile<<<nb, kBlock, 0, s>>>(in, out, bsum.get(), n);
    GLK_CHECK_LAUNCH();
    if (nb > 1) {
        scan_excl(bsum.get(), boff.get(), nb, s);
        k_scan_add<<<blocks_for(n), kBlock, 0, s>>>(out, boff.get(), n);
        GLK_CHECK_LAUNCH();
    }
    int last_out = 0, last_in = 0;
    GLK_HIP(hipMemcpyAsync(&last_out, out + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipMemcpyAsync(&last_in, in + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    return (int64_t)last_out + last_in;
}

// ---------------------------------------------------------- keys ------
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// aggregation priority: larger for the smaller index (0 stays free for "none")
__device__ __forceinline__ unsigned long long keyof(int i)
{
    return (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
}

// insert v into the ascending unique list buf[0..u); false on overflow
__device__ __forceinline__ bool sorted_insert(int *buf, int &u, int v)
{
    int lo = 0, hi = u;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (buf[mid] < v) lo = mid + 1; else hi = mid;
    }
    if (lo < u && buf[lo] == v) return true;
    if (u == kMaxRow) return false;
    for (int t = u; t > lo; --t) buf[t] = buf[t - 1];
    buf[lo] = v;
    ++u;
    return true;
}

__device__ __forceinline__ int find_col(const int *ci, int b, int e, int col)
{
    while (b < e) {
        const int mid = (b + e) >> 1;
        if (ci[mid] < col) b = mid + 1; else e = mid;
    }
    return b;
}

// ------------------------------------------------- level-0 CSR -------
template <int DIM>
__global__ void k_l0_count(Geom g, int *cnt)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    int k = 1;
    for (int a = 0; a < DIM; ++a) k += (c[a] > 0) + (c[a] < g.N[a] - 1);
    cnt[i] = k;
}

// columns ascending: lower neighbours (largest stride first), i, upper neighbours
template <int DIM>
__global__ void k_l0_cols(Geom g, const int *rp, int *ci)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    int st[3] = {1, g.N[0], g.N[0] * g.N[1]};
    int p = rp[i];
    for (int a = DIM - 1; a >= 0; --a)
        if (c[a] > 0) ci[p++] = i - st[a];
    ci[p++] = i;
    for (int a = 0; a < DIM; ++a)
        if (c[a] < g.N[a] - 1) ci[p++] = i + st[a];
}

// H = K-hat + 2 D |psi|^2 in the same entry order
template <int DIM>
struct L0Values {
    GeomT<double> g;
    const int *rp;
    LinkTab<double> U;
    const double2 *__restrict__ psi;
    double2 *v;
    double *diag;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double s[3];
        const double d = node_volume<DIM, double>(g, c, s);
        int p = rp[i];
        double asum = 0.0;
        for (int a = DIM - 1; a >= 0; --a)
            if (c[a] > 0) {
                const double al = d * s[a] * g.inv_h2[a];
                v[p++] = cscale(link_u<DIM, double>(U, a, c, c[a] - 1), -al);
            }
        const int pd = p++;
        for (int a = 0; a < DIM; ++a) {
            const double al = d * s[a] * g.inv_h2[a];
            if (c[a] < g.N[a] - 1) v[p++] = cscale(cconj(link_u<DIM, double>(U, a, c, c[a])), -al);
            asum += al * ((c[a] > 0) + (c[a] < g.N[a] - 1));
        }
        const double dg = asum + 2.0 * d * cabs2(psi[i]);
        v[pd] = make_double2(dg, 0.0);
        diag[i] = dg;
    }
};

// Level 0 of a simplicial mesh: its adjacency with the diagonal inserted
// (columns ascending), H_jj = K-hat_jj + 2 |V_j| |psi_j|^2, H_jk = -kw_jk
__global__ void k_l0s_count(int n, const int *arp, int *cnt)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cnt[i] = arp[i + 1] - arp[i] + 1;
}

__global__ void k_l0s_cols(int n, const int *arp, const int *aci, const int *rp, int *ci)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int p = rp[i];
    bool diag = false;
    for (int q = arp[i]; q < arp[i + 1]; ++q) {
        if (!diag && aci[q] > i) {
            ci[p++] = i;
            diag = true;
        }
        ci[p++] = aci[q];
    }
    if (!diag) ci[p] = i;
}

struct L0sValues {
    GeomT<double> g;
    const int *rp, *ci;
    const double2 *__restrict__ psi;
    double2 *v;
    double *diag;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int q = g.rp[i];
        const double dg = g.ks[i] + 2.0 * g.vol[i] * cabs2(psi[i]);
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            v[p] = ci[p] == i ? make_double2(dg, 0.0) : cscale(g.kw[q++], -1.0);
        diag[i] = dg;
    }
};

// --------------------------------------------------------- MIS-2 -----
__global__ void k_fill_int(int *a, int n, int val)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = val;
}

__global__ void k_mis_m1(int n, const int *rp, const int *ci, const int *state, unsigned long long *m1)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    unsigned long long best = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (state[j] == 0) best = max(best, keyof(j) + 1ull);
    }
    m1[i] = best;
}

__global__ void k_mis_select(int n, const int *rp, const int *ci, const unsigned long long *m1,
                             int *state)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    unsigned long long best = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) best = max(best, m1[ci[p]]);
    if (best == keyof(i) + 1ull) state[i] = 1;
}

__global__ void k_mis_near(int n, const int *rp, const int *ci, const int *state, int *near1)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int r = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) r |= (state[ci[p]] == 1);
    near1[i] = r;
}

__global__ void k_mis_remove(int n, const int *rp, const int *ci, const int *near1, int *state,
                             int *remaining)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    int r = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) r |= near1[ci[p]];
    if (r) state[i] = 2;
    else atomicAdd(remaining, 1);
}

__global__ void k_agg_phase_a(int n, const int *rp, const int *ci, const int *state, int *rootA)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (state[i] == 1) { rootA[i] = i; return; }
    int best = -1;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        if (j != i && state[j] == 1 && (best < 0 || keyof(j) > keyof(best))) best = j;
    }
    rootA[i] = best;
}

__global__ void k_agg_phase_b(int n, const int *rp, const int *ci, const int *rootA, int *root, int *err)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int best = rootA[i];
    if (best < 0) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j == i) continue;
            const int r = rootA[j];
            if (r >= 0 && (best < 0 || keyof(r) > keyof(best))) best = r;
        }
        if (best < 0) atomicOr(err, 1);
    }
    root[i] = best;
}

__global__ void k_root_flags(int n, const int *state, int *flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flag[i] = (state[i] == 1);
}

__global__ void k_agg_number(int n, const int *root, const int *id, const int *state, int *agg,
                             int *rootlist, int *aggsize)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int r = root[i];
    const int a = r >= 0 ? id[r] : 0;
    agg[i] = a;
    if (state[i] == 1) rootlist[id[i]] = i;
    atomicAdd(&aggsize[a], 1);
}

// ------------------------------------------------------ patterns -----
__global__ void k_p_pattern(int n, const int *rp, const int *ci, const int *agg, const int *prp,
                            int *cnt, int *pci, int *err)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int buf[kMaxRow];
    int u = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (!sorted_insert(buf, u, agg[ci[p]])) { atomicOr(err, 2); return; }
    if (pci) {
        const int o = prp[i];
        for (int t = 0; t < u; ++t) pci[o + t] = buf[t];
    } else {
        cnt[i] = u;
    }
}

__global__ void k_col_count(int nnz, const int *col, int *cnt)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[col[p]], 1);
}

__global__ void k_transpose_fill(int n, const int *prp, const int *pci, const int *rrp, int *fill,
                                 int *rci, int *rsrc)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int p = prp[i]; p < prp[i + 1]; ++p) {
        const int a = pci[p];
        const int q = rrp[a] + atomicAdd(&fill[a], 1);
        rci[q] = i;
        rsrc[q] = p;
    }
}

__global__ void k_sort_rows(int nr, const int *rrp, int *rci, int *rsrc)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nr) return;
    const int b = rrp[r], e = rrp[r + 1];
    for (int p = b + 1; p < e; ++p) {
        const int kc = rci[p], ks = rsrc[p];
        int q = p - 1;
        while (q >= b && rci[q] > kc) {
            rci[q + 1] = rci[q];
            rsrc[q + 1] = rsrc[q];
            --q;
        }
        rci[q + 1] = kc;
        rsrc[q + 1] = ks;
    }
}

// pattern of R A P, row by row
__global__ void k_rap_pattern(int nc, const int *rrp, const int *rci, const int *arp, const int *aci,
                              const int *prp, const int *pci, const int *crp, int *cnt, int *cci,
                              int *err)
{
    const int I = blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    int buf[kMaxRow];
    int u = 0;
    for (int p = rrp[I]; p < rrp[I + 1]; ++p) {
        const int i = rci[p];
        for (int q = arp[i]; q < arp[i + 1]; ++q) {
            const int j = aci[q];
            for (int s = prp[j]; s < prp[j + 1]; ++s)
                if (!sorted_insert(buf, u, pci[s])) { atomicOr(err, 4); return; }
        }
    }
    if (cci) {
        const int o = crp[I];
        for (int t = 0; t < u; ++t) cci[o + t] = buf[t];
    } else {
        cnt[I] = u;
    }
}

// --------------------------------------------------------- colours ----
template <int DIM>
__global__ void k_parity_colour(Geom g, int *col)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    col[i] = (c[0] + c[1] + c[2]) & 1;
}

constexpr int kRecolourPasses = 2;  // iterated-greedy passes after the colouring rounds

// colour priority: the smaller index first (the rounds then reproduce the
// serial greedy colouring in index order)
__device__ __forceinline__ unsigned long long colour_key(int i)
{
    return (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
}

__global__ void k_jp_ready(int n, const int *rp, const int *ci, const int *col, int *ready)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int r = 0;
    if (col[i] < 0) {
        r = 1;
        const unsigned long long k = colour_key(i);
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j != i && col[j] < 0 && colour_key(j) > k) { r = 0; break; }
        }
    }
    ready[i] = r;
}

__global__ void k_jp_colour(int n, const int *rp, const int *ci, const int *ready, int *col,
                            int *remaining, int *err)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (!ready[i]) {
        if (col[i] < 0) atomicAdd(remaining, 1);
        return;
    }
    unsigned long long used[4] = {0, 0, 0, 0};
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const int c = (j != i) ? col[j] : -1;
        if (c >= 0 && c < 256) used[c >> 6] |= 1ull << (c & 63);
    }
    int c = 0;
    while (c < 256 && (used[c >> 6] >> (c & 63) & 1ull)) ++c;
    if (c == 256) atomicOr(err, 8);
    col[i] = c;
}

// Iterated greedy (Culberson): the rows of one colour class (an independent
// set, so they do not see each other) take the smallest colour not yet given
// to a neighbour in this pass; classes are visited in reverse order.
__global__ void k_ig_class(int n, const int *rp, const int *ci, const int *old, int cls, int *nw, int *err)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || old[i] != cls) return;
    unsigned long long used[4] = {0, 0, 0, 0};
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const int c = (j != i) ? nw[j] : -1;
        if (c >= 0 && c < 256) used[c >> 6] |= 1ull << (c & 63);
    }
    int c = 0;
    while (c < 256 && (used[c >> 6] >> (c & 63) & 1ull)) ++c;
    if (c == 256) atomicOr(err, 8);
    nw[i] = c;
}

__global__ void k_colour_hist(int n, const int *col, int *hist)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&hist[col[i]], 1);
}

__global__ void k_flag_eq(int n, const int *col, int c, int *flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flag[i] = (col[i] == c);
}

__global__ void k_scatter_colour(int n, const int *col, int c, const int *pos, int *dst)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n && col[i] == c) dst[pos[i]] = i;
}

// --------------------------------------------------------- numeric ----
struct Diag {
    int n;
    const int *rp, *ci;
    const double2 *v;
    double *diag;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i >= n) return;
        const int p = find_col(ci, rp[i], rp[i + 1], i);
        diag[i] = (p < rp[i + 1] && ci[p] == i) ? v[p].x : 0.0;
    }
};

// Spectral radius of D^-1 A by power iteration from the counter-hash start
// s_i = (h1_i - 1/2) + i (h2_i - 1/2), h = fmix32(i ^ salt) / 2^32; the
// normalisation of each iterate is folded into the next step.
constexpr int kRhoSteps = 20;

struct PwStart {
    int n;
    double2 *x;
    RedSlot slot;
    __device__ void operator()(int, int) const
    {
        __shared__ double sm[kBlock / 64];
        const int i = blockIdx.x * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < n) {
            const double a = (double)fmix32((uint32_t)i ^ 0x2545F491u) / 4294967296.0 - 0.5;
            const double b = (double)fmix32((uint32_t)i ^ 0x6C8E9CF5u) / 4294967296.0 - 0.5;
            x[i] = make_double2(a, b);
            part = a * a + b * b;
        }
        block_reduce_store(part, slot, sm, blockIdx.x);
    }
};

// y = D^-1 A x / ||x|| (||x||^2 in *xn2), partial sums of |y|^2; kPwLanes
// lanes share a row (lane j takes entries j, j + kPwLanes, ... in order, then
// a fixed butterfly), so long coarse rows are not one serial chain of gathers.
// The grid is at most the partial-sum slot's size: a block strides over the
// rows by the grid (the same iterations for all its threads) and stores one
// partial.
constexpr int kPwLanes = 8;

struct PwStep {
    int n;
    const int *rp, *ci;
    const double2 *v;
    const double *diag;
    const double2 *x;
    const double *xn2;
    double2 *y;
    RedSlot slot;
    __device__ void operator()(int, int) const
    {
        __shared__ double sm[kBlock / 64];
        const int64_t total = (int64_t)n * kPwLanes;
        const double scale = 1.0 / sqrt(*xn2);
        double part = 0.0;
        for (int64_t base = (int64_t)blockIdx.x * kBlock; base < total; base += (int64_t)gridDim.x * kBlock) {
            const int64_t g = base + threadIdx.x;
            const int i = (int)(g / kPwLanes), lane = (int)(g % kPwLanes);
            const bool act = g < total;
            double2 acc = make_double2(0.0, 0.0);
            if (act)
                for (int p = rp[i] + lane; p < rp[i + 1]; p += kPwLanes) acc = cadd(acc, cmul(v[p], x[ci[p]]));
    #pragma unroll
            for (int o = kPwLanes / 2; o > 0; o >>= 1) {
                acc.x += __shfl_xor(acc.x, o, 64);
                acc.y += __shfl_xor(acc.y, o, 64);
            }
            if (act && lane == 0) {
                const double2 yi = cscale(acc, scale / diag[i]);
                y[i] = yi;
                part += cabs2(yi);
            }
        }
        block_reduce_store(part, slot, sm, blockIdx.x);
    }
};

// Level 0: the same step with H applied as the stencil (link factor tables
// and the diagonal; its CSR copy holds the same entries), so a step streams x
// and the diagonal instead of the CSR arrays.
template <int DIM>
struct PwStepL0 {
    GeomT<double> g;
    LinkTab<double> U;
    const double *diag;
    const double2 *x;
    const double *xn2;
    double2 *y;
    RedSlot slot;
    __device__ void operator()(int, int) const
    {
        __shared__ double sm[kBlock / 64];
        const int i = blockIdx.x * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            const double di = diag[i];
            const double2 acc = cadd(cscale(x[i], di), khat_offdiag<DIM, double>(g, i, c, x, U));
            const double2 yi = cscale(acc, 1.0 / (di * sqrt(*xn2)));
            y[i] = yi;
            part = cabs2(yi);
        }
        block_reduce_store(part, slot, sm, blockIdx.x);
    }
};

struct PwRho {
    const double *yn2;
    double *rho;
    __device__ void operator()(int, int) const
    {
        if (threadIdx.x == 0) *rho = sqrt(*yn2);
    }
};

static void rho_estimate(gl_precond *pre, Level &lev, const Launch &L)
{
    const gl_mesh *m = pre->mesh;
    const int n = lev.n, nb = blocks_for(n);
    const RedSlot slot = red_slot(m, 0);
    double2 *x = pre->vin.get(), *y = pre->cyc_r.get();
    double *nrm = pre->pwn.get();
    L.run(nb, PwStart{n, x, slot});
    launch_finalize(slot.partials, nb, FIN_STORE, nullptr, nrm, nullptr, L);
    // level 0 of a grid as the stencil, every other level (and level 0 of a
    // simplicial mesh) through its CSR matrix
    const bool l0 = &lev == &pre->L[0] && !m->g.simplicial;
    const GeomT<double> g = geom_t<double>(m->g);
    // CSR levels: kPwLanes threads per row, at most one partial per level-0 block
    const int nbl = std::min(blocks_for((int64_t)n * kPwLanes), blocks_for(m->g.n));
    for (int k = 1; k <= kRhoSteps; ++k) {
        const double *xn2 = nrm + ((k - 1) & 1);
        if (l0 && m->g.dim == 2)
            L.run(nb, PwStepL0<2>{g, link_tab<double>(m), lev.diag64.get(), x, xn2, y, slot});
        else if (l0)
            L.run(nb, PwStepL0<3>{g, link_tab<double>(m), lev.diag64.get(), x, xn2, y, slot});
        else
            L.run(nbl, PwStep{n, lev.A.rp.get(), lev.A.ci.get(), lev.A.v64.get(), lev.diag64.get(), x, xn2, y, slot});
        launch_finalize(slot.partials, l0 ? nb : nbl, FIN_STORE, nullptr, nrm + (k & 1), nullptr, L);
        std::swap(x, y);
    }
    L.run<PwRho, 64>(1, PwRho{nrm + (kRhoSteps & 1), lev.rho.get()});
}

struct PValues {
    int n;
    const int *arp, *aci;
    const double2 *av;
    const double *diag;
    const int *agg, *aggsize;
    const double *rho;
    const int *prp, *pci;
    double2 *pv;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i >= n) return;
        const double omega = (4.0 / 3.0) / *rho;
        const double dii = diag[i];
        const int ai = agg[i];
        for (int p = prp[i]; p < prp[i + 1]; ++p) {
            const int a = pci[p];
            const double ta = 1.0 / sqrt((double)aggsize[a]);
            double2 at = make_double2(0.0, 0.0);
            for (int q = arp[i]; q < arp[i + 1]; ++q)
                if (agg[aci[q]] == a) at = cadd(at, cscale(av[q], ta));
            const double t0 = (ai == a) ? ta : 0.0;
            const double f = omega / dii;
            pv[p] = make_double2(t0 - f * at.x, -f * at.y);
        }
    }
};

struct RValues {
    int nnz;
    const int *rsrc;
    const double2 *pv;
    double2 *rv;
    __device__ void operator()(int, int) const
    {
        const int q = blockIdx.x * kBlock + threadIdx.x;
        if (q < nnz) rv[q] = cconj(pv[rsrc[q]]);
    }
};

// Upper triangle (J >= I) of R A P.  The products of each stored entry are
// listed once per hierarchy (symbolic), in the order of the row traversal
// p (R row), q (A row), s (P row), and the numeric setup sums them in that
// order, one thread per entry.
template <class F>
__device__ __forceinline__ void rap_traverse(int I, const int *rrp, const int *rci, const int *arp,
                                             const int *aci, const int *prp, const int *pci, const int *cci,
                                             int cb, int ce, F &&f)
{
    for (int p = rrp[I]; p < rrp[I + 1]; ++p) {
        const int i = rci[p];
        for (int q = arp[i]; q < arp[i + 1]; ++q) {
            const int j = aci[q];
            for (int s = prp[j]; s < prp[j + 1]; ++s) {
                const int J = pci[s];
                if (J < I) continue;
                const int t = find_col(cci, cb, ce, J);
                if (t < ce && cci[t] == J) f(t, p, q, s);
            }
        }
    }
}

__global__ void k_rap_count(int nc, const int *rrp, const int *rci, const int *arp, const int *aci,
                            const int *prp, const int *pci, const int *crp, const int *cci, int *cnt)
{
    const int I = blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    rap_traverse(I, rrp, rci, arp, aci, prp, pci, cci, crp[I], crp[I + 1],
                 [&](int t, int, int, int) { cnt[t] += 1; });
}

__global__ void k_rap_fill(int nc, const int *rrp, const int *rci, const int *arp, const int *aci,
                           const int *prp, const int *pci, const int *crp, const int *cci, const int *tp,
                           int *fill, int *trip)
{
    const int I = blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    rap_traverse(I, rrp, rci, arp, aci, prp, pci, cci, crp[I], crp[I + 1], [&](int t, int p, int q, int s) {
        const int k = tp[t] + fill[t]++;
        trip[3 * k] = p;
        trip[3 * k + 1] = q;
        trip[3 * k + 2] = s;
    });
}

// cv[t] = sum of (R_p A_q) P_s over the products of entry t (0 for J < I).
// kRapLanes lanes share an entry: lane j sums products j, j + kRapLanes, ...
// of its list in order, then the lanes are added by a fixed butterfly, so a
// setup is bit-reproducible; neighbouring lanes read neighbouring triples.
constexpr int kRapLanes = 8;

struct RapValues {
    int nnz;
    const int *__restrict__ tp, *__restrict__ trip;
    const double2 *__restrict__ rv, *__restrict__ av, *__restrict__ pv;
    double2 *__restrict__ cv;
    __device__ void operator()(int, int) const
    {
        const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        const int t = (int)(g / kRapLanes), lane = (int)(g % kRapLanes);
        const bool act = t < nnz;
        double2 acc = make_double2(0.0, 0.0);
        if (act)
            for (int k = tp[t] + lane; k < tp[t + 1]; k += kRapLanes) {
                const double2 ra = cmul(rv[trip[3 * k]], av[trip[3 * k + 1]]);
                acc = cadd(acc, cmul(ra, pv[trip[3 * k + 2]]));
            }
    #pragma unroll
        for (int o = kRapLanes / 2; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (act && lane == 0) cv[t] = acc;
    }
};

struct RapMirror {
    int nc;
    const int *crp, *cci;
    double2 *cv;
    __device__ void operator()(int, int) const
    {
        const int I = blockIdx.x * kBlock + threadIdx.x;
        if (I >= nc) return;
        for (int t = crp[I]; t < crp[I + 1]; ++t) {
            const int J = cci[t];
            if (J > I) break;
            if (J == I) { cv[t].y = 0.0; break; }
            const int u = find_col(cci, crp[J], crp[J + 1], I);
            cv[t] = (u < crp[J + 1] && cci[u] == I) ? cconj(cv[u]) : make_double2(0.0, 0.0);
        }
    }
};

struct ToF32c {
    int n;
    const double2 *a;
    float2 *b;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
    }
};

struct ToF32r {
    int n;
    const double *a;
    float *b;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i < n) b[i] = (float)a[i];
    }
};

struct DenseFromCsr {
    int n;
    const int *rp, *ci;
    const double2 *v;
    double2 *M;
    __device__ void operator()(int, int) const
    {
        const int i = blockIdx.x * kBlock + threadIdx.x;
        if (i >= n) return;
        for (int j = 0; j < n; ++j) M[(size_t)i * n + j] = make_double2(0.0, 0.0);
        for (int p = rp[i]; p < rp[i + 1]; ++p) M[(size_t)i * n + ci[p]] = v[p];
    }
};

// Cholesky factor M = L L^H of the Hermitian coarsest operator, in place
// (row-major, lower triangle; the upper part zeroed at the end), blocked
// right-looking: a panel of pw columns is factored in LDS by one work-group
// (k_chol_panel), then every work-group updates its share of the trailing
// lower triangle with that panel (k_chol_update).  status = 1 when a pivot is
// not positive relative to the largest diagonal entry of M (k_chol_init);
// every later kernel returns at once then.
constexpr int kCholLds = (65536 - 1024) / sizeof(double2);  // panel entries held in LDS

int chol_panel_width(int n) { return std::max(1, std::min(32, kCholLds / std::max(n, 1))); }

struct CholInit {
    int n;
    const double2 *M;
    double *dmax;
    int *status;
    __device__ void operator()(int, int) const
    {
        __shared__ double sm[1024 / 64];
        double m = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(M[(size_t)i * n + i].x));
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
        if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sm[w]);
            *dmax = r;
            *status = 0;
        }
    }
};

// columns p0 .. p0 + pw - 1, rows p0 .. n - 1 (already updated by the
// earlier panels): P[r * pw + c] = M[p0 + r][p0 + c]
struct CholPanel {
    int n, p0, pw;
    double2 *M;
    const double *dmaxp;
    int *status;
    __device__ void operator()(int, int) const
    {
        __shared__ double2 P[kCholLds];
        __shared__ double piv;
        __shared__ int bad;
        if (*status) return;
        const int rows = n - p0;
        const double dmax = *dmaxp;
        for (int t = threadIdx.x; t < rows * pw; t += blockDim.x)
            P[t] = M[(size_t)(p0 + t / pw) * n + p0 + t % pw];
        if (threadIdx.x == 0) bad = 0;
        __syncthreads();
        for (int c = 0; c < pw; ++c) {
            if (threadIdx.x == 0) {
                const double d = P[c * pw + c].x;
                if (!(d > 1e-12 * dmax)) bad = 1;
                else {
                    piv = sqrt(d);
                    P[c * pw + c] = make_double2(piv, 0.0);
                }
            }
            __syncthreads();
            if (bad) break;
            const double inv = 1.0 / piv;
            for (int r = c + 1 + threadIdx.x; r < rows; r += blockDim.x) P[r * pw + c] = cscale(P[r * pw + c], inv);
            __syncthreads();
            // the panel's remaining columns c' > c, rows r >= c'
            const int w = pw - c - 1;
            for (int t = threadIdx.x; t < (rows - c - 1) * w; t += blockDim.x) {
                const int r = c + 1 + t / w, q = c + 1 + t % w;
                if (r >= q) P[r * pw + q] = csub(P[r * pw + q], cmul(P[r * pw + c], cconj(P[q * pw + c])));
            }
            __syncthreads();
        }
        if (bad) {
            if (threadIdx.x == 0) *status = 1;
            return;
        }
        for (int t = threadIdx.x; t < rows * pw; t += blockDim.x) {
            const int r = t / pw, c = t % pw;
            if (r >= c) M[(size_t)(p0 + r) * n + p0 + c] = P[t];
        }
    }
};

// M[i][k] -= sum_c L[i][p0 + c] conj(L[k][p0 + c]) for p0 + pw <= k <= i < n
// One 16 x 16 tile of the trailing matrix per work-group of 256 threads:
// tile bx = (tile row) * tiles + (tile column), tiles = ceil((n - p0 - pw) / 16).
struct CholUpdate {
    int n, p0, pw, tiles;
    double2 *M;
    const int *status;
    __device__ void operator()(int bx, int) const
    {
        if (*status) return;
        const int b = p0 + pw;
        const int i = b + (bx / tiles) * 16 + (int)(threadIdx.x >> 4);
        const int k = b + (bx % tiles) * 16 + (int)(threadIdx.x & 15);
        if (i >= n || k > i) return;
        const double2 *li = M + (size_t)i * n + p0, *lk = M + (size_t)k * n + p0;
        double2 acc = make_double2(0.0, 0.0);
        for (int c = 0; c < pw; ++c) acc = cadd(acc, cmul(li[c], cconj(lk[c])));
        M[(size_t)i * n + k] = csub(M[(size_t)i * n + k], acc);
    }
};

struct CholZeroUpper {
    int n;
    double2 *M;
    __device__ void operator()(int, int) const
    {
        const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (t >= (int64_t)n * n) return;
        if (t % n > t / n) M[t] = make_double2(0.0, 0.0);
    }
};

static void cholesky(int n, double2 *M, double *dmax, int *status, const Launch &L)
{
    L.run<CholInit, 1024>(1, CholInit{n, M, dmax, status});
    const int pb = chol_panel_width(n);
    for (int p0 = 0; p0 < n; p0 += pb) {
        const int pw = std::min(pb, n - p0);
        L.run<CholPanel, 1024>(1, CholPanel{n, p0, pw, M, dmax, status});
        const int m = n - p0 - pw;
        const int tiles = (m + 15) / 16;
        if (m > 0) L.run(tiles * tiles, CholUpdate{n, p0, pw, tiles, M, status});
    }
    L.run(blocks_for((int64_t)n * n), CholZeroUpper{n, M});
}

// Column j of (L L^H)^-1 (one work-group per column), stored row-major.
struct CholInverse {
    int n;
    const double2 *__restrict__ Lf;
    double2 *inv;
    const int *status;  // nonzero: the factorisation failed, nothing to invert
    __device__ void operator()(int, int) const
    {
        if (*status) return;
        __shared__ double2 y[kMaxDense];
        const int j = blockIdx.x;
        for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        __syncthreads();
        for (int k = j; k < n; ++k) {  // L y = e_j
            const double2 yk = cscale(y[k], 1.0 / Lf[(size_t)k * n + k].x);
            __syncthreads();
            for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) y[i] = csub(y[i], cmul(Lf[(size_t)i * n + k], yk));
            if (threadIdx.x == 0) y[k] = yk;
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {  // L^H x = y
            const double2 yk = cscale(y[k], 1.0 / Lf[(size_t)k * n + k].x);
            __syncthreads();
            for (int i = threadIdx.x; i < k; i += blockDim.x) y[i] = csub(y[i], cmulc(Lf[(size_t)k * n + i], yk));
            if (threadIdx.x == 0) y[k] = yk;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) inv[(size_t)i * n + j] = y[i];
    }
};

// ------------------------------------------------- colour renumbering --
__global__ void k_iperm(int n, const int *perm, int *iperm)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < n) iperm[perm[r]] = r;
}

// length of old row rowperm[r] (identity when rowperm is NULL)
__global__ void k_perm_count(int nrows, const int *rowperm, const int *rp, int *cnt)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nrows) return;
    const int o = rowperm ? rowperm[r] : r;
    cnt[r] = rp[o + 1] - rp[o];
}

// row r of the copy = old row rowperm[r] with columns relabelled by colmap
__global__ void k_perm_fill(int nrows, const int *rowperm, const int *rp, const int *ci, const int *colmap,
                            const int *nrp, int *nci, int *map)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nrows) return;
    const int o = rowperm ? rowperm[r] : r;
    int q = nrp[r];
    for (int p = rp[o]; p < rp[o + 1]; ++p, ++q) {
        nci[q] = colmap ? colmap[ci[p]] : ci[p];
        map[q] = p;
    }
}

// Level-0 restriction without the red columns: the level-0 residual the
// V-cycle restricts is zero on red nodes (their last pre-smoothing update
// zeroes it), so those entries only ever multiply zeros.  Row r keeps the
// entries of columns i with (c0 + c1 + c2) odd; map composes the copy's entry
// with the value map of the source copy.
__device__ __forceinline__ bool black_node(const GeomT<double> &g, int i)
{
    const int c0 = i % g.N[0], r = i / g.N[0];
    const int c1 = r % g.N[1], c2 = r / g.N[1];
    return ((c0 + c1 + c2) & 1) != 0;
}

__global__ void k_black_count(int nrows, GeomT<double> g, const int *rp, const int *ci, int *cnt)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nrows) return;
    int c = 0;
    for (int p = rp[r]; p < rp[r + 1]; ++p) c += black_node(g, ci[p]);
    cnt[r] = c;
}

// columns numbered as the V-cycle stores level-0 vectors: black node i of
// red-black pair t at npair + t
__global__ void k_black_fill(int nrows, GeomT<double> g, const int *rp, const int *ci, const int *srcmap,
                             const int *nrp, int *nci, int *map)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nrows) return;
    int q = nrp[r];
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
        const int i = ci[p];
        if (black_node(g, i)) {
            nci[q] = g.npair + (i / g.N[0]) * g.hr + (i % g.N[0]) / 2;
            map[q] = srcmap[p];
            ++q;
        }
    }
}

// Level-0 prolongation rows of the black nodes only, row t = the black node
// of red-black pair t (empty where the pair has none): the V-cycle corrects
// only black nodes from the coarse level, and the copy keeps those rows
// contiguous.  map composes with the value map of the source copy.
__device__ __forceinline__ int pair_black(const GeomT<double> &g, int t)
{
    const int row = t / g.hr, c0 = 2 * (t - row * g.hr);
    const int c1 = row % g.N[1], c2 = row / g.N[1];
    const int s = (1 + c1 + c2) & 1;
    return c0 + s < g.N[0] ? c0 + s + g.N[0] * row : -1;
}

__global__ void k_pblack_count(GeomT<double> g, const int *rp, int *cnt)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.npair) return;
    const int i = pair_black(g, t);
    cnt[t] = i < 0 ? 0 : rp[i + 1] - rp[i];
}

__global__ void k_pblack_fill(GeomT<double> g, const int *rp, const int *ci, const int *srcmap, const int *nrp,
                              int *nci, int *map)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.npair) return;
    const int i = pair_black(g, t);
    if (i < 0) return;
    int q = nrp[t];
    for (int p = rp[i]; p < rp[i + 1]; ++p, ++q) {
        nci[q] = ci[p];
        map[q] = srcmap[p];
    }
}

// the level-0 diagonal in the colour-split layout (an absent odd node's slot
// holds 1)
struct SplitDiag {
    GeomT<double> g;
    const double *d;
    double *s64;
    float *s32;
    __device__ void operator()(int, int) const
    {
        const int t = blockIdx.x * kBlock + threadIdx.x;
        if (t >= g.npair) return;
        const int row = t / g.hr, c0 = 2 * (t - row * g.hr);
        const int c1 = row % g.N[1], c2 = row / g.N[1];
        const int ie = c0 + g.N[0] * row, ce = (c0 + c1 + c2) & 1;
        const double de = d[ie], dodd = c0 + 1 < g.N[0] ? d[ie + 1] : 1.0;
        s64[ce * g.npair + t] = de;
        s32[ce * g.npair + t] = (float)de;
        s64[(1 - ce) * g.npair + t] = dodd;
        s32[(1 - ce) * g.npair + t] = (float)dodd;
    }
};

struct GatherC {
    int nnz;
    const int *map;
    const double2 *src;
    double2 *d64;
    float2 *d32;
    __device__ void operator()(int, int) const
    {
        const int q = blockIdx.x * kBlock + threadIdx.x;
        if (q >= nnz) return;
        const double2 v = src[map[q]];
        d64[q] = v;
        d32[q] = make_float2((float)v.x, (float)v.y);
    }
};

// padded block of one colour (rows row0 .. row0 + count - 1 of Aa), row-major:
// entry k of row r at r W + k
__global__ void k_ell_fill(int row0, int count, int W, const int *rp, const int *ci, int *eci, int *emap)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= count) return;
    const int i = row0 + r;
    const int b = rp[i], len = rp[i + 1] - rp[i];
    for (int k = 0; k < W; ++k) {
        eci[(size_t)r * W + k] = k < len ? ci[b + k] : i;
        emap[(size_t)r * W + k] = k < len ? b + k : -1;
    }
}

struct EllValues {
    int n;
    const int *emap;
    const double2 *src;
    double2 *d64;
    float2 *d32;
    __device__ void operator()(int, int) const
    {
        const int q = blockIdx.x * kBlock + threadIdx.x;
        if (q >= n) return;
        const int p = emap[q];
        const double2 v = p >= 0 ? src[p] : make_double2(0.0, 0.0);
        d64[q] = v;
        d32[q] = make_float2((float)v.x, (float)v.y);
    }
};

struct GatherR {
    int n;
    const int *perm;
    const double *src;
    double *d64;
    float *d32;
    __device__ void operator()(int, int) const
    {
        const int r = blockIdx.x * kBlock + threadIdx.x;
        if (r >= n) return;
        const double v = src[perm[r]];
        d64[r] = v;
        d32[r] = (float)v;
    }
};

// ------------------------------------------------------------- host ---
static int read_int(const int *d, hipStream_t s)
{
    int h = 0;
    GLK_HIP(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    return h;
}

static void check_err(const DevBuf<int> &err, hipStream_t s, const char *what)
{
    const int e = read_int(err.get(), s);
    if (e & 2 || e & 4) fail(GL_ERR_UNSUPPORTED, std::string(what) + ": a coarse row exceeds the setup row limit");
    if (e & 8) fail(GL_ERR_UNSUPPORTED, std::string(what) + ": more than 256 colours");
    if (e) fail(GL_ERR_HIP, std::string(what) + ": aggregation left a node unassigned");
}

// CSR pattern (rp from counts, then columns) helper
static void alloc_rowptr(Csr &M, const int *cnt, hipStream_t s)
{
    M.rp.alloc((size_t)M.n + 1);
    const int64_t nnz = scan_excl(cnt, M.rp.get(), M.n, s);
    if (nnz > INT32_MAX - 1) fail(GL_ERR_UNSUPPORTED, "sparse matrix too large");
    M.nnz = (int)nnz;
    GLK_HIP(hipMemcpyAsync(M.rp.get() + M.n, &M.nnz, sizeof(int), hipMemcpyHostToDevice, s));
    GLK_HIP(hipStreamSynchronize(s));
    M.ci.alloc((size_t)std::max(1, M.nnz));
}

static void colour_level(gl_precond *pre, int l, hipStream_t s)
{
    Level &L = pre->L[l];
    const int n = L.n, nb = blocks_for(n);
    L.color.alloc(n);
    const gl_mesh *m = pre->mesh;
    if (l == 0 && !m->g.simplicial) {
        if (m->g.dim == 2) k_parity_colour<2><<<nb, kBlock, 0, s>>>(m->g, L.color.get());
        else k_parity_colour<3><<<nb, kBlock, 0, s>>>(m->g, L.color.get());
        GLK_CHECK_LAUNCH();
        L.ncolors = n > 1 ? 2 : 1;
    } else {
        DevBuf<int> ready(n), cnt(1), err(1);
        GLK_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));
        k_fill_int<<<nb, kBlock, 0, s>>>(L.color.get(), n, -1);
        // index priorities colour in waves (many rounds): the host reads the
        // uncoloured count every few rounds (later rounds change nothing)
        for (int round = 0;; ++round) {
            if (round > n + 8) fail(GL_ERR_HIP, "colouring did not terminate");
            GLK_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int), s));
            k_jp_ready<<<nb, kBlock, 0, s>>>(n, L.A.rp.get(), L.A.ci.get(), L.color.get(), ready.get());
            k_jp_colour<<<nb, kBlock, 0, s>>>(n, L.A.rp.get(), L.A.ci.get(), ready.get(), L.color.get(),
                                              cnt.get(), err.get());
            GLK_CHECK_LAUNCH();
            if ((round & 3) == 3 && read_int(cnt.get(), s) == 0) break;
        }
        check_err(err, s, "colouring");
        // class sizes and the number of colours
        DevBuf<int> hist(257);
        std::vector<int> h;
        int nc = 0;
        auto count = [&] {
            GLK_HIP(hipMemsetAsync(hist.get(), 0, 257 * sizeof(int), s));
            k_colour_hist<<<nb, kBlock, 0, s>>>(n, L.color.get(), hist.get());
            GLK_CHECK_LAUNCH();
            h = to_host(hist.get(), 257, s);
            nc = 0;
            for (int c = 0; c < 257; ++c)
                if (h[c]) nc = c + 1;
        };
        count();
        // iterated greedy: never more colours, often fewer (each colour costs
        // two dependent passes per symmetric sweep)
        DevBuf<int> nw(n);
        for (int pass = 0; pass < kRecolourPasses; ++pass) {
            k_fill_int<<<nb, kBlock, 0, s>>>(nw.get(), n, -1);
            for (int c = nc - 1; c >= 0; --c)
                k_ig_class<<<nb, kBlock, 0, s>>>(n, L.A.rp.get(), L.A.ci.get(), L.color.get(), c, nw.get(), err.get());
            GLK_CHECK_LAUNCH();
            GLK_HIP(hipMemcpyAsync(L.color.get(), nw.get(), sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
            count();
        }
        check_err(err, s, "recolouring");
        L.ncolors = nc;
        // rows grouped by colour
        L.cperm.alloc(n);
        L.coff.assign(nc + 1, 0);
        DevBuf<int> flag(n), pos(n);
        for (int c = 0; c < nc; ++c) {
            L.coff[c + 1] = L.coff[c] + h[c];
            k_flag_eq<<<nb, kBlock, 0, s>>>(n, L.color.get(), c, flag.get());
            scan_excl(flag.get(), pos.get(), n, s);
            k_scatter_colour<<<nb, kBlock, 0, s>>>(n, L.color.get(), c, pos.get(), L.cperm.get() + L.coff[c]);
            GLK_CHECK_LAUNCH();
        }
    }
}

// aggregation of level l; returns the number of aggregates
static int aggregate_level(gl_precond *pre, int l, hipStream_t s)
{
    Level &L = pre->L[l];
    const int n = L.n, nb = blocks_for(n);
    const int *rp = L.A.rp.get(), *ci = L.A.ci.get();
    DevBuf<int> state(n), near1(n), cnt(1), err(1), rootA(n), rootB(n), flag(n), id(n);
    DevBuf<unsigned long long> m1(n);
    k_fill_int<<<nb, kBlock, 0, s>>>(state.get(), n, 0);
    GLK_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));
    // index priorities decide roots in waves across the grid (many rounds):
    // the host reads the undecided count every few rounds (rounds after the
    // last decision change nothing)
    for (int round = 0;; ++round) {
        if (round > n + 8) fail(GL_ERR_HIP, "aggregation did not terminate");
        GLK_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int), s));
        k_mis_m1<<<nb, kBlock, 0, s>>>(n, rp, ci, state.get(), m1.get());
        k_mis_select<<<nb, kBlock, 0, s>>>(n, rp, ci, m1.get(), state.get());
        k_mis_near<<<nb, kBlock, 0, s>>>(n, rp, ci, state.get(), near1.get());
        k_mis_remove<<<nb, kBlock, 0, s>>>(n, rp, ci, near1.get(), state.get(), cnt.get());
        GLK_CHECK_LAUNCH();
        if ((round & 3) == 3 && read_int(cnt.get(), s) == 0) break;
    }
    k_agg_phase_a<<<nb, kBlock, 0, s>>>(n, rp, ci, state.get(), rootA.get());
    k_agg_phase_b<<<nb, kBlock, 0, s>>>(n, rp, ci, rootA.get(), rootB.get(), err.get());
    k_root_flags<<<nb, kBlock, 0, s>>>(n, state.get(), flag.get());
    GLK_CHECK_LAUNCH();
    check_err(err, s, "aggregation");
    const int nc = (int)scan_excl(flag.get(), id.get(), n, s);
    L.nc = nc;
    L.agg.alloc(n);
    L.root.alloc(std::max(1, nc));
    L.aggsize.alloc(std::max(1, nc));
    GLK_HIP(hipMemsetAsync(L.aggsize.get(), 0, sizeof(int) * std::max(1, nc), s));
    k_agg_number<<<nb, kBlock, 0, s>>>(n, rootB.get(), id.get(), state.get(), L.agg.get(), L.root.get(),
                                       L.aggsize.get());
    GLK_CHECK_LAUNCH();
    return nc;
}

static void transfer_patterns(gl_precond *pre, int l, hipStream_t s)
{
    Level &L = pre->L[l];
    Level &Nx = pre->L[l + 1];
    const int n = L.n, nc = L.nc, nb = blocks_for(n), nbc = blocks_for(nc);
    DevBuf<int> cnt(std::max(n, nc)), err(1);
    GLK_HIP(hipMemsetAsync(err.get(), 0, sizeof(int), s));
    // P: n x nc
    L.P.n = n;
    L.P.m = nc;
    k_p_pattern<<<nb, kBlock, 0, s>>>(n, L.A.rp.get(), L.A.ci.get(), L.agg.get(), nullptr, cnt.get(),
                                      nullptr, err.get());
    GLK_CHECK_LAUNCH();
    check_err(err, s, "prolongator pattern");
    alloc_rowptr(L.P, cnt.get(), s);
    k_p_pattern<<<nb, kBlock, 0, s>>>(n, L.A.rp.get(), L.A.ci.get(), L.agg.get(), L.P.rp.get(), nullptr,
                                      L.P.ci.get(), err.get());
    // R = P^H: nc x n
    L.R.n = nc;
    L.R.m = n;
    GLK_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * nc, s));
    k_col_count<<<blocks_for(L.P.nnz), kBlock, 0, s>>>(L.P.nnz, L.P.ci.get(), cnt.get());
    GLK_CHECK_LAUNCH();
    alloc_rowptr(L.R, cnt.get(), s);
    L.rsrc.alloc(std::max(1, L.R.nnz));
    DevBuf<int> fill(nc);
    GLK_HIP(hipMemsetAsync(fill.get(), 0, sizeof(int) * nc, s));
    k_transpose_fill<<<nb, kBlock, 0, s>>>(n, L.P.rp.get(), L.P.ci.get(), L.R.rp.get(), fill.get(),
                                           L.R.ci.get(), L.rsrc.get());
    k_sort_rows<<<nbc, kBlock, 0, s>>>(nc, L.R.rp.get(), L.R.ci.get(), L.rsrc.get());
    GLK_CHECK_LAUNCH();
    // A_{l+1} = R A P pattern
    Nx.n = nc;
    Nx.A.n = nc;
    Nx.A.m = nc;
    k_rap_pattern<<<nbc, kBlock, 0, s>>>(nc, L.R.rp.get(), L.R.ci.get(), L.A.rp.get(), L.A.ci.get(),
                                         L.P.rp.get(), L.P.ci.get(), nullptr, cnt.get(), nullptr, err.get());
    GLK_CHECK_LAUNCH();
    check_err(err, s, "Galerkin pattern");
    alloc_rowptr(Nx.A, cnt.get(), s);
    k_rap_pattern<<<nbc, kBlock, 0, s>>>(nc, L.R.rp.get(), L.R.ci.get(), L.A.rp.get(), L.A.ci.get(),
                                         L.P.rp.get(), L.P.ci.get(), Nx.A.rp.get(), nullptr, Nx.A.ci.get(),
                                         err.get());
    GLK_CHECK_LAUNCH();
    // product lists of the upper triangle for the numeric Galerkin product
    const int nnzc = Nx.A.nnz;
    DevBuf<int> pc(std::max(1, nnzc));
    GLK_HIP(hipMemsetAsync(pc.get(), 0, sizeof(int) * std::max(1, nnzc), s));
    k_rap_count<<<nbc, kBlock, 0, s>>>(nc, L.R.rp.get(), L.R.ci.get(), L.A.rp.get(), L.A.ci.get(), L.P.rp.get(),
                                       L.P.ci.get(), Nx.A.rp.get(), Nx.A.ci.get(), pc.get());
    GLK_CHECK_LAUNCH();
    L.rap_tp.alloc((size_t)nnzc + 1);
    const int64_t ntrip = scan_excl(pc.get(), L.rap_tp.get(), nnzc, s);
    if (ntrip > (int64_t)1 << 30) fail(GL_ERR_UNSUPPORTED, "Galerkin product: too many products");
    const int total = (int)ntrip;
    GLK_HIP(hipMemcpyAsync(L.rap_tp.get() + nnzc, &total, sizeof(int), hipMemcpyHostToDevice, s));
    L.rap_trip.alloc((size_t)3 * std::max<int64_t>(1, ntrip));
    GLK_HIP(hipMemsetAsync(pc.get(), 0, sizeof(int) * std::max(1, nnzc), s));
    k_rap_fill<<<nbc, kBlock, 0, s>>>(nc, L.R.rp.get(), L.R.ci.get(), L.A.rp.get(), L.A.ci.get(), L.P.rp.get(),
                                      L.P.ci.get(), Nx.A.rp.get(), Nx.A.ci.get(), L.rap_tp.get(), pc.get(),
                                      L.rap_trip.get());
    GLK_CHECK_LAUNCH();
    GLK_HIP(hipStreamSynchronize(s));
}

static void alloc_values(gl_precond *pre)
{
    const bool simp = pre->mesh->g.simplicial;
    const int ns = simp ? 0 : 2 * geom_t<double>(pre->mesh->g).npair;  // level-0 split layout of a grid
    for (int l = 0; l < pre->nlev; ++l) {
        Level &L = pre->L[l];
        const int nv = l == 0 ? std::max(L.n, ns) : L.n;
        L.A.v64.alloc(std::max(1, L.A.nnz));
        L.A.v32.alloc(std::max(1, L.A.nnz));
        L.diag64.alloc(L.n);
        L.diag32.alloc(L.n);
        L.b64.alloc(nv);
        L.x64.alloc(nv);
        L.r64.alloc(nv);
        L.b32.alloc(nv);
        L.x32.alloc(nv);
        L.r32.alloc(nv);
        if (l == 0 && !simp) {
            L.hs64.alloc(ns);
            L.hs32.alloc(ns);
        }
        if (l < pre->nlev - 1) {
            L.P.v64.alloc(std::max(1, L.P.nnz));
            L.P.v32.alloc(std::max(1, L.P.nnz));
            L.R.v64.alloc(std::max(1, L.R.nnz));
            L.R.v32.alloc(std::max(1, L.R.nnz));
            L.rho.alloc(1);
        }
    }
    const int nl = pre->L[pre->nlev - 1].n;
    pre->cfac.alloc((size_t)nl * nl);
    pre->cinv64.alloc((size_t)nl * nl);
    pre->cinv32.alloc((size_t)nl * nl);
    pre->status.alloc(1);
    pre->cdmax.alloc(1);
    const int n0 = pre->L[0].n;
    pre->cyc_r.alloc(n0);
    pre->vin.alloc(n0);
    pre->pwn.alloc(2);
}

// copy of M with rows taken in the order rowperm and columns relabelled by colmap
static void permuted_copy(const Csr &M, const int *rowperm, const int *colmap, Csr &out, DevBuf<int> &map,
                          hipStream_t s)
{
    out.n = M.n;
    out.m = M.m;
    DevBuf<int> cnt(std::max(1, M.n));
    k_perm_count<<<blocks_for(M.n), kBlock, 0, s>>>(M.n, rowperm, M.rp.get(), cnt.get());
    GLK_CHECK_LAUNCH();
    alloc_rowptr(out, cnt.get(), s);
    map.alloc(std::max(1, out.nnz));
    k_perm_fill<<<blocks_for(M.n), kBlock, 0, s>>>(M.n, rowperm, M.rp.get(), M.ci.get(), colmap, out.rp.get(),
                                                   out.ci.get(), map.get());
    GLK_CHECK_LAUNCH();
    out.v64.alloc(std::max(1, out.nnz));
    out.v32.alloc(std::max(1, out.nnz));
}

// the colour-ordered copies the V-cycle works on
static void build_apply_copies(gl_precond *pre, hipStream_t s)
{
    // level 0 of a simplicial mesh is a CSR level like the coarse ones (when
    // it is not the coarsest, which is applied as a dense inverse in node order)
    const bool simp = pre->mesh->g.simplicial && pre->nlev > 1;
    const int lfirst = simp ? 0 : 1;
    for (int l = lfirst; l < pre->nlev; ++l) {
        Level &L = pre->L[l];
        L.perm.alloc(L.n);
        GLK_HIP(hipMemcpyAsync(L.perm.get(), L.cperm.get(), sizeof(int) * L.n, hipMemcpyDeviceToDevice, s));
        L.iperm.alloc(L.n);
        k_iperm<<<blocks_for(L.n), kBlock, 0, s>>>(L.n, L.perm.get(), L.iperm.get());
        GLK_CHECK_LAUNCH();
        L.dg64.alloc(L.n);
        L.dg32.alloc(L.n);
    }
    for (int l = 0; l < pre->nlev; ++l) {
        Level &L = pre->L[l];
        const bool generic = l >= lfirst;
        const int *rowp = generic ? L.perm.get() : nullptr;
        const int *colp = generic ? L.iperm.get() : nullptr;
        if (generic) permuted_copy(L.A, rowp, colp, L.Aa, L.amap, s);
        if (l + 1 < pre->nlev) {
            Level &Nx = pre->L[l + 1];
            permuted_copy(L.P, rowp, Nx.iperm.get(), L.Pa, L.pmap, s);
            permuted_copy(L.R, Nx.perm.get(), colp, L.Ra, L.rmap, s);
            if (l == 0 && !generic) {
                const GeomT<double> g = geom_t<double>(pre->mesh->g);
                Csr &B = L.Rb;
                B.n = L.Ra.n;
                B.m = 2 * g.npair;
                DevBuf<int> cnt(std::max(1, B.n));
                k_black_count<<<blocks_for(B.n), kBlock, 0, s>>>(B.n, g, L.Ra.rp.get(), L.Ra.ci.get(), cnt.get());
                GLK_CHECK_LAUNCH();
                alloc_rowptr(B, cnt.get(), s);
                L.bmap.alloc(std::max(1, B.nnz));
                k_black_fill<<<blocks_for(B.n), kBlock, 0, s>>>(B.n, g, L.Ra.rp.get(), L.Ra.ci.get(), L.rmap.get(),
                                                                B.rp.get(), B.ci.get(), L.bmap.get());
                GLK_CHECK_LAUNCH();
                B.v64.alloc(std::max(1, B.nnz));
                B.v32.alloc(std::max(1, B.nnz));
                Csr &Q = L.Pb;
                Q.n = g.npair;
                Q.m = L.Pa.m;
                DevBuf<int> qcnt(std::max(1, Q.n));
                k_pblack_count<<<blocks_for(Q.n), kBlock, 0, s>>>(g, L.Pa.rp.get(), qcnt.get());
                GLK_CHECK_LAUNCH();
                alloc_rowptr(Q, qcnt.get(), s);
                L.pbmap.alloc(std::max(1, Q.nnz));
                k_pblack_fill<<<blocks_for(Q.n), kBlock, 0, s>>>(g, L.Pa.rp.get(), L.Pa.ci.get(), L.pmap.get(),
                                                                 Q.rp.get(), Q.ci.get(), L.pbmap.get());
                GLK_CHECK_LAUNCH();
                Q.v64.alloc(std::max(1, Q.nnz));
                Q.v32.alloc(std::max(1, Q.nnz));
            }
        }
        if (generic) {
            // padded colour blocks for the Gauss-Seidel sweeps
            std::vector<int> rp = to_host(L.Aa.rp.get(), (size_t)L.n + 1, s);
            L.ewidth.assign(L.ncolors, 0);
            L.eoff.assign(L.ncolors + 1, 0);
            for (int c = 0; c < L.ncolors; ++c) {
                int w = 1;
                for (int r = L.coff[c]; r < L.coff[c + 1]; ++r) w = std::max(w, rp[r + 1] - rp[r]);
                L.ewidth[c] = w;
                L.eoff[c + 1] = L.eoff[c] + w * (L.coff[c + 1] - L.coff[c]);
            }
            const int ne = std::max(1, L.eoff[L.ncolors]);
            L.eci.alloc(ne);
            L.emap.alloc(ne);
            L.ev64.alloc(ne);
            L.ev32.alloc(ne);
            for (int c = 0; c < L.ncolors; ++c) {
                const int cnt = L.coff[c + 1] - L.coff[c];
                if (cnt == 0) continue;
                k_ell_fill<<<blocks_for(cnt), kBlock, 0, s>>>(L.coff[c], cnt, L.ewidth[c], L.Aa.rp.get(),
                                                             L.Aa.ci.get(), L.eci.get() + L.eoff[c],
                                                             L.emap.get() + L.eoff[c]);
                GLK_CHECK_LAUNCH();
            }
        }
    }
    GLK_HIP(hipStreamSynchronize(s));
}

void precond_symbolic(gl_precond *pre, hipStream_t s)
{
    const gl_mesh *m = pre->mesh;
    const int n0 = m->g.n, nb0 = blocks_for(n0);
    Level &L0 = pre->L[0];
    L0.n = n0;
    L0.A.n = L0.A.m = n0;
    {
        DevBuf<int> cnt(n0);
        if (m->g.simplicial) k_l0s_count<<<nb0, kBlock, 0, s>>>(n0, m->g.rp, cnt.get());
        else if (m->g.dim == 2) k_l0_count<2><<<nb0, kBlock, 0, s>>>(m->g, cnt.get());
        else k_l0_count<3><<<nb0, kBlock, 0, s>>>(m->g, cnt.get());
        GLK_CHECK_LAUNCH();
        alloc_rowptr(L0.A, cnt.get(), s);
        if (m->g.simplicial)
            k_l0s_cols<<<nb0, kBlock, 0, s>>>(n0, m->g.rp, m->g.ci, L0.A.rp.get(), L0.A.ci.get());
        else if (m->g.dim == 2) k_l0_cols<2><<<nb0, kBlock, 0, s>>>(m->g, L0.A.rp.get(), L0.A.ci.get());
        else k_l0_cols<3><<<nb0, kBlock, 0, s>>>(m->g, L0.A.rp.get(), L0.A.ci.get());
        GLK_CHECK_LAUNCH();
    }
    const int max_levels = std::min(pre->opts.max_levels, kMaxLevels);
    int l = 0;
    for (;;) {
        colour_level(pre, l, s);
        Level &L = pre->L[l];
        if (L.n <= pre->opts.max_coarse || l == max_levels - 1) break;
        const int nc = aggregate_level(pre, l, s);
        if ((double)nc > 0.85 * (double)L.n) {
            L.agg.release();
            L.root.release();
            L.aggsize.release();
            L.nc = 0;
            break;
        }
        transfer_patterns(pre, l, s);
        ++l;
    }
    pre->nlev = l + 1;
    if (pre->L[l].n > kMaxDense)
        fail(GL_ERR_UNSUPPORTED, "coarsest level too large for the dense solve");
    alloc_values(pre);
    build_apply_copies(pre, s);
    bottom_descriptors(pre, s);
    GLK_HIP(hipStreamSynchronize(s));
}

void precond_numeric_enqueue(gl_precond *pre, const double2 *psi, const Launch &L)
{
    const gl_mesh *m = pre->mesh;
    Level &L0 = pre->L[0];
    const int n0 = L0.n;
    const GeomT<double> g = geom_t<double>(m->g);
    const bool simp = m->g.simplicial;
    if (simp)
        L.run(blocks_for(n0), L0sValues{g, L0.A.rp.get(), L0.A.ci.get(), psi, L0.A.v64.get(), L0.diag64.get()});
    else if (m->g.dim == 2)
        L.run(blocks_for(n0), L0Values<2>{g, L0.A.rp.get(), link_tab<double>(m), psi, L0.A.v64.get(), L0.diag64.get()});
    else
        L.run(blocks_for(n0), L0Values<3>{g, L0.A.rp.get(), link_tab<double>(m), psi, L0.A.v64.get(), L0.diag64.get()});
    for (int l = 0; l + 1 < pre->nlev; ++l) {
        Level &lv = pre->L[l];
        Level &Nx = pre->L[l + 1];
        const int n = lv.n, nb = blocks_for(n);
        if (l > 0) L.run(nb, Diag{n, lv.A.rp.get(), lv.A.ci.get(), lv.A.v64.get(), lv.diag64.get()});
        rho_estimate(pre, lv, L);
        L.run(nb, PValues{n, lv.A.rp.get(), lv.A.ci.get(), lv.A.v64.get(), lv.diag64.get(), lv.agg.get(),
                          lv.aggsize.get(), lv.rho.get(), lv.P.rp.get(), lv.P.ci.get(), lv.P.v64.get()});
        L.run(blocks_for(lv.R.nnz), RValues{lv.R.nnz, lv.rsrc.get(), lv.P.v64.get(), lv.R.v64.get()});
        L.run(blocks_for((int64_t)Nx.A.nnz * kRapLanes),
              RapValues{Nx.A.nnz, lv.rap_tp.get(), lv.rap_trip.get(), lv.R.v64.get(), lv.A.v64.get(), lv.P.v64.get(),
                        Nx.A.v64.get()});
        L.run(blocks_for(lv.nc), RapMirror{lv.nc, Nx.A.rp.get(), Nx.A.ci.get(), Nx.A.v64.get()});
    }
    const int last = pre->nlev - 1;
    Level &Lc = pre->L[last];
    if (last > 0) L.run(blocks_for(Lc.n), Diag{Lc.n, Lc.A.rp.get(), Lc.A.ci.get(), Lc.A.v64.get(), Lc.diag64.get()});
    // level 0 in single precision (its stencil diagonal; the CSR copy serves export only)
    L.run(blocks_for(n0), ToF32r{n0, L0.diag64.get(), L0.diag32.get()});
    if (!simp) L.run(blocks_for(g.npair), SplitDiag{g, L0.diag64.get(), L0.hs64.get(), L0.hs32.get()});
    // colour-ordered copies for the V-cycle, FP64 and rounded to FP32
    for (int l = 0; l < pre->nlev; ++l) {
        Level &lv = pre->L[l];
        if (l >= 1 || (simp && last > 0)) {
            L.run(blocks_for(lv.Aa.nnz), GatherC{lv.Aa.nnz, lv.amap.get(), lv.A.v64.get(), lv.Aa.v64.get(), lv.Aa.v32.get()});
            L.run(blocks_for(lv.n), GatherR{lv.n, lv.perm.get(), lv.diag64.get(), lv.dg64.get(), lv.dg32.get()});
            const int ne = lv.eoff.empty() ? 0 : lv.eoff.back();
            if (ne > 0) L.run(blocks_for(ne), EllValues{ne, lv.emap.get(), lv.Aa.v64.get(), lv.ev64.get(), lv.ev32.get()});
        }
        if (l < last) {
            L.run(blocks_for(lv.Pa.nnz), GatherC{lv.Pa.nnz, lv.pmap.get(), lv.P.v64.get(), lv.Pa.v64.get(), lv.Pa.v32.get()});
            L.run(blocks_for(lv.Ra.nnz), GatherC{lv.Ra.nnz, lv.rmap.get(), lv.R.v64.get(), lv.Ra.v64.get(), lv.Ra.v32.get()});
            if (l == 0 && !simp) {
                L.run(blocks_for(lv.Rb.nnz),
                      GatherC{lv.Rb.nnz, lv.bmap.get(), lv.R.v64.get(), lv.Rb.v64.get(), lv.Rb.v32.get()});
                L.run(blocks_for(lv.Pb.nnz),
                      GatherC{lv.Pb.nnz, lv.pbmap.get(), lv.P.v64.get(), lv.Pb.v64.get(), lv.Pb.v32.get()});
            }
        }
    }
    // coarsest: Cholesky in FP64 (positive definiteness check), then the inverse
    // in the V-cycle's row order, applied as a dense product
    const Csr &Mc = last > 0 ? Lc.Aa : Lc.A;
    L.run(blocks_for(Lc.n), DenseFromCsr{Lc.n, Mc.rp.get(), Mc.ci.get(), Mc.v64.get(), pre->cfac.get()});
    cholesky(Lc.n, pre->cfac.get(), pre->cdmax.get(), pre->status.get(), L);
    L.run(Lc.n, CholInverse{Lc.n, pre->cfac.get(), pre->cinv64.get(), pre->status.get()});
    L.run(blocks_for((int64_t)Lc.n * Lc.n), ToF32c{Lc.n * Lc.n, pre->cinv64.get(), pre->cinv32.get()});
}

void precond_numeric_finish(gl_precond *pre, bool singular, hipStream_t s)
{
    if (singular) fail(GL_ERR_SINGULAR, "gl_precond_setup: coarsest operator is not positive definite");
    pre->has_values = true;
    form_tail(pre, s);
    if (pre->opts.cycles == 0) pcg_calibrate(pre, s);
}

void precond_numeric(gl_precond *pre, const double2 *psi, hipStream_t s)
{
    precond_numeric_enqueue(pre, psi, Launch{s});
    precond_numeric_finish(pre, read_int(pre->status.get(), s) != 0, s);
}

}  // namespace glk

using namespace glk;

namespace glk {
void check_amg_opts(const gl_amg_opts *opts, const char *who)
{
    const std::string w(who);
    if (opts->precision != GL_FP64 && opts->precision != GL_FP32 && opts->precision != GL_MIXED)
        fail(GL_ERR_INVALID_ARGUMENT, w + ": precision");
    if (opts->cycles < 0 || opts->cycles > 1000) fail(GL_ERR_INVALID_ARGUMENT, w + ": cycles must be in 0..1000");
    if (opts->cycles == 0 && opts->precision != GL_FP64)
        fail(GL_ERR_INVALID_ARGUMENT, w + ": R_inf (cycles 0) needs the FP64 V-cycle");
    if (opts->max_coarse < 1 || opts->max_coarse > kMaxDense)
        fail(GL_ERR_INVALID_ARGUMENT, w + ": max_coarse must be in 1..2048");
    if (opts->max_levels < 1 || opts->max_levels > kMaxLevels)
        fail(GL_ERR_INVALID_ARGUMENT, w + ": max_levels must be in 1..16");
}

uint64_t new_precond_uid()
{
    static std::atomic<uint64_t> next{1};
    return next++;
}
}  // namespace glk

extern "C" {

gl_status gl_precond_setup(const gl_mesh *mesh, const void *psi, const gl_amg_opts *opts,
                           gl_precond **inout, gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi || !inout) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_setup: NULL argument");
        hipStream_t s = as_stream(stream);
        gl_precond *pre = *inout;
        if (pre && pre->mesh != mesh)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_setup: handle belongs to another mesh");
        if (!pre && !opts) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_setup: opts required for a new handle");
        if (opts) check_amg_opts(opts, "gl_precond_setup");
        if (!pre) {
            pre = new gl_precond();
            try {
                pre->uid = new_precond_uid();
                pre->mesh = mesh;
                pre->opts = *opts;
                precond_symbolic(pre, s);
                precond_numeric(pre, (const double2 *)psi, s);
            } catch (...) {
                delete pre;
                throw;
            }
            *inout = pre;
        } else {
            if (opts) {
                if (opts->max_coarse != pre->opts.max_coarse || opts->max_levels != pre->opts.max_levels)
                    fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_setup: hierarchy limits differ from the handle's");
                pre->opts.precision = opts->precision;
                pre->opts.cycles = opts->cycles;
            }
            precond_numeric(pre, (const double2 *)psi, s);
        }
    });
}

gl_status gl_precond_inner_steps(const gl_precond *pre, int *steps)
{
    return guarded([&] {
        if (!pre || !steps) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_inner_steps: NULL argument");
        *steps = pre->opts.cycles == 0 ? pre->pcg_m : pre->opts.cycles;
    });
}

gl_status gl_precond_info(const gl_precond *pre, int *nlev, int64_t *sizes, int64_t *nnz, int *ncolors)
{
    return guarded([&] {
        if (!pre) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_info: NULL handle");
        if (nlev) *nlev = pre->nlev;
        for (int l = 0; l < pre->nlev; ++l) {
            if (sizes) sizes[l] = pre->L[l].n;
            if (nnz) nnz[l] = pre->L[l].A.nnz;
            if (ncolors) ncolors[l] = pre->L[l].ncolors;
        }
    });
}

gl_status gl_precond_export(const gl_precond *pre, int level, int what, void *host_buf, size_t *bytes)
{
    return guarded([&] {
        if (!pre || !bytes) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_export: NULL argument");
        if (level < 0 || level >= pre->nlev) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_export: level");
        const Level &L = pre->L[level];
        const bool last = level == pre->nlev - 1;
        if (last && ((what >= 6 && what <= 11) || what == 0 || what == 1))
            fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_export: the coarsest level has no transfer operators");
        const void *src = nullptr;
        size_t need = 0;
        switch (what) {
        case 0: src = L.agg.get(); need = sizeof(int) * L.n; break;
        case 1: src = L.root.get(); need = sizeof(int) * L.nc; break;
        case 2: src = L.color.get(); need = sizeof(int) * L.n; break;
        case 3: src = L.A.rp.get(); need = sizeof(int) * (L.n + 1); break;
        case 4: src = L.A.ci.get(); need = sizeof(int) * L.A.nnz; break;
        case 5: src = L.A.v64.get(); need = sizeof(double2) * L.A.nnz; break;
        case 6: src = L.P.rp.get(); need = sizeof(int) * (L.n + 1); break;
        case 7: src = L.P.ci.get(); need = sizeof(int) * L.P.nnz; break;
        case 8: src = L.P.v64.get(); need = sizeof(double2) * L.P.nnz; break;
        case 9: src = L.R.rp.get(); need = sizeof(int) * (L.nc + 1); break;
        case 10: src = L.R.ci.get(); need = sizeof(int) * L.R.nnz; break;
        case 11: src = L.R.v64.get(); need = sizeof(double2) * L.R.nnz; break;
        default: fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_export: unknown array");
        }
        if (!host_buf) { *bytes = need; return; }
        if (*bytes < need) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_export: buffer too small");
        *bytes = need;
        GLK_HIP(hipDeviceSynchronize());
        if (need) GLK_HIP(hipMemcpy(host_buf, src, need, hipMemcpyDeviceToHost));
    });
}

gl_status gl_precond_set_tiles(gl_precond *pre, const gl_tiles *tiles)
{
    return guarded([&] {
        if (!pre || !tiles) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_set_tiles: NULL argument");
        if (tiles->lane_shift < -2 || tiles->lane_shift > 2 || tiles->bottom_rows < 0 || tiles->bottom_rows > 65536 ||
            tiles->dense_rows < 0 || tiles->dense_rows > kMaxTail || tiles->l0_tiled < 0 || tiles->l0_tiled > 3)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_set_tiles: lane_shift in -2..2, bottom_rows in 0..65536, "
                                          "dense_rows in 0..8192, l0_tiled 0..3");
        const int rows = tiles->bottom_rows ? tiles->bottom_rows : kBottomRows;
        if (rows == pre->bottom_rows && tiles->lane_shift == pre->lane_shift && tiles->dense_rows == pre->dense_rows &&
            tiles->l0_tiled == pre->l0_tiled)
            return;
        pre->bottom_rows = rows;
        pre->lane_shift = tiles->lane_shift;
        pre->dense_rows = tiles->dense_rows;
        pre->l0_tiled = tiles->l0_tiled;
        pre->uid = new_precond_uid();  // captured graphs of the old shape are stale
        hipStream_t s = pre->mesh->ws;
        GLK_HIP(hipStreamSynchronize(s));  // no pending use of the buffers re-made here
        bottom_descriptors(pre, s);
        form_tail(pre, s);
        GLK_HIP(hipStreamSynchronize(s));
    });
}

gl_status gl_precond_get_tiles(const gl_precond *pre, gl_tiles *tiles)
{
    return guarded([&] {
        if (!pre || !tiles) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_get_tiles: NULL argument");
        tiles->lane_shift = pre->lane_shift;
        tiles->bottom_rows = pre->bottom_rows;
        tiles->dense_rows = pre->dense_rows;
        tiles->l0_tiled = pre->l0_tiled;
    });
}

void gl_precond_destroy(gl_precond *pre) { delete pre; }

}  // extern "C"
