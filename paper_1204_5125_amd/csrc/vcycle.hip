// Application of the preconditioner R_k = AMG_k(H, D .) (eq. prec2): k
// V-cycles from zero on H x = v with one symmetric Gauss-Seidel sweep before
// and after the coarse correction (Sec. 4.1).  A symmetric sweep visits the
// colours 0 .. C-1 and then C-2 .. 0; on level 0 (red-black, red = even index
// sum) that is red, black, red.  Every kernel is templated on the storage and
// arithmetic type (double or float); the input v and the output z are FP64.
//
// Level 0 needs six stencil passes instead of seven because a Gauss-Seidel
// update of a red node does not read the node's previous value:
//   - the first red update from x = 0 is x_r = b_r / H_rr, folded into the
//     black update that follows (which evaluates it for its red neighbours);
//   - after the pre-smoothing sweep the red residual is zero (the last update
//     made it so), and only black residuals are formed;
//   - after the coarse correction only the black values x_b + (P x_c)_b are
//     read (by the first red update), so only black nodes are prolonged.
// On the coarser levels the zero start and the first two colour passes of the
// pre-smoothing sweep are one dispatch for the same reason.  Below the first
// level with at most dense_rows rows (a tile choice) the cycle is a fixed
// linear map of that level's right-hand side; it is formed as a dense matrix
// at setup and applied as one product, like the coarsest inverse.
#include <cstring>
#include <type_traits>

#include "amg.h"
#include "stencil.h"

namespace glk {

#define GATE()                               \
    if (gate && *gate == 0) return

// The gate flag read together with a kernel's data and checked right before
// its stores, so that its load overlaps the others instead of delaying them;
// the flag is uniform, so every thread takes the same branch.
#define GATE_LOAD() const bool gate_go = gate == nullptr || *gate != 0

// a seeded right-hand side in [-1, 1]^2 per node (MurmurHash3 finaliser of
// the node index), for calibrating R_inf
__global__ void k_hash_rhs(int n, double2 *v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    auto mix = [](uint32_t h) {
        h ^= h >> 16;
        h *= 0x85ebca6bu;
        h ^= h >> 13;
        h *= 0xc2b2ae35u;
        h ^= h >> 16;
        return h;
    };
    const uint32_t a = mix(2u * (uint32_t)i + 0x9e3779b9u), b = mix(2u * (uint32_t)i + 1u + 0x9e3779b9u);
    v[i] = make_double2(a * (2.0 / 4294967295.0) - 1.0, b * (2.0 / 4294967295.0) - 1.0);
}

// Level-0 colour passes run one thread per red-black pair: thread t owns the
// nodes c0 = 2k and 2k + 1 of x-row `row` (k = t mod hr, row = t / hr), one
// of each colour, so every thread updates a node (a thread per node would
// leave half of them idle and need twice the waves).
struct Pair {
    int ie;      // index of the even node (c0 = 2k)
    int c[3];    // its coordinates
    bool odd;    // the odd node c0 = 2k + 1 exists
};

template <int DIM, class T>
__device__ __forceinline__ Pair pair_at(const GeomT<T> &g, int t)
{
    Pair P;
    const int row = t / g.hr, k = t - row * g.hr;
    P.c[0] = 2 * k;
    P.c[1] = DIM == 3 ? row % g.N[1] : row;
    P.c[2] = DIM == 3 ? row / g.N[1] : 0;
    P.ie = 2 * k + g.N[0] * row;
    P.odd = 2 * k + 1 < g.N[0];
    return P;
}

// the pair's node of colour col: offset s from the even node (false: absent)
__device__ __forceinline__ bool pair_colour(const Pair &P, int col, int &s)
{
    s = (col + P.c[1] + P.c[2]) & 1;
    return s == 0 || P.odd;
}

// The V-cycle's level-0 vectors (b, x, r) and the diagonal it divides by are
// stored split by colour: the node of colour col in pair t sits at
// col * npair + t.  A colour pass then reads and writes one contiguous half,
// and the neighbours of a node, all of the other colour, sit in the other
// half at pairs t +- 1 (x), t +- hr (y) and t +- hr N1 (z).  The sum below
// takes the terms in the order of khat_offdiag, so the results do not change.
template <int DIM, class T>
__device__ __forceinline__ C<T> khat_offdiag_rb(const GeomT<T> &g, const int c[3], int t,
                                                const C<T> *__restrict__ xo, const LinkTab<T> &U)
{
    T s[3];
    const T d = node_volume<DIM, T>(g, c, s);
    C<T> acc = mk<T>(0, 0);
    const int row0 = t - (c[0] >> 1);  // first pair of the node's x-row
    int pstride = g.hr;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T al = d * s[a] * g.inv_h2[a];
        int tl, tu;
        if (a == 0) {
            tl = row0 + ((c[0] - 1) >> 1);
            tu = row0 + ((c[0] + 1) >> 1);
        } else {
            tl = t - pstride;
            tu = t + pstride;
            pstride *= g.N[a];
        }
        if (c[a] > 0) acc = csub(acc, cscale(cmul(link_u<DIM, T>(U, a, c, c[a] - 1), xo[tl]), al));
        if (c[a] < g.N[a] - 1) acc = csub(acc, cscale(cmulc(link_u<DIM, T>(U, a, c, c[a]), xo[tu]), al));
    }
    return acc;
}

// pre-smoothing: b = round(v) into the split layout, and the black pass from
// zero (the red pass from zero, x_red = b / diag, folded in: it reads v and
// the natural-order diagonal hd at the red neighbours)
template <int DIM, class T>
struct L0PreBlack {
    GeomT<T> g;
    const double2 *v;
    C<T> *b, *x;
    LinkTab<T> U;
    const T *hd;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        const int t = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        if (t >= g.npair) return;
        const Pair P = pair_at<DIM, T>(g, t);
        const int np = g.npair, ce = (P.c[1] + P.c[2]) & 1;  // colour of the even node
        const C<T> b0 = narrow<T>(v[P.ie]);
        const C<T> b1 = P.odd ? narrow<T>(v[P.ie + 1]) : mk<T>(0, 0);
        if (gate_go) {
            b[ce * np + t] = b0;
            if (P.odd) b[(1 - ce) * np + t] = b1;
        }
        int sb;
        if (!pair_colour(P, 1, sb)) return;
        const int i = P.ie + sb;
        const int c[3] = {P.c[0] + sb, P.c[1], P.c[2]};
        const C<T> bi = sb ? b1 : b0;
        T s[3];
        const T d = node_volume<DIM, T>(g, c, s);
        C<T> off = mk<T>(0, 0);
        int stride = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const T al = d * s[a] * g.inv_h2[a];
            if (c[a] > 0) {
                const int k = i - stride;
                const C<T> xk = cscale(narrow<T>(v[k]), (T)1 / hd[k]);
                off = csub(off, cscale(cmul(link_u<DIM, T>(U, a, c, c[a] - 1), xk), al));
            }
            if (c[a] < g.N[a] - 1) {
                const int k = i + stride;
                const C<T> xk = cscale(narrow<T>(v[k]), (T)1 / hd[k]);
                off = csub(off, cscale(cmulc(link_u<DIM, T>(U, a, c, c[a]), xk), al));
            }
            stride *= g.N[a];
        }
        const C<T> xi = cscale(csub(bi, off), (T)1 / hd[i]);
        if (!gate_go) return;
        x[np + t] = xi;
    }
};

// x_i = (b_i - sum_{j != i} H_ij x_j) / H_ii on one colour (split layout; hs:
// the diagonal in that layout)
template <int DIM, class T>
struct L0Sweep {
    GeomT<T> g;
    int colour;
    const C<T> *b;
    C<T> *x;
    LinkTab<T> U;
    const T *hs;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        const int t = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        if (t >= g.npair) return;
        const Pair P = pair_at<DIM, T>(g, t);
        int sc;
        if (!pair_colour(P, colour, sc)) return;
        const int c[3] = {P.c[0] + sc, P.c[1], P.c[2]};
        const int q = colour * g.npair + t;
        const C<T> bi = b[q];
        const T di = hs[q];
        const C<T> off = khat_offdiag_rb<DIM, T>(g, c, t, x + (1 - colour) * g.npair, U);
        const C<T> xi = cscale(csub(bi, off), (T)1 / di);
        if (!gate_go) return;
        x[q] = xi;
    }
};

// r = b - H x on the black nodes (split layout); the red residual is zero and
// is neither stored nor read (the restriction has no red columns)
template <int DIM, class T>
struct L0Residual {
    GeomT<T> g;
    const C<T> *b, *x;
    LinkTab<T> U;
    const T *hs;
    C<T> *r;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        const int t = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        if (t >= g.npair) return;
        const Pair P = pair_at<DIM, T>(g, t);
        int sb;
        if (!pair_colour(P, 1, sb)) return;
        const int c[3] = {P.c[0] + sb, P.c[1], P.c[2]};
        const int q = g.npair + t;
        const C<T> bi = b[q];
        const C<T> xi = x[q];
        const T di = hs[q];
        const C<T> off = khat_offdiag_rb<DIM, T>(g, c, t, x, U);
        const C<T> ri = csub(csub(bi, cscale(xi, di)), off);
        if (!gate_go) return;
        r[q] = ri;
    }
};

// r = v - H z on every node, FP64 (between cycles of R_k, k > 1)
template <int DIM>
struct L0ResidualFull {
    GeomT<double> g;
    const double2 *v, *z;
    LinkTab<double> U;
    const double *hd;
    double2 *r;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE();
        const int i = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int c[3];
        node_coords<DIM>(g.N, i, c);
        const double2 off = khat_offdiag<DIM, double>(g, i, c, z, U);
        r[i] = csub(csub(v[i], cscale(z[i], hd[i])), off);
    }
};

// (P x_c)_k for one fine row
template <class T>
__device__ __forceinline__ C<T> prolong_row(const int *__restrict__ prp, const int *__restrict__ pci,
                                            const C<T> *__restrict__ pv, const C<T> *__restrict__ xc, int k)
{
    C<T> s = mk<T>(0, 0);
    for (int p = prp[k]; p < prp[k + 1]; ++p) s = cadd(s, cmul(pv[p], xc[pci[p]]));
    return s;
}

// coarse correction of the black nodes: x_b += (P x_c)_b (the red nodes are
// overwritten by the red pass that follows, which reads only black values);
// x in the split layout, P's black rows by pair (row t: the black node of
// pair t)
template <int DIM, class T, class TC = T>
struct L0ProlongBlack {
    GeomT<T> g;
    C<T> *x;
    const int *prp, *pci;
    const C<TC> *pv, *xc;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        const int t = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        if (t >= g.npair) return;
        const Pair P = pair_at<DIM, T>(g, t);
        int sb;
        if (!pair_colour(P, 1, sb)) return;
        const int q = g.npair + t;
        const C<T> xo = x[q];
        const C<T> xi = cadd(xo, as_c<T>(prolong_row<TC>(prp, pci, pv, xc, t)));
        if (!gate_go) return;
        x[q] = xi;
    }
};

// last red pass; z = x (ADD: z += x) on every node and partial sums of Re<vdot, z>
template <int DIM, class T, int ADD>
struct L0Last {
    GeomT<T> g;
    const C<T> *b;
    C<T> *x;
    LinkTab<T> U;
    const T *hs;
    double2 *z;
    const double2 *vdot;
    RedSlot slot;
    int want_dot;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        __shared__ double sm[kBlock / 64];
        const int t = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        const bool in = t < g.npair;
        const Pair P = pair_at<DIM, T>(g, in ? t : 0);
        // the red node's update, then z on both nodes (even first, natural
        // order); every load before the (uniform) gate check, every store
        // after it.  The red update goes to z only: the next cycle starts
        // from zero and writes every node before it reads it.
        int sr, sb;
        const bool red = in && pair_colour(P, 0, sr);
        const bool black = in && pair_colour(P, 1, sb);
        C<T> xr = mk<T>(0, 0);
        const C<T> xb = black ? x[g.npair + t] : mk<T>(0, 0);
        double2 zq[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
        double part = 0.0;
        if (red) {
            const int c[3] = {P.c[0] + sr, P.c[1], P.c[2]};
            const C<T> bi = b[t];
            const T di = hs[t];
            const C<T> off = khat_offdiag_rb<DIM, T>(g, c, t, x + g.npair, U);
            xr = cscale(csub(bi, off), (T)1 / di);
        }
        if (in) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (q == 1 && !P.odd) break;
                const int i = P.ie + q;
                double2 zi = widen(red && q == sr ? xr : xb);
                if (ADD) zi = cadd(z[i], zi);
                zq[q] = zi;
                if (want_dot) part += redot(vdot[i], zi);
            }
        }
        if (!gate_go) return;
        if (in) {
            z[P.ie] = zq[0];
            if (P.odd) z[P.ie + 1] = zq[1];
        }
        if (want_dot) block_reduce_store(part, slot, sm, bx);
    }
};

// ------------------------------------------- level 0 in LDS tiles (2D) ---
// The level-0 passes of a V-cycle fused into two kernels, each over a tile
// of S::TX x S::TY nodes held in LDS with a halo of three nodes: the three
// colour passes of a sweep need neighbours' values of the previous pass, so
// a pass is exact one node further inside than the one before, and three
// passes (or two and the residual) are exact on the tile itself.  Every node
// value is the same expression, in the same order, as in the
// one-pass-per-dispatch kernels above (red from zero folded, khat_offdiag
// order), so the cycle's output agrees with theirs to rounding (the compiler
// may contract multiply-adds differently in the two); the partial sums of
// Re<vdot, z> are grouped by tile.
// Tile shapes (gl_tiles.l0_tiled 1, 2, 3): fewer threads and smaller tiles
// keep more tiles resident per CU at the price of a larger halo share.
template <int X, int Y, int NT>
struct L0Shape {
    static constexpr int TX = X, TY = Y, H = 3, LX = X + 2 * H, LY = Y + 2 * H, LN = LX * LY, threads = NT;
};
using L0Shape1 = L0Shape<32, 32, 1024>;  // about 1.4 LDS nodes per thread and pass
using L0Shape2 = L0Shape<32, 16, 512>;
using L0Shape3 = L0Shape<16, 16, 256>;

// the forward links of node (gx, gy) along x and y (0 past the grid's edge),
// loaded once per tile so that the passes read only LDS
template <class T>
__device__ __forceinline__ void l0_links(const GeomT<T> &g, const LinkTab<T> &U, int gx, int gy, C<T> &ux, C<T> &uy)
{
    const int c[3] = {gx, gy, 0};
    ux = gx < g.N[0] - 1 ? link_u<2, T>(U, 0, c, gx) : mk<T>(0, 0);
    uy = gy < g.N[1] - 1 ? link_u<2, T>(U, 1, c, gy) : mk<T>(0, 0);
}

// The edge coefficients alpha = |V| s_a / h_a^2 of node (gx, gy) along x and
// y (the expression the one-pass kernels evaluate per node and pass), stored
// per LDS node in the tile's load phase.
template <class T>
__device__ __forceinline__ void l0_alphas(const GeomT<T> &g, int gx, int gy, T &a0, T &a1)
{
    const int c[3] = {gx, gy, 0};
    T s[3];
    const T d = node_volume<2, T>(g, c, s);
    a0 = d * s[0] * g.inv_h2[0];
    a1 = d * s[1] * g.inv_h2[1];
}

// (sum_{j != i} H_ij x_j) of node (gx, gy) at LDS position q (2D); the link
// of the edge towards the lower neighbour is that neighbour's forward link
template <class T, int LX>
__device__ __forceinline__ C<T> l0_offdiag_lds(const GeomT<T> &g, int gx, int gy, int q, const C<T> *sx,
                                               const C<T> *ux, const C<T> *uy, const T *sa0, const T *sa1)
{
    const T a0 = sa0[q], a1 = sa1[q];
    C<T> acc = mk<T>(0, 0);
    if (gx > 0) acc = csub(acc, cscale(cmul(ux[q - 1], sx[q - 1]), a0));
    if (gx < g.N[0] - 1) acc = csub(acc, cscale(cmulc(ux[q], sx[q + 1]), a0));
    if (gy > 0) acc = csub(acc, cscale(cmul(uy[q - LX], sx[q - LX]), a1));
    if (gy < g.N[1] - 1) acc = csub(acc, cscale(cmulc(uy[q], sx[q + LX]), a1));
    return acc;
}

struct L0TileAt {
    int x0, y0;  // grid coordinates of LDS position 0
};

template <class S>
__device__ __forceinline__ L0TileAt l0_tile(int tile, int ntx)
{
    return L0TileAt{(tile % ntx) * S::TX - S::H, (tile / ntx) * S::TY - S::H};
}

// LDS position q: grid coordinates, in the grid, and its ring (distance from
// the LDS border: 0 on the outermost ring, S::H inside the tile)
template <class S>
__device__ __forceinline__ void l0_pos(const L0TileAt &T0, int q, const int *N, int &gx, int &gy, bool &in,
                                       int &ring)
{
    const int lx = q % S::LX, ly = q / S::LX;
    gx = T0.x0 + lx;
    gy = T0.y0 + ly;
    in = gx >= 0 && gx < N[0] && gy >= 0 && gy < N[1];
    ring = min(min(lx, S::LX - 1 - lx), min(ly, S::LY - 1 - ly));
}

// Calls f(q, gx, gy) for the LDS nodes of colour col ((gx + gy) & 1) that
// are at least rmin rings in from the LDS border and lie in the grid, the
// threads taking them in turn: a pass visits only the nodes it updates, with
// no lane idle on the other colour or outside its rings.
template <class S, class F>
__device__ __forceinline__ void l0_colour_nodes(const L0TileAt &T0, const int *N, int col, int rmin, F &&f)
{
    const int w = (S::LX - 2 * rmin) / 2, h = S::LY - 2 * rmin;
    for (int k = threadIdx.x; k < w * h; k += S::threads) {
        const int ly = rmin + k / w;
        const int lx = rmin + 2 * (k % w) + ((col ^ (T0.x0 + T0.y0 + ly + rmin)) & 1);
        const int gx = T0.x0 + lx, gy = T0.y0 + ly;
        if (gx < 0 || gx >= N[0] || gy < 0 || gy >= N[1]) continue;
        f(ly * S::LX + lx, gx, gy);
    }
}

// Calls f(q, gx, gy) for the tile's own nodes (S::H rings in) that lie in the
// grid.
template <class S, class F>
__device__ __forceinline__ void l0_tile_nodes(const L0TileAt &T0, const int *N, F &&f)
{
    for (int k = threadIdx.x; k < S::TX * S::TY; k += S::threads) {
        const int ly = S::H + k / S::TX, lx = S::H + k % S::TX;
        const int gx = T0.x0 + lx, gy = T0.y0 + ly;
        if (gx >= N[0] || gy >= N[1]) continue;
        f(ly * S::LX + lx, gx, gy);
    }
}

// Down: b = round(v), red from zero, black, red, black residual (L0PreBlack,
// L0Sweep(0), L0Residual); writes b and x of the tile's nodes and r of its
// black nodes in the split layout.
template <class T, class S>
struct L0PreTile {
    GeomT<T> g;
    const double2 *v;
    const T *hd;
    LinkTab<T> U;
    C<T> *b, *x, *r;
    int ntx;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        __shared__ C<T> sb[S::LN], sx[S::LN], ux[S::LN], uy[S::LN];
        __shared__ T sd[S::LN], sa0[S::LN], sa1[S::LN];
        const L0TileAt T0 = l0_tile<S>(xcd_tile(bx, nbx), ntx);
        for (int q = threadIdx.x; q < S::LN; q += S::threads) {
            int gx, gy, ring;
            bool in;
            l0_pos<S>(T0, q, g.N, gx, gy, in, ring);
            const int i = gx + g.N[0] * gy;
            const C<T> bi = in ? narrow<T>(v[i]) : mk<T>(0, 0);
            const T di = in ? hd[i] : (T)1;
            C<T> lx = mk<T>(0, 0), ly = lx;
            T a0 = (T)0, a1 = (T)0;
            if (in) {
                l0_links<T>(g, U, gx, gy, lx, ly);
                l0_alphas<T>(g, gx, gy, a0, a1);
            }
            sb[q] = bi;
            sd[q] = di;
            ux[q] = lx;
            uy[q] = ly;
            sa0[q] = a0;
            sa1[q] = a1;
            // red from zero: x = b / d
            sx[q] = in && ((gx + gy) & 1) == 0 ? cscale(bi, (T)1 / di) : mk<T>(0, 0);
        }
        __syncthreads();
        // black (exact one ring in), then red (two rings in)
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            l0_colour_nodes<S>(T0, g.N, pass == 0 ? 1 : 0, pass + 1, [&](int q, int gx, int gy) {
                sx[q] = cscale(csub(sb[q], l0_offdiag_lds<T, S::LX>(g, gx, gy, q, sx, ux, uy, sa0, sa1)), (T)1 / sd[q]);
            });
            __syncthreads();
        }
        // the tile's nodes: b, x, and the black residual
        const int np = g.npair;
        l0_tile_nodes<S>(T0, g.N, [&](int q, int gx, int gy) {
            const int col = (gx + gy) & 1;
            const int t = (gx >> 1) + g.hr * gy;
            C<T> ri = mk<T>(0, 0);
            if (col == 1) ri = csub(csub(sb[q], cscale(sx[q], sd[q])), l0_offdiag_lds<T, S::LX>(g, gx, gy, q, sx, ux, uy, sa0, sa1));
            if (!gate_go) return;
            b[col * np + t] = sb[q];
            x[col * np + t] = sx[q];
            if (col == 1) r[np + t] = ri;
        });
    }
};

// Up: black += (P x_c)_b, red, black, last red; z = x on the tile's nodes (ADD:
// z += x) and partial sums of Re<vdot, z> (L0ProlongBlack, L0Sweep(0),
// L0Sweep(1), L0Last).
template <class T, class TC, int ADD, class S>
struct L0PostTile {
    GeomT<T> g;
    const C<T> *b, *x;
    const T *hd;
    LinkTab<T> U;
    const int *prp, *pci;
    const C<TC> *pv, *xc;
    double2 *z;
    const double2 *vdot;
    RedSlot slot;
    int want_dot;
    int ntx;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE_LOAD();
        __shared__ C<T> sb[S::LN], sx[S::LN], ux[S::LN], uy[S::LN];
        __shared__ T sd[S::LN], sa0[S::LN], sa1[S::LN];
        __shared__ double sm[S::threads / 64];
        const L0TileAt T0 = l0_tile<S>(xcd_tile(bx, nbx), ntx);
        const int np = g.npair;
        for (int q = threadIdx.x; q < S::LN; q += S::threads) {
            int gx, gy, ring;
            bool in;
            l0_pos<S>(T0, q, g.N, gx, gy, in, ring);
            C<T> bi = mk<T>(0, 0), xi = mk<T>(0, 0), lx = xi, ly = xi;
            T di = (T)1, a0 = (T)0, a1 = (T)0;
            if (in) {
                const int col = (gx + gy) & 1;
                const int t = (gx >> 1) + g.hr * gy;
                bi = b[col * np + t];
                di = hd[gx + g.N[0] * gy];
                l0_links<T>(g, U, gx, gy, lx, ly);
                l0_alphas<T>(g, gx, gy, a0, a1);
                // red values are recomputed from the black ones before any use
                if (col == 1) xi = cadd(x[np + t], as_c<T>(prolong_row<TC>(prp, pci, pv, xc, t)));
            }
            sb[q] = bi;
            sx[q] = xi;
            sd[q] = di;
            ux[q] = lx;
            uy[q] = ly;
            sa0[q] = a0;
            sa1[q] = a1;
        }
        __syncthreads();
        // red (one ring in), black (two rings in)
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            l0_colour_nodes<S>(T0, g.N, pass, pass + 1, [&](int q, int gx, int gy) {
                sx[q] = cscale(csub(sb[q], l0_offdiag_lds<T, S::LX>(g, gx, gy, q, sx, ux, uy, sa0, sa1)), (T)1 / sd[q]);
            });
            __syncthreads();
        }
        // last red on the tile, into z only; z on every node of the tile
        double part = 0.0;
        l0_tile_nodes<S>(T0, g.N, [&](int q, int gx, int gy) {
            C<T> xi = sx[q];
            if (((gx + gy) & 1) == 0)
                xi = cscale(csub(sb[q], l0_offdiag_lds<T, S::LX>(g, gx, gy, q, sx, ux, uy, sa0, sa1)), (T)1 / sd[q]);
            const int i = gx + g.N[0] * gy;
            double2 zi = widen(xi);
            if (ADD) zi = cadd(z[i], zi);
            if (want_dot) part += redot(vdot[i], zi);
            if (gate_go) z[i] = zi;
        });
        if (want_dot && gate_go) block_reduce_store(part, slot, sm, bx);
    }
};

// --------------------------------------------------------------- CSR ---
// LPR lanes of one wave share a row; partial sums are combined by shuffles.
template <class T, int LPR>
__device__ __forceinline__ C<T> lanes_sum(C<T> s)
{
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
        s.x += __shfl_xor(s.x, o, 64);
        s.y += __shfl_xor(s.y, o, 64);
    }
    return s;
}

// Gauss-Seidel update of one colour stored as a padded block (ELL, width W).
// The gate flag is loaded alongside the data and checked only before the
// store, so its latency overlaps the row loads.
template <class T, int LPR>
struct EllSgs {
    const int *eci;
    const C<T> *ev;
    int W;
    const T *diag;
    int row0, count;
    const C<T> *b;
    C<T> *x;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        const int go = gate ? *gate : 1;
        const int t = bx * kBlock + threadIdx.x;
        const int r = t / LPR, lane = t % LPR;
        const bool act = r < count;
        const int i = row0 + (act ? r : 0);
        // the row's b and diagonal are loaded before the gathers (they do not
        // depend on them), so the store waits for one memory round trip less
        const bool own = act && lane == 0;
        const C<T> bi = own ? b[i] : mk<T>(0, 0);
        const T di = own ? diag[i] : (T)1;
        C<T> s = mk<T>(0, 0);
        if (act) {
            const size_t base = (size_t)r * W;
            for (int k = lane; k < W; k += LPR) {
                const int j = eci[base + k];
                if (j != i) s = cadd(s, cmul(ev[base + k], x[j]));
            }
        }
        s = lanes_sum<T, LPR>(s);
        if (own && go) x[i] = cscale(csub(bi, s), (T)1 / di);
    }
};

// The first two passes of a sweep from x = 0, and the zero start, in one
// dispatch (rows are colour-ordered): colour 0 gets x = b / a_ii, colour 1
// its Gauss-Seidel update from those values (evaluated on the fly from b and
// the diagonal), every other row x = 0.  Same arithmetic as the three
// separate steps.
template <class T, int LPR>
struct EllSgsStart {
    const int *eci;  // colour-1 block
    const C<T> *ev;
    int W;
    const T *diag;
    int c1, c2, n;   // colour 0 = rows [0, c1), colour 1 = [c1, c2)
    const C<T> *b;
    C<T> *x;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        const int go = gate ? *gate : 1;
        const int t = bx * kBlock + threadIdx.x;
        const int r = t / LPR, lane = t % LPR;
        const bool valid = r < n, one = valid && r >= c1 && r < c2;
        const bool own = valid && lane == 0 && r < c2;
        const C<T> br = own ? b[r] : mk<T>(0, 0);
        const T dr = own ? diag[r] : (T)1;
        C<T> s = mk<T>(0, 0);
        if (one) {
            const size_t base = (size_t)(r - c1) * W;
            for (int k = lane; k < W; k += LPR) {
                const int j = eci[base + k];
                if (j != r && j < c1) s = cadd(s, cmul(ev[base + k], cscale(b[j], (T)1 / diag[j])));
            }
        }
        s = lanes_sum<T, LPR>(s);
        if (valid && lane == 0 && go) {
            if (r < c1) x[r] = cscale(br, (T)1 / dr);
            else if (r < c2) x[r] = cscale(csub(br, s), (T)1 / dr);
            else x[r] = mk<T>(0, 0);
        }
    }
};

// r = b - A x
template <class T, int LPR>
struct CsrResidual {
    int n;
    const int *rp, *ci;
    const C<T> *v, *b, *x;
    C<T> *r;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE_LOAD();
        const int t = bx * kBlock + threadIdx.x;
        const int i = t / LPR, lane = t % LPR;
        const bool act = i < n;
        const C<T> bi = act && lane == 0 ? b[i] : mk<T>(0, 0);
        C<T> s = mk<T>(0, 0);
        if (act)
            for (int p = rp[i] + lane; p < rp[i + 1]; p += LPR) s = cadd(s, cmul(v[p], as_c<T>(x[ci[p]])));
        s = lanes_sum<T, LPR>(s);
        if (act && lane == 0 && gate_go) r[i] = csub(bi, s);
    }
};

// y = A x (ADD = 0) or y += A x (ADD = 1); x may be held in the other precision
template <class T, int LPR, int ADD, class TX = T>
struct CsrSpmv {
    int n;
    const int *rp, *ci;
    const C<T> *v;
    const C<TX> *x;
    C<T> *y;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE_LOAD();
        const int t = bx * kBlock + threadIdx.x;
        const int i = t / LPR, lane = t % LPR;
        const bool act = i < n;
        const C<T> yi = ADD && act && lane == 0 ? y[i] : mk<T>(0, 0);
        C<T> s = mk<T>(0, 0);
        if (act)
            for (int p = rp[i] + lane; p < rp[i + 1]; p += LPR) s = cadd(s, cmul(v[p], as_c<T>(x[ci[p]])));
        s = lanes_sum<T, LPR>(s);
        if (act && lane == 0 && gate_go) y[i] = ADD ? cadd(yi, s) : s;
    }
};

template <class T>
struct FillZero {
    int n;
    C<T> *x;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) x[i] = mk<T>(0, 0);
    }
};

template <class T>
struct Narrow {
    int n;
    const double2 *v;
    C<T> *b;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) b[i] = narrow<T>(v[i]);
    }
};

// z = x (ADD = 0) or z += x (ADD = 1); partial sums of Re<vdot, z>
template <class T, int ADD>
struct Output {
    int n;
    const C<T> *x;
    const double2 *vdot;
    double2 *z;
    RedSlot slot;
    int want_dot;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        __shared__ double sm[kBlock / 64];
        const int i = bx * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < n) {
            double2 zi = widen(x[i]);
            if (ADD) zi = cadd(z[i], zi);
            z[i] = zi;
            if (want_dot) part = redot(vdot[i], zi);
        }
        if (want_dot) block_reduce_store(part, slot, sm, bx);
    }
};

// b[r] = round(v[perm[r]]): level 0 of a simplicial mesh, whose V-cycle
// vectors are in colour order (row r is node perm[r])
template <class T>
struct NarrowPerm {
    int n;
    const double2 *v;
    const int *perm;
    C<T> *b;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        const int r = bx * kBlock + threadIdx.x;
        if (r < n) b[r] = narrow<T>(v[perm[r]]);
    }
};

// z[perm[r]] = x[r] (ADD: +=), partial sums of Re<vdot, z> in row order
template <class T, int ADD>
struct OutputPerm {
    int n;
    const C<T> *x;
    const int *perm;
    const double2 *vdot;
    double2 *z;
    RedSlot slot;
    int want_dot;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        __shared__ double sm[kBlock / 64];
        const int r = bx * kBlock + threadIdx.x;
        double part = 0.0;
        if (r < n) {
            const int i = perm[r];
            double2 zi = widen(x[r]);
            if (ADD) zi = cadd(z[i], zi);
            z[i] = zi;
            if (want_dot) part = redot(vdot[i], zi);
        }
        if (want_dot) block_reduce_store(part, slot, sm, bx);
    }
};

// x = M b for a dense row-major operator (the coarsest inverse or an explicit
// sub-cycle), a wave per row.  Each lane issues kDenseUnroll loads before it
// uses any (a row of a few thousand entries is otherwise one memory round
// trip per 64 entries); the sum still runs over j = lane, lane + 64, ... in
// that order.
constexpr int kDenseUnroll = 8;

template <class T>
struct DenseApply {
    int n;
    const C<T> *M, *b;
    C<T> *x;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE_LOAD();
        const int t = bx * kBlock + threadIdx.x;
        const int i = t / 64, lane = t % 64;
        const bool act = i < n;
        C<T> s = mk<T>(0, 0);
        if (act) {
            const C<T> *row = M + (size_t)i * n;
            for (int j0 = 0; j0 < n; j0 += 64 * kDenseUnroll) {
                C<T> m[kDenseUnroll], v[kDenseUnroll];
#pragma unroll
                for (int u = 0; u < kDenseUnroll; ++u) {
                    const int j = j0 + u * 64 + lane;
                    m[u] = j < n ? row[j] : mk<T>(0, 0);
                    v[u] = j < n ? b[j] : mk<T>(0, 0);
                }
#pragma unroll
                for (int u = 0; u < kDenseUnroll; ++u)
                    if (j0 + u * 64 + lane < n) s = cadd(s, cmul(m[u], v[u]));
            }
        }
        s = lanes_sum<T, 64>(s);
        if (act && lane == 0 && gate_go) x[i] = s;
    }
};

// ------------------------------------------------------------ bottom ---
// Every level from D.first down to the coarsest, in one work-group of
// kBottomThreads threads: the same V-cycle steps as the multi-kernel levels,
// separated by work-group barriers, and the dense solve.  One work-group
// avoids a dispatch per colour pass, but a step costs about 3 us even over a
// handful of rows (a dependent global load is about 1 us away, measured on
// MI355X) and one compute unit streams about 20-25 GB/s, so this pays only for
// levels of a few hundred rows; the tile autotuner chooses the bound
// (bottom_rows).  Eight lanes share a row, so a colour pass of such a level
// is one round of loads.
constexpr int kBottomThreads = 1024;
constexpr int kBottomLpr = 8;

// one colour of a level, from its ELL block; x in LDS or global memory
template <class T>
__device__ __forceinline__ void bottom_rows_sgs(const BottomLevel<T> &L, int colour, const C<T> *b, C<T> *x)
{
    const int cnt = L.coff[colour + 1] - L.coff[colour];
    const int row0 = L.coff[colour];
    const int W = L.ewidth[colour];
    const int *eci = L.eci + L.eoff[colour];
    const C<T> *ev = L.ev + L.eoff[colour];
    const int per = kBottomThreads / kBottomLpr;
    const int lane = threadIdx.x % kBottomLpr;
    for (int base = 0; base < cnt; base += per) {
        const int r = base + threadIdx.x / kBottomLpr;
        const bool act = r < cnt;
        const int i = row0 + (act ? r : 0);
        C<T> s = mk<T>(0, 0);
        if (act)
            for (int k = lane; k < W; k += kBottomLpr) {
                const int j = eci[(size_t)r * W + k];
                if (j != i) s = cadd(s, cmul(ev[(size_t)r * W + k], x[j]));
            }
        s = lanes_sum<T, kBottomLpr>(s);
        if (act && lane == 0) x[i] = cscale(csub(b[i], s), (T)1 / L.diag[i]);
    }
}

// MODE 0: y = M x, 1: y += M x, 2: y = b - M x
template <class T, int MODE>
__device__ __forceinline__ void bottom_rows_spmv(int nrows, const int *rp, const int *ci, const C<T> *v,
                                                 const C<T> *x, const C<T> *b, C<T> *y)
{
    const int per = kBottomThreads / kBottomLpr;
    const int lane = threadIdx.x % kBottomLpr;
    for (int base = 0; base < nrows; base += per) {
        const int i = base + threadIdx.x / kBottomLpr;
        const bool act = i < nrows;
        C<T> s = mk<T>(0, 0);
        if (act)
            for (int p = rp[i] + lane; p < rp[i + 1]; p += kBottomLpr) s = cadd(s, cmul(v[p], x[ci[p]]));
        s = lanes_sum<T, kBottomLpr>(s);
        if (act && lane == 0) {
            if (MODE == 0) y[i] = s;
            else if (MODE == 1) y[i] = cadd(y[i], s);
            else y[i] = csub(b[i], s);
        }
    }
}

// y = M b for a dense row-major n x n matrix
template <class T>
__device__ __forceinline__ void bottom_dense(int n, const C<T> *M, const C<T> *b, C<T> *y)
{
    const int per = kBottomThreads / kBottomLpr;
    const int lane = threadIdx.x % kBottomLpr;
    for (int base = 0; base < n; base += per) {
        const int i = base + threadIdx.x / kBottomLpr;
        const bool act = i < n;
        C<T> s = mk<T>(0, 0);
        if (act)
            for (int j = lane; j < n; j += kBottomLpr) s = cadd(s, cmul(M[(size_t)i * n + j], b[j]));
        s = lanes_sum<T, kBottomLpr>(s);
        if (act && lane == 0) y[i] = s;
    }
}

template <class T>
__device__ __forceinline__ void bottom_sgs(const BottomLevel<T> &L, const C<T> *b, C<T> *x)
{
    for (int t = 0; t < 2 * L.ncolors - 1; ++t) {
        bottom_rows_sgs<T>(L, t < L.ncolors ? t : 2 * L.ncolors - 2 - t, b, x);
        __syncthreads();
    }
}

// The V-cycle over levels D.first .. D.last in one work-group: the same
// steps as the multi-kernel levels, then the dense operator of level D.last.
// vec(l, k) is level l's right-hand side (k = 0), iterate (1) or residual (2).
template <class T, class V>
__device__ __forceinline__ void bottom_cycle(const BottomDesc<T> &D, V vec)
{
    for (int l = D.first; l < D.last; ++l) {
        const BottomLevel<T> &L = D.L[l];
        C<T> *b = vec(l, 0), *x = vec(l, 1), *r = vec(l, 2);
        for (int i = threadIdx.x; i < L.n; i += kBottomThreads) x[i] = mk<T>(0, 0);
        __syncthreads();
        bottom_sgs<T>(L, b, x);
        bottom_rows_spmv<T, 2>(L.n, L.rp, L.ci, L.v, x, b, r);
        __syncthreads();
        bottom_rows_spmv<T, 0>(L.nc, L.rrp, L.rci, L.rv, r, nullptr, vec(l + 1, 0));
        __syncthreads();
    }
    bottom_dense<T>(D.L[D.last].n, D.cinv, vec(D.last, 0), vec(D.last, 1));
    __syncthreads();
    for (int l = D.last - 1; l >= D.first; --l) {
        const BottomLevel<T> &L = D.L[l];
        C<T> *x = vec(l, 1);
        bottom_rows_spmv<T, 1>(L.n, L.prp, L.pci, L.pv, vec(l + 1, 1), nullptr, x);
        __syncthreads();
        bottom_sgs<T>(L, vec(l, 0), x);
    }
}

// The level D.lds_level (the largest one handled here, when it fits) keeps
// its iterate in LDS for the whole cycle and writes it out at the end.
template <class T>
struct Bottom {
    const BottomDesc<T> *Dp;
    const int *gate;
    __device__ void operator()(int, int) const
    {
        GATE();
        extern __shared__ double2 glk_bottom_lds[];
        const BottomDesc<T> &D = *Dp;
        C<T> *xs = reinterpret_cast<C<T> *>(glk_bottom_lds);
        bottom_cycle<T>(D, [&](int l, int k) -> C<T> * {
            const BottomLevel<T> &L = D.L[l];
            return k == 0 ? L.b : k == 1 ? (l == D.lds_level ? xs : L.x) : L.r;
        });
        if (D.lds_level >= 0) {
            const BottomLevel<T> &L = D.L[D.lds_level];
            for (int i = threadIdx.x; i < L.n; i += kBottomThreads) L.x[i] = xs[i];
            __syncthreads();
        }
    }
};

// Block forms of the bottom kernel's steps, for forming an explicit sub-cycle
// kTailBlock columns at a time: vectors are [n][kTailBlock] blocks (the
// columns of a row contiguous), thread t works on row t / kTailBlock and
// column t % kTailBlock, and the kTailBlock threads of a row read the same
// matrix entries, so a level's matrix is read once per block of columns
// instead of once per column.  A thread takes its row's entries in groups of
// kTailUnroll, every gather of a group issued before any is used, and sums
// them in order.  A null right-hand side stands for columns bid .. bid +
// kTailBlock - 1 of the identity.
constexpr int kTailBlock = 16;
constexpr int kTailRows = kBottomThreads / kTailBlock;  // rows per round
constexpr int kTailUnroll = 8;

template <class T>
__device__ __forceinline__ C<T> blk_rhs(const C<T> *b, int bid, int i, int c)
{
    return b ? b[(size_t)i * kTailBlock + c] : mk<T>(i == bid + c ? 1 : 0, 0);
}

// sum over k in [k0, k1) of v[k] x[idx[k]][c], skipping idx[k] == skip
template <class T>
__device__ __forceinline__ C<T> blk_row_sum(const int *idx, const C<T> *v, int k0, int k1, const C<T> *x, int c,
                                            int skip)
{
    C<T> acc = mk<T>(0, 0);
    int k = k0;
    for (; k + kTailUnroll <= k1; k += kTailUnroll) {
        int j[kTailUnroll];
        C<T> a[kTailUnroll], xv[kTailUnroll];
#pragma unroll
        for (int u = 0; u < kTailUnroll; ++u) {
            j[u] = idx[k + u];
            a[u] = v[k + u];
        }
#pragma unroll
        for (int u = 0; u < kTailUnroll; ++u) xv[u] = x[(size_t)j[u] * kTailBlock + c];
#pragma unroll
        for (int u = 0; u < kTailUnroll; ++u)
            if (j[u] != skip) acc = cadd(acc, cmul(a[u], xv[u]));
    }
    for (; k < k1; ++k) {
        const int jj = idx[k];
        if (jj != skip) acc = cadd(acc, cmul(v[k], x[(size_t)jj * kTailBlock + c]));
    }
    return acc;
}

// one colour of a level, from its ELL block
template <class T>
__device__ __forceinline__ void blk_sgs_colour(const BottomLevel<T> &L, int colour, const C<T> *b, int bid, C<T> *x)
{
    const int cnt = L.coff[colour + 1] - L.coff[colour];
    const int row0 = L.coff[colour];
    const int W = L.ewidth[colour];
    const int *eci = L.eci + L.eoff[colour];
    const C<T> *ev = L.ev + L.eoff[colour];
    const int c = threadIdx.x % kTailBlock;
    for (int r = threadIdx.x / kTailBlock; r < cnt; r += kTailRows) {
        const int i = row0 + r;
        const C<T> bi = blk_rhs<T>(b, bid, i, c);
        const size_t e0 = (size_t)r * W;
        const C<T> acc = blk_row_sum<T>(eci + e0, ev + e0, 0, W, x, c, i);
        x[(size_t)i * kTailBlock + c] = cscale(csub(bi, acc), (T)1 / L.diag[i]);
    }
}

template <class T>
__device__ __forceinline__ void blk_sgs(const BottomLevel<T> &L, const C<T> *b, int bid, C<T> *x)
{
    for (int t = 0; t < 2 * L.ncolors - 1; ++t) {
        blk_sgs_colour<T>(L, t < L.ncolors ? t : 2 * L.ncolors - 2 - t, b, bid, x);
        __syncthreads();
    }
}

// MODE 0: y = M x, 1: y += M x, 2: y = b - M x
template <class T, int MODE>
__device__ __forceinline__ void blk_spmv(int nrows, const int *rp, const int *ci, const C<T> *v, const C<T> *x,
                                         const C<T> *b, int bid, C<T> *y)
{
    const int c = threadIdx.x % kTailBlock;
    for (int i = threadIdx.x / kTailBlock; i < nrows; i += kTailRows) {
        const C<T> acc = blk_row_sum<T>(ci, v, rp[i], rp[i + 1], x, c, -1);
        C<T> &yi = y[(size_t)i * kTailBlock + c];
        if (MODE == 0) yi = acc;
        else if (MODE == 1) yi = cadd(yi, acc);
        else yi = csub(blk_rhs<T>(b, bid, i, c), acc);
    }
}

// y = M b for a dense row-major n x n matrix
template <class T>
__device__ __forceinline__ void blk_dense(int n, const C<T> *M, const C<T> *b, C<T> *y)
{
    const int c = threadIdx.x % kTailBlock;
    for (int i = threadIdx.x / kTailBlock; i < n; i += kTailRows) {
        const C<T> *row = M + (size_t)i * n;
        C<T> acc = mk<T>(0, 0);
        int j = 0;
        for (; j + kTailUnroll <= n; j += kTailUnroll) {
            C<T> a[kTailUnroll], xv[kTailUnroll];
#pragma unroll
            for (int u = 0; u < kTailUnroll; ++u) {
                a[u] = row[j + u];
                xv[u] = b[(size_t)(j + u) * kTailBlock + c];
            }
#pragma unroll
            for (int u = 0; u < kTailUnroll; ++u) acc = cadd(acc, cmul(a[u], xv[u]));
        }
        for (; j < n; ++j) acc = cadd(acc, cmul(row[j], b[(size_t)j * kTailBlock + c]));
        y[(size_t)i * kTailBlock + c] = acc;
    }
}

// The V-cycle over levels D.first .. D.last on kTailBlock identity columns
// (the steps of bottom_cycle); vec(l, k): level l's b (k = 0, unused on
// D.first), x (1) or r (2) block.
template <class T, class V>
__device__ __forceinline__ void blk_cycle(const BottomDesc<T> &D, V vec, int bid)
{
    for (int l = D.first; l < D.last; ++l) {
        const BottomLevel<T> &L = D.L[l];
        const C<T> *b = l == D.first ? nullptr : vec(l, 0);
        C<T> *x = vec(l, 1), *r = vec(l, 2);
        for (int t = threadIdx.x; t < L.n * kTailBlock; t += kBottomThreads) x[t] = mk<T>(0, 0);
        __syncthreads();
        blk_sgs<T>(L, b, bid, x);
        blk_spmv<T, 2>(L.n, L.rp, L.ci, L.v, x, b, bid, r);
        __syncthreads();
        blk_spmv<T, 0>(L.nc, L.rrp, L.rci, L.rv, r, nullptr, 0, vec(l + 1, 0));
        __syncthreads();
    }
    blk_dense<T>(D.L[D.last].n, D.cinv, vec(D.last, 0), vec(D.last, 1));
    __syncthreads();
    for (int l = D.last - 1; l >= D.first; --l) {
        const BottomLevel<T> &L = D.L[l];
        C<T> *x = vec(l, 1);
        blk_spmv<T, 1>(L.n, L.prp, L.pci, L.pv, vec(l + 1, 1), nullptr, 0, x);
        __syncthreads();
        blk_sgs<T>(L, l == D.first ? nullptr : vec(l, 0), bid, x);
    }
}

// Columns of the explicit sub-cycle of level D.first: work-group g forms
// columns col0 + g kTailBlock .. + kTailBlock - 1 (those below n) with
// blocks of its own (ws + g * ws_blk: b, x, r of each level in turn) and
// stores them into the row-major n x n matrix out.
template <class T>
struct TailColumns {
    const BottomDesc<T> *Dp;
    C<T> *ws;
    size_t ws_blk;
    int col0, nblk;
    C<T> *out;
    __device__ void operator()(int bx, int) const
    {
        if (bx >= nblk) return;
        const BottomDesc<T> &D = *Dp;
        const int n = D.L[D.first].n, bid = col0 + bx * kTailBlock;
        C<T> *base = ws + (size_t)bx * ws_blk;
        auto vec = [&](int l, int k) -> C<T> * {
            size_t off = 0;
            for (int q = D.first; q < l; ++q) off += 3 * (size_t)D.L[q].n;
            return base + (off + (size_t)k * D.L[l].n) * kTailBlock;
        };
        blk_cycle<T>(D, vec, bid);
        const C<T> *x = vec(D.first, 1);
        for (int t = threadIdx.x; t < n * kTailBlock; t += kBottomThreads) {
            const int i = t / kTailBlock, col = bid + t % kTailBlock;
            if (col < n) out[(size_t)i * n + col] = x[t];
        }
    }
};

// ---------------------------------------------------------------- host -
template <class T> static C<T> *vec_b(Level &L);
template <class T> static C<T> *vec_x(Level &L);
template <class T> static C<T> *vec_r(Level &L);
template <> double2 *vec_b<double>(Level &L) { return L.b64.get(); }
template <> double2 *vec_x<double>(Level &L) { return L.x64.get(); }
template <> double2 *vec_r<double>(Level &L) { return L.r64.get(); }
template <> float2 *vec_b<float>(Level &L) { return L.b32.get(); }
template <> float2 *vec_x<float>(Level &L) { return L.x32.get(); }
template <> float2 *vec_r<float>(Level &L) { return L.r32.get(); }
template <class T> static const C<T> *vals(const Csr &M);
template <> const double2 *vals<double>(const Csr &M) { return M.v64.get(); }
template <> const float2 *vals<float>(const Csr &M) { return M.v32.get(); }
// level-0 diagonal (natural order) and the colour-ordered diagonal of l >= 1
template <class T> static const T *diag(const Level &L);
template <> const double *diag<double>(const Level &L) { return L.diag64.get(); }
template <> const float *diag<float>(const Level &L) { return L.diag32.get(); }
// level-0 diagonal in the colour-split layout of the V-cycle's level-0 vectors
template <class T> static const T *hsplit(const Level &L);
template <> const double *hsplit<double>(const Level &L) { return L.hs64.get(); }
template <> const float *hsplit<float>(const Level &L) { return L.hs32.get(); }
template <class T> static const T *dgn(const Level &L);
template <> const double *dgn<double>(const Level &L) { return L.dg64.get(); }
template <> const float *dgn<float>(const Level &L) { return L.dg32.get(); }

// dense operator of level pre->tail: the coarsest inverse, or the explicit sub-cycle
template <class T> static const C<T> *cinv(const gl_precond *p);
template <> const double2 *cinv<double>(const gl_precond *p)
{
    return p->tail < p->nlev - 1 ? p->tinv64.get() : p->cinv64.get();
}
template <> const float2 *cinv<float>(const gl_precond *p)
{
    return p->tail < p->nlev - 1 ? p->tinv32.get() : p->cinv32.get();
}
template <class T> static int bottom_lds(const gl_precond *p);
template <> int bottom_lds<double>(const gl_precond *p) { return p->lds64; }
template <> int bottom_lds<float>(const gl_precond *p) { return p->lds32; }
template <class T> static const BottomDesc<T> *bdesc(const gl_precond *p);
template <> const BottomDesc<double> *bdesc<double>(const gl_precond *p)
{
    return reinterpret_cast<const BottomDesc<double> *>(p->bdesc64.get());
}
template <> const BottomDesc<float> *bdesc<float>(const gl_precond *p)
{
    return reinterpret_cast<const BottomDesc<float> *>(p->bdesc32.get());
}

// lanes per row: about one lane per 2.5 entries, scaled by 2^shift, in 1 .. 32
static int shifted(int lpr, int shift)
{
    while (shift > 0 && lpr < 32) { lpr *= 2; --shift; }
    while (shift < 0 && lpr > 1) { lpr /= 2; ++shift; }
    return lpr;
}

static int lanes_for(const Csr &M, int shift)
{
    const double avg = M.n ? (double)M.nnz / M.n : 1.0;
    const int lpr = avg <= 2.5 ? 1 : avg <= 5.0 ? 2 : avg <= 10.0 ? 4 : avg <= 20.0 ? 8 : avg <= 40.0 ? 16 : 32;
    return shifted(lpr, shift);
}

// dispatch a CSR kernel over LPR in {1, 2, 4, 8, 16, 32}
#define GLK_LPR_SWITCH(lpr, ...)                              \
    switch (lpr) {                                            \
    case 1: { constexpr int LPR = 1; __VA_ARGS__; } break;    \
    case 2: { constexpr int LPR = 2; __VA_ARGS__; } break;    \
    case 4: { constexpr int LPR = 4; __VA_ARGS__; } break;    \
    case 8: { constexpr int LPR = 8; __VA_ARGS__; } break;    \
    case 16: { constexpr int LPR = 16; __VA_ARGS__; } break;  \
    default: { constexpr int LPR = 32; __VA_ARGS__; } break;  \
    }

template <class T, class TX = T>
static void csr_spmv(const Csr &M, const C<TX> *x, C<T> *y, bool add, int shift, const int *gate,
                     const Launch &L)
{
    const int lpr = lanes_for(M, shift);
    const int nb = blocks_for((int64_t)M.n * lpr);
    GLK_LPR_SWITCH(lpr, {
        if (add) L.run(nb, CsrSpmv<T, LPR, 1, TX>{M.n, M.rp.get(), M.ci.get(), vals<T>(M), x, y, gate});
        else L.run(nb, CsrSpmv<T, LPR, 0, TX>{M.n, M.rp.get(), M.ci.get(), vals<T>(M), x, y, gate});
    });
}

template <class T> static const C<T> *evals(const Level &L);
template <> const double2 *evals<double>(const Level &L) { return L.ev64.get(); }
template <> const float2 *evals<float>(const Level &L) { return L.ev32.get(); }

static int ell_lanes(int W, int shift) { return shifted(W <= 3 ? 2 : W <= 6 ? 4 : W <= 16 ? 8 : 16, shift); }

// One symmetric sweep on a level >= 1: colours 0 .. C-1, then C-2 .. 0.
// from_zero: the sweep starts from x = 0 (its first two passes and the zero
// start are one dispatch).
template <class T>
static void csr_sgs(Level &Lv, int shift, bool from_zero, const int *gate, const Launch &L)
{
    const int nco = Lv.ncolors;
    const int t0 = from_zero ? std::min(2, 2 * nco - 1) : 0;
    // algorithmic bytes of a pass: the colour's padded rows (index + value),
    // one x value per stored entry, b and the diagonal of each row, x written
    double bytes = 0.0;
    int passes = 0;
    for (int t = 0; t < 2 * nco - 1; ++t) {
        const int c = t < nco ? t : 2 * nco - 2 - t;
        const int cnt = Lv.coff[c + 1] - Lv.coff[c];
        if (cnt == 0) continue;
        bytes += (double)cnt * Lv.ewidth[c] * (4.0 + 2.0 * sizeof(C<T>)) + cnt * (2.0 * sizeof(C<T>) + sizeof(T));
        ++passes;
    }
    if (from_zero) passes -= t0 - 1;
    // the passes of one sweep share one event bracket
    prof_launch(PROF_COARSE_SWEEP, bytes, L, [&] {
        if (from_zero) {
            const int c1 = Lv.coff[1], c2 = nco > 1 ? Lv.coff[2] : Lv.n;
            const int W = nco > 1 ? Lv.ewidth[1] : 1;
            const int lpr = ell_lanes(W, shift);
            const int nb = blocks_for((int64_t)Lv.n * lpr);
            GLK_LPR_SWITCH(lpr, {
                L.run(nb, EllSgsStart<T, LPR>{Lv.eci.get() + (nco > 1 ? Lv.eoff[1] : 0), evals<T>(Lv) +
                                              (nco > 1 ? Lv.eoff[1] : 0), W, dgn<T>(Lv), c1, c2, Lv.n,
                                              vec_b<T>(Lv), vec_x<T>(Lv), gate});
            });
        }
        for (int t = t0; t < 2 * nco - 1; ++t) {
            const int c = t < nco ? t : 2 * nco - 2 - t;
            const int cnt = Lv.coff[c + 1] - Lv.coff[c];
            if (cnt == 0) continue;
            const int W = Lv.ewidth[c];
            const int lpr = ell_lanes(W, shift);
            const int nb = blocks_for((int64_t)cnt * lpr);
            GLK_LPR_SWITCH(lpr, {
                L.run(nb, EllSgs<T, LPR>{Lv.eci.get() + Lv.eoff[c], evals<T>(Lv) + Lv.eoff[c], W, dgn<T>(Lv),
                                         Lv.coff[c], cnt, vec_b<T>(Lv), vec_x<T>(Lv), gate});
            });
        }
    }, passes);
}

template <class T>
static void csr_residual(Level &Lv, int shift, const int *gate, const Launch &L)
{
    const int lpr = lanes_for(Lv.Aa, shift);
    const int nb = blocks_for((int64_t)Lv.n * lpr);
    GLK_LPR_SWITCH(lpr, {
        L.run(nb, CsrResidual<T, LPR>{Lv.n, Lv.Aa.rp.get(), Lv.Aa.ci.get(), vals<T>(Lv.Aa), vec_b<T>(Lv),
                                      vec_x<T>(Lv), vec_r<T>(Lv), gate});
    });
}

// calls f with the tile shape of gl_tiles.l0_tiled (1, 2 or 3)
template <class F>
static void l0_tiled_shape(int which, F &&f)
{
    if (which == 1) f(L0Shape1{});
    else if (which == 2) f(L0Shape2{});
    else f(L0Shape3{});
}

// T: level 0 (stencil sweeps, where the bytes are); TC: levels >= 1 and the
// coarsest solve (latency-bound: their precision costs no bandwidth)
// The V-cycle below level 0, from b of level 1 to x of level 1: the
// multi-kernel levels down (sweep from zero, residual, restriction), the
// small levels and the dense operator of level `tail` (the coarsest inverse
// or the explicit sub-cycle) in one work-group, or that dense product alone
// over many work-groups, then the multi-kernel levels up (prolongation,
// sweep).
template <class TC>
static void coarse_levels(gl_precond *pre, const int *gate, const Launch &L)
{
    const int nb_first = pre->bottom;
    const int sh = pre->lane_shift;
    for (int l = 1; l < nb_first; ++l) {
        Level &Lv = pre->L[l];
        csr_sgs<TC>(Lv, sh, true, gate, L);
        csr_residual<TC>(Lv, sh, gate, L);
        csr_spmv<TC>(Lv.Ra, vec_r<TC>(Lv), vec_b<TC>(pre->L[l + 1]), false, sh, gate, L);
    }
    if (pre->bottom < pre->tail) {
        L.run<Bottom<TC>, kBottomThreads>(1, Bottom<TC>{bdesc<TC>(pre), gate}, bottom_lds<TC>(pre));
    } else {
        Level &Lc = pre->L[pre->tail];
        L.run(blocks_for((int64_t)Lc.n * 64),
              DenseApply<TC>{Lc.n, cinv<TC>(pre), vec_b<TC>(Lc), vec_x<TC>(Lc), gate});
    }
    for (int l = nb_first - 1; l >= 1; --l) {
        Level &Lv = pre->L[l];
        csr_spmv<TC>(Lv.Pa, vec_x<TC>(pre->L[l + 1]), vec_x<TC>(Lv), true, sh, gate, L);
        csr_sgs<TC>(Lv, sh, false, gate, L);
    }
}

template <int DIM, class T, class TC>
static void vcycle_once_grid(const gl_precond *cpre, const double2 *v, const double2 *vdot, double2 *z,
                        const int *gate, KrylovScalars *ks, int mode, int add, const Launch &L,
                        double *store = nullptr)
{
    gl_precond *pre = const_cast<gl_precond *>(cpre);
    const gl_mesh *m = pre->mesh;
    const GeomT<T> g = geom_t<T>(m->g);
    const LinkTab<T> U = link_tab<T>(m);
    const RedSlot slot = red_slot(m, 1);
    Level &L0 = pre->L[0];
    const int n0 = L0.n, nb0 = blocks_for(n0);
    const int nl = pre->nlev;
    const bool f32 = std::is_same<T, float>::value;
    C<T> *b0 = vec_b<T>(L0);
    C<T> *x0 = vec_x<T>(L0);
    // Re<vdot, z> is reduced for the Krylov scalars (ks) or stored (store)
    const int want = ks != nullptr || store != nullptr;
    const int fmode = store ? (int)FIN_STORE : mode;
    if (nl == 1) {
        C<TC> *xc0 = vec_x<TC>(L0);
        L.run(nb0, Narrow<TC>{n0, v, vec_b<TC>(L0), gate});
        L.run(blocks_for((int64_t)n0 * 64), DenseApply<TC>{n0, cinv<TC>(pre), vec_b<TC>(L0), xc0, gate});
        if (add) L.run(nb0, Output<TC, 1>{n0, xc0, vdot, z, slot, want, gate});
        else L.run(nb0, Output<TC, 0>{n0, xc0, vdot, z, slot, want, gate});
        if (want) launch_finalize(slot.partials, nb0, fmode, ks, store, gate, L);
        return;
    }
    const T *hd = diag<T>(L0), *hs = hsplit<T>(L0);
    Level &L1 = pre->L[1];
    // algorithmic bytes of the level-0 kernels (each array touched once)
    // (the link factor tables are a few KB and stay in cache)
    const double sz = sizeof(C<T>), szr = sizeof(T), nn = n0, mc = 0.5 * nn;
    const double b_pre = nn * 16 + nn * sz + nn * szr + mc * sz;
    const double b_sweep = mc * (sz + szr + sz) + (nn - mc) * sz;
    const double b_resid = b_sweep + (nn - mc) * sz;
    const double szc = sizeof(C<TC>);
    const double b_prol = (g.npair + 1 + L0.Pb.nnz) * 4.0 + L0.Pb.nnz * szc + L0.nc * szc + 2.0 * mc * sz;
    const double b_last = b_sweep - mc * sz + (nn - mc) * sz + nn * 16 * (want ? 2 : 1) + (add ? nn * 16 : 0);
    const double b_restr = (L0.nc + 1 + L0.Rb.nnz) * 4.0 + L0.Rb.nnz * szc + (nn - mc) * sz + L0.nc * szc;
    // level 0 (one thread per red-black pair), down: red (from zero, folded) +
    // black, red, black residual, restriction; in 2D by default the three
    // passes in one LDS-tiled kernel (L0PreTile)
    const int nbp = blocks_for(g.npair);
    const int tiled = DIM == 2 ? pre->l0_tiled : 0;
    if (tiled) {
        // each array once (the halo's re-reads come from cache)
        const double b_tile = nn * 16 + nn * szr + 2 * nn * sz + mc * sz;
        prof_launch(PROF_L0_SWEEP, b_tile, L, [&] {
            l0_tiled_shape(tiled, [&](auto sh) {
                using S = decltype(sh);
                const int ntx = (g.N[0] + S::TX - 1) / S::TX, nbt = ntx * ((g.N[1] + S::TY - 1) / S::TY);
                L.run<L0PreTile<T, S>, S::threads>(nbt,
                                                   L0PreTile<T, S>{g, v, hd, U, vec_b<T>(L0), x0, vec_r<T>(L0), ntx, gate});
            });
        });
    } else {
        prof_launch(PROF_L0_SWEEP, b_pre, L, [&] {
            L.run(nbp, L0PreBlack<DIM, T>{g, v, vec_b<T>(L0), x0, U, hd, gate});
        });
        prof_launch(PROF_L0_SWEEP, b_sweep, L, [&] {
            L.run(nbp, L0Sweep<DIM, T>{g, 0, b0, x0, U, hs, gate});
        });
        prof_launch(PROF_L0_RESIDUAL, b_resid, L, [&] {
            L.run(nbp, L0Residual<DIM, T>{g, b0, x0, U, hs, vec_r<T>(L0), gate});
        });
    }
    prof_launch(PROF_L0_TRANSFER, b_restr, L, [&] {
        csr_spmv<TC, T>(L0.Rb, vec_r<T>(L0), vec_b<TC>(L1), false, 0, gate, L);
    });
    // levels >= 1: b of level 1 in, x of level 1 out
    coarse_levels<TC>(pre, gate, L);
    // level 0, up: red with the coarse correction, black, red + output
    // black coarse correction, then the red pass (fusing the two reads every
    // black correction four times and was measured slower); in 2D by default
    // all four in one LDS-tiled kernel (L0PostTile), each tile correcting the
    // black nodes of its halo once
    if (tiled) {
        const double b_tile = (g.npair + 1 + L0.Pb.nnz) * 4.0 + L0.Pb.nnz * szc + L0.nc * szc + mc * sz +
                              nn * sz + nn * szr + nn * 16 * (want ? 2 : 1) + (add ? nn * 16 : 0);
        int nbt = 0;
        prof_launch(PROF_L0_SWEEP, b_tile, L, [&] {
            l0_tiled_shape(tiled, [&](auto sh) {
                using S = decltype(sh);
                const int ntx = (g.N[0] + S::TX - 1) / S::TX;
                nbt = ntx * ((g.N[1] + S::TY - 1) / S::TY);
                if (add)
                    L.run<L0PostTile<T, TC, 1, S>, S::threads>(
                        nbt, L0PostTile<T, TC, 1, S>{g, b0, x0, hd, U, L0.Pb.rp.get(), L0.Pb.ci.get(), vals<TC>(L0.Pb),
                                                     vec_x<TC>(L1), z, vdot, slot, want, ntx, gate});
                else
                    L.run<L0PostTile<T, TC, 0, S>, S::threads>(
                        nbt, L0PostTile<T, TC, 0, S>{g, b0, x0, hd, U, L0.Pb.rp.get(), L0.Pb.ci.get(), vals<TC>(L0.Pb),
                                                     vec_x<TC>(L1), z, vdot, slot, want, ntx, gate});
            });
        });
        if (want) launch_finalize(slot.partials, nbt, fmode, ks, store, gate, L);
        return;
    }
    prof_launch(PROF_L0_TRANSFER, b_prol, L, [&] {
        L.run(nbp, L0ProlongBlack<DIM, T, TC>{g, x0, L0.Pb.rp.get(), L0.Pb.ci.get(), vals<TC>(L0.Pb),
                                              vec_x<TC>(L1), gate});
    });
    prof_launch(PROF_L0_SWEEP, b_sweep, L, [&] {
        L.run(nbp, L0Sweep<DIM, T>{g, 0, b0, x0, U, hs, gate});
    });
    prof_launch(PROF_L0_SWEEP, b_sweep, L, [&] {
        L.run(nbp, L0Sweep<DIM, T>{g, 1, b0, x0, U, hs, gate});
    });
    prof_launch(PROF_L0_SWEEP, b_last, L, [&] {
        if (add) L.run(nbp, L0Last<DIM, T, 1>{g, b0, x0, U, hs, z, vdot, slot, want, gate});
        else L.run(nbp, L0Last<DIM, T, 0>{g, b0, x0, U, hs, z, vdot, slot, want, gate});
    });
    if (want) launch_finalize(slot.partials, nbp, fmode, ks, store, gate, L);
}

// Level 0 of a simplicial mesh is a CSR level like the coarse ones: its
// rows in colour order (perm), padded colour blocks for the sweeps, the full
// restriction and prolongation.
template <class T, class TC>
static void vcycle_once_simplicial(const gl_precond *cpre, const double2 *v, const double2 *vdot, double2 *z,
                                   const int *gate, KrylovScalars *ks, int mode, int add, const Launch &L,
                                   double *store)
{
    gl_precond *pre = const_cast<gl_precond *>(cpre);
    const gl_mesh *m = pre->mesh;
    const RedSlot slot = red_slot(m, 1);
    Level &L0 = pre->L[0];
    const int n0 = L0.n, nb0 = blocks_for(n0);
    const int want = ks != nullptr || store != nullptr;
    const int fmode = store ? (int)FIN_STORE : mode;
    if (pre->nlev == 1) {  // the coarsest inverse in node order
        C<TC> *xc0 = vec_x<TC>(L0);
        L.run(nb0, Narrow<TC>{n0, v, vec_b<TC>(L0), gate});
        L.run(blocks_for((int64_t)n0 * 64), DenseApply<TC>{n0, cinv<TC>(pre), vec_b<TC>(L0), xc0, gate});
        if (add) L.run(nb0, Output<TC, 1>{n0, xc0, vdot, z, slot, want, gate});
        else L.run(nb0, Output<TC, 0>{n0, xc0, vdot, z, slot, want, gate});
        if (want) launch_finalize(slot.partials, nb0, fmode, ks, store, gate, L);
        return;
    }
    Level &L1 = pre->L[1];
    const int sh = pre->lane_shift;
    const int *perm = L0.perm.get();
    C<T> *x0 = vec_x<T>(L0);
    L.run(nb0, NarrowPerm<T>{n0, v, perm, vec_b<T>(L0), gate});
    csr_sgs<T>(L0, sh, true, gate, L);
    csr_residual<T>(L0, sh, gate, L);
    csr_spmv<TC, T>(L0.Ra, vec_r<T>(L0), vec_b<TC>(L1), false, sh, gate, L);
    coarse_levels<TC>(pre, gate, L);
    csr_spmv<T, TC>(L0.Pa, vec_x<TC>(L1), x0, true, sh, gate, L);
    csr_sgs<T>(L0, sh, false, gate, L);
    if (add) L.run(nb0, OutputPerm<T, 1>{n0, x0, perm, vdot, z, slot, want, gate});
    else L.run(nb0, OutputPerm<T, 0>{n0, x0, perm, vdot, z, slot, want, gate});
    if (want) launch_finalize(slot.partials, nb0, fmode, ks, store, gate, L);
}

// One V-cycle on H x = D v from x = 0 (DIM 0: a simplicial mesh)
template <int DIM, class T, class TC>
static void vcycle_once(const gl_precond *cpre, const double2 *v, const double2 *vdot, double2 *z,
                        const int *gate, KrylovScalars *ks, int mode, int add, const Launch &L,
                        double *store = nullptr)
{
    if constexpr (DIM == 0) vcycle_once_simplicial<T, TC>(cpre, v, vdot, z, gate, ks, mode, add, L, store);
    else vcycle_once_grid<DIM, T, TC>(cpre, v, vdot, z, gate, ks, mode, add, L, store);
}

// ------------------------------------------------------------- R_inf ---
// R_inf = H^-1 (eq. prec1; the scaled form of H^-1 D): preconditioned
// conjugate gradients on H x = v from x = 0 with one V-cycle per step, run
// for a fixed number m of steps (chosen at each setup, pcg_calibrate), so
// that the operator is a fixed linear map to the calibration's accuracy and
// the steps can be captured in the MINRES iteration graph.  Scalars of step
// j live at fixed places: rz[j] = <r_j, z_j>, pq[j] = <p_j, H p_j>.

// q = H p (level 0 as the FP64 stencil with its diagonal), partials of Re<p, q>
template <int DIM>
struct PcgHp {
    GeomT<double> g;
    const double2 *p;
    LinkTab<double> U;
    const double *hd;
    double2 *q;
    RedSlot slot;
    const int *gate;
    __device__ void operator()(int bx, int nbx) const
    {
        GATE();
        __shared__ double sm[kBlock / 64];
        const int i = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            const double2 pi = p[i];
            const double2 qi = cadd(khat_offdiag<DIM, double>(g, i, c, p, U), cscale(pi, hd[i]));
            q[i] = qi;
            part = redot(pi, qi);
        }
        block_reduce_store(part, slot, sm, bx);
    }
};

// x += alpha p (x = alpha p at the first step), r -= alpha q, alpha = rz / pq
// (0 when pq is not positive: nothing left to reduce); partials of |r|^2
// when asked (calibration)
struct PcgStep {
    int n;
    const double2 *p, *q;
    double2 *x, *r;
    const double *rz, *pq;
    int first;
    RedSlot slot;
    int want_rr;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        __shared__ double sm[kBlock / 64];
        const double den = *pq;
        const double alpha = den > 0.0 ? *rz / den : 0.0;
        const int i = bx * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < n) {
            const double2 pi = p[i], qi = q[i];
            x[i] = first ? cscale(pi, alpha) : cadd(x[i], cscale(pi, alpha));
            const double2 ri = csub(r[i], cscale(qi, alpha));
            r[i] = ri;
            part = cabs2(ri);
        }
        if (want_rr) block_reduce_store(part, slot, sm, bx);
    }
};

// p = z + beta p, beta = rz_new / rz (0 when rz is not positive)
struct PcgDir {
    int n;
    const double2 *z;
    double2 *p;
    const double *rz, *rz_new;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        const double den = *rz;
        const double beta = den > 0.0 ? *rz_new / den : 0.0;
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) p[i] = cadd(z[i], cscale(p[i], beta));
    }
};

// partials of |r|^2 (calibration)
struct PcgNorm {
    int n;
    const double2 *r;
    RedSlot slot;
    __device__ void operator()(int bx, int) const
    {
        __shared__ double sm[kBlock / 64];
        const int i = bx * kBlock + threadIdx.x;
        block_reduce_store(i < n ? cabs2(r[i]) : 0.0, slot, sm, bx);
    }
};

// r = v (the first residual, x = 0)
struct PcgInit {
    int n;
    const double2 *v;
    double2 *r;
    const int *gate;
    __device__ void operator()(int bx, int) const
    {
        GATE();
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) r[i] = v[i];
    }
};

struct PcgBufs {
    double2 *x, *r, *p, *q, *z;
    double *rz, *pq;
};

static PcgBufs pcg_bufs(const gl_precond *pre)
{
    gl_precond *p = const_cast<gl_precond *>(pre);
    const size_t n = (size_t)pre->L[0].n;
    double2 *b = p->pcg.get();
    double *sc = p->pcg_sc.get();
    return PcgBufs{b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, sc, sc + kPcgMaxSteps + 1};
}

// m steps of CG; z = x with the Krylov partials of Re<vdot, z> when ks is set
template <int DIM, class T, class TC>
static void vcycle_pcg(const gl_precond *pre, const double2 *v, double2 *z, const int *gate, KrylovScalars *ks,
                       int mode, const Launch &L)
{
    const gl_mesh *m = pre->mesh;
    const GeomT<double> g = geom_t<double>(m->g);
    const int n = pre->L[0].n, nb = blocks_for(n);
    const PcgBufs B = pcg_bufs(pre);
    const int steps = std::max(1, pre->pcg_m);
    const RedSlot hslot = red_slot(m, 0);
    L.run(nb, PcgInit{n, v, B.r, gate});
    // z_0 = V(r_0) straight into p_0
    vcycle_once<DIM, T, TC>(pre, B.r, B.r, B.p, gate, nullptr, 0, 0, L, B.rz);
    for (int j = 0; j < steps; ++j) {
        L.run(nb, PcgHp<DIM>{g, B.p, link_tab<double>(m), pre->L[0].diag64.get(), B.q, hslot, gate});
        launch_finalize(hslot.partials, nb, FIN_STORE, nullptr, B.pq + j, gate, L);
        L.run(nb, PcgStep{n, B.p, B.q, B.x, B.r, B.rz + j, B.pq + j, j == 0, hslot, 0, gate});
        if (j + 1 < steps) {
            vcycle_once<DIM, T, TC>(pre, B.r, B.r, B.z, gate, nullptr, 0, 0, L, B.rz + j + 1);
            L.run(nb, PcgDir{n, B.z, B.p, B.rz + j, B.rz + j + 1, gate});
        }
    }
    const RedSlot slot = red_slot(m, 1);
    L.run(nb, Output<double, 0>{n, B.x, v, z, slot, ks != nullptr, gate});
    if (ks) launch_finalize(slot.partials, nb, mode, ks, nullptr, gate, L);
}

template <int DIM>
static void pcg_calibrate_dim(gl_precond *pre, hipStream_t s)
{
    // CG from a seeded counter-hash right-hand side with the norm of the
    // residual read after every step: m = the steps to 1e-12, plus 2
    const gl_mesh *m = pre->mesh;
    const GeomT<double> g = geom_t<double>(m->g);
    const int n = pre->L[0].n, nb = blocks_for(n);
    const PcgBufs B = pcg_bufs(pre);
    const RedSlot hslot = red_slot(m, 0), rslot = red_slot(m, 2);
    double2 *v = pre->vin.get();
    k_hash_rhs<<<nb, kBlock, 0, s>>>(n, v);
    GLK_CHECK_LAUNCH();
    const Launch L{s};
    double *rr = m->dscal.get() + 8;
    auto host_rr = [&]() {
        double h = 0.0;
        GLK_HIP(hipMemcpyAsync(&h, rr, sizeof(double), hipMemcpyDeviceToHost, s));
        GLK_HIP(hipStreamSynchronize(s));
        return h;
    };
    L.run(nb, PcgInit{n, v, B.r, nullptr});
    L.run(nb, PcgNorm{n, B.r, rslot});
    launch_finalize(rslot.partials, nb, FIN_STORE, nullptr, rr, nullptr, L);
    const double rr0 = host_rr();
    vcycle_once<DIM, double, double>(pre, B.r, B.r, B.p, nullptr, nullptr, 0, 0, L, B.rz);
    int steps = kPcgMaxSteps;
    for (int j = 0; j < kPcgMaxSteps; ++j) {
        L.run(nb, PcgHp<DIM>{g, B.p, link_tab<double>(m), pre->L[0].diag64.get(), B.q, hslot, nullptr});
        launch_finalize(hslot.partials, nb, FIN_STORE, nullptr, B.pq + j, nullptr, L);
        L.run(nb, PcgStep{n, B.p, B.q, B.x, B.r, B.rz + j, B.pq + j, j == 0, rslot, 1, nullptr});
        launch_finalize(rslot.partials, nb, FIN_STORE, nullptr, rr, nullptr, L);
        if (!(host_rr() > 1e-24 * rr0)) {
            steps = std::min(kPcgMaxSteps, j + 1 + 2);
            break;
        }
        if (j + 1 < kPcgMaxSteps) {
            vcycle_once<DIM, double, double>(pre, B.r, B.r, B.z, nullptr, nullptr, 0, 0, L, B.rz + j + 1);
            L.run(nb, PcgDir{n, B.z, B.p, B.rz + j, B.rz + j + 1, nullptr});
        }
    }
    pre->pcg_m = steps;
}

void pcg_calibrate(gl_precond *pre, hipStream_t s)
{
    const size_t n = (size_t)pre->L[0].n;
    if (pre->pcg.count < 5 * n) pre->pcg.alloc(5 * n);
    if (pre->pcg_sc.count < 2 * kPcgMaxSteps + 2) pre->pcg_sc.alloc(2 * kPcgMaxSteps + 2);
    with_dim(pre->mesh->g, [&](auto D) { pcg_calibrate_dim<decltype(D)::value>(pre, s); });
}

template <int DIM, class T, class TC>
static void vcycle_k(const gl_precond *pre, const double2 *v, double2 *z, const int *gate,
                     KrylovScalars *ks, int mode, const Launch &L)
{
    const int k = pre->opts.cycles;
    if (k == 0) {
        vcycle_pcg<DIM, T, TC>(pre, v, z, gate, ks, mode, L);
        return;
    }
    if (k <= 1) {
        vcycle_once<DIM, T, TC>(pre, v, v, z, gate, ks, mode, 0, L);
        return;
    }
    // x <- x + V(v - H x), k times from x = 0
    const gl_mesh *m = pre->mesh;
    const GeomT<double> g = geom_t<double>(m->g);
    const int nb0 = blocks_for(pre->L[0].n);
    vcycle_once<DIM, T, TC>(pre, v, v, z, gate, nullptr, 0, 0, L);
    for (int c = 1; c < k; ++c) {
        L.run(nb0, L0ResidualFull<DIM>{g, v, z, link_tab<double>(m), pre->L[0].diag64.get(), pre->cyc_r.get(),
                                       gate});
        const bool lastc = (c == k - 1);
        vcycle_once<DIM, T, TC>(pre, pre->cyc_r.get(), v, z, gate, lastc ? ks : nullptr, mode, 1, L);
    }
}

void vcycle_enqueue(const gl_precond *pre, const double2 *v, double2 *z, const int *gate,
                    KrylovScalars *ks, int mode, const Launch &L, gl_precision p)
{
    with_dim(pre->mesh->g, [&](auto D) {
        constexpr int K = decltype(D)::value;
        if (p == GL_FP32) vcycle_k<K, float, float>(pre, v, z, gate, ks, mode, L);
        else if (p == GL_MIXED) vcycle_k<K, float, double>(pre, v, z, gate, ks, mode, L);
        else vcycle_k<K, double, double>(pre, v, z, gate, ks, mode, L);
    });
}

void vcycle_enqueue(const gl_precond *pre, const double2 *v, double2 *z, const int *gate,
                    KrylovScalars *ks, int mode, const Launch &L)
{
    vcycle_enqueue(pre, v, z, gate, ks, mode, L, pre->opts.precision);
}

// Device descriptors of the bottom levels (pointers fixed after setup).
template <class T>
static void fill_bottom(gl_precond *pre, BottomDesc<T> &D)
{
    std::memset(&D, 0, sizeof(D));
    D.first = pre->bottom;
    D.last = pre->tail;
    D.cinv = cinv<T>(pre);
    for (int l = 1; l < pre->nlev; ++l) {
        Level &L = pre->L[l];
        BottomLevel<T> &B = D.L[l];
        B.n = L.n;
        B.nc = L.nc;
        B.ncolors = L.ncolors;
        B.rp = L.Aa.rp.get();
        B.ci = L.Aa.ci.get();
        B.v = vals<T>(L.Aa);
        B.diag = dgn<T>(L);
        for (int c = 0; c <= L.ncolors && c <= kMaxColors && c < (int)L.coff.size(); ++c) B.coff[c] = L.coff[c];
        if (l + 1 < pre->nlev) {
            B.prp = L.Pa.rp.get();
            B.pci = L.Pa.ci.get();
            B.pv = vals<T>(L.Pa);
            B.rrp = L.Ra.rp.get();
            B.rci = L.Ra.ci.get();
            B.rv = vals<T>(L.Ra);
        }
        B.b = vec_b<T>(L);
        B.x = vec_x<T>(L);
        B.r = vec_r<T>(L);
        B.eci = L.eci.get();
        B.ev = evals<T>(L);
        for (int c = 0; c < L.ncolors && c < kMaxColors && c < (int)L.ewidth.size(); ++c) {
            B.ewidth[c] = L.ewidth[c];
            B.eoff[c] = L.eoff[c];
        }
    }
    // the first bottom level keeps its iterate in LDS when it fits
    D.lds_level = -1;
    if (D.first < D.last) {
        int dev = 0, lmax = 0;
        GLK_HIP(hipGetDevice(&dev));
        GLK_HIP(hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t need = (size_t)pre->L[D.first].n * sizeof(C<T>);
        if (need + 1024 <= (size_t)lmax) D.lds_level = D.first;
    }
}

void bottom_descriptors(gl_precond *pre, hipStream_t s)
{
    const int last = pre->nlev - 1;
    // level with an explicit sub-cycle: the first l >= 1 with at most
    // dense_rows rows and a bottom-kernel colouring (the coarsest if none)
    int tail = last;
    if (pre->dense_rows > 0)
        for (int l = 1; l < last; ++l) {
            const Level &L = pre->L[l];
            if (L.n <= pre->dense_rows) {
                bool fits = true;
                for (int q = l; q < last; ++q) fits = fits && pre->L[q].ncolors <= kMaxColors;
                if (fits) tail = l;
                break;
            }
        }
    pre->tail = tail;
    // first level of the bottom kernel: the smallest l >= 1 from which every
    // level above the tail fits (size and colour count); a single-level
    // hierarchy is just the dense solve on level 0.  One work-group applies
    // an explicit sub-cycle only up to kBottomDenseRows rows: a larger one is
    // a product for many work-groups, so no level goes to the bottom kernel.
    int first = tail;
    if (tail == last || pre->L[tail].n <= kBottomDenseRows)
        for (int l = tail - 1; l >= 1; --l) {
            const Level &L = pre->L[l];
            if (L.n > pre->bottom_rows || L.ncolors > kMaxColors) break;
            first = l;
        }
    pre->bottom = first;
    if (tail < last) {
        const int nt = pre->L[tail].n;
        pre->tinv64.alloc((size_t)nt * nt);
        pre->tinv32.alloc((size_t)nt * nt);
        size_t col = 0;
        for (int l = tail; l <= last; ++l) col += 3 * (size_t)pre->L[l].n;
        pre->tws_col = col * kTailBlock;  // elements per block of columns
        const int nblk = (nt + kTailBlock - 1) / kTailBlock;
        const size_t fit = kTailWorkspace / (pre->tws_col * sizeof(double2));
        pre->tws_cols = (int)std::max<size_t>(1, std::min<size_t>(nblk, fit));  // blocks per launch
        pre->tws.alloc(pre->tws_col * pre->tws_cols);
        // formation: levels tail .. coarsest with the coarsest inverse
        BottomDesc<double> dt;
        const int keep = pre->tail;
        pre->tail = last;
        const int keep_b = pre->bottom;
        pre->bottom = tail;
        fill_bottom<double>(pre, dt);
        pre->tail = keep;
        pre->bottom = keep_b;
        dt.lds_level = -1;
        pre->tdesc64.alloc(sizeof(dt));
        GLK_HIP(hipMemcpyAsync(pre->tdesc64.get(), &dt, sizeof(dt), hipMemcpyHostToDevice, s));
    } else {
        pre->tinv64.release();
        pre->tinv32.release();
        pre->tws.release();
        pre->tdesc64.release();
        pre->tws_col = 0;
        pre->tws_cols = 0;
    }
    BottomDesc<double> d64;
    BottomDesc<float> d32;
    fill_bottom<double>(pre, d64);
    fill_bottom<float>(pre, d32);
    pre->lds64 = d64.lds_level >= 0 ? (int)(pre->L[d64.lds_level].n * sizeof(double2)) : 0;
    pre->lds32 = d32.lds_level >= 0 ? (int)(pre->L[d32.lds_level].n * sizeof(float2)) : 0;
    pre->bdesc64.alloc(sizeof(d64));
    pre->bdesc32.alloc(sizeof(d32));
    GLK_HIP(hipMemcpyAsync(pre->bdesc64.get(), &d64, sizeof(d64), hipMemcpyHostToDevice, s));
    GLK_HIP(hipMemcpyAsync(pre->bdesc32.get(), &d32, sizeof(d32), hipMemcpyHostToDevice, s));
    GLK_HIP(hipStreamSynchronize(s));
}

// The explicit sub-cycle of level `tail` from the current values: FP64
// columns, kTailBlock per work-group and as many work-groups per launch as
// the workspace holds, then the FP32 copy.
void form_tail(gl_precond *pre, hipStream_t s)
{
    if (!pre->has_values || pre->tail >= pre->nlev - 1) return;
    const int nt = pre->L[pre->tail].n;
    const auto *D = reinterpret_cast<const BottomDesc<double> *>(pre->tdesc64.get());
    const Launch L{s};
    const int nblk = (nt + kTailBlock - 1) / kTailBlock;
    for (int b0 = 0; b0 < nblk; b0 += pre->tws_cols) {
        const int nb = std::min(pre->tws_cols, nblk - b0);
        L.run<TailColumns<double>, kBottomThreads>(
            nb, TailColumns<double>{D, pre->tws.get(), pre->tws_col, b0 * kTailBlock, nb, pre->tinv64.get()});
    }
    const int64_t nn = (int64_t)nt * nt;
    L.run(blocks_for(nn), Narrow<float>{(int)nn, pre->tinv64.get(), pre->tinv32.get(), nullptr});
}

}  // namespace glk

using namespace glk;

extern "C" gl_status gl_precond_apply(const gl_precond *pre, const void *r, void *z, gl_stream stream)
{
    return guarded([&] {
        if (!pre || !r || !z) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_apply: NULL argument");
        if (r == z) fail(GL_ERR_INVALID_ARGUMENT, "gl_precond_apply: r and z alias");
        hipStream_t s = as_stream(stream);
        // R_k r = AMG_k(H, D r)
        double2 *vin = const_cast<gl_precond *>(pre)->vin.get();
        scale_by_volume(pre->mesh, (const double2 *)r, vin, s);
        vcycle_enqueue(pre, vin, (double2 *)z, nullptr, nullptr, 0, Launch{s});
    });
}
