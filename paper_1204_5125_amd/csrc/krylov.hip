// Preconditioned MINRES for the Jacobian system and the Newton iteration.
//
// Sec. 4: J(psi) is self-adjoint in <u,v>_R = Re sum |V_i| conj(u_i) v_i and
// generally indefinite, so the Krylov method is MINRES, preconditioned by
// R_k(psi) = AMG_k(H, D .) (eq. prec2).  Internally the system is scaled by D:
// A = D J(psi), b_hat = D b, M^-1 = AMG_k(H, .), with the Euclidean real inner
// product; the iterates equal those of MINRES on J in <.,.>_R with M^-1 = R_k,
// because <D r, z>_E = <r, z>_R.  Without a preconditioner M^-1 = D^-1.
//
// Iteration j, gated by device flags so that the host can enqueue (or replay
// a graph of) several iterations between convergence checks:
//   1. the w / x update of iteration j-1 (w_j = (z_{j-1}/gamma_{j-1} - a3 w_{j-2}
//      - a2 w_{j-1}) / a1, x += c eta w_j), fused with q = D J(psi)(z_j / gamma_j)
//      and the partial sums of delta = Re<q, z_j / gamma_j>
//   2. finalize: delta
//   3. v_{j+1} = q - (delta / gamma) v_j - (gamma / gamma_prev) v_{j-1}
//   4. z_{j+1} = M^-1 v_{j+1} (V-cycle) with partial sums of gamma_{j+1}^2
//   5. finalize: the Givens recurrence (minres_finalize)
// The w / x update of the last iteration is applied after the loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "amg.h"
#include "stencil.h"

namespace glk {

// stride of the stored Krylov basis of reorthogonalised solves: n rounded up
// to a multiple of 4 (aligned wide loads)
__host__ __device__ inline size_t reorth_ld(int n) { return ((size_t)n + 3) & ~(size_t)3; }

// A complex number as two BF16 halves of one 32-bit word (real part low),
// rounded to nearest even from FP32: the reorthogonalisation's copy of Z
// with a reduced-precision V-cycle (it only steers the coefficients h_i,
// whose rounding moves the basis' orthogonality, not the recorded relation)
__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t pack_bf16(double2 v)
{
    return bf16_bits((float)v.x) | (bf16_bits((float)v.y) << 16);
}
__device__ __forceinline__ double2 unpack_bf16(uint32_t w)
{
    return make_double2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
}

__global__ void k_ks_init_running(KrylovScalars *ks)
{
    ks->running = (ks->eta0 > 0.0) && (ks->max_iter > 0) && (ks->status == 0);
    ks->iter = 0;
    ks->wx_valid = 0;
}

struct KsInit {
    KrylovScalars *ks;
    double rtol;
    int max_iter;
    __device__ void operator()(int, int) const
    {
        if (threadIdx.x != 0) return;
        ks->rtol = rtol;
        ks->max_iter = max_iter;
        ks->running = 1;
        ks->wx_valid = 0;
        ks->iter = 0;
        ks->status = 0;
        ks->converged = 0;
        ks->delta = 0.0;
    }
};

// v = D b, v_prev = w = w_prev = x = 0
template <int DIM>
struct MinresInit {
    GeomT<double> g;
    const double2 *b;
    double2 *v, *vp, *w, *wp, *x;
    __device__ void operator()(int bx, int) const
    {
        const int i = bx * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 zero = make_double2(0.0, 0.0);
        v[i] = cscale(b[i], d);
        vp[i] = zero;
        w[i] = zero;
        wp[i] = zero;
        x[i] = zero;
    }
};

// no preconditioner: M^-1 = I in <.,.>_R, i.e. z = D^-1 v in the scaled form,
// with the partial sums of gamma^2 = Re<v, z>
template <int DIM>
struct Unprec {
    GeomT<double> g;
    const double2 *v;
    double2 *z;
    const int *gate;
    RedSlot slot;
    __device__ void operator()(int bx, int) const
    {
        if (gate && *gate == 0) return;
        __shared__ double sm[kBlock / 64];
        const int i = bx * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            double sf[3];
            const double d = node_volume<DIM, double>(g, c, sf);
            const double2 vi = v[i];
            const double2 zi = cscale(vi, 1.0 / d);
            z[i] = zi;
            part = redot(vi, zi);
        }
        block_reduce_store(part, slot, sm, bx);
    }
};

// w / x update of the previous iteration (when iter >= 1) and q = D J (z / gamma)
template <int DIM>
struct MinresJapply {
    GeomT<double> g;
    const double2 *psi, *z;
    LinkTab<double> U;
    double2 *q;
    const double2 *zprev, *w;
    double2 *wp, *x;
    const KrylovScalars *ks;
    RedSlot slot;
    RedSlot slot_u;  // deflation: partials of <u, q>_E, u = i psi (unused otherwise)
    int defl;
    double2 *zb = nullptr;  // reorthogonalised solves: the basis Z (z_j / gamma_j stored
                            // at slot j); no w / x update then
    uint32_t *zbh = nullptr; // and its BF16 copy (reduced-precision V-cycles)
    __device__ void operator()(int bx, int nbx) const
    {
        // the scalars and the vectors are loaded together; the (uniform)
        // running flag is checked before the first store
        __shared__ double sm[kBlock / 64];
        const int running = ks->running;
        const double ig = 1.0 / ks->gamma;
        const int jt = ks->iter;
        const bool upd = zb == nullptr && jt >= 1;
        const int i = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        const bool in = i < g.n;
        double part = 0.0, part_u = 0.0;
        double2 wn = make_double2(0.0, 0.0), xn = wn, qi = wn;
        if (in) {
            if (upd) {
                const double2 zp = cscale(zprev[i], ks->wx_inv_gamma);
                wn = cscale(csub(csub(zp, cscale(wp[i], ks->wx_a3)), cscale(w[i], ks->wx_a2)), 1.0 / ks->wx_a1);
                xn = cadd(x[i], cscale(wn, ks->wx_coef));
            }
            int c[3];
            node_coords<DIM>(g.N, i, c);
            const double2 zi = z[i];
            double d, asum;
            const double2 kz = khat_node<DIM, double>(g, i, c, z, U, zi, d, asum);
            const double2 zn = cscale(zi, ig);
            const double2 p = psi[i];
            const double2 react = cadd(cscale(zn, 2.0 * cabs2(p) - 1.0), cmul(cmul(p, p), cconj(zn)));
            qi = cadd(cscale(kz, ig), cscale(react, d));
            part = redot(qi, zn);
            // Re(conj(i psi) q) = Im(conj(psi) q)
            part_u = p.x * qi.y - p.y * qi.x;
        }
        if (running == 0) return;
        if (in) {
            if (upd) {
                wp[i] = wn;
                x[i] = xn;
            }
            if (zb) {
                const double2 zs = cscale(z[i], ig);
                const size_t at = (size_t)jt * reorth_ld(g.n) + i;
                zb[at] = zs;
                if (zbh) zbh[at] = pack_bf16(zs);
            }
            q[i] = qi;
        }
        block_reduce_store(part, slot, sm, bx);
        if (defl) block_reduce_store(part_u, slot_u, sm, bx);
    }
};

// a basis vector entry in FP64 or FP32 (whichever buffer is given)
__device__ __forceinline__ void store_basis(double2 *b64, float2 *b32, size_t at, double2 v)
{
    if (b64) b64[at] = v;
    if (b32) b32[at] = make_float2((float)v.x, (float)v.y);
}

struct MinresVupdate {
    int n;
    const double2 *q, *v;
    double2 *vp;
    const KrylovScalars *ks;
    double2 *vb = nullptr;  // reorthogonalised solves: the basis V (v_j / gamma_j at slot j)
    float2 *vb32 = nullptr; // or its FP32 form (reduced-precision V-cycles)
    __device__ void operator()(int bx, int) const
    {
        const int running = ks->running;
        const double a = ks->delta / ks->gamma, b = ks->gamma / ks->gamma_prev;
        const int jt = ks->iter;
        const int i = bx * kBlock + threadIdx.x;
        if (i >= n) return;
        const double2 qi = q[i], vi = v[i], vpi = vp[i];
        if (running == 0) return;
        vp[i] = csub(csub(qi, cscale(vi, a)), cscale(vpi, b));
        store_basis(vb, vb32, (size_t)jt * reorth_ld(n) + i, cscale(vi, 1.0 / ks->gamma));
    }
};

// ------------------------------ MINRES with the basis reorthogonalised ----
// Sec. 4 traces the iteration peaks of the continuation runs to the loss of
// orthogonality of the MINRES basis and names the remedy: store the basis
// and fully reorthogonalise it in every step, as GMRES does.  Iteration j
// keeps the MINRES step (the Japply, delta and the Lanczos update above, which
// store V_j = v_j / gamma_j and Z_j = z_j / gamma_j in the basis) and then
//   h_i = <Z_i, v_{j+1}>_E for every i <= j          (ReorthDots, ReorthSum)
//   v_{j+1} -= sum_i h_i V_i                          (ReorthUpdate)
//   z_{j+1} = M^-1 v_{j+1}, gamma_{j+1}^2 = <v_{j+1}, z_{j+1}>
//   column j of the projected matrix: h_i, plus delta on the diagonal and
//   gamma_j above it, gamma_{j+1} below; the previous Givens rotations, a new
//   one, and |g_{j+1}| (the preconditioned residual norm) tested against
//   rtol eta_0                                        (ReorthColumn)
// classical Gram-Schmidt: every h_i from the same vector.  After the loop the
// host solves R y = g and x += Z y (k_basis_combine).  Every kernel reads j
// from the device scalars, so the graph of two iterations replays.

// The multiply-adds of the passes are written as fma, so their rounding does
// not depend on the compiler's contraction choices.

// Basis vectors are stored with the padded stride ld = n rounded up to a
// multiple of 4, four nodes per thread: the FP32 entries of a thread are two
// aligned 16-byte loads, the BF16 ones one.  Entries past n are never used
// (selected away).
constexpr int kReorthNodes = 4;

__device__ __forceinline__ void load4(const uint32_t *p, double2 out[4])
{
    const uint4 w = reinterpret_cast<const uint4 *>(p)[0];
    out[0] = unpack_bf16(w.x);
    out[1] = unpack_bf16(w.y);
    out[2] = unpack_bf16(w.z);
    out[3] = unpack_bf16(w.w);
}

template <class T>
__device__ __forceinline__ void load4(const C<T> *p, double2 out[4]);
__device__ __forceinline__ void load4(const double2 *p, double2 out[4]) { load4<double>(p, out); }

template <class T>
__device__ __forceinline__ void load4(const C<T> *p, double2 out[4])
{
    if constexpr (sizeof(T) == 4) {
        const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
        out[0] = make_double2(a.x, a.y);
        out[1] = make_double2(a.z, a.w);
        out[2] = make_double2(b.x, b.y);
        out[3] = make_double2(b.z, b.w);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = p[e];
    }
}

// partials of h_i = <Z_i, q>_E, i = 0 .. j, one per wave: part[i * nparts +
// wave].  The basis is read in FP64 with an FP64 V-cycle and as BF16 with a
// reduced-precision one (the coefficients are of the size of the loss of
// orthogonality, and every one subtracted is also the one recorded in the
// projected matrix, so the relation J Z = V H holds to FP64 rounding either
// way; their rounding only sets how orthogonal the basis stays).  No
// barrier: each wave keeps G rows of the basis in flight.
template <class S>
struct ReorthDots {
    // rows in flight per thread: 4 (16 bytes each in BF16, 64 in FP64)
    static constexpr int G = 4;
    int n, nparts;
    const S *zb;  // double2 (FP64) or uint32_t (BF16 pairs)
    const double2 *q;
    double *part;
    const KrylovScalars *ks;
    __device__ void operator()(int bx, int) const
    {
        if (ks->running == 0) return;  // uniform
        const int j = ks->iter;
        const size_t ld = reorth_ld(n);
        const int t = bx * kBlock + threadIdx.x, base = t * kReorthNodes;
        const int wave = t >> 6, lane = threadIdx.x & 63;
        // a thread past n reads the first nodes (always present) and selects
        // its terms away
        const int cb = base < n ? base : 0;
        double2 qv[kReorthNodes];
        bool ok[kReorthNodes];
#pragma unroll
        for (int e = 0; e < kReorthNodes; ++e) {
            ok[e] = base + e < n;
            qv[e] = ok[e] ? q[base + e] : make_double2(0.0, 0.0);
        }
        for (int k0 = 0; k0 <= j; k0 += G) {
            // every load of the group first, with no branch between them, so
            // that all are in flight together (rows past j re-read row j)
            double2 zv[G][kReorthNodes];
#pragma unroll
            for (int g = 0; g < G; ++g) load4(zb + (size_t)min(k0 + g, j) * ld + cb, zv[g]);
            double sv[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double acc = 0.0;
#pragma unroll
                for (int e = 0; e < kReorthNodes; ++e)
                    acc = ok[e] ? fma(zv[g][e].y, qv[e].y, fma(zv[g][e].x, qv[e].x, acc)) : acc;
                sv[g] = wave_sum(acc);
            }
            if (lane == 0) {
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (k0 + g <= j) part[(size_t)(k0 + g) * nparts + wave] = sv[g];
            }
        }
    }
};

// h_i = sum of the nparts partials of coefficient i (block i, fixed order)
struct ReorthSum {
    int nparts;
    const double *part;
    double *h;
    const KrylovScalars *ks;
    __device__ void operator()(int bx, int) const
    {
        __shared__ double sm[kBlock / 64];
        if (ks->running == 0 || bx > ks->iter) return;  // uniform per block
        double sv = 0.0;
        for (int k = threadIdx.x; k < nparts; k += kBlock) sv += part[(size_t)bx * nparts + k];
        sv = block_sum(sv, sm);
        if (threadIdx.x == 0) h[bx] = sv;
    }
};

// q -= sum_{i <= j} h_i V_i (V in FP64 or FP32 as in ReorthDots)
template <class T>
struct ReorthUpdate {
    int n;
    const C<T> *vb;
    const double *h;
    double2 *q;
    const KrylovScalars *ks;
    __device__ void operator()(int bx, int) const
    {
        if (ks->running == 0) return;
        const int j = ks->iter;
        const size_t ld = reorth_ld(n);
        const int base = (bx * kBlock + threadIdx.x) * kReorthNodes;
        if (base >= n) return;
        double2 acc[kReorthNodes];
#pragma unroll
        for (int e = 0; e < kReorthNodes; ++e) acc[e] = base + e < n ? q[base + e] : make_double2(0.0, 0.0);
#pragma unroll 4
        for (int k = 0; k <= j; ++k) {
            double2 vv[kReorthNodes];
            load4<T>(vb + (size_t)k * ld + base, vv);
            const double hk = h[k];
#pragma unroll
            for (int e = 0; e < kReorthNodes; ++e)
                acc[e] = make_double2(fma(-vv[e].x, hk, acc[e].x), fma(-vv[e].y, hk, acc[e].y));
        }
#pragma unroll
        for (int e = 0; e < kReorthNodes; ++e)
            if (base + e < n) q[base + e] = acc[e];
    }
};

// Column j of the projected matrix, its rotations and the convergence test.
// The rotations are a chain on thread 0; the block stages their
// coefficients and the column's entries in LDS, 64 at a time.  R is
// column-major with kmax + 1 rows.
struct ReorthColumn {
    int kmax;
    double *R, *cs, *sn, *gv;
    const double *h;
    KrylovScalars *ks;
    __device__ void operator()(int, int) const
    {
        __shared__ double scs[64], ssn[64], sh[64];
        const int running = ks->running, j = ks->iter;
        const double delta = ks->delta, gam = ks->gamma;
        __syncthreads();  // every thread has read the scalars before thread 0 writes them
        if (running == 0) return;  // uniform
        auto entry = [&](int i) { return h[i] + (i == j ? delta : 0.0) + (i == j - 1 ? gam : 0.0); };
        double *col = R + (size_t)j * (kmax + 1);
        double carry = threadIdx.x == 0 ? entry(0) : 0.0;
        for (int i0 = 0; i0 < j; i0 += 64) {
            const int cnt = min(64, j - i0);
            if ((int)threadIdx.x < cnt) {
                scs[threadIdx.x] = cs[i0 + threadIdx.x];
                ssn[threadIdx.x] = sn[i0 + threadIdx.x];
                sh[threadIdx.x] = entry(i0 + threadIdx.x + 1);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int t = 0; t < cnt; ++t) {
                    const double a1 = sh[t];
                    col[i0 + t] = scs[t] * carry + ssn[t] * a1;
                    carry = -ssn[t] * carry + scs[t] * a1;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x != 0) return;
        const double g2 = ks->rg2;
        if (!(g2 >= 0.0)) {
            ks->status = GL_ERR_BREAKDOWN;
            ks->running = 0;
            return;
        }
        const double gnew = sqrt(g2);
        if (j == 0) gv[0] = ks->eta0;
        const double rr = sqrt(carry * carry + gnew * gnew);
        if (!(rr > 0.0)) {
            ks->status = GL_ERR_BREAKDOWN;
            ks->running = 0;
            return;
        }
        cs[j] = carry / rr;
        sn[j] = gnew / rr;
        col[j] = rr;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        ks->eta = gv[j + 1];
        ks->iter = j + 1;
        ks->gamma_prev = gam;
        ks->gamma = gnew;
        if (fabs(gv[j + 1]) <= ks->rtol * ks->eta0 || gnew == 0.0) {
            ks->converged = 1;
            ks->running = 0;
        } else if (j + 1 >= kmax || j + 1 >= ks->max_iter) {
            ks->running = 0;
        }
    }
};

// x += sum_{k < cols} y_k Z_k
__global__ __launch_bounds__(kBlock) void k_basis_combine(int n, int cols, const double2 *__restrict__ zb,
                                                          const double *__restrict__ y, double2 *__restrict__ x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t ld = reorth_ld(n);
    double2 acc = x[i];
    for (int k = 0; k < cols; ++k) acc = cadd(acc, cscale(zb[(size_t)k * ld + i], y[k]));
    x[i] = acc;
}

// ---------------------------------------------- deflation of i psi ----
// The solve restricted to the <.,.>_R-orthogonal complement of the gauge
// mode u = i psi: at a solution J(psi) u = 0 (eq. jacobian nullspace), and
// near one J is nearly singular along u; Sec. 3 names deflation among the
// remedies.  In the D-scaled form the projector of solution-space vectors
// (z, w, x) is Pi z = z - u <u, z>_R / c and that of residual-space vectors
// (v, q = D J z) its transpose Pi' v = v - D u Re(sum conj(u) v) / c, with
// c = <u, u>_R.  MINRES runs on Pi' (D J) Pi with the preconditioner
// Pi AMG Pi': q is projected before the Lanczos update (its coefficient comes
// with delta from MinresJapply) and every preconditioner output after it.
// delta and gamma need no correction: <q, z> and <v, M^-1 v> are unchanged by
// the projections when z and v already lie in the complements.

// partials of c = <u, u>_R = sum d |psi|^2 and <u, b>_R = sum d Im(conj(psi) b)
template <int DIM>
struct DeflInit {
    GeomT<double> g;
    const double2 *psi, *b;
    RedSlot sc, sb;
    __device__ void operator()(int bx, int) const
    {
        __shared__ double sm[kBlock / 64];
        const int i = bx * kBlock + threadIdx.x;
        double pc = 0.0, pb = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            double sf[3];
            const double d = node_volume<DIM, double>(g, c, sf);
            const double2 p = psi[i], bi = b[i];
            pc = d * cabs2(p);
            pb = d * (p.x * bi.y - p.y * bi.x);
        }
        block_reduce_store(pc, sc, sm, bx);
        block_reduce_store(pb, sb, sm, bx);
    }
};

// v = D Pi b = D (b - u <u, b>_R / c), v_prev = w = w_prev = x = 0
template <int DIM>
struct MinresInitDefl {
    GeomT<double> g;
    const double2 *psi, *b;
    double2 *v, *vp, *w, *wp, *x;
    const KrylovScalars *ks;
    __device__ void operator()(int bx, int) const
    {
        const double cu = ks->defl_c;
        const double sb = cu > 0.0 ? ks->defl_sq / cu : 0.0;
        const int i = bx * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 p = psi[i], bi = b[i];
        const double2 zero = make_double2(0.0, 0.0);
        // u = i psi = (-Im psi, Re psi)
        v[i] = cscale(make_double2(bi.x + sb * p.y, bi.y - sb * p.x), d);
        vp[i] = zero;
        w[i] = zero;
        wp[i] = zero;
        x[i] = zero;
    }
};

// v_{j+1} = Pi'(q) - (delta / gamma) v_j - (gamma / gamma_prev) v_{j-1}
template <int DIM>
struct MinresVupdateDefl {
    GeomT<double> g;
    const double2 *psi, *q, *v;
    double2 *vp;
    const KrylovScalars *ks;
    double2 *vb = nullptr;  // as in MinresVupdate
    float2 *vb32 = nullptr;
    __device__ void operator()(int bx, int) const
    {
        const int running = ks->running;
        const double a = ks->delta / ks->gamma, b = ks->gamma / ks->gamma_prev;
        const int jt = ks->iter;
        const double cu = ks->defl_c;
        const double sq = cu > 0.0 ? ks->defl_sq / cu : 0.0;
        const int i = bx * kBlock + threadIdx.x;
        if (i >= g.n) return;
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 qi = q[i], vi = v[i], vpi = vp[i], p = psi[i];
        if (running == 0) return;
        const double2 pq = make_double2(qi.x + sq * d * p.y, qi.y - sq * d * p.x);
        vp[i] = csub(csub(pq, cscale(vi, a)), cscale(vpi, b));
        store_basis(vb, vb32, (size_t)jt * reorth_ld(g.n) + i, cscale(vi, 1.0 / ks->gamma));
    }
};

// partials of <u, z>_R = sum d Im(conj(psi) z) for a new preconditioner output
template <int DIM>
struct DeflZ {
    GeomT<double> g;
    const double2 *psi, *z;
    const KrylovScalars *ks;
    RedSlot slot;
    __device__ void operator()(int bx, int) const
    {
        if (!ks->defl_pending) return;  // the finalisation then stores 0
        __shared__ double sm[kBlock / 64];
        const int i = bx * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            double sf[3];
            const double d = node_volume<DIM, double>(g, c, sf);
            const double2 p = psi[i], zi = z[i];
            part = d * (p.x * zi.y - p.y * zi.x);
        }
        block_reduce_store(part, slot, sm, bx);
    }
};

// z = Pi z = z - u defl_sy / c
struct DeflApply {
    int n;
    const double2 *psi;
    double2 *z;
    const KrylovScalars *ks;
    __device__ void operator()(int bx, int) const
    {
        const double cu = ks->defl_c, sy = ks->defl_sy;
        if (!(cu > 0.0) || sy == 0.0) return;
        const double s = sy / cu;
        const int i = bx * kBlock + threadIdx.x;
        if (i >= n) return;
        const double2 p = psi[i], zi = z[i];
        z[i] = make_double2(zi.x + s * p.y, zi.y - s * p.x);
    }
};

// the pending w / x update after the last iteration
__global__ __launch_bounds__(kBlock) void k_minres_wx(int n, const double2 *__restrict__ z,
                                                      const double2 *__restrict__ w, double2 *__restrict__ wp,
                                                      double2 *__restrict__ x, const KrylovScalars *ks)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double2 zn = cscale(z[i], ks->wx_inv_gamma);
    const double2 wn = cscale(csub(csub(zn, cscale(wp[i], ks->wx_a3)), cscale(w[i], ks->wx_a2)), 1.0 / ks->wx_a1);
    wp[i] = wn;
    x[i] = cadd(x[i], cscale(wn, ks->wx_coef));
}

// partial sums of ||b - J x||_D^2 and ||b||_D^2
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_true_residual(GeomT<double> g, const double2 *__restrict__ psi,
                                                          const double2 *__restrict__ x,
                                                          const double2 *__restrict__ b,
                                                          const LinkTab<double> U, RedSlot s1, RedSlot s2)
{
    __shared__ double sm[kBlock / 64];
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    double pr = 0.0, pb = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        const double2 xi = x[i];
        double d, asum;
        const double2 kx = khat_node<DIM, double>(g, i, c, x, U, xi, d, asum);
        const double2 p = psi[i];
        const double2 jx = cadd(cadd(cscale(kx, 1.0 / d), cscale(xi, 2.0 * cabs2(p) - 1.0)),
                                cmul(cmul(p, p), cconj(xi)));
        const double2 bi = b[i];
        pr = d * cabs2(csub(bi, jx));
        pb = d * cabs2(bi);
    }
    block_reduce_store(pr, s1, sm, blockIdx.x);
    block_reduce_store(pb, s2, sm, blockIdx.x);
}

// deflated solves: partials of <u, r>_R and <u, b>_R (u = i psi), with r the
// residual vector b - J x already formed
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_defl_dots(GeomT<double> g, const double2 *__restrict__ psi,
                                                      const double2 *__restrict__ r,
                                                      const double2 *__restrict__ b, RedSlot s1, RedSlot s2)
{
    __shared__ double sm[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double pr = 0.0, pb = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 p = psi[i], ri = r[i], bi = b[i];
        pr = d * (p.x * ri.y - p.y * ri.x);
        pb = d * (p.x * bi.y - p.y * bi.x);
    }
    block_reduce_store(pr, s1, sm, blockIdx.x);
    block_reduce_store(pb, s2, sm, blockIdx.x);
}

// partials of ||Pi r||_D^2 and ||Pi b||_D^2, Pi y = y - u <u, y>_R / c (the
// projections formed explicitly: the residual carries the phase condition's
// multiplier along u, which a difference of squares would cancel badly)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_defl_norms(GeomT<double> g, const double2 *__restrict__ psi,
                                                       const double2 *__restrict__ r,
                                                       const double2 *__restrict__ b,
                                                       const KrylovScalars *__restrict__ ks, RedSlot s1,
                                                       RedSlot s2)
{
    __shared__ double sm[kBlock / 64];
    const double cu = ks->defl_c;
    const double sr = cu > 0.0 ? ks->res_u_num / cu : 0.0, sb = cu > 0.0 ? ks->res_u_den / cu : 0.0;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double pr = 0.0, pb = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 p = psi[i], ri = r[i], bi = b[i];
        // y - s u with u = i psi = (-Im psi, Re psi)
        pr = d * cabs2(make_double2(ri.x + sr * p.y, ri.y - sr * p.x));
        pb = d * cabs2(make_double2(bi.x + sb * p.y, bi.y - sb * p.x));
    }
    block_reduce_store(pr, s1, sm, blockIdx.x);
    block_reduce_store(pb, s2, sm, blockIdx.x);
}

// psi -= dx (the Newton update)
struct NewtonSub {
    int n;
    double2 *psi;
    const double2 *dx;
    __device__ void operator()(int bx, int) const
    {
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) psi[i] = csub(psi[i], dx[i]);
    }
};

// x += d
__global__ void k_add(int n, double2 *x, const double2 *d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = cadd(x[i], d[i]);
}

// x += c d (a backtracking step of the Newton line search)
struct NewtonAxpy {
    int n;
    double c;
    double2 *x;
    const double2 *d;
    __device__ void operator()(int bx, int) const
    {
        const int i = bx * kBlock + threadIdx.x;
        if (i < n) x[i] = cadd(x[i], cscale(d[i], c));
    }
};

// Sufficient decrease of the Newton line search: a step of length alpha is
// kept when the residual norm falls by the factor 1 - 1e-4 alpha (false for
// NaN).
static bool newton_accepts(double res_new, double res_old, double alpha)
{
    return res_new <= (1.0 - 1e-4 * alpha) * res_old;
}

// r = b - J(psi) x
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_vec(GeomT<double> g, const double2 *__restrict__ psi,
                                                         const double2 *__restrict__ x,
                                                         const double2 *__restrict__ b,
                                                         const LinkTab<double> U, double2 *__restrict__ r)
{
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    const double2 xi = x[i];
    double d, asum;
    const double2 kx = khat_node<DIM, double>(g, i, c, x, U, xi, d, asum);
    const double2 p = psi[i];
    const double2 jx = cadd(cadd(cscale(kx, 1.0 / d), cscale(xi, 2.0 * cabs2(p) - 1.0)),
                            cmul(cmul(p, p), cconj(xi)));
    r[i] = csub(b[i], jx);
}

__global__ void k_ks_set(KrylovScalars *ks, double rtol, int max_iter)
{
    ks->rtol = rtol;
    ks->max_iter = max_iter;
}

// continue a recurrence stopped at an intermediate tolerance
__global__ void k_ks_resume(KrylovScalars *ks, double rtol)
{
    ks->rtol = rtol;
    ks->converged = 0;
    ks->running = 1;
}

__global__ void k_zero(int n, double2 *x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = make_double2(0.0, 0.0);
}

__global__ void k_copy(int n, double2 *dst, const double2 *src)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

static void read_scalars(const gl_mesh *m, KrylovScalars *h, hipStream_t s)
{
    GLK_HIP(hipMemcpyAsync(m->hscal, m->kscal.get(), sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    std::memcpy(h, m->hscal, sizeof(KrylovScalars));
}

// Buffers of one MINRES solve.  Two iterations rotate (v, vp), (z, zn), (w, wp)
// back to their starting roles, so a captured pair of iterations can be
// replayed any number of times.
struct Ksolve {
    const gl_mesh *m;
    const double2 *psi;
    const gl_precond *pre;
    const double2 *rhs;
    double2 *x;
    double2 *v, *vp, *z, *zn, *q, *w, *wp;
    gl_precision prec;  // of the V-cycle applications
    bool defl;          // restricted to the complement of i psi
    // reorthogonalised solves: the basis (V then Z, kmax vectors each) and
    // the projected matrix's state; rb == nullptr: plain MINRES
    double2 *rb = nullptr;
    float2 *rb32 = nullptr;  // non-null: the reorthogonalisation reads the BF16 Z and FP32 V copies
    double *rs = nullptr;
    int kmax = 0;
};

// blocks of the reorthogonalisation kernels and their partials (one per wave)
static int reorth_blocks(int n) { return (n + kBlock * kReorthNodes - 1) / (kBlock * kReorthNodes); }
static int reorth_parts(int n) { return reorth_blocks(n) * (kBlock / 64); }

// Layout of gl_mesh::rstate for a basis of kmax vectors and nbd dot partials
struct ReorthLayout {
    double *R, *cs, *sn, *gv, *h, *part;
};

static ReorthLayout reorth_layout(double *rs, int kmax)
{
    ReorthLayout L;
    L.R = rs;
    L.cs = L.R + (size_t)(kmax + 1) * kmax;
    L.sn = L.cs + kmax;
    L.gv = L.sn + kmax;
    L.h = L.gv + kmax + 1;
    L.part = L.h + kmax + 1;
    return L;
}

// After a reorthogonalised run of `cols` columns: R y = g on the host (cols
// x cols, upper triangular) and x += Z y on the device.  Synchronises s.
static void reorth_combine(const gl_mesh *m, double *rs, int kmax, int cols, double2 *x, hipStream_t s)
{
    if (cols <= 0) return;
    const int n = m->g.n;
    const ReorthLayout RL = reorth_layout(rs, kmax);
    std::vector<double> Rh((size_t)cols * (kmax + 1)), gh((size_t)cols), y((size_t)cols, 0.0);
    GLK_HIP(hipMemcpyAsync(Rh.data(), RL.R, sizeof(double) * Rh.size(), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipMemcpyAsync(gh.data(), RL.gv, sizeof(double) * gh.size(), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    for (int i = cols - 1; i >= 0; --i) {
        double acc = gh[(size_t)i];
        for (int c = i + 1; c < cols; ++c) acc -= Rh[(size_t)c * (kmax + 1) + i] * y[(size_t)c];
        y[(size_t)i] = acc / Rh[(size_t)i * (kmax + 1) + i];
    }
    GLK_HIP(hipMemcpyAsync(RL.h, y.data(), sizeof(double) * cols, hipMemcpyHostToDevice, s));
    k_basis_combine<<<blocks_for(n), kBlock, 0, s>>>(n, cols, m->rbasis.get(), RL.h, x);
    GLK_CHECK_LAUNCH();
    GLK_HIP(hipStreamSynchronize(s));
}

// starts of a reorthogonalised solve at most (as the refinement's outer
// rounds); each one measures the true residual
constexpr int kMaxStarts = 64;

// The mesh's basis and state for kmax vectors (grown, never shrunk).  The
// cached iteration graphs are dropped when the buffers move (a graph holds
// their addresses; the stream is idle between solves).
static void ensure_reorth(gl_mesh *m, int kmax, bool fp32)
{
    if (m->rcap >= kmax && (fp32 ? m->rcap_32 : m->rcap_v64)) return;
    const bool v64 = m->rcap_v64 || !fp32, b32 = m->rcap_32 || fp32;
    kmax = std::max(kmax, m->rcap);
    const size_t n = reorth_ld(m->g.n), nbd = (size_t)reorth_parts(m->g.n);
    for (auto &e : m->graphs) (void)hipGraphExecDestroy(e.exec);
    m->graphs.clear();
    m->rbasis.release();
    m->rbasis32.release();
    m->rstate.release();
    m->rcap = 0;
    m->rcap_v64 = m->rcap_32 = false;
    m->rbasis.alloc((v64 ? 2 : 1) * (size_t)kmax * n);
    if (b32) m->rbasis32.alloc(3 * (size_t)kmax * n / 2);  // BF16 Z (half a float2 each), FP32 V
    m->rstate.alloc((size_t)(kmax + 1) * kmax + 2 * (size_t)kmax + 2 * (size_t)(kmax + 1) + nbd * kmax);
    m->rcap = kmax;
    m->rcap_v64 = v64;
    m->rcap_32 = b32;
}

static Ksolve make_ksolve(const gl_mesh *m, const double2 *psi, const gl_precond *pre, const double2 *rhs,
                          double2 *x, bool defl)
{
    const size_t n = (size_t)m->g.n;
    double2 *W = m->work.get();
    return Ksolve{m,         psi,       pre,       rhs,       x,         W,
                  W + n,     W + 2 * n, W + 3 * n, W + 4 * n, W + 5 * n, W + 6 * n,
                  pre ? pre->opts.precision : GL_FP64, defl};
}

// z = Pi z after a new preconditioner output (deflated solves)
template <int DIM>
static void defl_project_z(const Ksolve &k, double2 *z, const Launch &L)
{
    const gl_mesh *m = k.m;
    const int n = m->g.n, nb = blocks_for(n);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    L.run(nb, DeflZ<DIM>{geom_t<double>(m->g), k.psi, z, ks, red_slot(m, 3)});
    launch_finalize(red_slot(m, 3).partials, nb, FIN_DEFL_Y, ks, nullptr, nullptr, L);
    L.run(nb, DeflApply{n, k.psi, z, ks});
}

// the roles of the rotating buffers after `iters` further iterations
static Ksolve rotated(Ksolve k, int iters)
{
    if (iters & 1) {
        std::swap(k.v, k.vp);
        std::swap(k.z, k.zn);
        std::swap(k.w, k.wp);
    }
    return k;
}

// x = 0, v = D rhs, z = M^-1 v, gamma_1, eta_0
template <int DIM>
static void ksolve_init(const Ksolve &k, double rtol, int max_iter, const Launch &L)
{
    const gl_mesh *m = k.m;
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    L.run<KsInit, 64>(1, KsInit{ks, rtol, max_iter});
    if (k.defl) {
        L.run(nb, DeflInit<DIM>{g, k.psi, k.rhs, red_slot(m, 2), red_slot(m, 3)});
        launch_finalize(red_slot(m, 2).partials, nb, FIN_STORE, nullptr, &ks->defl_c, nullptr, L);
        launch_finalize(red_slot(m, 3).partials, nb, FIN_STORE, nullptr, &ks->defl_sq, nullptr, L);
        L.run(nb, MinresInitDefl<DIM>{g, k.psi, k.rhs, k.v, k.vp, k.w, k.wp, k.x, ks});
    } else {
        L.run(nb, MinresInit<DIM>{g, k.rhs, k.v, k.vp, k.w, k.wp, k.x});
    }
    if (k.pre) {
        vcycle_enqueue(k.pre, k.v, k.z, nullptr, ks, FIN_MINRES_INIT, L, k.prec);
    } else {
        L.run(nb, Unprec<DIM>{g, k.v, k.z, nullptr, red_slot(m, 1)});
        launch_finalize(red_slot(m, 1).partials, nb, FIN_MINRES_INIT, ks, nullptr, nullptr, L);
    }
    if (k.defl) defl_project_z<DIM>(k, k.z, L);
}

template <int DIM>
static void enqueue_iteration(Ksolve &k, const Launch &L)
{
    const gl_mesh *m = k.m;
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    const int *gate = &ks->running;
    // the basis: Z (FP64) and V (FP64), or Z (FP64) plus Z in BF16 and V in
    // FP32 (kn is even: ld is a multiple of 4, so V starts 16-byte aligned)
    const size_t kn = (size_t)k.kmax * reorth_ld(n);
    const int nbr = reorth_blocks(n), npr = reorth_parts(n);
    double2 *zb = k.rb;
    double2 *vb = k.rb && !k.rb32 ? k.rb + kn : nullptr;
    uint32_t *zbh = k.rb32 ? reinterpret_cast<uint32_t *>(k.rb32) : nullptr;  // BF16 Z, then FP32 V
    float2 *vb32 = k.rb32 ? k.rb32 + kn / 2 : nullptr;
    prof_launch(PROF_MINRES_JAPPLY, 48.0 * n + 96.0 * n, L, [&] {
        L.run(nb, MinresJapply<DIM>{g, k.psi, k.z, link_tab<double>(m), k.q, k.zn, k.w, k.wp, k.x, ks,
                                    red_slot(m, 0), red_slot(m, 2), k.defl ? 1 : 0, zb, zbh});
    });
    launch_finalize(red_slot(m, 0).partials, nb, FIN_DELTA, ks, nullptr, gate, L);
    if (k.defl) {
        launch_finalize(red_slot(m, 2).partials, nb, FIN_STORE, nullptr, &ks->defl_sq, gate, L);
        prof_launch(PROF_VUPDATE, 80.0 * n, L,
                    [&] { L.run(nb, MinresVupdateDefl<DIM>{g, k.psi, k.q, k.v, k.vp, ks, vb, vb32}); });
    } else {
        prof_launch(PROF_VUPDATE, 64.0 * n, L,
                    [&] { L.run(nb, MinresVupdate{n, k.q, k.v, k.vp, ks, vb, vb32}); });
    }
    const int fin = k.rb ? FIN_REORTH : FIN_MINRES_STEP;
    ReorthLayout R{};
    if (k.rb) {
        R = reorth_layout(k.rs, k.kmax);
        if (k.rb32) {
            L.run(nbr, ReorthDots<uint32_t>{n, npr, zbh, k.vp, R.part, ks});
            L.run(k.kmax, ReorthSum{npr, R.part, R.h, ks});
            L.run(nbr, ReorthUpdate<float>{n, vb32, R.h, k.vp, ks});
        } else {
            L.run(nbr, ReorthDots<double2>{n, npr, zb, k.vp, R.part, ks});
            L.run(k.kmax, ReorthSum{npr, R.part, R.h, ks});
            L.run(nbr, ReorthUpdate<double>{n, vb, R.h, k.vp, ks});
        }
    }
    if (k.pre) {
        vcycle_enqueue(k.pre, k.vp, k.zn, gate, ks, fin, L, k.prec);
    } else {
        L.run(nb, Unprec<DIM>{g, k.vp, k.zn, gate, red_slot(m, 1)});
        launch_finalize(red_slot(m, 1).partials, nb, fin, ks, nullptr, gate, L);
    }
    if (k.defl) defl_project_z<DIM>(k, k.zn, L);
    if (k.rb) L.run<ReorthColumn, 64>(1, ReorthColumn{k.kmax, R.R, R.cs, R.sn, R.gv, R.h, ks});
    std::swap(k.v, k.vp);
    std::swap(k.z, k.zn);
    std::swap(k.w, k.wp);
}

// The graph of two iterations for this (psi, rhs, x, preconditioner) set.
template <int DIM>
static hipGraphExec_t iteration_graph(Ksolve k, hipStream_t s)
{
    gl_mesh *m = const_cast<gl_mesh *>(k.m);
    const uint64_t key[8] = {(uint64_t)(uintptr_t)k.psi, (uint64_t)(uintptr_t)k.rhs, (uint64_t)(uintptr_t)k.x,
                             k.pre ? k.pre->uid : 0,
                             (k.pre ? (uint64_t)(k.prec * 4096 + k.pre->opts.cycles) : 0) | ((uint64_t)k.defl << 40) |
                                 (k.pre ? (uint64_t)k.pre->pcg_m << 48 : 0),
                             (uint64_t)(uintptr_t)k.v, (uint64_t)(uintptr_t)k.rb ^ (uint64_t)(uintptr_t)k.rb32,
                             (uint64_t)k.kmax | ((uint64_t)(k.rb32 != nullptr) << 40)};
    for (auto &e : m->graphs)
        if (std::memcmp(e.key, key, sizeof(key)) == 0) return e.exec;
    hipGraph_t graph = nullptr;
    GLK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_iteration<DIM>(k, Launch{s});
        enqueue_iteration<DIM>(k, Launch{s});
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(s, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    GLK_HIP(hipStreamEndCapture(s, &graph));
    hipGraphExec_t exec;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GLK_HIP(e);
    if (m->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(m->graphs.front().exec);
        m->graphs.erase(m->graphs.begin());
    }
    GraphEntry ge;
    std::memcpy(ge.key, key, sizeof(key));
    ge.exec = exec;
    m->graphs.push_back(ge);
    return exec;
}

// The pending w / x update of the last iteration; k0 holds the buffer roles of
// device iteration iter0.
static void ksolve_finish(const Ksolve &k0, int iter0, const KrylovScalars &h, hipStream_t s)
{
    if (!h.wx_valid || h.iter < 1) return;
    const Ksolve kk = rotated(k0, h.iter - iter0);
    const int n = k0.m->g.n;
    k_minres_wx<<<blocks_for(n), kBlock, 0, s>>>(n, kk.zn, kk.w, kk.wp, kk.x,
                                                reinterpret_cast<const KrylovScalars *>(k0.m->kscal.get()));
    GLK_CHECK_LAUNCH();
}

// Iterate until the device flags stop (convergence, breakdown or max_iter),
// then apply the pending w / x update of the last iteration (finish), or
// leave it to a continuation of the same recurrence.  k holds the buffer
// roles of device iteration iter0 (the first one this call runs).
template <int DIM>
static void ksolve_iterate(Ksolve k, int max_iter, int poll, hipStream_t s, KrylovScalars &h,
                           bool finish = true, int iter0 = 0)
{
    const bool graphs = profiler().kernel == 0;
    hipGraphExec_t exec = graphs ? iteration_graph<DIM>(k, s) : nullptr;
    const Ksolve k0 = k;
    int launched = 0;
    for (;;) {
        read_scalars(k.m, &h, s);
        if (!h.running || launched >= max_iter) break;
        if (graphs) {
            for (int t = 0; t < std::max(1, poll / 2) && launched < max_iter; ++t, launched += 2)
                GLK_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int t = 0; t < poll && launched < max_iter; ++t, ++launched) enqueue_iteration<DIM>(k, Launch{s});
        }
    }
    if (finish) ksolve_finish(k0, iter0, h, s);
}

template <int DIM>
static void true_residual(const gl_mesh *m, const double2 *psi, const double2 *x, const double2 *b, bool defl,
                          hipStream_t s)
{
    const int nb = blocks_for(m->g.n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    if (defl) {
        // r = b - J x into the refinement's residual buffer (free once the solve has ended)
        double2 *r = m->work.get() + 10 * (size_t)m->g.n;
        k_residual_vec<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, link_tab<double>(m), r);
        k_defl_dots<DIM><<<nb, kBlock, 0, s>>>(g, psi, r, b, red_slot(m, 0), red_slot(m, 1));
        GLK_CHECK_LAUNCH();
        launch_finalize(red_slot(m, 0).partials, nb, FIN_STORE, nullptr, &ks->res_u_num, nullptr, s);
        launch_finalize(red_slot(m, 1).partials, nb, FIN_STORE, nullptr, &ks->res_u_den, nullptr, s);
        k_defl_norms<DIM><<<nb, kBlock, 0, s>>>(g, psi, r, b, ks, red_slot(m, 2), red_slot(m, 3));
        GLK_CHECK_LAUNCH();
        launch_finalize(red_slot(m, 2).partials, nb, FIN_RESNUM, ks, nullptr, nullptr, s);
        launch_finalize(red_slot(m, 3).partials, nb, FIN_RESDEN, ks, nullptr, nullptr, s);
        return;
    }
    k_true_residual<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, link_tab<double>(m), red_slot(m, 2), red_slot(m, 3));
    GLK_CHECK_LAUNCH();
    launch_finalize(red_slot(m, 2).partials, nb, FIN_RESNUM, ks, nullptr, nullptr, s);
    launch_finalize(red_slot(m, 3).partials, nb, FIN_RESDEN, ks, nullptr, nullptr, s);
}

template <int DIM>
static gl_status minres_run(const gl_mesh *m, const double2 *psi, const gl_precond *pre,
                            const double2 *b, double2 *x, const gl_krylov_opts &o,
                            gl_krylov_info *info, hipStream_t s)
{
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    const int poll = std::max(1, o.poll_every);
    KrylovScalars h;
    gl_status st = GL_OK;
    int iters = 0;
    bool converged = false;
    double eta0 = 0.0, res_est = 0.0;
    const bool fp64 = !pre || pre->opts.precision == GL_FP64;
    const bool defl = o.deflate != 0;
    if (o.reorth > 0) {
        // the basis of at most kmax vectors; each start measures the true
        // residual r = b - J x: the solve ends when its preconditioned norm
        // meets rtol, and restarts otherwise (a full basis, or rounding)
        const int kmax = o.reorth;
        gl_mesh *mm = const_cast<gl_mesh *>(m);
        ensure_reorth(mm, kmax, !fp64);
        // the recurrence's own x (zeroed by every start, never updated with a
        // basis) is scratch; the solution accumulates x += Z y in x
        double2 *r = m->work.get() + 10 * (size_t)n, *scratch = m->work.get() + 9 * (size_t)n;
        k_copy<<<nb, kBlock, 0, s>>>(n, r, b);
        k_zero<<<nb, kBlock, 0, s>>>(n, x);
        GLK_CHECK_LAUNCH();
        Ksolve k = make_ksolve(m, psi, pre, r, scratch, defl);
        k.rb = mm->rbasis.get();
        k.rb32 = fp64 ? nullptr : mm->rbasis32.get();
        k.rs = mm->rstate.get();
        k.kmax = kmax;
        double eta_first = 0.0, eta_prev = 0.0;
        for (int start = 0; start < kMaxStarts; ++start) {
            ksolve_init<DIM>(k, 0.0, 0, Launch{s});
            read_scalars(m, &h, s);
            if (h.status) { st = (gl_status)h.status; break; }
            if (eta_first == 0.0) eta_first = h.eta0;
            res_est = eta_first > 0 ? h.eta0 / eta_first : 0.0;
            if (h.eta0 <= o.rtol * eta_first || h.eta0 == 0.0) { converged = true; break; }
            if (iters >= o.max_iter) break;
            // a restart that has not halved the true residual: the system's
            // attainable accuracy is above rtol (near a singular J); stop
            if (start > 0 && h.eta0 > 0.5 * eta_prev) break;
            eta_prev = h.eta0;
            const int budget = o.max_iter - iters;
            k_ks_set<<<1, 1, 0, s>>>(ks, o.rtol * eta_first / h.eta0, budget);
            k_ks_init_running<<<1, 1, 0, s>>>(ks);
            ksolve_iterate<DIM>(k, budget, poll, s, h, false);
            const int cols = h.iter;
            iters += cols;
            reorth_combine(m, k.rs, kmax, cols, x, s);
            res_est = eta_first > 0 ? std::fabs(h.eta) / eta_first : 0.0;
            if (h.status) { st = (gl_status)h.status; break; }
            // also after convergence of the estimate: the next start measures
            // the true residual's norm and ends the solve, or restarts
            if (cols == 0) break;
            k_residual_vec<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, link_tab<double>(m), r);
            GLK_CHECK_LAUNCH();
        }
        eta0 = eta_first;
    } else if (fp64 && o.inner_rtol <= 0.0) {
        Ksolve k = make_ksolve(m, psi, pre, b, x, defl);
        ksolve_init<DIM>(k, o.rtol, o.max_iter, Launch{s});
        ksolve_iterate<DIM>(k, o.max_iter, poll, s, h);
        iters = h.iter;
        converged = h.converged;
        eta0 = h.eta0;
        res_est = h.eta0 > 0 ? std::fabs(h.eta) / h.eta0 : 0.0;
        if (h.status) st = (gl_status)h.status;
    } else {
        // iterative refinement in FP64 around MINRES solves, each to the inner
        // tolerance (FP32 V-cycle: a fixed rounded preconditioner, whose
        // rounding caps what one MINRES run attains), stopped on the true
        // residual in the preconditioner norm.  relax: each MINRES run applies
        // the FP64 V-cycle until its estimate reaches relax_rtol and the
        // reduced-precision one after that (the error of an operator
        // application may grow in inverse proportion to the residual in an
        // inexact Krylov method), to rtol in one run
        const bool relax = !fp64 && o.relax_rtol > 0.0;
        const double inner = o.inner_rtol > 0.0 ? o.inner_rtol : relax ? o.rtol : 1e-5;
        double2 *d = m->work.get() + 9 * (size_t)n, *r = m->work.get() + 10 * (size_t)n;
        k_copy<<<nb, kBlock, 0, s>>>(n, r, b);
        k_zero<<<nb, kBlock, 0, s>>>(n, x);
        Ksolve k = make_ksolve(m, psi, pre, r, d, defl);
        if (relax) k.prec = GL_FP64;
        double eta_first = 0.0;
        for (int outer = 0; outer < 64; ++outer) {
            ksolve_init<DIM>(k, inner, 0, Launch{s});
            read_scalars(m, &h, s);
            if (h.status) { st = (gl_status)h.status; break; }
            if (outer == 0) eta_first = h.eta0;
            res_est = eta_first > 0 ? h.eta0 / eta_first : 0.0;
            if (h.eta0 <= o.rtol * eta_first || h.eta0 == 0.0) { converged = true; break; }
            if (iters >= o.max_iter) break;
            const double rt = std::max(inner, o.rtol * eta_first / h.eta0);
            const int budget = o.max_iter - iters;
            const bool two = relax && rt < o.relax_rtol;
            k_ks_set<<<1, 1, 0, s>>>(ks, two ? o.relax_rtol : rt, budget);
            // re-open the gate: max_iter was 0 during the norm-only start
            k_ks_init_running<<<1, 1, 0, s>>>(ks);
            ksolve_iterate<DIM>(k, budget, poll, s, h, !two);
            if (two) {
                const int ia = h.iter;
                if (h.status == 0 && h.converged && h.gamma > 0.0 && ia < budget &&
                    std::fabs(h.eta) > rt * h.eta0) {
                    Ksolve kb = rotated(k, ia);
                    kb.prec = pre->opts.precision;
                    k_ks_resume<<<1, 1, 0, s>>>(ks, rt);
                    ksolve_iterate<DIM>(kb, budget - ia, poll, s, h, true, ia);
                } else {
                    ksolve_finish(k, 0, h, s);
                }
            }
            iters += h.iter;
            if (h.status) { st = (gl_status)h.status; break; }
            k_add<<<nb, kBlock, 0, s>>>(n, x, d);
            k_residual_vec<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, link_tab<double>(m), r);
            GLK_CHECK_LAUNCH();
        }
        eta0 = eta_first;
    }
    true_residual<DIM>(m, psi, x, b, defl, s);
    read_scalars(m, &h, s);
    if (info) {
        info->iterations = iters;
        info->converged = converged;
        info->eta0 = eta0;
        info->res_est = res_est;
        info->res_true = h.res_den > 0 ? std::sqrt(h.res_num / h.res_den) : 0.0;
    }
    if (st != GL_OK) return st;
    if (!std::isfinite(res_est) || !std::isfinite(h.res_num)) return GL_ERR_NONFINITE;
    return converged ? GL_OK : GL_ERR_NOT_CONVERGED;
}

// All Krylov work runs on the mesh's own stream (graph capture needs a
// non-default stream); it is ordered after, and before, the caller's stream.
gl_status minres_solve(const gl_mesh *m, const double2 *psi, const gl_precond *pre, const double2 *b,
                       double2 *x, const gl_krylov_opts &o, gl_krylov_info *info, hipStream_t s)
{
    GLK_HIP(hipEventRecord(m->ev_in, s));
    GLK_HIP(hipStreamWaitEvent(m->ws, m->ev_in, 0));
    gl_status st = GL_OK;
    with_dim(m->g, [&](auto D) { st = minres_run<decltype(D)::value>(m, psi, pre, b, x, o, info, m->ws); });
    GLK_HIP(hipEventRecord(m->ev_out, m->ws));
    GLK_HIP(hipStreamWaitEvent(s, m->ev_out, 0));
    return st;
}

static void check_krylov_opts(const gl_krylov_opts *o, const char *who)
{
    if (!o) fail(GL_ERR_INVALID_ARGUMENT, std::string(who) + ": NULL options");
    if (!(o->rtol >= 0.0) || o->max_iter < 0 || o->max_iter > 100000000 || o->poll_every < 1 ||
        !(o->inner_rtol >= 0.0 && o->inner_rtol < 1.0) || !(o->relax_rtol >= 0.0 && o->relax_rtol < 1.0) ||
        (o->deflate != 0 && o->deflate != 1) || o->reorth < 0 || o->reorth > 100000 ||
        (o->reorth > 0 && (o->inner_rtol > 0.0 || o->relax_rtol > 0.0)))
        fail(GL_ERR_INVALID_ARGUMENT, std::string(who) + ": invalid Krylov options");
}

}  // namespace glk

using namespace glk;

extern "C" {

gl_status gl_jacobian_solve(const gl_mesh *mesh, const void *psi, const gl_precond *pre, const void *b,
                            void *x, const gl_krylov_opts *opts, gl_krylov_info *info, gl_stream stream)
{
    gl_status rc = GL_OK;
    gl_status g = guarded([&] {
        if (!mesh || !psi || !b || !x) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: NULL argument");
        if (x == b || x == psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: x aliases an input");
        if (pre && pre->mesh != mesh) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: preconditioner of another mesh");
        check_krylov_opts(opts, "gl_jacobian_solve");
        rc = minres_solve(mesh, (const double2 *)psi, pre, (const double2 *)b, (double2 *)x, *opts, info,
                          as_stream(stream));
        if (rc != GL_OK) set_last_error(std::string("gl_jacobian_solve: ") + gl_status_string(rc));
    });
    return g != GL_OK ? g : rc;
}

gl_status gl_newton_solve(const gl_mesh *mesh, void *psi_inout, const gl_newton_opts *opts,
                          gl_precond **pre_inout, gl_newton_info *info, gl_stream stream)
{
    gl_status rc = GL_OK;
    gl_precond *pre = pre_inout ? *pre_inout : nullptr;
    gl_status g = guarded([&] {
        if (!mesh || !psi_inout || !opts) fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: NULL argument");
        if (pre && pre->mesh != mesh) fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: preconditioner of another mesh");
        check_krylov_opts(&opts->krylov, "gl_newton_solve");
        if (opts->max_steps < 0 || opts->max_steps > 63 || opts->fixed_steps < 0 || opts->fixed_steps > 63)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: steps must be in 0..63");
        if (opts->linesearch < 0 || opts->linesearch > 30)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: linesearch must be in 0..30");
        hipStream_t s = as_stream(stream);
        const int n = mesh->g.n;
        double2 *psi = (double2 *)psi_inout;
        double2 *r = mesh->work.get() + 7 * (size_t)n;
        double2 *dx = mesh->work.get() + 8 * (size_t)n;
        gl_newton_info ni;
        std::memset(&ni, 0, sizeof(ni));
        auto residual = [&]() {
            gl_residual_enqueue(mesh, psi, r, mesh->dscal.get(), s);
            GLK_HIP(hipMemcpyAsync(mesh->hscal, mesh->dscal.get(), sizeof(double), hipMemcpyDeviceToHost, s));
            GLK_HIP(hipStreamSynchronize(s));
            return std::sqrt(mesh->hscal[0]);
        };
        double res = residual();
        ni.res[0] = res;
        int k = 0;
        for (;;) {
            if (!std::isfinite(res)) { rc = GL_ERR_NONFINITE; break; }
            if (opts->fixed_steps > 0) { if (k == opts->fixed_steps) break; }
            else if (res < opts->tol || k == opts->max_steps) break;
            if (opts->use_precond) {
                gl_status ps = gl_precond_setup(mesh, psi, &opts->amg, &pre, stream);
                if (ps != GL_OK) fail(ps, gl_last_error());
                if (pre_inout) *pre_inout = pre;
            }
            gl_krylov_info ki;
            gl_status ks = minres_solve(mesh, psi, opts->use_precond ? pre : nullptr, r, dx, opts->krylov, &ki, s);
            if (ks != GL_OK && ks != GL_ERR_NOT_CONVERGED) { rc = ks; break; }
            Launch{s}.run(blocks_for(n), NewtonSub{n, psi, dx});
            GLK_CHECK_LAUNCH();
            ni.krylov_iters[k] = ki.iterations;
            double res_new = residual(), alpha = 1.0;
            // backtracking: psi = psi_k - alpha dpsi_k with alpha halved
            for (int h = 0; h < opts->linesearch && !newton_accepts(res_new, res, alpha); ++h) {
                Launch{s}.run(blocks_for(n), NewtonAxpy{n, 0.5 * alpha, psi, dx});
                GLK_CHECK_LAUNCH();
                alpha *= 0.5;
                res_new = residual();
            }
            ni.alpha[k] = alpha;
            ++k;
            res = res_new;
            ni.res[k] = res;
        }
        ni.steps = k;
        ni.converged = std::isfinite(res) && res < opts->tol;
        if (rc == GL_OK && opts->fixed_steps == 0 && !ni.converged) rc = GL_ERR_NOT_CONVERGED;
        if (rc != GL_OK) set_last_error(std::string("gl_newton_solve: ") + gl_status_string(rc));
        if (info) *info = ni;
    });
    if (!pre_inout) gl_precond_destroy(pre);
    return g != GL_OK ? g : rc;
}

}  // extern "C"

// ================================================================ batch ===
// Many instances in lock-step.  Every kernel of a MINRES iteration is a step
// struct; recording one iteration pair per instance and zipping the records of
// instances with identical launch shapes gives one batched dispatch per step
// (grid: work-groups x instances).  One captured graph holds the iteration
// pair of every group (groups on parallel branches); it is replayed between
// host convergence checks, and converged instances idle on their flags.
namespace glk {

struct BatchScalars {
    KrylovScalars ks;
    double res2;
};

__global__ void k_gather_scalars(const KrylovScalars *const *ks, const double *const *ds, BatchScalars *out,
                                 int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[i].ks = *ks[i];
    out[i].res2 = *ds[i];
}

__global__ void k_ks_stop(KrylovScalars *ks)
{
    ks->running = 0;
    ks->wx_valid = 0;
    ks->iter = 0;
    ks->status = 0;
}

// A zipped step sequence: the steps of the first member and, per step, the
// byte offset of the packed argument array (one struct per member).
struct Zip {
    std::vector<Step> steps;
    std::vector<size_t> off;
    int count = 0;
};

static bool same_shape(const std::vector<Step> &a, const std::vector<Step> &b)
{
    if (a.size() != b.size()) return false;
    for (size_t p = 0; p < a.size(); ++p)
        if (a[p].many != b[p].many || a[p].nbx != b[p].nbx || a[p].lds != b[p].lds ||
            a[p].args.size() != b[p].args.size())
            return false;
    return true;
}

// Append the packed arguments of recs (same shape) to buf; returns the zip.
static Zip zip_records(const std::vector<std::vector<Step>> &recs, std::vector<unsigned char> &buf)
{
    Zip z;
    z.count = (int)recs.size();
    z.steps = recs[0];
    for (auto &st : z.steps) st.args.clear();
    z.off.resize(recs[0].size());
    for (size_t p = 0; p < recs[0].size(); ++p) {
        size_t o = (buf.size() + 255) & ~(size_t)255;
        const size_t sz = recs[0][p].args.size();
        buf.resize(o + sz * recs.size());
        for (size_t i = 0; i < recs.size(); ++i) std::memcpy(buf.data() + o + i * sz, recs[i][p].args.data(), sz);
        z.off[p] = o;
    }
    return z;
}

static void launch_zip(const Zip &z, const unsigned char *dev, hipStream_t s)
{
    for (size_t p = 0; p < z.steps.size(); ++p)
        z.steps[p].many(dev + z.off[p], z.steps[p].nbx, z.count, z.steps[p].lds, s);
    GLK_CHECK_LAUNCH();
}

// A captured iteration pair for a subset of one group's instances.
struct GroupGraph {
    std::vector<uint64_t> key;
    std::vector<int> members;
    hipGraphExec_t exec = nullptr;
    DevBuf<unsigned char> args;
    int64_t dispatches = 0;
};

// Instances whose iteration pairs have the same launch shape; each group
// replays its graph on its own stream, so groups run concurrently.
struct BatchGroup {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<GroupGraph> cache;  // most recent last
};

}  // namespace glk

struct gl_batch {
    std::vector<gl_mesh *> meshes;
    std::vector<gl_precond *> pre;
    std::vector<gl_tiles> tiles;
    hipStream_t s = nullptr;
    std::vector<glk::BatchGroup> groups;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int64_t dispatches = 0;  // batched dispatches per iteration pair (all groups)
    int ngroups = 0;
    glk::DevBuf<const glk::KrylovScalars *> ks_ptr;
    glk::DevBuf<const double *> ds_ptr;
    glk::DevBuf<glk::BatchScalars> gathered;
    glk::BatchScalars *host_sc = nullptr;
    int *host_status = nullptr;  // per instance: the coarsest factor's failure flag of the last setup
    glk::DevBuf<unsigned char> init_args;
    unsigned char *staging = nullptr;
    size_t staging_cap = 0;
    int64_t graph_launches = 0;
    double seconds[3] = {0.0, 0.0, 0.0};  // residuals, preconditioner setups, Krylov solves
    int deflate = 0;                      // Krylov options of the running solve
    int reorth = 0;
    ~gl_batch();
};

namespace glk {

static KrylovScalars *kscal_of(const gl_mesh *m) { return reinterpret_cast<KrylovScalars *>(m->kscal.get()); }

static void batch_gather(gl_batch *B)
{
    const int N = (int)B->meshes.size();
    k_gather_scalars<<<blocks_for(N, 64), 64, 0, B->s>>>(B->ks_ptr.get(), B->ds_ptr.get(), B->gathered.get(), N);
    GLK_CHECK_LAUNCH();
    GLK_HIP(hipMemcpyAsync(B->host_sc, B->gathered.get(), sizeof(BatchScalars) * N, hipMemcpyDeviceToHost, B->s));
    GLK_HIP(hipStreamSynchronize(B->s));
}

// Krylov buffers of instance i: x = dx (W8) for a single run, d (W9) with rhs
// r_ref (W10) in refinement; otherwise rhs = GL (W7).
static Ksolve batch_ksolve(gl_batch *B, double2 *const *psi, int i, bool refine, bool use_pre)
{
    gl_mesh *m = B->meshes[i];
    const size_t n = (size_t)m->g.n;
    double2 *W = m->work.get();
    Ksolve k = make_ksolve(m, psi[i], use_pre ? B->pre[i] : nullptr, refine ? W + 10 * n : W + 7 * n,
                           refine ? W + 9 * n : W + 8 * n, B->deflate != 0);
    if (B->reorth > 0) {
        // the basis of the mesh (ensure_reorth before the solve); the
        // recurrence's x is the scratch vector, the solution W + 8 n
        k.rb = m->rbasis.get();
        k.rb32 = k.prec == GL_FP64 ? nullptr : m->rbasis32.get();
        k.rs = m->rstate.get();
        k.kmax = B->reorth;
    }
    return k;
}

// Group instances by the shape of a recorded sequence; rec(i, out) records one.
template <class Rec>
static void group_records(const std::vector<int> &members, Rec &&rec, std::vector<std::vector<int>> &groups,
                          std::vector<std::vector<std::vector<Step>>> &records)
{
    for (int i : members) {
        std::vector<Step> r;
        rec(i, r);
        size_t g = 0;
        for (; g < groups.size(); ++g)
            if (same_shape(records[g][0], r)) break;
        if (g == groups.size()) {
            groups.emplace_back();
            records.emplace_back();
        }
        groups[g].push_back(i);
        records[g].push_back(std::move(r));
    }
}

// Record, zip and run a sequence for the given instances directly (not captured).
template <class Rec>
static void batch_run_direct(gl_batch *B, const std::vector<int> &members, Rec &&rec)
{
    if (members.empty()) return;
    std::vector<std::vector<int>> groups;
    std::vector<std::vector<std::vector<Step>>> records;
    group_records(members, rec, groups, records);
    std::vector<unsigned char> buf;
    std::vector<Zip> zips;
    for (auto &r : records) zips.push_back(zip_records(r, buf));
    // the previous contents of the staging buffer were consumed by a copy that
    // completed before the last synchronisation of B->s
    if (buf.size() > B->staging_cap) {
        if (B->staging) (void)hipHostFree(B->staging);
        B->staging = nullptr;
        B->staging_cap = 0;
        GLK_HIP(hipHostMalloc(&B->staging, buf.size(), hipHostMallocDefault));
        B->staging_cap = buf.size();
    }
    if (buf.size() > B->init_args.count) B->init_args.alloc(buf.size());
    std::memcpy(B->staging, buf.data(), buf.size());
    GLK_HIP(hipMemcpyAsync(B->init_args.get(), B->staging, buf.size(), hipMemcpyHostToDevice, B->s));
    for (auto &z : zips) launch_zip(z, B->init_args.get(), B->s);
}

static void record_iterations(gl_batch *B, double2 *const *psi, int i, bool refine, bool use_pre,
                              std::vector<Step> &out)
{
    Launch L{nullptr, &out};
    Ksolve k = batch_ksolve(B, psi, i, refine, use_pre);
    with_dim(B->meshes[i]->g, [&](auto D) {
        enqueue_iteration<decltype(D)::value>(k, L);
        enqueue_iteration<decltype(D)::value>(k, L);
    });
}

static GroupGraph build_group_graph(gl_batch *B, BatchGroup &G, const std::vector<int> &members,
                                    const std::vector<std::vector<Step>> &recs, std::vector<uint64_t> key)
{
    GroupGraph gg;
    gg.key = std::move(key);
    gg.members = members;
    std::vector<unsigned char> buf;
    Zip z = zip_records(recs, buf);
    gg.dispatches = (int64_t)z.steps.size();
    gg.args.alloc(buf.size());
    GLK_HIP(hipMemcpy(gg.args.get(), buf.data(), buf.size(), hipMemcpyHostToDevice));
    hipGraph_t graph = nullptr;
    GLK_HIP(hipStreamBeginCapture(G.s, hipStreamCaptureModeThreadLocal));
    try {
        launch_zip(z, gg.args.get(), G.s);
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(G.s, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    GLK_HIP(hipStreamEndCapture(G.s, &graph));
    hipError_t e = hipGraphInstantiate(&gg.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GLK_HIP(e);
    return gg;
}

// Replay iteration pairs until no instance runs (or max_iter iterations).
// The running instances are grouped by launch shape; a group's graph covers
// a set of instances that contains its running ones and is rebuilt for the
// running subset once at most half of its instances still run (finished
// instances idle on their flags, but their work-groups are still launched).
static void batch_iterate(gl_batch *B, double2 *const *psi, bool refine, bool use_pre, int max_iter, int poll)
{
    const int N = (int)B->meshes.size();
    batch_gather(B);
    std::vector<int> running;
    for (int i = 0; i < N; ++i)
        if (B->host_sc[i].ks.running) running.push_back(i);
    if (running.empty()) return;
    // shapes of the running instances
    std::vector<std::vector<int>> gm;
    std::vector<std::vector<std::vector<Step>>> grec;
    group_records(running, [&](int i, std::vector<Step> &r) { record_iterations(B, psi, i, refine, use_pre, r); },
                  gm, grec);
    const int G = (int)gm.size();
    while ((int)B->groups.size() < G) {
        BatchGroup bg;
        GLK_HIP(hipStreamCreateWithFlags(&bg.s, hipStreamNonBlocking));
        GLK_HIP(hipEventCreateWithFlags(&bg.fork, hipEventDisableTiming));
        GLK_HIP(hipEventCreateWithFlags(&bg.join, hipEventDisableTiming));
        B->groups.push_back(std::move(bg));
    }
    auto key_of = [&](const std::vector<int> &mem) {
        std::vector<uint64_t> key{(uint64_t)refine, (uint64_t)use_pre, (uint64_t)B->deflate};
        for (int i : mem) {
            const gl_precond *p = use_pre ? B->pre[i] : nullptr;
            key.push_back((uint64_t)i);
            key.push_back((uint64_t)(uintptr_t)psi[i]);
            key.push_back(p ? p->uid : 0);
            key.push_back(p ? (uint64_t)(p->opts.precision * 4096 + p->opts.cycles) : 0);
            key.push_back(p ? (uint64_t)p->pcg_m : 0);
            if (B->reorth > 0) {
                const gl_mesh *m = B->meshes[i];
                key.push_back((uint64_t)B->reorth);
                key.push_back((uint64_t)(uintptr_t)m->rbasis.get());
                key.push_back((uint64_t)(uintptr_t)m->rbasis32.get());
                key.push_back((uint64_t)(uintptr_t)m->rstate.get());
            }
        }
        return key;
    };
    // graph of group g for the member subset `mem`
    auto graph_for = [&](int g, const std::vector<int> &mem) -> GroupGraph & {
        BatchGroup &bg = B->groups[g];
        std::vector<uint64_t> key = key_of(mem);
        for (size_t c = 0; c < bg.cache.size(); ++c)
            if (bg.cache[c].key == key) return bg.cache[c];
        std::vector<std::vector<Step>> recs;
        for (int i : mem)
            for (size_t k = 0; k < gm[g].size(); ++k)
                if (gm[g][k] == i) recs.push_back(grec[g][k]);
        if (bg.cache.size() >= 8) {
            (void)hipGraphExecDestroy(bg.cache.front().exec);
            bg.cache.erase(bg.cache.begin());
        }
        bg.cache.push_back(build_group_graph(B, bg, mem, recs, std::move(key)));
        return bg.cache.back();
    };
    std::vector<GroupGraph *> cur(G);
    int64_t disp = 0;
    for (int g = 0; g < G; ++g) {
        cur[g] = &graph_for(g, gm[g]);
        disp += cur[g]->dispatches;
    }
    B->dispatches = std::max(B->dispatches, disp);
    B->ngroups = std::max(B->ngroups, G);
    int launched = 0;
    for (;;) {
        // one window: every group's graph poll / 2 times on its own stream
        const int reps = std::max(1, poll / 2);
        for (int g = 0; g < G; ++g) {
            if (!cur[g]) continue;
            BatchGroup &bg = B->groups[g];
            GLK_HIP(hipEventRecord(bg.fork, B->s));
            GLK_HIP(hipStreamWaitEvent(bg.s, bg.fork, 0));
            for (int t = 0; t < reps && launched + 2 * t < max_iter; ++t) {
                GLK_HIP(hipGraphLaunch(cur[g]->exec, bg.s));
                ++B->graph_launches;
            }
            GLK_HIP(hipEventRecord(bg.join, bg.s));
            GLK_HIP(hipStreamWaitEvent(B->s, bg.join, 0));
        }
        launched += 2 * reps;
        batch_gather(B);
        if (launched >= max_iter) break;
        bool any = false;
        for (int g = 0; g < G; ++g) {
            if (!cur[g]) continue;
            std::vector<int> still;
            for (int i : cur[g]->members)
                if (B->host_sc[i].ks.running) still.push_back(i);
            if (still.empty()) {
                cur[g] = nullptr;
                continue;
            }
            any = true;
            if (2 * still.size() <= cur[g]->members.size()) cur[g] = &graph_for(g, still);
        }
        if (!any) break;
    }
}

// pending w / x update of instance i after its run stopped (roles by parity)
static void batch_flush(gl_batch *B, double2 *const *psi, int i, bool refine, bool use_pre)
{
    const KrylovScalars &h = B->host_sc[i].ks;
    if (!(h.wx_valid && h.iter >= 1)) return;
    Ksolve kk = batch_ksolve(B, psi, i, refine, use_pre);
    if (h.iter & 1) {
        std::swap(kk.v, kk.vp);
        std::swap(kk.z, kk.zn);
        std::swap(kk.w, kk.wp);
    }
    const int n = B->meshes[i]->g.n;
    k_minres_wx<<<blocks_for(n), kBlock, 0, B->s>>>(n, kk.zn, kk.w, kk.wp, kk.x, kscal_of(B->meshes[i]));
    GLK_CHECK_LAUNCH();
}

static void batch_init(gl_batch *B, double2 *const *psi, const std::vector<int> &members, bool refine,
                       bool use_pre, double rtol, int max_iter)
{
    batch_run_direct(B, members, [&](int i, std::vector<Step> &r) {
        Launch L{nullptr, &r};
        Ksolve k = batch_ksolve(B, psi, i, refine, use_pre);
        with_dim(B->meshes[i]->g, [&](auto D) { ksolve_init<decltype(D)::value>(k, rtol, max_iter, L); });
    });
}

// Solve J(psi_i) dx_i = GL(psi_i) for the instances in `act`; iters, st per instance.
static void batch_solve(gl_batch *B, double2 *const *psi, const std::vector<int> &act, const gl_newton_opts &o,
                        std::vector<int> &iters, std::vector<gl_status> &st)
{
    const gl_krylov_opts &ko = o.krylov;
    const bool use_pre = o.use_precond != 0;
    const bool fp32 = use_pre && o.amg.precision != GL_FP64;
    const bool refine = fp32 || ko.inner_rtol > 0.0;
    const int poll = std::max(1, ko.poll_every);
    for (int i : act) iters[i] = 0;
    if (B->reorth > 0) {
        // as a single reorthogonalised solve, instance by instance between
        // the batched runs: every start measures the true residual, every
        // run ends with x += Z y and r = b - J x
        for (int i : act) {
            gl_mesh *m = B->meshes[i];
            ensure_reorth(m, B->reorth, use_pre && B->pre[i]->opts.precision != GL_FP64);
            const int n = m->g.n;
            double2 *W = m->work.get();
            k_copy<<<blocks_for(n), kBlock, 0, B->s>>>(n, W + 10 * (size_t)n, W + 7 * (size_t)n);
            k_zero<<<blocks_for(n), kBlock, 0, B->s>>>(n, W + 8 * (size_t)n);
            GLK_CHECK_LAUNCH();
        }
        std::vector<double> eta_first(B->meshes.size(), 0.0), eta_prev(B->meshes.size(), 0.0);
        std::vector<int> solving = act;
        for (int outer = 0; outer < kMaxStarts && !solving.empty(); ++outer) {
            batch_init(B, psi, solving, true, use_pre, 0.0, 0);
            batch_gather(B);
            std::vector<int> next;
            for (int i : solving) {
                const KrylovScalars &h = B->host_sc[i].ks;
                if (h.status) { st[i] = (gl_status)h.status; continue; }
                if (outer == 0) eta_first[i] = h.eta0;
                if (h.eta0 <= ko.rtol * eta_first[i] || h.eta0 == 0.0) continue;  // converged
                if (iters[i] >= ko.max_iter) continue;
                if (outer > 0 && h.eta0 > 0.5 * eta_prev[i]) continue;  // stagnated, as a single solve
                eta_prev[i] = h.eta0;
                KrylovScalars *ks = kscal_of(B->meshes[i]);
                k_ks_set<<<1, 1, 0, B->s>>>(ks, ko.rtol * eta_first[i] / h.eta0, ko.max_iter - iters[i]);
                k_ks_init_running<<<1, 1, 0, B->s>>>(ks);
                GLK_CHECK_LAUNCH();
                next.push_back(i);
            }
            solving.swap(next);
            if (solving.empty()) break;
            batch_iterate(B, psi, true, use_pre, ko.max_iter, poll);
            std::vector<int> keep;
            for (int i : solving) {
                const KrylovScalars &h = B->host_sc[i].ks;
                if (h.status) { st[i] = (gl_status)h.status; continue; }
                const gl_mesh *m = B->meshes[i];
                const int n = m->g.n;
                double2 *W = m->work.get();
                iters[i] += h.iter;
                reorth_combine(m, m->rstate.get(), B->reorth, h.iter, W + 8 * (size_t)n, B->s);
                if (h.iter == 0) continue;
                const GeomT<double> g = geom_t<double>(m->g);
                with_dim(m->g, [&](auto D) {
                    k_residual_vec<decltype(D)::value><<<blocks_for(n), kBlock, 0, B->s>>>(
                        g, psi[i], W + 8 * (size_t)n, W + 7 * (size_t)n, link_tab<double>(m), W + 10 * (size_t)n);
                });
                GLK_CHECK_LAUNCH();
                keep.push_back(i);
            }
            solving.swap(keep);
        }
        return;
    }
    if (!refine) {
        batch_init(B, psi, act, false, use_pre, ko.rtol, ko.max_iter);
        batch_iterate(B, psi, false, use_pre, ko.max_iter, poll);
        for (int i : act) {
            const KrylovScalars &h = B->host_sc[i].ks;
            batch_flush(B, psi, i, false, use_pre);
            iters[i] = h.iter;
            if (h.status) st[i] = (gl_status)h.status;
        }
        return;
    }
    const double inner = ko.inner_rtol > 0.0 ? ko.inner_rtol : 1e-5;
    std::vector<double> eta_first(B->meshes.size(), 0.0);
    for (int i : act) {
        const gl_mesh *m = B->meshes[i];
        const int n = m->g.n;
        double2 *W = m->work.get();
        k_copy<<<blocks_for(n), kBlock, 0, B->s>>>(n, W + 10 * (size_t)n, W + 7 * (size_t)n);
        k_zero<<<blocks_for(n), kBlock, 0, B->s>>>(n, W + 8 * (size_t)n);
        GLK_CHECK_LAUNCH();
    }
    std::vector<int> solving = act;
    for (int outer = 0; outer < 64 && !solving.empty(); ++outer) {
        batch_init(B, psi, solving, true, use_pre, inner, 0);
        batch_gather(B);
        std::vector<int> next;
        for (int i : solving) {
            const KrylovScalars &h = B->host_sc[i].ks;
            if (h.status) { st[i] = (gl_status)h.status; continue; }
            if (outer == 0) eta_first[i] = h.eta0;
            if (h.eta0 <= ko.rtol * eta_first[i] || h.eta0 == 0.0) continue;  // converged
            if (iters[i] >= ko.max_iter) continue;
            const double rt = std::max(inner, ko.rtol * eta_first[i] / h.eta0);
            KrylovScalars *ks = kscal_of(B->meshes[i]);
            k_ks_set<<<1, 1, 0, B->s>>>(ks, rt, ko.max_iter - iters[i]);
            k_ks_init_running<<<1, 1, 0, B->s>>>(ks);
            GLK_CHECK_LAUNCH();
            next.push_back(i);
        }
        solving.swap(next);
        if (solving.empty()) break;
        batch_iterate(B, psi, true, use_pre, ko.max_iter, poll);
        for (int i : solving) {
            const KrylovScalars &h = B->host_sc[i].ks;
            batch_flush(B, psi, i, true, use_pre);
            iters[i] += h.iter;
            if (h.status) st[i] = (gl_status)h.status;
            const gl_mesh *m = B->meshes[i];
            const int n = m->g.n;
            double2 *W = m->work.get();
            k_add<<<blocks_for(n), kBlock, 0, B->s>>>(n, W + 8 * (size_t)n, W + 9 * (size_t)n);
            const GeomT<double> g = geom_t<double>(m->g);
            with_dim(m->g, [&](auto D) {
                k_residual_vec<decltype(D)::value><<<blocks_for(n), kBlock, 0, B->s>>>(
                    g, psi[i], W + 8 * (size_t)n, W + 7 * (size_t)n, link_tab<double>(m), W + 10 * (size_t)n);
            });
            GLK_CHECK_LAUNCH();
        }
        std::vector<int> keep;
        for (int i : solving)
            if (st[i] == GL_OK) keep.push_back(i);
        solving.swap(keep);
    }
}

// Numeric setups of the instances in `which`, whose handles exist: every
// kernel of every setup recorded and run as one batched dispatch per step and
// shape group, one synchronisation, then each instance's failure flag (as
// gl_precond_setup on an existing handle, instance by instance).
static void batch_setups(gl_batch *B, double2 *const *psi, const std::vector<int> &which, const gl_amg_opts &amg,
                         std::vector<gl_status> &st, std::vector<char> &active)
{
    std::vector<int> run;
    for (int i : which) {
        gl_precond *p = B->pre[i];
        if (amg.max_coarse != p->opts.max_coarse || amg.max_levels != p->opts.max_levels) {
            set_last_error("gl_batch_newton_solve: hierarchy limits differ from the handle's");
            st[i] = GL_ERR_INVALID_ARGUMENT;
            active[i] = 0;
            continue;
        }
        p->opts.precision = amg.precision;
        p->opts.cycles = amg.cycles;
        run.push_back(i);
    }
    if (run.empty()) return;
    batch_run_direct(B, run, [&](int i, std::vector<Step> &r) {
        precond_numeric_enqueue(B->pre[i], psi[i], Launch{nullptr, &r});
    });
    for (int i : run)
        GLK_HIP(hipMemcpyAsync(B->host_status + i, B->pre[i]->status.get(), sizeof(int), hipMemcpyDeviceToHost, B->s));
    GLK_HIP(hipStreamSynchronize(B->s));
    for (int i : run) {
        const gl_status r = guarded([&] { precond_numeric_finish(B->pre[i], B->host_status[i] != 0, B->s); });
        if (r != GL_OK) {
            st[i] = r;
            active[i] = 0;
        }
    }
}

static gl_status batch_newton(gl_batch *B, double2 *const *psi, const gl_newton_opts &o, gl_newton_info *infos)
{
    const int N = (int)B->meshes.size();
    std::vector<gl_newton_info> ni(N);
    std::memset(ni.data(), 0, sizeof(gl_newton_info) * N);
    std::vector<gl_status> st(N, GL_OK);
    std::vector<char> active(N, 1);
    std::vector<double> res(N, 0.0);
    std::vector<int> iters(N, 0);
    B->deflate = o.krylov.deflate;
    B->reorth = o.krylov.reorth;
    for (int i = 0; i < N; ++i) k_ks_stop<<<1, 1, 0, B->s>>>(kscal_of(B->meshes[i]));
    GLK_CHECK_LAUNCH();
    // Residual norms of the instances in `which` into out[i], batched: per
    // instance first the update `before` records (the Newton step or a
    // backtracking step; nothing for the start), then the residual.
    auto residuals_of = [&](const std::vector<int> &which, std::vector<double> &out, auto &&before) {
        batch_run_direct(B, which, [&](int i, std::vector<Step> &r) {
            const Launch L{nullptr, &r};
            gl_mesh *m = B->meshes[i];
            before(i, L);
            gl_residual_enqueue(m, psi[i], m->work.get() + 7 * (size_t)m->g.n, m->dscal.get(), L);
        });
        batch_gather(B);
        for (int i : which) out[i] = std::sqrt(B->host_sc[i].res2);
    };
    auto residuals = [&]() {
        std::vector<int> all;
        for (int i = 0; i < N; ++i)
            if (active[i]) all.push_back(i);
        residuals_of(all, res, [](int, const Launch &) {});
    };
    auto dpsi = [&](int i) { return B->meshes[i]->work.get() + 8 * (size_t)B->meshes[i]->g.n; };
    using clk = std::chrono::steady_clock;
    auto since = [](clk::time_point t) { return std::chrono::duration<double>(clk::now() - t).count(); };
    auto t0 = clk::now();
    residuals();
    B->seconds[0] += since(t0);
    for (int i = 0; i < N; ++i) ni[i].res[0] = res[i];
    for (int k = 0;; ++k) {
        std::vector<int> act;
        for (int i = 0; i < N; ++i) {
            if (!active[i]) continue;
            bool stop;
            if (!std::isfinite(res[i])) { st[i] = GL_ERR_NONFINITE; stop = true; }
            else if (o.fixed_steps > 0) stop = (k == o.fixed_steps);
            else stop = res[i] < o.tol || k == o.max_steps;
            if (stop) active[i] = 0;
            else act.push_back(i);
        }
        if (act.empty()) break;
        t0 = clk::now();
        if (o.use_precond) {
            // a new handle is built (and its tiles set) instance by instance;
            // the numeric setups of existing handles run batched
            std::vector<int> built;
            for (int i : act) {
                if (B->pre[i]) {
                    built.push_back(i);
                    continue;
                }
                gl_status ps = gl_precond_setup(B->meshes[i], psi[i], &o.amg, &B->pre[i], B->s);
                if (ps == GL_OK) ps = gl_precond_set_tiles(B->pre[i], &B->tiles[i]);
                if (ps != GL_OK) {
                    st[i] = ps;
                    active[i] = 0;
                }
            }
            batch_setups(B, psi, built, o.amg, st, active);
            std::vector<int> keep;
            for (int i : act)
                if (active[i]) keep.push_back(i);
            act.swap(keep);
            if (act.empty()) break;
        }
        B->seconds[1] += since(t0);
        t0 = clk::now();
        batch_solve(B, psi, act, o, iters, st);
        std::vector<int> upd;
        for (int i : act) {
            if (st[i] != GL_OK && st[i] != GL_ERR_NOT_CONVERGED) {
                active[i] = 0;
                continue;
            }
            st[i] = GL_OK;
            ni[i].krylov_iters[k] = iters[i];
            ni[i].steps = k + 1;
            upd.push_back(i);
        }
        B->seconds[2] += since(t0);
        t0 = clk::now();
        std::vector<double> res_new(N, 0.0), alpha(N, 1.0);
        // psi -= dpsi and the new residuals
        residuals_of(upd, res_new, [&](int i, const Launch &L) {
            const int n = B->meshes[i]->g.n;
            L.run(blocks_for(n), NewtonSub{n, psi[i], dpsi(i)});
        });
        // backtracking, the instances whose step does not reduce the residual
        // enough halve theirs together (as in gl_newton_solve)
        for (int h = 0; h < o.linesearch; ++h) {
            std::vector<int> back;
            for (int i : upd)
                if (!newton_accepts(res_new[i], res[i], alpha[i])) back.push_back(i);
            if (back.empty()) break;
            residuals_of(back, res_new, [&](int i, const Launch &L) {
                const int n = B->meshes[i]->g.n;
                L.run(blocks_for(n), NewtonAxpy{n, 0.5 * alpha[i], psi[i], dpsi(i)});
            });
            for (int i : back) alpha[i] *= 0.5;
        }
        B->seconds[0] += since(t0);
        for (int i : upd) {
            res[i] = res_new[i];
            ni[i].res[k + 1] = res[i];
            ni[i].alpha[k] = alpha[i];
        }
    }
    gl_status rc = GL_OK;
    for (int i = 0; i < N; ++i) {
        ni[i].converged = std::isfinite(ni[i].res[ni[i].steps]) && ni[i].res[ni[i].steps] < o.tol;
        if (rc == GL_OK && st[i] != GL_OK) rc = st[i];
    }
    if (rc == GL_OK && o.fixed_steps == 0)
        for (int i = 0; i < N; ++i)
            if (!ni[i].converged) rc = GL_ERR_NOT_CONVERGED;
    if (infos) std::memcpy(infos, ni.data(), sizeof(gl_newton_info) * N);
    return rc;
}

}  // namespace glk

gl_batch::~gl_batch()
{
    (void)hipDeviceSynchronize();
    for (auto &g : groups) {
        for (auto &gg : g.cache)
            if (gg.exec) (void)hipGraphExecDestroy(gg.exec);
        if (g.s) (void)hipStreamDestroy(g.s);
        if (g.fork) (void)hipEventDestroy(g.fork);
        if (g.join) (void)hipEventDestroy(g.join);
    }
    for (gl_precond *p : pre) gl_precond_destroy(p);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (s) (void)hipStreamDestroy(s);
    if (host_sc) (void)hipHostFree(host_sc);
    if (host_status) (void)hipHostFree(host_status);
    if (staging) (void)hipHostFree(staging);
}

extern "C" {

gl_status gl_batch_create(int count, gl_mesh *const *meshes, gl_batch **out)
{
    return guarded([&] {
        if (!meshes || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_create: NULL argument");
        if (count < 1 || count > 4096) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_create: count must be in 1..4096");
        for (int i = 0; i < count; ++i) {
            if (!meshes[i]) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_create: NULL mesh");
            for (int j = 0; j < i; ++j)
                if (meshes[j] == meshes[i]) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_create: repeated mesh");
        }
        gl_batch *B = new gl_batch();
        try {
            B->meshes.assign(meshes, meshes + count);
            B->pre.assign(count, nullptr);
            B->tiles.assign(count, gl_tiles{0, 0, 0, 0});
            GLK_HIP(hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking));
            GLK_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
            GLK_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
            std::vector<const KrylovScalars *> kp(count);
            std::vector<const double *> dp(count);
            for (int i = 0; i < count; ++i) {
                kp[i] = kscal_of(meshes[i]);
                dp[i] = meshes[i]->dscal.get();
            }
            B->ks_ptr.alloc(count);
            B->ds_ptr.alloc(count);
            B->gathered.alloc(count);
            GLK_HIP(hipMemcpy(B->ks_ptr.get(), kp.data(), sizeof(void *) * count, hipMemcpyHostToDevice));
            GLK_HIP(hipMemcpy(B->ds_ptr.get(), dp.data(), sizeof(void *) * count, hipMemcpyHostToDevice));
            GLK_HIP(hipHostMalloc(&B->host_sc, sizeof(BatchScalars) * count, hipHostMallocDefault));
            GLK_HIP(hipHostMalloc(&B->host_status, sizeof(int) * count, hipHostMallocDefault));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
    });
}

gl_status gl_batch_newton_solve(gl_batch *batch, void *const *psi_inout, const gl_newton_opts *opts,
                                gl_newton_info *infos, gl_stream stream)
{
    gl_status rc = GL_OK;
    gl_status g = guarded([&] {
        if (!batch || !psi_inout || !opts) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_newton_solve: NULL argument");
        const int N = (int)batch->meshes.size();
        for (int i = 0; i < N; ++i) {
            if (!psi_inout[i]) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_newton_solve: NULL psi");
            for (int j = 0; j < i; ++j)
                if (psi_inout[j] == psi_inout[i]) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_newton_solve: repeated psi");
        }
        check_krylov_opts(&opts->krylov, "gl_batch_newton_solve");
        if (opts->use_precond) check_amg_opts(&opts->amg, "gl_batch_newton_solve");
        if (opts->max_steps < 0 || opts->max_steps > 63 || opts->fixed_steps < 0 || opts->fixed_steps > 63)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_newton_solve: steps must be in 0..63");
        if (opts->linesearch < 0 || opts->linesearch > 30)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_newton_solve: linesearch must be in 0..30");
        if (profiler().kernel != 0) fail(GL_ERR_UNSUPPORTED, "gl_batch_newton_solve: not under gl_profile_start");
        hipStream_t s = as_stream(stream);
        batch->graph_launches = 0;
        batch->dispatches = 0;
        batch->ngroups = 0;
        for (double &v : batch->seconds) v = 0.0;
        GLK_HIP(hipEventRecord(batch->ev_in, s));
        GLK_HIP(hipStreamWaitEvent(batch->s, batch->ev_in, 0));
        rc = batch_newton(batch, reinterpret_cast<double2 *const *>(psi_inout), *opts, infos);
        GLK_HIP(hipEventRecord(batch->ev_out, batch->s));
        GLK_HIP(hipStreamWaitEvent(s, batch->ev_out, 0));
        if (rc != GL_OK) set_last_error(std::string("gl_batch_newton_solve: ") + gl_status_string(rc));
    });
    return g != GL_OK ? g : rc;
}

gl_status gl_batch_set_tiles(gl_batch *batch, int index, const gl_tiles *tiles)
{
    return guarded([&] {
        if (!batch || !tiles) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_set_tiles: NULL argument");
        const int N = (int)batch->meshes.size();
        if (index < -1 || index >= N) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_set_tiles: index");
        for (int i = 0; i < N; ++i) {
            if (index >= 0 && i != index) continue;
            if (batch->pre[i]) {
                gl_status r = gl_precond_set_tiles(batch->pre[i], tiles);
                if (r != GL_OK) fail(r, gl_last_error());
            } else if (tiles->lane_shift < -2 || tiles->lane_shift > 2 || tiles->bottom_rows < 0 ||
                       tiles->bottom_rows > 65536 || tiles->dense_rows < 0 || tiles->dense_rows > kMaxTail ||
                       tiles->l0_tiled < 0 || tiles->l0_tiled > 3) {
                fail(GL_ERR_INVALID_ARGUMENT,
                     "gl_batch_set_tiles: lane_shift in -2..2, bottom_rows in 0..65536, dense_rows in 0..8192, "
                     "l0_tiled 0..3");
            }
            batch->tiles[i] = *tiles;
        }
    });
}

gl_status gl_batch_stats(const gl_batch *batch, int64_t *graph_launches, int64_t *dispatches_per_graph,
                         int *groups, double *seconds)
{
    return guarded([&] {
        if (!batch) fail(GL_ERR_INVALID_ARGUMENT, "gl_batch_stats: NULL handle");
        if (graph_launches) *graph_launches = batch->graph_launches;
        if (dispatches_per_graph) *dispatches_per_graph = batch->dispatches;
        if (groups) *groups = batch->ngroups;
        if (seconds)
            for (int k = 0; k < 3; ++k) seconds[k] = batch->seconds[k];
    });
}

void gl_batch_destroy(gl_batch *batch) { delete batch; }

}  // extern "C"
