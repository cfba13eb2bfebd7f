// Grid construction, link variables, GL residual and Jacobian apply.
//   link variables : Sec. 3, U_jk = exp(-i int e.A), midpoint rule (exact for linear A)
//   GL residual    : eq. discr ginla, GL_i = (K psi)_i - psi_i (1 - |psi_i|^2)
//   Jacobian apply : discrete Jacobian of Sec. 3
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include <algorithm>
#include <array>
#include "amg.h"
#include "stencil.h"

namespace glk {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(gl_status s, const std::string &msg) { throw Error{s, msg}; }

hipStream_t as_stream(gl_stream s) { return reinterpret_cast<hipStream_t>(s); }

Profiler &profiler()
{
    static Profiler p;
    return p;
}

Allocator &allocator()
{
    static Allocator a;
    return a;
}

RedSlot red_slot(const gl_mesh *m, int k)
{
    const size_t per = m->partials.count / kMaxSlots;
    return RedSlot{m->partials.get() + per * k};
}

struct Finalize {
    const double *partials;
    int nparts, mode;
    KrylovScalars *ks;
    double *out;
    const int *gate;
    __device__ void operator()(int, int) const
    {
        // the (uniform) gate flag is loaded with the partials and checked
        // before the barrier of the block sum
        const bool go = gate == nullptr || *gate != 0;
        __shared__ double sm[1024 / 64];
        double s = 0.0;
        for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += partials[k];
        if (!go) return;
        s = block_sum(s, sm);
        if (threadIdx.x == 0) {
            if (mode == FIN_STORE) *out = s;
            else minres_finalize(ks, mode, s);
        }
    }
};

void launch_finalize(const double *partials, int nparts, int mode, KrylovScalars *ks, double *out,
                     const int *gate, const Launch &L)
{
    L.run<Finalize, 1024>(1, Finalize{partials, nparts, mode, ks, out, gate});
}

struct Potential {
    double m[9];
    double L[3];
};

// Factor tables of the link variables (LinkTab): entry j of F_ab is
// exp(-i h_a M_ab mid_b(j)), mid_b(j) = -L_b/2 + j h_b (+ h_a/2 when b = a),
// so that prod_b F_ab[c_b] = exp(-i h_a A_a(edge midpoint)) with A = M r.
// Grid (max_b N_b / kBlock, DIM * DIM): blockIdx.y = a DIM + b.
struct TableOffsets {
    int off[3][3];
};

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_link_tables(Geom g, Potential pot, TableOffsets t,
                                                        double2 *__restrict__ F64, float2 *__restrict__ F32)
{
    const int a = blockIdx.y / DIM, b = blockIdx.y % DIM;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (t.off[a][b] < 0 || j >= g.N[b]) return;
    double mid = -0.5 * pot.L[b] + (double)j * g.h[b];
    if (b == a) mid += 0.5 * g.h[a];
    const double ph = g.h[a] * pot.m[3 * a + b] * mid;
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double2 u = make_double2(cs, -sn);
    F64[t.off[a][b] + j] = u;
    F32[t.off[a][b] + j] = make_float2((float)u.x, (float)u.y);
}

// Links of the dipole potential mu A_d, A_d(r) = m x (r - x0) / |r - x0|^3, one
// per node and axis (the forward edge; 0 on the axis's upper face).  Along
// the edge from node k (a = x_k - x0) in unit direction t of length h, the
// integrand e . A_d = m . (a x e) / |a + s t|^3 has a constant numerator;
// with d the distance of x0 from the edge's line and s the coordinate along
// it (s0 = a . t at node k, s1 = s0 + h),
//   int e . A_d = m . (a x t) [s / (d^2 sqrt(d^2 + s^2))]_{s0}^{s1},
// evaluated without the division by d^2 when s0 and s1 have the same sign
// (the two terms then nearly cancel far from x0):
//   m . (a x t) (s1 - s0)(s1 + s0) / (r0 r1 (s1 r0 + s0 r1)), r = sqrt(d^2 + s^2).
struct Dipole {
    double mu;
    double m[3], x0[3];
    double lo[3];  // coordinate of node 0 along each axis
};

__device__ __forceinline__ double dipole_phase(const Dipole &D, const double xk[3], int axis, double h)
{
    double a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] = xk[c] - D.x0[c];
    // a x t with t the unit vector of `axis`
    double axt[3] = {0.0, 0.0, 0.0};
    if (axis == 0) { axt[1] = a[2]; axt[2] = -a[1]; }
    else if (axis == 1) { axt[0] = -a[2]; axt[2] = a[0]; }
    else { axt[0] = a[1]; axt[1] = -a[0]; }
    const double num = D.m[0] * axt[0] + D.m[1] * axt[1] + D.m[2] * axt[2];
    const double d2 = axt[0] * axt[0] + axt[1] * axt[1] + axt[2] * axt[2];
    if (!(d2 > 0.0)) return 0.0;  // the line passes through x0: no transverse part, num = 0
    const double s0 = a[axis], s1 = s0 + h;
    const double r0 = sqrt(d2 + s0 * s0), r1 = sqrt(d2 + s1 * s1);
    if (s0 * s1 > 0.0) return num * (s1 - s0) * (s1 + s0) / (r0 * r1 * (s1 * r0 + s0 * r1));
    return num / d2 * (s1 / r1 - s0 / r0);
}

// The same integral along the edge from xk to xj in any direction (unit t,
// length L): m . (a x t) [s / (d^2 sqrt(d^2 + s^2))] between s0 = a . t and
// s0 + L, d^2 = |a x t|^2, with the cancellation-free form when s0 and s1
// have the same sign.  D.mu is not applied.
__device__ __forceinline__ double dipole_phase_edge(const Dipole &D, const double xk[3], const double xj[3])
{
    double a[3], t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c] = xk[c] - D.x0[c];
        t[c] = xj[c] - xk[c];
    }
    const double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] /= L;
    const double axt[3] = {a[1] * t[2] - a[2] * t[1], a[2] * t[0] - a[0] * t[2], a[0] * t[1] - a[1] * t[0]};
    const double num = D.m[0] * axt[0] + D.m[1] * axt[1] + D.m[2] * axt[2];
    const double d2 = axt[0] * axt[0] + axt[1] * axt[1] + axt[2] * axt[2];
    if (!(d2 > 0.0)) return 0.0;
    const double s0 = a[0] * t[0] + a[1] * t[1] + a[2] * t[2], s1 = s0 + L;
    const double r0 = sqrt(d2 + s0 * s0), r1 = sqrt(d2 + s1 * s1);
    if (s0 * s1 > 0.0) return num * (s1 - s0) * (s1 + s0) / (r0 * r1 * (s1 * r0 + s0 * r1));
    return num / d2 * (s1 / r1 - s0 / r0);
}

// ------------------------------------------------- simplicial meshes ---
struct P3 {
    double x, y, z;
};

__device__ __forceinline__ P3 node_at(const double *__restrict__ x, int i)
{
    return P3{x[3 * i], x[3 * i + 1], x[3 * i + 2]};
}

__device__ __forceinline__ P3 sub(P3 a, P3 b) { return P3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ P3 cross(P3 a, P3 b)
{
    return P3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Triangle: 1/2 cot of the angle at o between the edges o -> p and o -> q
// (the Remark's edge coefficient of the edge pq in that triangle).
__device__ __forceinline__ double half_cot_at(P3 o, P3 p, P3 q)
{
    const P3 u = sub(p, o), v = sub(q, o);
    return 0.5 * dot(u, v) / fabs(u.x * v.y - u.y * v.x);
}

// Tetrahedron (p, q, u, v): the coefficient of the edge uv in it,
// |pq| cot(theta_pq) / 6 with theta_pq the dihedral angle at the opposite
// edge pq.  With n_u = (q - p) x (u - p) and n_v = (q - p) x (v - p),
// cot theta = n_u . n_v / |n_u x n_v| and |n_u x n_v| = |pq| |det(q - p,
// u - p, v - p)|, so the coefficient is n_u . n_v / (6 |det|).
__device__ __forceinline__ double dihedral_coef(P3 p, P3 q, P3 u, P3 v)
{
    const P3 e = sub(q, p), a = sub(u, p), b = sub(v, p);
    return dot(cross(e, a), cross(e, b)) / (6.0 * fabs(dot(e, cross(a, b))));
}

// Per adjacency entry (row j, column k): alpha_jk, the sum over the cells at
// the edge of its coefficient there (triangles: 1/2 cot of the opposite
// angle; tetrahedra: the dihedral form above; both the Corollary's
// coefficients), and phi_jk = int_{x_k}^{x_j} A_1 . dl, the link phase at
// unit field strength (linear A_1 = M r: exact at the midpoint; the dipole:
// dipole_phase_edge).  Both entries of an edge evaluate the same expressions
// with the lower-numbered node first, so alpha_jk = alpha_kj and
// phi_jk = -phi_kj hold exactly (K-hat stays exactly Hermitian whatever the
// rounding of the contracted products).
__global__ __launch_bounds__(kBlock) void k_simp_edges(int n, int dim, const int *__restrict__ rp,
                                                       const int *__restrict__ ci, const int *__restrict__ erp,
                                                       const int *__restrict__ eo, const double *__restrict__ x,
                                                       int dipole, Potential pot, Dipole D,
                                                       double *__restrict__ alpha, double *__restrict__ phi)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    for (int p = rp[j]; p < rp[j + 1]; ++p) {
        const int k = ci[p];
        const P3 lo = node_at(x, min(j, k)), hi = node_at(x, max(j, k));
        double al = 0.0;
        for (int t = erp[p]; t < erp[p + 1]; ++t)
            al += dim == 2 ? half_cot_at(node_at(x, eo[2 * t]), lo, hi)
                           : dihedral_coef(node_at(x, eo[2 * t]), node_at(x, eo[2 * t + 1]), lo, hi);
        alpha[p] = al;
        // the phase from lo to hi
        const double a3[3] = {lo.x, lo.y, lo.z}, b3[3] = {hi.x, hi.y, hi.z};
        double ph = 0.0;
        if (dipole) {
            ph = dipole_phase_edge(D, a3, b3);
        } else {
            const double mid[3] = {0.5 * (a3[0] + b3[0]), 0.5 * (a3[1] + b3[1]), 0.5 * (a3[2] + b3[2])};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                ph += (b3[a] - a3[a]) * (pot.m[3 * a] * mid[0] + pot.m[3 * a + 1] * mid[1] + pot.m[3 * a + 2] * mid[2]);
        }
        phi[p] = j > k ? ph : -ph;
    }
}

// Per node: K-hat_jj = sum of alpha over its edges, and |V_j| = sum over its
// cells T and the edges e of T at j of 1/(2 dim) alpha_e^T |e|^2, alpha_e^T
// the cell's own coefficient of e (triangle: others a, b; tetrahedron:
// others a, b, c, the edge ja opposite bc and so on).
__global__ __launch_bounds__(kBlock) void k_simp_nodes(int n, int dim, const int *__restrict__ rp,
                                                       const double *__restrict__ alpha, const int *__restrict__ trp,
                                                       const int *__restrict__ tv, const double *__restrict__ x,
                                                       double *ks64, float *ks32, double *vol64, float *vol32)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    double ks = 0.0;
    for (int p = rp[j]; p < rp[j + 1]; ++p) ks += alpha[p];
    const P3 xj = node_at(x, j);
    double v = 0.0;
    for (int q = trp[j]; q < trp[j + 1]; ++q) {
        if (dim == 2) {
            const P3 xa = node_at(x, tv[2 * q]), xb = node_at(x, tv[2 * q + 1]);
            const P3 da = sub(xj, xa), db = sub(xj, xb);
            v += 0.25 * (half_cot_at(xb, xj, xa) * dot(da, da) + half_cot_at(xa, xj, xb) * dot(db, db));
        } else {
            const P3 o[3] = {node_at(x, tv[3 * q]), node_at(x, tv[3 * q + 1]), node_at(x, tv[3 * q + 2])};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const P3 d = sub(xj, o[a]);
                v += dihedral_coef(o[(a + 1) % 3], o[(a + 2) % 3], xj, o[a]) * dot(d, d) / 6.0;
            }
        }
    }
    ks64[j] = ks;
    ks32[j] = (float)ks;
    vol64[j] = v;
    vol32[j] = (float)v;
}

// kw_jk = alpha_jk U_jk, U_jk = exp(-i mu phi_jk), per row j; the sine and
// cosine are taken of the edge's phase from its lower-numbered node, so
// U_kj = conj(U_jk) exactly.
__global__ __launch_bounds__(kBlock) void k_simp_links(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       double mu, const double *__restrict__ alpha,
                                                       const double *__restrict__ phi, double2 *__restrict__ kw64,
                                                       float2 *__restrict__ kw32)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    for (int p = rp[j]; p < rp[j + 1]; ++p) {
        const bool up = j > ci[p];
        double sn, cs;
        sincos(mu * (up ? phi[p] : -phi[p]), &sn, &cs);
        const double a = alpha[p];
        const double2 w = make_double2(a * cs, up ? -(a * sn) : a * sn);
        kw64[p] = w;
        kw32[p] = make_float2((float)w.x, (float)w.y);
    }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_link_dipole(Geom g, Dipole D, double2 *__restrict__ F64,
                                                        float2 *__restrict__ F32)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    double xk[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) xk[a] = D.lo[a] + c[a] * g.h[a];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double2 u = make_double2(0.0, 0.0);
        if (c[a] < g.N[a] - 1) {
            double sn, cs;
            sincos(D.mu * dipole_phase(D, xk, a, g.h[a]), &sn, &cs);
            u = make_double2(cs, -sn);
        }
        F64[(int64_t)a * g.n + i] = u;
        F32[(int64_t)a * g.n + i] = make_float2((float)u.x, (float)u.y);
    }
}

// the forward-edge links of one axis per node (0 on the axis's upper face)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_link_export(Geom g, LinkTab<double> U, int a, double2 *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    out[i] = c[a] < g.N[a] - 1 ? link_u<DIM, double>(U, a, c, c[a]) : make_double2(0.0, 0.0);
}

static void compute_amat(const gl_grid_desc &d, double mu, double out[9])
{
    if (d.potential == 1) {
        std::memcpy(out, d.a_matrix, sizeof(double) * 9);
        return;
    }
    if (d.potential == 2) {  // not linear: links per edge
        for (int k = 0; k < 9; ++k) out[k] = 0.0;
        return;
    }
    double b[3] = {d.b_dir[0], d.b_dir[1], d.b_dir[2]};
    double nb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    for (double &v : b) v /= nb;
    // A(r) = mu/2 (b x r)
    const double cr[9] = {0.0, -b[2], b[1], b[2], 0.0, -b[0], -b[1], b[0], 0.0};
    for (int k = 0; k < 9; ++k) out[k] = 0.5 * mu * cr[k];
}

static void launch_links(gl_mesh *m, hipStream_t s)
{
    if (m->g.simplicial) {
        // the matrix potential carries its strength in phi
        const double mu = m->desc.potential == 1 ? 1.0 : m->desc.mu;
        const int n = m->g.n;
        k_simp_links<<<blocks_for(n), kBlock, 0, s>>>(n, m->s_rp.get(), m->s_ci.get(), mu, m->s_alpha.get(),
                                                     m->s_phi.get(), m->s_kw64.get(), m->s_kw32.get());
        GLK_CHECK_LAUNCH();
        return;
    }
    if (m->per_edge) {
        Dipole D;
        D.mu = m->desc.mu;
        for (int a = 0; a < 3; ++a) {
            D.m[a] = m->desc.dipole_m[a];
            D.x0[a] = m->desc.dipole_x0[a];
            D.lo[a] = a < m->g.dim ? -0.5 * m->desc.side[a] : 0.0;
        }
        const int nb = blocks_for(m->g.n);
        if (m->g.dim == 2) k_link_dipole<2><<<nb, kBlock, 0, s>>>(m->g, D, m->F64.get(), m->F32.get());
        else k_link_dipole<3><<<nb, kBlock, 0, s>>>(m->g, D, m->F64.get(), m->F32.get());
        GLK_CHECK_LAUNCH();
        return;
    }
    Potential pot;
    std::memcpy(pot.m, m->amat, sizeof(pot.m));
    for (int a = 0; a < 3; ++a) pot.L[a] = m->desc.side[a];
    TableOffsets t;
    std::memcpy(t.off, m->foff, sizeof(t.off));
    const int dim = m->g.dim;
    const dim3 grid(blocks_for(std::max(m->g.N[0], std::max(m->g.N[1], m->g.N[2]))), dim * dim);
    if (dim == 2)
        k_link_tables<2><<<grid, kBlock, 0, s>>>(m->g, pot, t, m->F64.get(), m->F32.get());
    else
        k_link_tables<3><<<grid, kBlock, 0, s>>>(m->g, pot, t, m->F64.get(), m->F32.get());
    GLK_CHECK_LAUNCH();
}

// ------------------------------------------------------- GL residual ---
template <int DIM>
struct GlResidual {
    GeomT<double> g;
    const double2 *__restrict__ psi;
    LinkTab<double> U;
    double2 *__restrict__ out;
    RedSlot slot;
    __device__ void operator()(int bx, int nbx) const
    {
        __shared__ double sm[kBlock / 64];
        const int i = xcd_tile(bx, nbx) * kBlock + threadIdx.x;
        double part = 0.0;
        if (i < g.n) {
            int c[3];
            node_coords<DIM>(g.N, i, c);
            const double2 p = psi[i];
            double d, asum;
            const double2 kp = khat_node<DIM, double>(g, i, c, psi, U, p, d, asum);
            const double a2 = cabs2(p);
            const double2 r = csub(cscale(kp, 1.0 / d), cscale(p, 1.0 - a2));
            if (out) out[i] = r;
            part = d * cabs2(r);
        }
        block_reduce_store(part, slot, sm, bx);
    }
};

// residual into out (nullable) and its block partials in `slot`, then their
// fixed-order sum into dresult
static void residual_steps(const gl_mesh *m, const double2 *psi, double2 *out, RedSlot slot, double *dresult,
                           const Launch &L, bool profiled)
{
    const int nb = blocks_for(m->g.n);
    const GeomT<double> g = geom_t<double>(m->g);
    const LinkTab<double> U = link_tab<double>(m);
    const double bytes = 16.0 * m->g.n * (out ? 2 : 1);
    auto run = [&] {
        with_dim(m->g, [&](auto D) { L.run(nb, GlResidual<decltype(D)::value>{g, psi, U, out, slot}); });
    };
    if (profiled) prof_launch(PROF_GL, bytes, L, run);
    else run();
    launch_finalize(slot.partials, nb, FIN_STORE, nullptr, dresult, nullptr, L);
}

void gl_residual_enqueue(const gl_mesh *m, const double2 *psi, double2 *out, double *dresult,
                         hipStream_t s)
{
    residual_steps(m, psi, out, red_slot(m, 0), dresult, Launch{s}, true);
}

void gl_residual_enqueue(const gl_mesh *m, const double2 *psi, double2 *out, double *dresult,
                         const Launch &L)
{
    residual_steps(m, psi, out, red_slot(m, 0), dresult, L, false);
}

// ------------------------------------- GL residual without allocation ---
// gl_residual_noalloc keeps its block partial sums and its result in this
// file-scope device array instead of the mesh's reduction buffers.  Each GPU
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, once per device, and only
// that address is passed to kernels.
constexpr int kNoAllocParts = 1 << 16;  // block partials: n <= 2^16 * 256 nodes
constexpr int kNoAllocSlots = kNoAllocParts + 64;
static __device__ __align__(256) double scratch[kNoAllocSlots];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on first use).
static double *scratch_on_current_device()
{
    int dev = -1;
    GLK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(GL_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        GLK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(GL_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

// ---------------------------------------------------- Jacobian apply ---
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_jacobian(GeomT<double> g, const double2 *__restrict__ psi,
                                                     const double2 *__restrict__ phi,
                                                     const LinkTab<double> U,
                                                     double2 *__restrict__ out)
{
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    const double2 f = phi[i];
    double d, asum;
    const double2 kf = khat_node<DIM, double>(g, i, c, phi, U, f, d, asum);
    const double2 p = psi[i];
    const double2 p2 = cmul(p, p);
    const double2 r = cadd(cadd(cscale(kf, 1.0 / d), cscale(f, 2.0 * cabs2(p) - 1.0)),
                           cmul(p2, cconj(f)));
    out[i] = r;
}

void jacobian_enqueue(const gl_mesh *m, const double2 *psi, const double2 *phi, double2 *out,
                      hipStream_t s)
{
    const int nb = blocks_for(m->g.n);
    const GeomT<double> g = geom_t<double>(m->g);
    with_dim(m->g, [&](auto D) {
        k_jacobian<decltype(D)::value><<<nb, kBlock, 0, s>>>(g, psi, phi, link_tab<double>(m), out);
    });
    GLK_CHECK_LAUNCH();
}

// partial sums of Re and Im of sum |V_i| conj(u_i) v_i
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cdot(GeomT<double> g, const double2 *__restrict__ u,
                                                 const double2 *__restrict__ v, RedSlot sre, RedSlot sim)
{
    __shared__ double sm[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double pre = 0.0, pim = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 p = cmulc(u[i], v[i]);
        pre = d * p.x;
        pim = d * p.y;
    }
    block_reduce_store(pre, sre, sm, blockIdx.x);
    block_reduce_store(pim, sim, sm, blockIdx.x);
}

// out = psi + ratio (psi - e^{i chi} prev), e^{i chi} = ip / |ip|
__global__ __launch_bounds__(kBlock) void k_secant(int n, const double2 *__restrict__ psi,
                                                   const double2 *__restrict__ prev, const double *ip,
                                                   double ratio, double2 *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double a = hypot(ip[0], ip[1]);
    const double2 ph = a > 0.0 ? make_double2(ip[0] / a, ip[1] / a) : make_double2(1.0, 0.0);
    const double2 p = psi[i];
    out[i] = cadd(p, cscale(csub(p, cmul(ph, prev[i])), ratio));
}

void secant_enqueue(const gl_mesh *m, const double2 *psi, const double2 *prev, double ratio, double2 *out,
                    hipStream_t s)
{
    const int nb = blocks_for(m->g.n);
    const GeomT<double> g = geom_t<double>(m->g);
    with_dim(m->g, [&](auto D) {
        k_cdot<decltype(D)::value><<<nb, kBlock, 0, s>>>(g, prev, psi, red_slot(m, 2), red_slot(m, 3));
    });
    GLK_CHECK_LAUNCH();
    double *ip = m->dscal.get() + 2;
    launch_finalize(red_slot(m, 2).partials, nb, FIN_STORE, nullptr, ip, nullptr, s);
    launch_finalize(red_slot(m, 3).partials, nb, FIN_STORE, nullptr, ip + 1, nullptr, s);
    k_secant<<<nb, kBlock, 0, s>>>(m->g.n, psi, prev, ip, ratio, out);
    GLK_CHECK_LAUNCH();
}

// ----------------------------------------- parameter derivative of GL ---
// d GL(psi; mu) / d mu for A = mu A_1 (the continuation parameter of Sec. 4):
// the diagonal of K-hat does not depend on mu, and the link variable of the
// forward edge along axis a leaving node c is U = exp(-i mu phi1) with
// phi1 = h_a A_1,a(edge midpoint), so dU/dmu = -i phi1 U.  With the stencil
// of K-hat, (dK-hat/dmu x)_i = sum_a alpha_a [ i phi1(k) U_a[k] x_k
// - i phi1(i) conj(U_a[i]) x_j ] (k = i - s_a, j = i + s_a), and
// GL_mu = D^-1 (dK-hat/dmu) psi.
struct FieldDeriv {
    double m1[3][3];  // A_1 = m1 r
    double lo[3];     // coordinate of node 0 along each axis
};

template <int DIM>
__device__ __forceinline__ double edge_phase1(const GeomT<double> &g, const FieldDeriv &fd, int a, const int c[3],
                                              int ca)
{
    double ph = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const double mid = fd.lo[b] + (b == a ? ca : c[b]) * g.h[b] + (b == a ? 0.5 * g.h[a] : 0.0);
        ph += fd.m1[a][b] * mid;
    }
    return g.h[a] * ph;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_gl_dmu(GeomT<double> g, const double2 *__restrict__ psi,
                                                   const LinkTab<double> U, FieldDeriv fd,
                                                   double2 *__restrict__ out)
{
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= g.n) return;
    if constexpr (DIM == 0) {
        // dK-hat_jk / dmu = -alpha dU_jk/dmu = i phi_jk kw_jk (the diagonal does not depend on mu)
        double2 acc = make_double2(0.0, 0.0);
        for (int p = g.rp[i]; p < g.rp[i + 1]; ++p) {
            const double2 w = cmul(g.kw[p], psi[g.ci[p]]);
            const double ph = g.phi[p];
            acc.x -= ph * w.y;
            acc.y += ph * w.x;
        }
        out[i] = cscale(acc, 1.0 / g.vol[i]);
        return;
    }
    int c[3];
    node_coords<DIM>(g.N, i, c);
    double s[3];
    const double d = node_volume<DIM, double>(g, c, s);
    double2 acc = make_double2(0.0, 0.0);
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double al = d * s[a] * g.inv_h2[a];
        if (c[a] > 0) {
            const double ph = edge_phase1<DIM>(g, fd, a, c, c[a] - 1);
            const double2 w = cmul(link_u<DIM, double>(U, a, c, c[a] - 1), psi[i - stride]);
            // + al i ph w
            acc.x -= al * ph * w.y;
            acc.y += al * ph * w.x;
        }
        if (c[a] < g.N[a] - 1) {
            const double ph = edge_phase1<DIM>(g, fd, a, c, c[a]);
            const double2 w = cmulc(link_u<DIM, double>(U, a, c, c[a]), psi[i + stride]);
            // - al i ph w
            acc.x += al * ph * w.y;
            acc.y -= al * ph * w.x;
        }
        stride *= g.N[a];
    }
    out[i] = cscale(acc, 1.0 / d);
}

// out = a x + b y (out may alias x or y)
__global__ void k_axpby(int n, double a, const double2 *x, double b, const double2 *y, double2 *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double2 xi = x[i], yi = y[i];
        out[i] = make_double2(a * xi.x + b * yi.x, a * xi.y + b * yi.y);
    }
}

// y = D x
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_scale_volume(GeomT<double> g, const double2 *__restrict__ x,
                                                         double2 *__restrict__ y)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    double sf[3];
    y[i] = cscale(x[i], node_volume<DIM, double>(g, c, sf));
}

void scale_by_volume(const gl_mesh *m, const double2 *x, double2 *y, hipStream_t s)
{
    const GeomT<double> g = geom_t<double>(m->g);
    with_dim(m->g, [&](auto D) {
        k_scale_volume<decltype(D)::value><<<blocks_for(m->g.n), kBlock, 0, s>>>(g, x, y);
    });
    GLK_CHECK_LAUNCH();
}

}  // namespace glk

gl_mesh::~gl_mesh()
{
    if (ws) (void)hipStreamSynchronize(ws);
    for (auto &e : graphs) (void)hipGraphExecDestroy(e.exec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ws) (void)hipStreamDestroy(ws);
    if (hscal) (void)hipHostFree(hscal);
}

using namespace glk;

extern "C" {

const char *gl_status_string(gl_status s)
{
    switch (s) {
    case GL_OK: return "ok";
    case GL_ERR_INVALID_ARGUMENT: return "invalid argument";
    case GL_ERR_HIP: return "HIP runtime error";
    case GL_ERR_OUT_OF_MEMORY: return "out of device memory";
    case GL_ERR_NOT_CONVERGED: return "not converged";
    case GL_ERR_BREAKDOWN: return "Krylov breakdown";
    case GL_ERR_NONFINITE: return "non-finite value";
    case GL_ERR_SINGULAR: return "singular preconditioner matrix";
    case GL_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *gl_last_error(void) { return g_last_error.c_str(); }

gl_status gl_mesh_create_grid(const gl_grid_desc *desc, gl_stream stream, gl_mesh **out)
{
    return guarded([&] {
        if (!desc || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: NULL argument");
        *out = nullptr;
        if (desc->dim != 2 && desc->dim != 3)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: dim must be 2 or 3");
        if (desc->potential < 0 || desc->potential > 2)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: potential must be 0, 1 or 2");
        if (desc->potential == 2) {
            const double *mm = desc->dipole_m, *x0 = desc->dipole_x0;
            if (!(mm[0] * mm[0] + mm[1] * mm[1] + mm[2] * mm[2] > 0.0) || !std::isfinite(desc->mu) ||
                !std::isfinite(x0[0] + x0[1] + x0[2]) || !std::isfinite(mm[0] + mm[1] + mm[2]))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: dipole moment, position or mu");
        }
        int64_t n = 1;
        for (int a = 0; a < desc->dim; ++a) {
            if (desc->n_axis[a] < 2 || desc->n_axis[a] > (int64_t)1 << 30)
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: n_axis out of range");
            if (!(desc->side[a] > 0.0) || !std::isfinite(desc->side[a]))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: side must be positive");
            n *= desc->n_axis[a];
            if (n > ((int64_t)1 << 31) - 2)
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: too many nodes");
        }
        if (desc->potential == 0) {
            const double *b = desc->b_dir;
            if (!(b[0] * b[0] + b[1] * b[1] + b[2] * b[2] > 0.0))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: b_dir is zero");
            if (!std::isfinite(desc->mu)) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_grid: mu");
        }
        hipStream_t s = as_stream(stream);
        gl_mesh *m = new gl_mesh();
        try {
            m->desc = *desc;
            m->g.dim = desc->dim;
            m->g.n = (int)n;
            for (int a = 0; a < 3; ++a) {
                if (a < desc->dim) {
                    m->g.N[a] = (int)desc->n_axis[a];
                    m->g.h[a] = desc->side[a] / (double)(desc->n_axis[a] - 1);
                    m->g.inv_h2[a] = 1.0 / (m->g.h[a] * m->g.h[a]);
                } else {
                    m->g.N[a] = 1;
                    m->g.h[a] = 1.0;
                    m->g.inv_h2[a] = 1.0;
                }
            }
            compute_amat(*desc, desc->mu, m->amat);
            // tables only where M_ab can be nonzero (the pattern of M at mu = 1)
            double pat[9];
            compute_amat(*desc, 1.0, pat);
            int tot = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    m->foff[a][b] = -1;
                    if (a < desc->dim && b < desc->dim && pat[3 * a + b] != 0.0) {
                        m->foff[a][b] = tot;
                        tot += m->g.N[b];
                    }
                }
            if (desc->potential == 2) {
                m->per_edge = true;
                m->F64.alloc((size_t)desc->dim * n);
                m->F32.alloc((size_t)desc->dim * n);
            } else {
                m->F64.alloc(std::max(tot, 1));
                m->F32.alloc(std::max(tot, 1));
            }
            // one partial per block, or per level-0 tile of the smallest
            // tiled shape (16 x 16 nodes) on a 2D grid
            size_t per = (size_t)blocks_for(n);
            if (desc->dim == 2)
                per = std::max(per, (size_t)((desc->n_axis[0] + 15) / 16) * (size_t)((desc->n_axis[1] + 15) / 16));
            per += 64;
            m->partials.alloc(per * kMaxSlots);
            m->dscal.alloc(64);
            m->work.alloc((size_t)kWorkVecs * n);
            m->kscal.alloc(4096);
            GLK_HIP(hipHostMalloc(&m->hscal, 64 * sizeof(double), hipHostMallocDefault));
            GLK_HIP(hipStreamCreateWithFlags(&m->ws, hipStreamNonBlocking));
            GLK_HIP(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
            GLK_HIP(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
            GLK_HIP(hipMemsetAsync(m->dscal.get(), 0, 64 * sizeof(double), s));
            GLK_HIP(hipMemsetAsync(m->kscal.get(), 0, 4096, s));
            launch_links(m, s);
            GLK_HIP(hipStreamSynchronize(s));
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

gl_status gl_mesh_create_simplicial(const gl_simplicial_desc *desc, gl_stream stream, gl_mesh **out)
{
    return guarded([&] {
        if (!desc || !out || !desc->x || !desc->cells)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: NULL argument");
        *out = nullptr;
        const int dim = desc->dim, nv = dim + 1;
        if (dim != 2 && dim != 3) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: dim must be 2 or 3");
        const int64_t n = desc->n_nodes, nc = desc->n_cells;
        // every (cell, ordered vertex pair) is an int-indexed incidence
        if (n < nv || n > ((int64_t)1 << 31) - 2 || nc < 1 || nc > ((int64_t)1 << 31) || nc * nv * dim > ((int64_t)1 << 31) - 1)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: node or cell count out of range");
        if (desc->potential < 0 || desc->potential > 2)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: potential must be 0, 1 or 2");
        if (!std::isfinite(desc->mu)) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: mu");
        if (desc->potential == 0) {
            const double *b = desc->b_dir;
            if (!(b[0] * b[0] + b[1] * b[1] + b[2] * b[2] > 0.0))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: b_dir is zero");
        }
        if (desc->potential == 2) {
            const double *mm = desc->dipole_m, *x0 = desc->dipole_x0;
            if (!(mm[0] * mm[0] + mm[1] * mm[1] + mm[2] * mm[2] > 0.0) || !std::isfinite(x0[0] + x0[1] + x0[2]) ||
                !std::isfinite(mm[0] + mm[1] + mm[2]))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: dipole moment or position");
        }
        const int64_t *cell = desc->cells;
        std::vector<double> pts((size_t)3 * n, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < dim; ++c) {
                const double v = desc->x[dim * i + c];
                if (!std::isfinite(v)) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: coordinates");
                pts[(size_t)(3 * i + c)] = v;
            }
        // topology on the host: directed edge entries (row, column, the
        // cell's other vertices: the third one of a triangle, the opposite
        // edge of a tetrahedron), and the faces to check that no face lies in
        // more than two cells
        struct Ent {
            int r, c, o1, o2;
        };
        std::vector<Ent> ents;
        ents.reserve((size_t)(nc * nv * dim));
        std::vector<std::array<int, 3>> faces;
        faces.reserve((size_t)(nc * nv));
        std::vector<int> tdeg((size_t)n, 0);
        for (int64_t t = 0; t < nc; ++t) {
            int v[4];
            for (int e = 0; e < nv; ++e) {
                const int64_t x = cell[nv * t + e];
                if (x < 0 || x >= n) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: node index out of range");
                v[e] = (int)x;
            }
            double u[3][3];
            for (int e = 0; e < dim; ++e)
                for (int c = 0; c < 3; ++c) u[e][c] = pts[(size_t)(3 * v[e + 1] + c)] - pts[(size_t)(3 * v[0] + c)];
            const double det = dim == 2 ? u[0][0] * u[1][1] - u[0][1] * u[1][0]
                                        : u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
                                              u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
                                              u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
            if (!(std::fabs(det) > 0.0)) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: degenerate cell");
            for (int a = 0; a < nv; ++a) {
                ++tdeg[(size_t)v[a]];
                std::array<int, 3> f{-1, -1, -1};
                for (int b = 0, q = 0; b < nv; ++b)
                    if (b != a) f[(size_t)q++] = v[b];
                std::sort(f.begin(), f.begin() + dim);
                faces.push_back(f);
                for (int b = 0; b < nv; ++b) {
                    if (b == a) continue;
                    int o[2] = {-1, -1};
                    for (int c = 0, q = 0; c < nv; ++c)
                        if (c != a && c != b) o[q++] = v[c];
                    ents.push_back({v[a], v[b], o[0], o[1]});
                }
            }
        }
        std::sort(faces.begin(), faces.end());
        for (size_t q = 0; q + 2 < faces.size(); ++q)
            if (faces[q] == faces[q + 2])
                fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: a face in more than two cells");
        faces = {};
        std::sort(ents.begin(), ents.end(), [](const Ent &x, const Ent &y) {
            if (x.r != y.r) return x.r < y.r;
            if (x.c != y.c) return x.c < y.c;
            return x.o1 != y.o1 ? x.o1 < y.o1 : x.o2 < y.o2;
        });
        std::vector<int> rp((size_t)n + 1, 0), ci, erp(1, 0), eo;
        eo.reserve((size_t)2 * ents.size());
        for (size_t q = 0; q < ents.size();) {
            size_t e = q;
            while (e < ents.size() && ents[e].r == ents[q].r && ents[e].c == ents[q].c) {
                eo.push_back(ents[e].o1);
                eo.push_back(ents[e].o2);
                ++e;
            }
            ci.push_back(ents[q].c);
            erp.push_back((int)(eo.size() / 2));
            ++rp[(size_t)ents[q].r + 1];
            q = e;
        }
        ents = {};
        for (int64_t i = 0; i < n; ++i) {
            if (tdeg[(size_t)i] == 0) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_create_simplicial: a node in no cell");
            rp[(size_t)i + 1] += rp[(size_t)i];
        }
        // per node: the other dim vertices of each of its cells, in cell order
        std::vector<int> trp((size_t)n + 1, 0), tv((size_t)(nc * nv * dim)), fill((size_t)n, 0);
        for (int64_t i = 0; i < n; ++i) trp[(size_t)i + 1] = trp[(size_t)i] + tdeg[(size_t)i];
        for (int64_t t = 0; t < nc; ++t)
            for (int e = 0; e < nv; ++e) {
                const int j = (int)cell[nv * t + e];
                const size_t q = (size_t)trp[j] + fill[j]++;
                for (int b = 1; b < nv; ++b) tv[(size_t)dim * q + b - 1] = (int)cell[nv * t + (e + b) % nv];
            }
        const int nnz = (int)ci.size();
        hipStream_t s = as_stream(stream);
        gl_mesh *m = new gl_mesh();
        try {
            gl_grid_desc &d = m->desc;
            std::memset(&d, 0, sizeof(d));
            d.dim = dim;
            d.n_axis[0] = n;
            d.n_axis[1] = d.n_axis[2] = 1;
            d.potential = desc->potential;
            d.mu = desc->mu;
            for (int a = 0; a < 3; ++a) {
                d.b_dir[a] = desc->b_dir[a];
                d.dipole_m[a] = desc->dipole_m[a];
                d.dipole_x0[a] = desc->dipole_x0[a];
            }
            std::memcpy(d.a_matrix, desc->a_matrix, sizeof(d.a_matrix));
            m->g.dim = dim;
            m->g.n = (int)n;
            m->g.N[0] = (int)n;
            m->g.N[1] = m->g.N[2] = 1;
            for (int a = 0; a < 3; ++a) m->g.h[a] = m->g.inv_h2[a] = 1.0;
            compute_amat(d, d.mu, m->amat);
            m->F64.alloc(1);
            m->F32.alloc(1);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) m->foff[a][b] = -1;
            auto upload = [&](auto &buf, const auto &v) {
                buf.alloc(std::max<size_t>(1, v.size()));
                if (!v.empty())
                    GLK_HIP(hipMemcpyAsync(buf.get(), v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice, s));
            };
            upload(m->s_rp, rp);
            upload(m->s_ci, ci);
            upload(m->s_erp, erp);
            upload(m->s_eo, eo);
            upload(m->s_trp, trp);
            upload(m->s_tv, tv);
            upload(m->s_x, pts);
            m->s_alpha.alloc(std::max(1, nnz));
            m->s_phi.alloc(std::max(1, nnz));
            m->s_kw64.alloc(std::max(1, nnz));
            m->s_kw32.alloc(std::max(1, nnz));
            m->s_ks64.alloc(n);
            m->s_ks32.alloc(n);
            m->s_vol64.alloc(n);
            m->s_vol32.alloc(n);
            Geom &g = m->g;
            g.simplicial = true;
            g.rp = m->s_rp.get();
            g.ci = m->s_ci.get();
            g.kw64 = m->s_kw64.get();
            g.kw32 = m->s_kw32.get();
            g.ks64 = m->s_ks64.get();
            g.ks32 = m->s_ks32.get();
            g.vol64 = m->s_vol64.get();
            g.vol32 = m->s_vol32.get();
            g.phi = m->s_phi.get();
            m->partials.alloc(((size_t)blocks_for(n) + 64) * kMaxSlots);
            m->dscal.alloc(64);
            m->work.alloc((size_t)kWorkVecs * n);
            m->kscal.alloc(4096);
            GLK_HIP(hipHostMalloc(&m->hscal, 64 * sizeof(double), hipHostMallocDefault));
            GLK_HIP(hipStreamCreateWithFlags(&m->ws, hipStreamNonBlocking));
            GLK_HIP(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
            GLK_HIP(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
            GLK_HIP(hipMemsetAsync(m->dscal.get(), 0, 64 * sizeof(double), s));
            GLK_HIP(hipMemsetAsync(m->kscal.get(), 0, 4096, s));
            // the edge phases at unit strength: the field direction's matrix, the
            // given matrix, or the dipole
            Potential pot;
            compute_amat(d, 1.0, pot.m);
            for (int a = 0; a < 3; ++a) pot.L[a] = 0.0;
            Dipole D;
            D.mu = 1.0;
            for (int a = 0; a < 3; ++a) {
                D.m[a] = d.dipole_m[a];
                D.x0[a] = d.dipole_x0[a];
                D.lo[a] = 0.0;
            }
            const int nb = blocks_for(n);
            k_simp_edges<<<nb, kBlock, 0, s>>>((int)n, dim, m->s_rp.get(), m->s_ci.get(), m->s_erp.get(),
                                               m->s_eo.get(), m->s_x.get(), d.potential == 2, pot, D,
                                               m->s_alpha.get(), m->s_phi.get());
            k_simp_nodes<<<nb, kBlock, 0, s>>>((int)n, dim, m->s_rp.get(), m->s_alpha.get(), m->s_trp.get(),
                                               m->s_tv.get(), m->s_x.get(), m->s_ks64.get(), m->s_ks32.get(),
                                               m->s_vol64.get(), m->s_vol32.get());
            GLK_CHECK_LAUNCH();
            launch_links(m, s);
            GLK_HIP(hipStreamSynchronize(s));
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

gl_status gl_mesh_set_field(gl_mesh *mesh, double mu, gl_stream stream)
{
    return guarded([&] {
        if (!mesh) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_set_field: NULL mesh");
        if (mesh->desc.potential == 1)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_set_field: mesh has a matrix potential");
        if (!std::isfinite(mu)) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_set_field: mu");
        mesh->desc.mu = mu;
        compute_amat(mesh->desc, mu, mesh->amat);
        launch_links(mesh, as_stream(stream));
    });
}

gl_status gl_mesh_num_nodes(const gl_mesh *mesh, int64_t *n)
{
    return guarded([&] {
        if (!mesh || !n) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_num_nodes: NULL argument");
        *n = mesh->g.n;
    });
}

gl_status gl_mesh_export_links(const gl_mesh *mesh, int axis, void *host_out)
{
    return guarded([&] {
        if (!mesh || !host_out) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_export_links: NULL argument");
        if (mesh->g.simplicial) fail(GL_ERR_UNSUPPORTED, "gl_mesh_export_links: a simplicial mesh has no axes");
        if (axis < 0 || axis >= mesh->g.dim) fail(GL_ERR_INVALID_ARGUMENT, "gl_mesh_export_links: axis");
        GLK_HIP(hipDeviceSynchronize());
        // staged in the first Krylov vector (no solve is in flight after the synchronisation)
        double2 *stage = mesh->work.get();
        const int nb = blocks_for(mesh->g.n);
        if (mesh->g.dim == 2)
            k_link_export<2><<<nb, kBlock>>>(mesh->g, link_tab<double>(mesh), axis, stage);
        else
            k_link_export<3><<<nb, kBlock>>>(mesh->g, link_tab<double>(mesh), axis, stage);
        GLK_CHECK_LAUNCH();
        GLK_HIP(hipMemcpy(host_out, stage, sizeof(double2) * (size_t)mesh->g.n, hipMemcpyDeviceToHost));
    });
}

void gl_mesh_destroy(gl_mesh *mesh) { delete mesh; }

gl_status gl_residual(const gl_mesh *mesh, const void *psi, void *out, double *norm_D, gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual: NULL mesh or psi");
        if (out == psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual: out aliases psi");
        hipStream_t s = as_stream(stream);
        gl_residual_enqueue(mesh, (const double2 *)psi, (double2 *)out, mesh->dscal.get(), s);
        if (norm_D) {
            GLK_HIP(hipMemcpyAsync(mesh->hscal, mesh->dscal.get(), sizeof(double), hipMemcpyDeviceToHost, s));
            GLK_HIP(hipStreamSynchronize(s));
            *norm_D = std::sqrt(mesh->hscal[0]);
        }
    });
}

gl_status gl_residual_noalloc(const gl_mesh *mesh, const void *psi, void *out, double *norm_D,
                              gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual_noalloc: NULL mesh or psi");
        if (out == psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual_noalloc: out aliases psi");
        const int nb = blocks_for(mesh->g.n);
        if (nb > kNoAllocParts)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_residual_noalloc: more than " +
                                              std::to_string((int64_t)kNoAllocParts * kBlock) + " nodes");
        double *sc = scratch_on_current_device();
        hipStream_t s = as_stream(stream);
        // every partial is written by its block and the result by the
        // finalisation, so nothing has to be cleared between calls
        double *res = sc + kNoAllocParts;
        residual_steps(mesh, (const double2 *)psi, (double2 *)out, RedSlot{sc}, res, Launch{s}, false);
        if (norm_D) {
            double v = 0.0;
            GLK_HIP(hipMemcpyAsync(&v, res, sizeof(double), hipMemcpyDeviceToHost, s));
            GLK_HIP(hipStreamSynchronize(s));
            *norm_D = std::sqrt(v);
        }
    });
}

gl_status gl_secant_predict(const gl_mesh *mesh, const void *psi_m, const void *psi_prev, double ratio,
                            void *out, gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi_m || !psi_prev || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_secant_predict: NULL argument");
        if (out == psi_m || out == psi_prev) fail(GL_ERR_INVALID_ARGUMENT, "gl_secant_predict: out aliases an input");
        if (!std::isfinite(ratio)) fail(GL_ERR_INVALID_ARGUMENT, "gl_secant_predict: ratio");
        secant_enqueue(mesh, (const double2 *)psi_m, (const double2 *)psi_prev, ratio, (double2 *)out,
                       as_stream(stream));
    });
}

gl_status gl_set_allocator(gl_alloc_fn alloc, gl_free_fn release, void *ctx)
{
    return guarded([&] {
        if ((alloc == nullptr) != (release == nullptr))
            fail(GL_ERR_INVALID_ARGUMENT, "gl_set_allocator: set both functions or neither");
        Allocator &a = allocator();
        a.alloc = alloc;
        a.release = release;
        a.ctx = alloc ? ctx : nullptr;
    });
}

gl_status gl_residual_dmu(const gl_mesh *mesh, const void *psi, void *out, gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual_dmu: NULL argument");
        if (out == psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_residual_dmu: out aliases psi");
        if (mesh->desc.potential == 1)
            fail(GL_ERR_UNSUPPORTED, "gl_residual_dmu: the mesh has no field-strength parameter");
        if (mesh->desc.potential == 2 && !mesh->g.simplicial)
            fail(GL_ERR_UNSUPPORTED, "gl_residual_dmu: the dipole potential on a grid");
        FieldDeriv fd;
        double m1[9];
        compute_amat(mesh->desc, 1.0, m1);
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) fd.m1[a][b] = m1[3 * a + b];
            fd.lo[a] = -0.5 * mesh->g.h[a] * (mesh->g.N[a] - 1);
        }
        const int nb = blocks_for(mesh->g.n);
        const GeomT<double> g = geom_t<double>(mesh->g);
        hipStream_t s = as_stream(stream);
        with_dim(mesh->g, [&](auto D) {
            k_gl_dmu<decltype(D)::value><<<nb, kBlock, 0, s>>>(g, (const double2 *)psi, link_tab<double>(mesh), fd,
                                                               (double2 *)out);
        });
        GLK_CHECK_LAUNCH();
    });
}

gl_status gl_inner(const gl_mesh *mesh, const void *u, const void *v, double *out, gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !u || !v || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_inner: NULL argument");
        const int nb = blocks_for(mesh->g.n);
        const GeomT<double> g = geom_t<double>(mesh->g);
        hipStream_t s = as_stream(stream);
        with_dim(mesh->g, [&](auto D) {
            k_cdot<decltype(D)::value><<<nb, kBlock, 0, s>>>(g, (const double2 *)u, (const double2 *)v,
                                                             red_slot(mesh, 2), red_slot(mesh, 3));
        });
        GLK_CHECK_LAUNCH();
        launch_finalize(red_slot(mesh, 2).partials, nb, FIN_STORE, nullptr, mesh->dscal.get() + 6, nullptr, s);
        GLK_HIP(hipMemcpyAsync(mesh->hscal + 6, mesh->dscal.get() + 6, sizeof(double), hipMemcpyDeviceToHost, s));
        GLK_HIP(hipStreamSynchronize(s));
        *out = mesh->hscal[6];
    });
}

gl_status gl_axpby(const gl_mesh *mesh, double a, const void *x, double b, const void *y, void *out,
                   gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !x || !y || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_axpby: NULL argument");
        if (!std::isfinite(a) || !std::isfinite(b)) fail(GL_ERR_INVALID_ARGUMENT, "gl_axpby: coefficient");
        const int n = mesh->g.n;
        k_axpby<<<blocks_for(n), kBlock, 0, as_stream(stream)>>>(n, a, (const double2 *)x, b, (const double2 *)y,
                                                                 (double2 *)out);
        GLK_CHECK_LAUNCH();
    });
}

gl_status gl_profile_start(int kernel_id)
{
    return guarded([&] {
        if (kernel_id < 1 || kernel_id > 8) fail(GL_ERR_INVALID_ARGUMENT, "gl_profile_start: kernel id");
        Profiler &p = profiler();
        p.kernel = kernel_id;
        p.used = 0;
        p.launches = 0;
        p.bytes = 0.0;
    });
}

gl_status gl_profile_stop(double *ms_total, double *bytes_total, int64_t *launches)
{
    return guarded([&] {
        Profiler &p = profiler();
        GLK_HIP(hipDeviceSynchronize());
        double ms = 0.0;
        for (size_t k = 0; k < p.used; ++k) {
            float t = 0.f;
            GLK_HIP(hipEventElapsedTime(&t, p.ev[k].first, p.ev[k].second));
            ms += t;
        }
        if (ms_total) *ms_total = ms;
        if (bytes_total) *bytes_total = p.bytes;
        if (launches) *launches = p.launches;
        p.kernel = 0;
        p.used = 0;
        p.launches = 0;
        p.bytes = 0.0;
    });
}

gl_status gl_jacobian_apply(const gl_mesh *mesh, const void *psi, const void *phi, void *out,
                            gl_stream stream)
{
    return guarded([&] {
        if (!mesh || !psi || !phi || !out) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_apply: NULL argument");
        if (out == psi || out == phi) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_apply: out aliases an input");
        jacobian_enqueue(mesh, (const double2 *)psi, (const double2 *)phi, (double2 *)out, as_stream(stream));
    });
}

}  // extern "C"
