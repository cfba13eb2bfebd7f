// Internal declarations of libglnk: error handling, device buffers, complex
// arithmetic on double2 / float2, wave64 reductions and the deterministic
// last-block finalisation used by every fused dot product.
#pragma once

#include <cstring>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/glnk.h"

namespace glk {

// ------------------------------------------------------------ errors ----
struct Error {
    gl_status status;
    std::string msg;
};

[[noreturn]] void fail(gl_status s, const std::string &msg);
void set_last_error(const std::string &msg);

#define GLK_HIP(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::glk::fail(e_ == hipErrorOutOfMemory ? GL_ERR_OUT_OF_MEMORY : GL_ERR_HIP,   \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define GLK_CHECK_LAUNCH() GLK_HIP(hipGetLastError())

// Run body, translating internal errors into a gl_status (no exception ever
// crosses the C ABI).
template <class F>
gl_status guarded(F &&body)
{
    try {
        body();
        return GL_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return GL_ERR_OUT_OF_MEMORY;
    } catch (...) {
        set_last_error("unexpected internal error");
        return GL_ERR_HIP;
    }
}

// ---------------------------------------------------- device buffers ----
// Device memory of every handle comes from here: the caller's allocator when
// one is set (gl_set_allocator), hipMalloc otherwise.  A buffer remembers the
// release function of the allocator that gave it its memory.
struct Allocator {
    gl_alloc_fn alloc = nullptr;
    gl_free_fn release = nullptr;
    void *ctx = nullptr;
};
Allocator &allocator();

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t count = 0;
    gl_free_fn rel = nullptr;  // null: hipFree
    void *rctx = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t c) { alloc(c); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), count(o.count), rel(o.rel), rctx(o.rctx)
    {
        o.p = nullptr;
        o.count = 0;
        o.rel = nullptr;
        o.rctx = nullptr;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            count = o.count;
            rel = o.rel;
            rctx = o.rctx;
            o.p = nullptr;
            o.count = 0;
            o.rel = nullptr;
            o.rctx = nullptr;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t c)
    {
        release();
        if (!c) return;
        const Allocator &A = allocator();
        if (A.alloc) {
            p = static_cast<T *>(A.alloc(c * sizeof(T), nullptr, A.ctx));
            if (!p) fail(GL_ERR_OUT_OF_MEMORY, "the caller's allocator returned no memory");
            rel = A.release;
            rctx = A.ctx;
        } else {
            GLK_HIP(hipMalloc(&p, c * sizeof(T)));
        }
        count = c;
    }
    void release()
    {
        if (p) {
            if (rel) {
                // the memory goes back to an allocator that may hand it out
                // at once: nothing may still be using it
                (void)hipDeviceSynchronize();
                rel(p, nullptr, rctx);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        count = 0;
        rel = nullptr;
        rctx = nullptr;
    }
    T *get() const { return p; }
};

template <class T>
std::vector<T> to_host(const T *d, size_t count, hipStream_t s)
{
    std::vector<T> h(count);
    if (count) {
        GLK_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
        GLK_HIP(hipStreamSynchronize(s));
    }
    return h;
}

template <class T>
void to_device(T *d, const std::vector<T> &h, hipStream_t s)
{
    if (!h.empty()) {
        GLK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
        GLK_HIP(hipStreamSynchronize(s));
    }
}

// ------------------------------------------------- complex on device ----
template <class T> struct cx;
template <> struct cx<double> { using t = double2; };
template <> struct cx<float> { using t = float2; };
template <class T> using C = typename cx<T>::t;

template <class T> __host__ __device__ __forceinline__ C<T> mk(T re, T im) { C<T> r; r.x = re; r.y = im; return r; }
template <class V> __host__ __device__ __forceinline__ V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <class V> __host__ __device__ __forceinline__ V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
template <class V, class T> __host__ __device__ __forceinline__ V cscale(V a, T s) { a.x *= s; a.y *= s; return a; }
// a * b
template <class V> __host__ __device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// conj(a) * b
template <class V> __host__ __device__ __forceinline__ V cmulc(V a, V b)
{
    V r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.x * b.y - a.y * b.x;
    return r;
}
template <class V> __host__ __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
// Re(conj(a) b)
template <class V> __host__ __device__ __forceinline__ auto redot(V a, V b) { return a.x * b.x + a.y * b.y; }
template <class V> __host__ __device__ __forceinline__ auto cabs2(V a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double2 widen(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 widen(double2 a) { return a; }
template <class T> __device__ __forceinline__ C<T> narrow(double2 a);
template <> __device__ __forceinline__ double2 narrow<double>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 narrow<float>(double2 a) { return make_float2((float)a.x, (float)a.y); }
// complex value in the precision T, from either precision
template <class T, class V> __device__ __forceinline__ C<T> as_c(V a) { return narrow<T>(widen(a)); }

// ----------------------------------------------------- launch shapes ----
constexpr int kBlock = 256;
constexpr int kXcds = 8;

inline int blocks_for(int64_t n, int bs = kBlock) { return (int)((n + bs - 1) / bs); }

// Work-groups of one dispatch are handed to the 8 XCDs round-robin; renumber
// them so that each XCD walks one contiguous range of tiles, which keeps the
// neighbouring rows of a stencil in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    int q = nb / kXcds, r = nb % kXcds;
    int x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// ------------------------------------------------------- reductions ----
template <class T> __device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over the block (blockDim.x a multiple of 64, <= 1024); result valid in
// thread 0.  Fixed combination order, so the result is reproducible.
__device__ __forceinline__ double block_sum(double v, double *sm)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double r = 0.0;
    if (w == 0) {
        r = lane < nw ? sm[lane] : 0.0;
        r = wave_sum(r);
    }
    return r;
}

// Per-dispatch reduction slot: one partial per block.  A producer kernel
// stores its block sums; a one-work-group finalize kernel that follows in the
// same stream adds them in block order (fixed tree), so totals are
// reproducible and no counter is contended.
struct RedSlot {
    double *partials;
};

__device__ __forceinline__ void block_reduce_store(double part, RedSlot slot, double *sm, int bx)
{
    const double bs = block_sum(part, sm);
    if (threadIdx.x == 0) slot.partials[bx] = bs;
}

// ------------------------------------------------------- grid geometry --
// Tensor grid: nodes i = c0 + N0 (c1 + N1 c2).  |V_i| = prod_a e_a with
// e_a = h_a (interior) or h_a / 2 (boundary); the edge coefficient along axis
// a at node i is alpha_a = |V_i| s_a / h_a^2, s_a = 2 on a boundary of axis a
// (so alpha_a = prod_{b != a} e_b / h_a, the dual-facet area over the edge length).
// A 2D simplicial mesh (simplicial = true) keeps its operator per edge
// instead: the node adjacency in CSR (rp, ci: the other end of each edge at
// a node, ascending), kw = alpha_jk U_jk for the entry (row j, column k), so
// that K-hat_jk = -kw, the diagonal ks_j = K-hat_jj = sum of alpha at j, the
// volumes |V_j|, and phi_jk, the link phase at mu = 1 (U_jk = exp(-i mu phi)).
// Kernels templated on DIM take it as DIM == 0.
struct Geom {
    int dim;
    int N[3];
    int n;
    double h[3];
    double inv_h2[3];
    bool simplicial = false;
    const int *rp = nullptr, *ci = nullptr;
    const double2 *kw64 = nullptr;
    const float2 *kw32 = nullptr;
    const double *ks64 = nullptr, *vol64 = nullptr, *phi = nullptr;
    const float *ks32 = nullptr, *vol32 = nullptr;
};

template <class T>
struct GeomT {
    int N[3];
    int n;
    int hr, npair;  // red-black pairs: ceil(N0 / 2) per x-row, hr * n / N0 in all
    T h[3];
    T inv_h2[3];
    // simplicial meshes (DIM == 0)
    const int *rp, *ci;
    const C<T> *kw;
    const T *ks, *vol;
    const double *phi;
};

template <class T> inline GeomT<T> geom_t(const Geom &g)
{
    GeomT<T> r;
    for (int a = 0; a < 3; ++a) {
        r.N[a] = g.N[a];
        r.h[a] = (T)g.h[a];
        r.inv_h2[a] = (T)g.inv_h2[a];
    }
    r.n = g.n;
    r.hr = (g.N[0] + 1) / 2;
    r.npair = r.hr * (g.n / g.N[0]);
    r.rp = g.rp;
    r.ci = g.ci;
    r.phi = g.phi;
    if constexpr (std::is_same<T, double>::value) {
        r.kw = g.kw64;
        r.ks = g.ks64;
        r.vol = g.vol64;
    } else {
        r.kw = g.kw32;
        r.ks = g.ks32;
        r.vol = g.vol32;
    }
    return r;
}

// Calls f(std::integral_constant<int, K>) with the mesh kind: 0 for a
// simplicial mesh, else its dimension (2 or 3).
template <class F>
inline void with_dim(const Geom &g, F &&f)
{
    if (g.simplicial) f(std::integral_constant<int, 0>{});
    else if (g.dim == 2) f(std::integral_constant<int, 2>{});
    else f(std::integral_constant<int, 3>{});
}

// Link variables of the linear potential A(r) = M r as factor tables.  The
// phase of the forward edge along axis a leaving the node with coordinates c
// is h_a A_a(midpoint) = sum_b h_a M_ab mid_b(c_b), one term per coordinate,
// so U_a(c) = prod_b F_ab[c_b] with F_ab[j] = exp(-i h_a M_ab mid_b(j)) and
// mid_b(j) the midpoint's coordinate b (the node's, plus h_a / 2 along a).
// Table F_ab has N_b entries at f + off[a][b]; off[a][b] = -1 where M_ab is
// zero for every field strength (the diagonal of the uniform-field potential,
// components the field direction lacks, zeros of a given matrix), whose
// factor is 1.  The offsets depend on the grid and that pattern only, so a
// field change rewrites the values in place.
// Potentials that are not linear (the dipole) have no factor tables: then
// n_edge > 0 and f holds one link per node and axis, the forward edge along
// axis a leaving node i at f[a n_edge + i] (N0, N1: the grid's first two
// extents, to index the node).
template <class T>
struct LinkTab {
    const C<T> *__restrict__ f;
    int off[3][3];
    int n_edge;
    int N0, N1;
};

}  // namespace glk

// --------------------------------------------------- public handles ----
namespace glk {
struct GraphEntry {
    uint64_t key[8];
    hipGraphExec_t exec;
};
}  // namespace glk

struct gl_mesh {
    glk::Geom g;
    gl_grid_desc desc;
    double amat[9];
    glk::DevBuf<double2> F64;  // link factor tables (glk::LinkTab), FP64 and rounded to FP32
    glk::DevBuf<float2> F32;
    int foff[3][3] = {};
    bool per_edge = false;           // links stored per edge (non-linear potential)
    // simplicial meshes: topology (device), per-entry and per-node arrays
    glk::DevBuf<int> s_rp, s_ci;     // node adjacency (CSR without the diagonal)
    glk::DevBuf<int> s_erp, s_eo;    // per entry: its cells' other vertices (2D: one and -1; 3D: the opposite edge)
    glk::DevBuf<int> s_trp, s_tv;    // per node: the dim other vertices of each cell at the node
    glk::DevBuf<double> s_x;         // node coordinates (x, y, z), z = 0 in 2D
    glk::DevBuf<double> s_alpha, s_phi, s_ks64, s_vol64;
    glk::DevBuf<float> s_ks32, s_vol32;
    glk::DevBuf<double2> s_kw64;
    glk::DevBuf<float2> s_kw32;
    // reductions
    glk::DevBuf<double> partials;
    glk::DevBuf<double> dscal;       // device scalar results
    double *hscal = nullptr;         // pinned host mirror
    // Krylov workspace (allocated with the mesh so that solves allocate nothing)
    glk::DevBuf<double2> work;       // kWorkVecs * n
    // reorthogonalised solves (rcap vectors): Z in FP64 (x = Z y) then, for
    // FP64 V-cycles, V in FP64; for reduced-precision V-cycles the basis
    // the reorthogonalisation reads, Z in BF16 then V in FP32; the projected
    // matrix's state (R, rotations, g, coefficients, partials)
    glk::DevBuf<double2> rbasis;
    glk::DevBuf<float2> rbasis32;
    glk::DevBuf<double> rstate;
    int rcap = 0;
    bool rcap_v64 = false, rcap_32 = false;
    glk::DevBuf<char> kscal;         // Krylov scalar state
    hipStream_t ws = nullptr;        // Krylov work stream (graph capture)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<glk::GraphEntry> graphs;
    ~gl_mesh();
};

namespace glk {
template <class T> LinkTab<T> link_tab(const gl_mesh *m);
template <> inline LinkTab<double> link_tab<double>(const gl_mesh *m)
{
    LinkTab<double> t;
    t.f = m->F64.get();
    std::memcpy(t.off, m->foff, sizeof(t.off));
    t.n_edge = m->per_edge ? m->g.n : 0;
    t.N0 = m->g.N[0];
    t.N1 = m->g.N[1];
    return t;
}
template <> inline LinkTab<float> link_tab<float>(const gl_mesh *m)
{
    LinkTab<float> t;
    t.f = m->F32.get();
    std::memcpy(t.off, m->foff, sizeof(t.off));
    t.n_edge = m->per_edge ? m->g.n : 0;
    t.N0 = m->g.N[0];
    t.N1 = m->g.N[1];
    return t;
}
}  // namespace glk

namespace glk {
// ------------------------------------------------------------ profiling -
// Event-bracketed launches of one selected kernel (see gl_profile_start).
struct Profiler {
    int kernel = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    int64_t launches = 0;
    double bytes = 0.0;
};
Profiler &profiler();
enum ProfId {
    PROF_MINRES_JAPPLY = 1, PROF_L0_SWEEP = 2, PROF_L0_RESIDUAL = 3, PROF_L0_TRANSFER = 4,
    PROF_VUPDATE = 5, PROF_WX = 6, PROF_GL = 7, PROF_COARSE_SWEEP = 8
};

// count: kernel launches inside the bracket (consecutive launches of one
// class can share one event pair, so that the bracket adds no gaps between them)
template <class F>
void prof_launch(int id, double bytes, hipStream_t s, F &&launch, int count = 1)
{
    Profiler &p = profiler();
    if (p.kernel != id) {
        launch();
        return;
    }
    if (p.used == p.ev.size()) {
        hipEvent_t a, b;
        GLK_HIP(hipEventCreate(&a));
        GLK_HIP(hipEventCreate(&b));
        p.ev.emplace_back(a, b);
    }
    auto &e = p.ev[p.used++];
    GLK_HIP(hipEventRecord(e.first, s));
    launch();
    GLK_HIP(hipEventRecord(e.second, s));
    p.bytes += bytes;
    p.launches += count;
}


constexpr int kWorkVecs = 11;
constexpr int kMaxSlots = 4;  // independent reduction slots per mesh
RedSlot red_slot(const gl_mesh *m, int k);
hipStream_t as_stream(gl_stream s);
}  // namespace glk
