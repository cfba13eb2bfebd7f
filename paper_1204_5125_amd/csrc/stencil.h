// Node-centred application of K-hat on the tensor grid (discrete kinetic
// energy operator, Sec. 3): for node i and each axis a with lower neighbour
// k = i - s_a and upper neighbour j = i + s_a,
//   (K-hat x)_i = sum_a alpha_a [ (x_i - U_a[k] x_k) + (x_i - conj(U_a[i]) x_j) ]
// where U_a[k] is the link variable of the forward edge leaving node k along
// axis a, a product of factor-table entries (LinkTab).  |V_i| and alpha_a are
// computed from the node's position, so the operator streams only x.
// On a simplicial mesh (DIM == 0) the same quantities come from its edge
// arrays: (K-hat x)_j = ks_j x_j - sum_k kw_jk x_k over the node's adjacency.
#pragma once

#include "common.h"

namespace glk {

// U of the forward edge along axis a whose lower node has coordinates c,
// except c[a] -> ca
template <int DIM, class T>
__device__ __forceinline__ C<T> link_u(const LinkTab<T> &L, int a, const int c[3], int ca)
{
    if (L.n_edge > 0) {
        const int i0 = a == 0 ? ca : c[0], i1 = a == 1 ? ca : c[1];
        const int i2 = DIM == 3 ? (a == 2 ? ca : c[2]) : 0;
        return L.f[(int64_t)a * L.n_edge + i0 + L.N0 * (i1 + L.N1 * i2)];
    }
    C<T> u = mk<T>(1, 0);
    bool first = true;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int o = L.off[a][b];
        if (o >= 0) {
            const C<T> f = L.f[o + (a == b ? ca : c[b])];
            u = first ? f : cmul(u, f);
            first = false;
        }
    }
    return u;
}

template <int DIM>
__device__ __forceinline__ void node_coords(const int *N, int i, int c[3])
{
    if constexpr (DIM == 0) {  // a simplicial mesh: the node index itself
        c[0] = i;
        c[1] = c[2] = 0;
        return;
    }
    c[0] = i % N[0];
    int t = i / N[0];
    if (DIM == 3) {
        c[1] = t % N[1];
        c[2] = t / N[1];
    } else {
        c[1] = t;
        c[2] = 0;
    }
}

// |V_i| and the boundary factors s_a (1 interior, 2 boundary) of node c.
template <int DIM, class T>
__device__ __forceinline__ T node_volume(const GeomT<T> &g, const int c[3], T s[3])
{
    if constexpr (DIM == 0) {
        s[0] = s[1] = s[2] = (T)1;
        return g.vol[c[0]];
    }
    T d = (T)1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        bool bnd = (c[a] == 0) || (c[a] == g.N[a] - 1);
        s[a] = bnd ? (T)2 : (T)1;
        d *= bnd ? (T)0.5 * g.h[a] : g.h[a];
    }
    return d;
}

// Returns (K-hat x)_i; d = |V_i|, asum = K-hat_ii = sum of alpha over the
// edges at i.  x_i is passed in (already loaded by the caller).
template <int DIM, class T>
__device__ __forceinline__ C<T> khat_node(const GeomT<T> &g, int i, const int c[3],
                                          const C<T> *__restrict__ x,
                                          const LinkTab<T> &U, C<T> xi, T &d, T &asum)
{
    if constexpr (DIM == 0) {
        d = g.vol[i];
        asum = g.ks[i];
        C<T> acc = mk<T>(0, 0);
        for (int p = g.rp[i]; p < g.rp[i + 1]; ++p) acc = csub(acc, cmul(g.kw[p], x[g.ci[p]]));
        return cadd(acc, cscale(xi, asum));
    }
    T s[3];
    d = node_volume<DIM, T>(g, c, s);
    C<T> acc = mk<T>(0, 0);
    asum = 0;
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T al = d * s[a] * g.inv_h2[a];
        if (c[a] > 0) {
            const C<T> u = link_u<DIM, T>(U, a, c, c[a] - 1);
            const C<T> xk = x[i - stride];
            acc = csub(acc, cscale(cmul(u, xk), al));
            asum += al;
        }
        if (c[a] < g.N[a] - 1) {
            const C<T> u = link_u<DIM, T>(U, a, c, c[a]);
            const C<T> xj = x[i + stride];
            acc = csub(acc, cscale(cmulc(u, xj), al));
            asum += al;
        }
        stride *= g.N[a];
    }
    return cadd(acc, cscale(xi, asum));
}

// Off-diagonal part only: sum_{j != i} K-hat_ij x_j.
template <int DIM, class T>
__device__ __forceinline__ C<T> khat_offdiag(const GeomT<T> &g, int i, const int c[3],
                                             const C<T> *__restrict__ x,
                                             const LinkTab<T> &U)
{
    if constexpr (DIM == 0) {
        C<T> acc = mk<T>(0, 0);
        for (int p = g.rp[i]; p < g.rp[i + 1]; ++p) acc = csub(acc, cmul(g.kw[p], x[g.ci[p]]));
        return acc;
    }
    T s[3];
    const T d = node_volume<DIM, T>(g, c, s);
    C<T> acc = mk<T>(0, 0);
    int stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T al = d * s[a] * g.inv_h2[a];
        if (c[a] > 0) acc = csub(acc, cscale(cmul(link_u<DIM, T>(U, a, c, c[a] - 1), x[i - stride]), al));
        if (c[a] < g.N[a] - 1) acc = csub(acc, cscale(cmulc(link_u<DIM, T>(U, a, c, c[a]), x[i + stride]), al));
        stride *= g.N[a];
    }
    return acc;
}

}  // namespace glk
