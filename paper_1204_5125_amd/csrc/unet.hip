// Learned continuation predictor: a 2D vertex-grid U-Net with BF16 weights
// and activations and FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), trained with the library's own forward,
// backward and Adam kernels.
//
// Network (levels L, base channels c, C_l = c 2^l):
//   x = (Re psi, Im psi, Re s, Im s, mu, 50 dmu), s = (psi_b - psi) / dmu the
//       slope of the base start psi_b (the secant step)  (padded to 32 channels)
//   encoder level l: [subsample if l > 0] conv3x3 + SiLU, conv3x3 + SiLU
//   decoder level l = L-2 .. 0: linear vertex interpolation of the coarser
//     output, concatenation [upsampled, encoder output l], 2 x (conv3x3 + SiLU)
//   head: 1x1 convolution to (o_re, o_im); psi_pred = psi_b + dmu (o_re + i o_im)
// Loss of an aligned sample: sum_i d_i |o_i - (t_i - psi_b,i)/dmu|^2 / sum d.
//
// Layouts: activations pixel-major with channels contiguous ([P][C], BF16,
// P = N^2, x fastest); weights per layer [c_out][tap][c_in] (tap = 3 ky + kx,
// offsets -1..1), their transposes [c_in][8 - tap][c_out] for the input
// gradient; the parameter vector is FP32, per layer W then b, the head W[2][C_0]
// then b[2].
//
// Convolutions are implicit GEMMs: rows = pixels, columns = output channels,
// reduction = 9 taps x input channels in slices of 32.  A work-group owns an
// 8 x 16-pixel block and 32 or 64 output channels (a wave two block rows:
// 2 x 2 or 2 x 4 MFMA tiles), with each slice's input block (and halo) and
// weights staged in LDS.
// The weight gradient is a GEMM over pixels (split over work-groups, partial
// sums reduced in a fixed order), staged through LDS.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "amg.h"
#include "stencil.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

namespace glk {

constexpr int kCi = 32;  // input channels per reduction slice

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_d(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ bf16x8 load8(const __bf16 *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    return z;
}

enum ConvMode { CONV_FWD = 0, CONV_DGRAD = 1, CONV_DGRAD_SILU = 2 };

// out[p][co] = sum_{tap, ci} in[p + off(tap)][ci] w[co][tap][ci] (+ epilogue)
//   FWD:        z = acc + bias -> out0 (z), out1 (SiLU(z))
//   DGRAD:      acc -> out0
//   DGRAD_SILU: acc * SiLU'(zs[p][co]) -> out0
// A work-group computes an 8 x 16-pixel block of the image for 16 WCO output
// channels; wave w owns the block's rows 2w and 2w + 1 (one 16-pixel MFMA
// row tile each).  The reduction runs over 32-channel input slices: per
// slice, the block's input with a one-pixel halo (10 x 18 pixels, zero
// outside the image) and the slice's weights of all nine taps are staged in
// LDS, so an input value is read from memory once per slice and channel tile
// instead of once per tap, and a weight once per work-group instead of once
// per wave.  The next slice's global loads are issued before the current
// slice's products.
constexpr int kBH = 8, kBW = 16;              // pixel block
constexpr int kHH = kBH + 2, kHW = kBW + 2;   // with its halo
constexpr int kSP = kCi + 8;                  // LDS row pitch (bf16): 80 bytes

template <int WCO>
struct ConvLds {
    static constexpr int a_rows = kHH * kHW;        // halo pixels
    static constexpr int b_rows = 9 * 16 * WCO;     // (tap, output channel)
    static constexpr int na = a_rows * (kCi / 8);   // 16-byte pieces per slice
    static constexpr int nb = b_rows * (kCi / 8);
    static constexpr int ca = (na + 255) / 256;     // pieces per thread
    static constexpr int cb = (nb + 255) / 256;
    static constexpr int tile = 16 * WCO + 8;       // epilogue row pitch (bf16)
    static constexpr int elems = (a_rows + b_rows) * kSP;
    static_assert(4 * 32 * tile <= b_rows * kSP, "the epilogue tiles reuse the weight slice's LDS");
};

template <int MODE, int WCO>
__global__ __launch_bounds__(256) void k_conv3x3(const __bf16 *__restrict__ in, int ldi, int cin, int H, int W,
                                                 const __bf16 *__restrict__ w, int cout,
                                                 const float *__restrict__ bias, __bf16 *out0, int ld0, int off0,
                                                 __bf16 *out1, int ld1, int off1, const __bf16 *__restrict__ zs,
                                                 int ldzs, int bxs)
{
    using G = ConvLds<WCO>;
    __shared__ __attribute__((aligned(16))) __bf16 lds[G::elems];
    __bf16 *sA = lds, *sB = lds + G::a_rows * kSP;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int x0 = (blockIdx.x % bxs) * kBW, y0 = (blockIdx.x / bxs) * kBH;
    const int co0 = blockIdx.y * (16 * WCO);
    const int kk = 8 * (lane >> 4), m = lane & 15;
    const int nci = cin / kCi;
    bf16x8 ra[G::ca], rb[G::cb];
    // global loads of slice s into registers (zero outside the image)
    auto fetch = [&](int s) {
        const int ci0 = s * kCi;
#pragma unroll
        for (int j = 0; j < G::ca; ++j) {
            const int q = threadIdx.x + 256 * j;
            bf16x8 v = zero8();
            if (q < G::na) {
                const int h = q >> 2, part = (q & 3) * 8;
                const int y = y0 - 1 + h / kHW, x = x0 - 1 + h % kHW;
                if (y >= 0 && y < H && x >= 0 && x < W) v = load8(in + (size_t)(y * W + x) * ldi + ci0 + part);
            }
            ra[j] = v;
        }
#pragma unroll
        for (int j = 0; j < G::cb; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < G::nb) {
                const int row = q >> 2, part = (q & 3) * 8;
                const int tap = row / (16 * WCO), col = row % (16 * WCO);
                rb[j] = load8(w + (size_t)(co0 + col) * 9 * cin + tap * cin + ci0 + part);
            }
        }
    };
    f4 acc[2][WCO];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < WCO; ++c) acc[r][c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    fetch(0);
    for (int s = 0; s < nci; ++s) {
        __syncthreads();  // the previous slice's products are done with the LDS
#pragma unroll
        for (int j = 0; j < G::ca; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < G::na) *reinterpret_cast<bf16x8 *>(sA + (q >> 2) * kSP + (q & 3) * 8) = ra[j];
        }
#pragma unroll
        for (int j = 0; j < G::cb; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < G::nb) *reinterpret_cast<bf16x8 *>(sB + (q >> 2) * kSP + (q & 3) * 8) = rb[j];
        }
        __syncthreads();
        if (s + 1 < nci) fetch(s + 1);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3 - 1, dx = tap % 3 - 1;
            bf16x8 a[2], b[WCO];
#pragma unroll
            for (int r = 0; r < 2; ++r)
                a[r] = *reinterpret_cast<const bf16x8 *>(sA + ((2 * wave + r + 1 + dy) * kHW + m + 1 + dx) * kSP + kk);
#pragma unroll
            for (int c = 0; c < WCO; ++c)
                b[c] = *reinterpret_cast<const bf16x8 *>(sB + (tap * 16 * WCO + 16 * c + m) * kSP + kk);
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < WCO; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], b[c], acc[r][c], 0, 0, 0);
        }
    }
    __syncthreads();  // every wave is done with the weight slice: its LDS holds the epilogue tiles
    // D layout: row (pixel) 4 (lane / 16) + i of the row tile, column (channel)
    // lane % 16.  Each output tile goes through the wave's LDS tile so that a
    // lane stores eight channels of one pixel (16 bytes) at a time.
    __bf16 *stile = sB + wave * 32 * G::tile;
    auto emit = [&](auto value, __bf16 *out, int ld, int off) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < WCO; ++c)
#pragma unroll
                for (int i = 0; i < 4; ++i) stile[(16 * r + 4 * (lane >> 4) + i) * G::tile + 16 * c + m] = value(r, c, i);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = lane; q < 64 * WCO; q += 64) {
            const int row = q / (2 * WCO), ch = (q % (2 * WCO)) * 8;
            const int y = y0 + 2 * wave + row / 16, x = x0 + row % 16;
            if (y < H && x < W)
                *reinterpret_cast<bf16x8 *>(out + (size_t)(y * W + x) * ld + off + co0 + ch) =
                    *reinterpret_cast<const bf16x8 *>(stile + row * G::tile + ch);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    if constexpr (MODE == CONV_FWD) {
        float bs[WCO];
#pragma unroll
        for (int c = 0; c < WCO; ++c) bs[c] = bias[co0 + 16 * c + m];
        emit([&](int r, int c, int i) { return (__bf16)(acc[r][c][i] + bs[c]); }, out0, ld0, off0);
        emit([&](int r, int c, int i) { return (__bf16)silu_f(acc[r][c][i] + bs[c]); }, out1, ld1, off1);
    } else if constexpr (MODE == CONV_DGRAD) {
        emit([&](int r, int c, int i) { return (__bf16)acc[r][c][i]; }, out0, ld0, off0);
    } else {
        emit(
            [&](int r, int c, int i) {
                const int y = y0 + 2 * wave + r, x = x0 + 4 * (lane >> 4) + i;
                const float z = (y < H && x < W) ? (float)zs[(size_t)(y * W + x) * ldzs + co0 + 16 * c + m] : 0.0f;
                return (__bf16)(acc[r][c][i] * silu_d(z));
            },
            out0, ld0, off0);
    }
}

// Weight gradient partials: part[s][co][tap][ci] = sum over the pixels of
// split s of dz[p][co] in[p + off(tap)][ci]; tiles of 32 x 32 (co, ci), one
// 16 x 16 MFMA tile per wave and tap, 32-pixel slices staged in LDS.
__global__ __launch_bounds__(256) void k_conv_wgrad(const __bf16 *__restrict__ dz, int ldz, int cout,
                                                    const __bf16 *__restrict__ in, int ldi, int cin, int H, int W,
                                                    int pix_per_split, float *__restrict__ part)
{
    __shared__ __bf16 sdz[32][32 + 8];
    __shared__ __bf16 sin_[9][32][32 + 8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int co0 = blockIdx.x * 32, ci0 = blockIdx.y * 32, s = blockIdx.z;
    const int P = H * W;
    const int pbeg = s * pix_per_split, pend = min(P, pbeg + pix_per_split);
    const int cb = wave >> 1, ib = wave & 1, m = lane & 15, kk = 8 * (lane >> 4);
    f4 acc[9];
    for (int t = 0; t < 9; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int c0 = pbeg; c0 < pend; c0 += 32) {
        // dz slice: 32 pixels x 32 channels (8 channels per thread)
        if (threadIdx.x < 128) {
            const int px = threadIdx.x >> 2, part8 = (threadIdx.x & 3) * 8;
            const int p = c0 + px;
            const bf16x8 v = p < pend ? load8(dz + (size_t)p * ldz + co0 + part8) : zero8();
            for (int j = 0; j < 8; ++j) sdz[px][part8 + j] = v[j];
        }
        // input slices for the 9 taps
        for (int idx = threadIdx.x; idx < 9 * 128; idx += 256) {
            const int tap = idx >> 7, rem = idx & 127, px = rem >> 2, part8 = (rem & 3) * 8;
            const int p = c0 + px;
            bf16x8 v = zero8();
            if (p < pend) {
                const int y = p / W, x = p - (p / W) * W;
                const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = load8(in + (size_t)(yy * W + xx) * ldi + ci0 + part8);
            }
            for (int j = 0; j < 8; ++j) sin_[tap][px][part8 + j] = v[j];
        }
        __syncthreads();
        bf16x8 a;
        for (int j = 0; j < 8; ++j) a[j] = sdz[kk + j][16 * cb + m];
        for (int t = 0; t < 9; ++t) {
            bf16x8 b;
            for (int j = 0; j < 8; ++j) b[j] = sin_[t][kk + j][16 * ib + m];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int t = 0; t < 9; ++t)
        for (int i = 0; i < 4; ++i) {
            const int co = co0 + 16 * cb + 4 * (lane >> 4) + i, ci = ci0 + 16 * ib + m;
            part[(((size_t)s * cout + co) * 9 + t) * cin + ci] = acc[t][i];
        }
}

// grad[co][tap][ci] += sum_s part[s][co][tap][ci] (ci < cin_real), fixed order
__global__ void k_wgrad_reduce(const float *__restrict__ part, int splits, int cout, int cin_pad, int cin_real,
                               float *__restrict__ grad)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = cout * 9 * cin_real;
    if (idx >= total) return;
    const int ci = idx % cin_real, rest = idx / cin_real;  // rest = co * 9 + tap
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += part[((size_t)k * cout * 9 + rest) * cin_pad + ci];
    grad[idx] += s;
}

// bias gradient partials: part[s][co] = sum over split s of dz[p][co]
// (256 threads; cout divides 256: thread t sums channel t mod cout over every
// (256 / cout)-th pixel of the split, and the lanes of a channel are added in
// lane order)
__global__ __launch_bounds__(256) void k_bias_partial(const __bf16 *__restrict__ dz, int ldz, int cout, int P,
                                                      int pix_per_split, float *__restrict__ part)
{
    __shared__ float sm[256];
    const int s = blockIdx.x;
    const int pbeg = s * pix_per_split, pend = min(P, pbeg + pix_per_split);
    const int lanes = 256 / cout, co = threadIdx.x % cout, l = threadIdx.x / cout;
    float acc = 0.0f;
    for (int p = pbeg + l; p < pend; p += lanes) acc += (float)dz[(size_t)p * ldz + co];
    sm[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < cout) {
        float t = 0.0f;
        for (int k = 0; k < lanes; ++k) t += sm[k * cout + threadIdx.x];
        part[(size_t)s * cout + threadIdx.x] = t;
    }
}

__global__ void k_bias_reduce(const float *__restrict__ part, int splits, int cout, float *__restrict__ grad)
{
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= cout) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += part[(size_t)k * cout + co];
    grad[co] += s;
}

// input planes (Re psi, Im psi, Re s, Im s, mu, 50 dmu, 0 ...) with 32
// channels, s = (psi_b - psi) / dmu
__global__ void k_unet_input(int P, const double2 *__restrict__ psi, const double2 *__restrict__ psib, double dmu,
                             float mu, __bf16 *__restrict__ x)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double2 v = psi[p], b = psib[p];
    __bf16 *o = x + (size_t)p * 32;
    o[0] = (__bf16)(float)v.x;
    o[1] = (__bf16)(float)v.y;
    o[2] = (__bf16)(float)((b.x - v.x) / dmu);
    o[3] = (__bf16)(float)((b.y - v.y) / dmu);
    o[4] = (__bf16)mu;
    o[5] = (__bf16)(float)(50.0 * dmu);
    for (int c = 6; c < 32; ++c) o[c] = (__bf16)0.0f;
}

// vertex subsampling: out[i][j] = in[2i][2j]
__global__ void k_down(int Nc, int C, const __bf16 *__restrict__ in, int ldi, int offi, __bf16 *__restrict__ out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nc * Nc * C) return;
    const int c = idx % C, q = idx / C, i = q / Nc, j = q % Nc;
    const int Nf = 2 * Nc - 1;
    out[(size_t)q * C + c] = in[(size_t)(2 * i * Nf + 2 * j) * ldi + offi + c];
}

// linear vertex interpolation to the finer grid, into channels [off, off + C) of out
// (eight channels per thread: C, ldo and off are multiples of 8)
__global__ void k_up(int Nc, int C, const __bf16 *__restrict__ in, __bf16 *__restrict__ out, int ldo, int off)
{
    const int Nf = 2 * Nc - 1, C8 = C / 8;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nf * Nf * C8) return;
    const int c = (idx % C8) * 8, q = idx / C8, y = q / Nf, x = q % Nf;
    const int i0 = y >> 1, j0 = x >> 1, i1 = i0 + (y & 1), j1 = j0 + (x & 1);
    const bf16x8 a = load8(in + (size_t)(i0 * Nc + j0) * C + c), b = load8(in + (size_t)(i1 * Nc + j0) * C + c);
    const bf16x8 d = load8(in + (size_t)(i0 * Nc + j1) * C + c), e = load8(in + (size_t)(i1 * Nc + j1) * C + c);
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)(0.25f * ((float)a[j] + (float)b[j] + (float)d[j] + (float)e[j]));
    *reinterpret_cast<bf16x8 *>(out + (size_t)q * ldo + off + c) = v;
}

// transpose of k_up: coarse node (i, j) gathers its fine neighbours
__global__ void k_up_backward(int Nc, int C, const __bf16 *__restrict__ dy, int ldy, __bf16 *__restrict__ dx)
{
    const int Nf = 2 * Nc - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nc * Nc * C) return;
    const int c = idx % C, q = idx / C, i = q / Nc, j = q % Nc;
    float s = 0.0f;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) {
            const int y = 2 * i + a, x = 2 * j + b;
            if (y < 0 || y >= Nf || x < 0 || x >= Nf) continue;
            const float wgt = (a == 0 ? 1.0f : 0.5f) * (b == 0 ? 1.0f : 0.5f);
            s += wgt * (float)dy[(size_t)(y * Nf + x) * ldy + c];
        }
    dx[(size_t)q * C + c] = (__bf16)s;
}

// dh = dskip (nullable) + scatter of the coarse gradient to the even nodes
__global__ void k_down_backward_add(int Nc, int C, const __bf16 *__restrict__ dcoarse,
                                    const __bf16 *__restrict__ dskip, int lds, int offs, __bf16 *__restrict__ dh)
{
    const int Nf = 2 * Nc - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nf * Nf * C) return;
    const int c = idx % C, q = idx / C, y = q / Nf, x = q % Nf;
    float v = dskip ? (float)dskip[(size_t)q * lds + offs + c] : 0.0f;
    if (!(y & 1) && !(x & 1)) v += (float)dcoarse[(size_t)((y >> 1) * Nc + (x >> 1)) * C + c];
    dh[(size_t)q * C + c] = (__bf16)v;
}

// dz = dh * SiLU'(z)
__global__ void k_silu_backward(int n, const __bf16 *__restrict__ dh, const __bf16 *__restrict__ z,
                                __bf16 *__restrict__ dz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dz[i] = (__bf16)((float)dh[i] * silu_d((float)z[i]));
}

// head: o[p][k] = b[k] + sum_ci W[k][ci] h[p][ci] (FP32), k = 0, 1
__global__ void k_head(int P, int C, const __bf16 *__restrict__ h, const float *__restrict__ Wb,
                       float *__restrict__ o)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float a0 = Wb[2 * C], a1 = Wb[2 * C + 1];
    for (int c = 0; c < C; ++c) {
        const float v = (float)h[(size_t)p * C + c];
        a0 += Wb[c] * v;
        a1 += Wb[C + c] * v;
    }
    o[2 * p] = a0;
    o[2 * p + 1] = a1;
}

// psi_out = psi_b + dmu (o_re + i o_im)
__global__ void k_predict(int P, const double2 *__restrict__ psi, const float *__restrict__ o, double dmu,
                          double2 *__restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    out[p] = make_double2(psi[p].x + dmu * o[2 * p], psi[p].y + dmu * o[2 * p + 1]);
}

// partial sums of the loss normaliser sum_i d_i (|w_i|^2 + kLossEps),
// w = (t - psi_b) / dmu: the base start's error with an absolute floor (slope^2
// units) so that samples whose secant start is already nearly exact cannot
// dominate
constexpr double kLossEps = 1e-4;

__global__ __launch_bounds__(kBlock) void k_loss_norm(GeomT<double> g, const double2 *__restrict__ psi,
                                                      const double2 *__restrict__ psib,
                                                      const double2 *__restrict__ tgt, double dmu, RedSlot slot)
{
    __shared__ double sm[kBlock / 64];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    double part = 0.0;
    if (p < g.n) {
        int c[3];
        node_coords<2>(g.N, p, c);
        double sf[3];
        const double d = node_volume<2, double>(g, c, sf);
        const double wr = (tgt[p].x - psib[p].x) / dmu, wi = (tgt[p].y - psib[p].y) / dmu;
        part = d * (wr * wr + wi * wi + kLossEps);
    }
    block_reduce_store(part, slot, sm, blockIdx.x);
}

// partial sums of sum_i d_i |o_i - w_i|^2 and do = dL/do with
// L = that sum / *norm (scaled by `scale`, 1 / count for minibatches)
__global__ __launch_bounds__(kBlock) void k_loss(GeomT<double> g, const double2 *__restrict__ psib,
                                                 const double2 *__restrict__ tgt, const float *__restrict__ o,
                                                 double dmu, const double *__restrict__ norm, float scale,
                                                 float *__restrict__ dout, RedSlot slot)
{
    __shared__ double sm[kBlock / 64];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const double inv = *norm > 0.0 ? 1.0 / *norm : 0.0;
    double part = 0.0;
    if (p < g.n) {
        int c[3];
        node_coords<2>(g.N, p, c);
        double sf[3];
        const double d = node_volume<2, double>(g, c, sf);
        const double wr = (tgt[p].x - psib[p].x) / dmu, wi = (tgt[p].y - psib[p].y) / dmu;
        const double rr = o[2 * p] - wr, ri = o[2 * p + 1] - wi;
        part = d * (rr * rr + ri * ri);
        dout[2 * p] = (float)(2.0 * d * rr * inv) * scale;
        dout[2 * p + 1] = (float)(2.0 * d * ri * inv) * scale;
    }
    block_reduce_store(part, slot, sm, blockIdx.x);
}

// head backward: dh[p][ci] = sum_k W[k][ci] do[p][k] (BF16); weight and bias
// gradient partials per split
__global__ void k_head_backward(int P, int C, const __bf16 *__restrict__ h, const float *__restrict__ Wb,
                                const float *__restrict__ dout, __bf16 *__restrict__ dh)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * C) return;
    const int p = idx / C, c = idx % C;
    dh[idx] = (__bf16)(Wb[c] * dout[2 * p] + Wb[C + c] * dout[2 * p + 1]);
}

__global__ void k_head_wgrad_partial(int P, int C, const __bf16 *__restrict__ h, const float *__restrict__ dout,
                                     int pix_per_split, float *__restrict__ part)
{
    // part[s][k * C + ci] and part[s][2 C + k]
    const int s = blockIdx.x;
    const int pbeg = s * pix_per_split, pend = min(P, pbeg + pix_per_split);
    for (int e = threadIdx.x; e < 2 * C + 2; e += blockDim.x) {
        float acc = 0.0f;
        if (e < 2 * C) {
            const int k = e / C, ci = e % C;
            for (int p = pbeg; p < pend; ++p) acc += dout[2 * p + k] * (float)h[(size_t)p * C + ci];
        } else {
            const int k = e - 2 * C;
            for (int p = pbeg; p < pend; ++p) acc += dout[2 * p + k];
        }
        part[(size_t)s * (2 * C + 2) + e] = acc;
    }
}

// BF16 weights of one layer from the FP32 parameters: forward [co][tap][ci_pad]
// (zero padding) and, when wt != NULL, transposed [ci][8 - tap][co]
__global__ void k_pack_weights(const float *__restrict__ W, int cout, int cin, int cin_pad, __bf16 *__restrict__ wf,
                               __bf16 *__restrict__ wt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cout * 9 * cin_pad) return;
    const int ci = idx % cin_pad, rest = idx / cin_pad, tap = rest % 9, co = rest / 9;
    const float v = ci < cin ? W[((size_t)co * 9 + tap) * cin + ci] : 0.0f;
    wf[idx] = (__bf16)v;
    if (wt && ci < cin) wt[((size_t)ci * 9 + (8 - tap)) * cout + co] = (__bf16)v;
}

__global__ void k_adam(int n, float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// grad[e] += sum_s part[s][e], fixed order
__global__ void k_sum_partials(const float *__restrict__ part, int splits, int n, float *__restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += part[(size_t)k * n + e];
    grad[e] += s;
}

__global__ void k_fill_f32(int n, float *x, float v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

}  // namespace glk

// ------------------------------------------------------------ handle ---
struct gl_unet {
    int levels = 0, base = 0;
    std::vector<int> cin, cout, ksz;       // per layer
    std::vector<size_t> woff, boff;        // offsets in the parameter vector
    size_t nparams = 0;
    glk::DevBuf<float> theta, m, v, grad;
    std::vector<glk::DevBuf<__bf16>> wf, wt;
    int64_t adam_t = 0;
    // activations for grid size N
    int N = 0;
    std::vector<int> Nl;
    glk::DevBuf<__bf16> x0;                            // input planes [P0][32]
    std::vector<glk::DevBuf<__bf16>> a0, ez0, eh1, ez1; // encoder: input, z0, h1, z1 per level
    glk::DevBuf<__bf16> hbott;                         // output of the last encoder level
    std::vector<glk::DevBuf<__bf16>> cat, dz0, dh1, dz1, dh; // decoder per level (index l)
    glk::DevBuf<float> o, dout, part;
    glk::DevBuf<__bf16> g1, g2, g3, dcat_tmp;
    std::vector<glk::DevBuf<__bf16>> dcat;             // decoder concat gradients per level
    size_t part_cap = 0;
    ~gl_unet() = default;
};

namespace glk {

static int enc_layer(int l, int k) { return 2 * l + k; }
static int dec_layer(const gl_unet *u, int l, int k) { return 2 * u->levels + 2 * (u->levels - 2 - l) + k; }
static int head_layer(const gl_unet *u) { return 4 * u->levels - 2; }

static void unet_pack(gl_unet *u, hipStream_t s)
{
    for (size_t li = 0; li + 1 < u->cin.size(); ++li) {
        const int ci = u->cin[li], co = u->cout[li], cp = li == 0 ? 32 : ci;
        const int n = co * 9 * cp;
        k_pack_weights<<<blocks_for(n), kBlock, 0, s>>>(u->theta.get() + u->woff[li], co, ci, cp, u->wf[li].get(),
                                                        li == 0 ? nullptr : u->wt[li].get());
    }
    GLK_CHECK_LAUNCH();
}

static void unet_alloc(gl_unet *u, int N)
{
    if (u->N == N) return;
    const int L = u->levels;
    u->N = N;
    u->Nl.assign(L, 0);
    for (int l = 0; l < L; ++l) u->Nl[l] = (N - 1) / (1 << l) + 1;
    auto P = [&](int l) { return (size_t)u->Nl[l] * u->Nl[l]; };
    auto C = [&](int l) { return (size_t)u->base << l; };
    u->x0.alloc(P(0) * 32);
    u->a0.resize(L);
    u->ez0.resize(L);
    u->eh1.resize(L);
    u->ez1.resize(L);
    u->cat.resize(L);
    u->dz0.resize(L);
    u->dh1.resize(L);
    u->dz1.resize(L);
    u->dh.resize(L);
    u->dcat.resize(L);
    size_t gmax = 0;
    for (int l = 0; l < L; ++l) {
        if (l > 0) u->a0[l].alloc(P(l) * C(l - 1));
        u->ez0[l].alloc(P(l) * C(l));
        u->eh1[l].alloc(P(l) * C(l));
        u->ez1[l].alloc(P(l) * C(l));
        gmax = std::max(gmax, P(l) * C(l) * 3);
        if (l < L - 1) {
            const size_t cc = C(l + 1) + C(l);
            u->cat[l].alloc(P(l) * cc);
            u->dcat[l].alloc(P(l) * cc);
            u->dz0[l].alloc(P(l) * C(l));
            u->dh1[l].alloc(P(l) * C(l));
            u->dz1[l].alloc(P(l) * C(l));
            u->dh[l].alloc(P(l) * C(l));
        }
    }
    u->hbott.alloc(P(L - 1) * C(L - 1));
    u->o.alloc(P(0) * 2);
    u->dout.alloc(P(0) * 2);
    u->g1.alloc(gmax);
    u->g2.alloc(gmax);
    u->g3.alloc(gmax);
    // weight-gradient partials: at most 32 MB
    u->part_cap = (size_t)8 << 20;
    u->part.alloc(u->part_cap);
}

// A 3 x 3 convolution on an H x H grid: 64 output channels per work-group
// where cout allows and the grid still gets at least two work-groups per
// compute unit, else 32.
template <int MODE>
static void launch_conv(const __bf16 *in, int ldi, int cin, int H, const __bf16 *w, int cout, const float *bias,
                        __bf16 *out0, int ld0, int off0, __bf16 *out1, int ld1, int off1, const __bf16 *zs, int ldzs,
                        hipStream_t s)
{
    if (cin % kCi != 0 || cout % 32 != 0 || ldi < cin || ldi % 8 != 0)
        fail(GL_ERR_INVALID_ARGUMENT, "conv3x3: channels must be multiples of 32");
    const int bxs = (H + kBW - 1) / kBW, bys = (H + kBH - 1) / kBH;
    const int64_t blocks = (int64_t)bxs * bys;
    const int wco = (cout % 64 == 0 && blocks * (cout / 64) >= 512) ? 4 : 2;
    const dim3 grid((unsigned)blocks, cout / (16 * wco));
    auto go = [&](auto kern) {
        kern<<<grid, 256, 0, s>>>(in, ldi, cin, H, H, w, cout, bias, out0, ld0, off0, out1, ld1, off1, zs, ldzs,
                                  bxs);
    };
    if (wco == 4) go(k_conv3x3<MODE, 4>);
    else go(k_conv3x3<MODE, 2>);
    GLK_CHECK_LAUNCH();
}

static void conv_fwd(gl_unet *u, int li, const __bf16 *in, int ldi, int H, __bf16 *z, __bf16 *h, int ldh, int offh,
                     hipStream_t s)
{
    const int cin = li == 0 ? 32 : u->cin[li], co = u->cout[li];
    launch_conv<CONV_FWD>(in, ldi, cin, H, u->wf[li].get(), co, u->theta.get() + u->boff[li], z, co, 0, h, ldh, offh,
                          nullptr, 0, s);
}

// input gradient of layer li: out = W^T dz (* SiLU'(zs) when zs != NULL)
static void conv_dgrad(gl_unet *u, int li, const __bf16 *dz, int H, __bf16 *out, int ldo, const __bf16 *zs,
                       hipStream_t s)
{
    const int ci = u->cin[li], co = u->cout[li];
    if (zs)
        launch_conv<CONV_DGRAD_SILU>(dz, co, co, H, u->wt[li].get(), ci, nullptr, out, ldo, 0, nullptr, 0, 0, zs, ci, s);
    else
        launch_conv<CONV_DGRAD>(dz, co, co, H, u->wt[li].get(), ci, nullptr, out, ldo, 0, nullptr, 0, 0, nullptr, 0, s);
}

static void conv_wgrad(gl_unet *u, int li, const __bf16 *dz, const __bf16 *in, int ldi, int H, hipStream_t s)
{
    const int cin_pad = li == 0 ? 32 : u->cin[li], cin = u->cin[li], co = u->cout[li];
    const int P = H * H;
    const int tiles = (co / 32) * (cin_pad / 32);
    int splits = std::max(1, std::min((P + 31) / 32, 1024 / tiles));
    while ((size_t)splits * co * 9 * cin_pad > u->part_cap && splits > 1) splits /= 2;
    const int pps = ((P + splits - 1) / splits + 31) / 32 * 32;
    splits = (P + pps - 1) / pps;
    k_conv_wgrad<<<dim3(co / 32, cin_pad / 32, splits), 256, 0, s>>>(dz, co, co, in, ldi, cin_pad, H, H, pps,
                                                                     u->part.get());
    const int n = co * 9 * cin;
    k_wgrad_reduce<<<blocks_for(n), kBlock, 0, s>>>(u->part.get(), splits, co, cin_pad, cin,
                                                    u->grad.get() + u->woff[li]);
    if (co > 256 || 256 % co != 0) fail(GL_ERR_INVALID_ARGUMENT, "bias gradient: c_out must divide 256");
    const int bs = std::min(256, std::max(1, P / 1024));
    const int bpps = (P + bs - 1) / bs;
    k_bias_partial<<<bs, 256, 0, s>>>(dz, co, co, P, bpps, u->part.get());
    k_bias_reduce<<<blocks_for(co), kBlock, 0, s>>>(u->part.get(), bs, co, u->grad.get() + u->boff[li]);
}

// forward pass; leaves o in u->o
static void unet_forward(gl_unet *u, const gl_mesh *m, const double2 *psi, const double2 *psib, double mu,
                         double dmu, hipStream_t s)
{
    const int L = u->levels;
    const int P0 = u->Nl[0] * u->Nl[0];
    k_unet_input<<<blocks_for(P0), kBlock, 0, s>>>(P0, psi, psib, dmu, (float)mu, u->x0.get());
    const __bf16 *in = u->x0.get();
    int ldi = 32;
    for (int l = 0; l < L; ++l) {
        const int H = u->Nl[l], Cl = u->base << l;
        if (l > 0) {
            const int Cp = u->base << (l - 1);
            // the previous level's output lives in its concat buffer (skip slice) or hbott
            k_down<<<blocks_for((int64_t)H * H * Cp), kBlock, 0, s>>>(H, Cp, in, ldi, ldi - Cp, u->a0[l].get());
            in = u->a0[l].get();
            ldi = Cp;
        }
        conv_fwd(u, enc_layer(l, 0), in, ldi, H, u->ez0[l].get(), u->eh1[l].get(), Cl, 0, s);
        __bf16 *hout;
        int ldh, offh;
        if (l < L - 1) {
            hout = u->cat[l].get();
            ldh = (u->base << (l + 1)) + Cl;
            offh = u->base << (l + 1);
        } else {
            hout = u->hbott.get();
            ldh = Cl;
            offh = 0;
        }
        conv_fwd(u, enc_layer(l, 1), u->eh1[l].get(), Cl, H, u->ez1[l].get(), hout, ldh, offh, s);
        in = hout;  // the next level subsamples the skip slice
        ldi = ldh;
    }
    // decoder
    const __bf16 *hc = u->hbott.get();
    for (int l = L - 2; l >= 0; --l) {
        const int H = u->Nl[l], Hc = u->Nl[l + 1], Cl = u->base << l, Cu = u->base << (l + 1);
        const int cc = Cu + Cl;
        k_up<<<blocks_for((int64_t)H * H * Cu / 8), kBlock, 0, s>>>(Hc, Cu, hc, u->cat[l].get(), cc, 0);
        conv_fwd(u, dec_layer(u, l, 0), u->cat[l].get(), cc, H, u->dz0[l].get(), u->dh1[l].get(), Cl, 0, s);
        conv_fwd(u, dec_layer(u, l, 1), u->dh1[l].get(), Cl, H, u->dz1[l].get(), u->dh[l].get(), Cl, 0, s);
        hc = u->dh[l].get();
    }
    const int hl = head_layer(u);
    k_head<<<blocks_for(P0), kBlock, 0, s>>>(P0, u->base, L > 1 ? u->dh[0].get() : u->hbott.get(),
                                             u->theta.get() + u->woff[hl], u->o.get());
    GLK_CHECK_LAUNCH();
}

// backward pass from u->dout; adds the parameter gradient to u->grad
static void unet_backward(gl_unet *u, hipStream_t s)
{
    const int L = u->levels;
    const int P0 = u->Nl[0] * u->Nl[0];
    const int C0 = u->base;
    const int hl = head_layer(u);
    const __bf16 *hlast = L > 1 ? u->dh[0].get() : u->hbott.get();
    // head
    {
        const int bs = std::min(256, std::max(1, P0 / 1024));
        const int pps = (P0 + bs - 1) / bs;
        k_head_wgrad_partial<<<bs, 256, 0, s>>>(P0, C0, hlast, u->dout.get(), pps, u->part.get());
        k_sum_partials<<<blocks_for(2 * C0 + 2), kBlock, 0, s>>>(u->part.get(), bs, 2 * C0 + 2,
                                                                u->grad.get() + u->woff[hl]);
        k_head_backward<<<blocks_for((int64_t)P0 * C0), kBlock, 0, s>>>(P0, C0, hlast, u->theta.get() + u->woff[hl],
                                                                       u->dout.get(), u->g1.get());
    }
    // g1 = gradient w.r.t. the current level's output h
    for (int l = 0; l <= L - 2; ++l) {
        const int H = u->Nl[l], P = H * H, Cl = u->base << l, Cu = u->base << (l + 1), cc = Cu + Cl;
        const int l1 = dec_layer(u, l, 1), l0 = dec_layer(u, l, 0);
        k_silu_backward<<<blocks_for((int64_t)P * Cl), kBlock, 0, s>>>(P * Cl, u->g1.get(), u->dz1[l].get(),
                                                                       u->g2.get());
        conv_wgrad(u, l1, u->g2.get(), u->dh1[l].get(), Cl, H, s);
        conv_dgrad(u, l1, u->g2.get(), H, u->g3.get(), Cl, u->dz0[l].get(), s);  // g3 = dz0
        conv_wgrad(u, l0, u->g3.get(), u->cat[l].get(), cc, H, s);
        conv_dgrad(u, l0, u->g3.get(), H, u->dcat[l].get(), cc, nullptr, s);
        const int Hc = u->Nl[l + 1];
        k_up_backward<<<blocks_for((int64_t)Hc * Hc * Cu), kBlock, 0, s>>>(Hc, Cu, u->dcat[l].get(), cc, u->g1.get());
    }
    // encoder, from the coarsest level; g1 = gradient w.r.t. its output
    for (int l = L - 1; l >= 0; --l) {
        const int H = u->Nl[l], P = H * H, Cl = u->base << l;
        // g1: gradient w.r.t. this level's output (skip and subsampling paths)
        k_silu_backward<<<blocks_for((int64_t)P * Cl), kBlock, 0, s>>>(P * Cl, u->g1.get(), u->ez1[l].get(),
                                                                       u->g2.get());
        conv_wgrad(u, enc_layer(l, 1), u->g2.get(), u->eh1[l].get(), Cl, H, s);
        conv_dgrad(u, enc_layer(l, 1), u->g2.get(), H, u->g3.get(), Cl, u->ez0[l].get(), s);  // g3 = dz0
        const __bf16 *ain = l == 0 ? u->x0.get() : u->a0[l].get();
        const int lda = l == 0 ? 32 : (u->base << (l - 1));
        conv_wgrad(u, enc_layer(l, 0), u->g3.get(), ain, lda, H, s);
        if (l > 0) {
            const int Cp = u->base << (l - 1), Hf = u->Nl[l - 1];
            conv_dgrad(u, enc_layer(l, 0), u->g3.get(), H, u->g2.get(), Cp, nullptr, s);  // g2 = d a0
            // gradient w.r.t. the output of level l - 1: skip part + subsampling part
            const int ccp = Cl + Cp;
            k_down_backward_add<<<blocks_for((int64_t)Hf * Hf * Cp), kBlock, 0, s>>>(
                H, Cp, u->g2.get(), u->dcat[l - 1].get(), ccp, Cl, u->g1.get());
        }
    }
    GLK_CHECK_LAUNCH();
}

static double read_double(const double *d, hipStream_t s)
{
    double h = 0.0;
    GLK_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    return h;
}

static void check_grid(const gl_unet *u, const gl_mesh *m)
{
    if (m->g.simplicial || m->g.dim != 2 || m->g.N[0] != m->g.N[1])
        fail(GL_ERR_UNSUPPORTED, "gl_unet: the predictor needs a square 2D grid");
    const int N = m->g.N[0], q = 1 << (u->levels - 1);
    if ((N - 1) % q != 0 || (N - 1) / q < 1)
        fail(GL_ERR_INVALID_ARGUMENT, "gl_unet: grid nodes per axis must be 2^(levels-1) k + 1");
}

// loss of one sample; leaves do in u->dout (scaled) and returns L
static double unet_loss(gl_unet *u, const gl_mesh *m, const double2 *psi, const double2 *psib, const double2 *tgt,
                        double mu, double dmu, float scale, hipStream_t s)
{
    unet_forward(u, m, psi, psib, mu, dmu, s);
    const int P0 = m->g.n, nb = blocks_for(P0);
    const GeomT<double> g = geom_t<double>(m->g);
    double *norm = m->dscal.get() + 5;
    k_loss_norm<<<nb, kBlock, 0, s>>>(g, psi, psib, tgt, dmu, red_slot(m, 3));
    launch_finalize(red_slot(m, 3).partials, nb, FIN_STORE, nullptr, norm, nullptr, s);
    k_loss<<<nb, kBlock, 0, s>>>(g, psib, tgt, u->o.get(), dmu, norm, scale, u->dout.get(), red_slot(m, 2));
    launch_finalize(red_slot(m, 2).partials, nb, FIN_STORE, nullptr, m->dscal.get() + 4, nullptr, s);
    GLK_HIP(hipMemcpyAsync(m->hscal + 4, m->dscal.get() + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    return m->hscal[5] > 0.0 ? m->hscal[4] / m->hscal[5] : 0.0;
}

}  // namespace glk

using namespace glk;

extern "C" {

gl_status gl_unet_create(int levels, int base_channels, gl_unet **out)
{
    return guarded([&] {
        if (!out) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_create: NULL out");
        if (levels < 1 || levels > 6 || base_channels < 32 || base_channels % 32 != 0 || (base_channels << (levels - 1)) > 1024)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_create: levels in 1..6, base channels a multiple of 32");
        gl_unet *u = new gl_unet();
        try {
            u->levels = levels;
            u->base = base_channels;
            const int L = levels;
            auto add = [&](int ci, int co, int k) {
                u->cin.push_back(ci);
                u->cout.push_back(co);
                u->ksz.push_back(k);
            };
            int c = 6;
            for (int l = 0; l < L; ++l) {
                add(c, base_channels << l, 3);
                add(base_channels << l, base_channels << l, 3);
                c = base_channels << l;
            }
            for (int l = L - 2; l >= 0; --l) {
                add(c + (base_channels << l), base_channels << l, 3);
                add(base_channels << l, base_channels << l, 3);
                c = base_channels << l;
            }
            add(c, 2, 1);
            size_t o = 0;
            for (size_t li = 0; li < u->cin.size(); ++li) {
                u->woff.push_back(o);
                o += (size_t)u->cout[li] * u->ksz[li] * u->ksz[li] * u->cin[li];
                u->boff.push_back(o);
                o += u->cout[li];
            }
            u->nparams = o;
            u->theta.alloc(o);
            u->m.alloc(o);
            u->v.alloc(o);
            u->grad.alloc(o);
            u->wf.resize(u->cin.size());
            u->wt.resize(u->cin.size());
            for (size_t li = 0; li + 1 < u->cin.size(); ++li) {
                const int cp = li == 0 ? 32 : u->cin[li];
                u->wf[li].alloc((size_t)u->cout[li] * 9 * cp);
                if (li > 0) u->wt[li].alloc((size_t)u->cout[li] * 9 * u->cin[li]);
            }
            GLK_HIP(hipMemset(u->theta.get(), 0, o * sizeof(float)));
            GLK_HIP(hipMemset(u->m.get(), 0, o * sizeof(float)));
            GLK_HIP(hipMemset(u->v.get(), 0, o * sizeof(float)));
            GLK_HIP(hipMemset(u->grad.get(), 0, o * sizeof(float)));
            unet_pack(u, nullptr);
            GLK_HIP(hipDeviceSynchronize());
        } catch (...) {
            delete u;
            throw;
        }
        *out = u;
    });
}

gl_status gl_unet_num_params(const gl_unet *u, int64_t *n)
{
    return guarded([&] {
        if (!u || !n) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_num_params: NULL argument");
        *n = (int64_t)u->nparams;
    });
}

gl_status gl_unet_set_params(gl_unet *u, const float *host_params)
{
    return guarded([&] {
        if (!u || !host_params) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_set_params: NULL argument");
        GLK_HIP(hipMemcpy(u->theta.get(), host_params, u->nparams * sizeof(float), hipMemcpyHostToDevice));
        GLK_HIP(hipMemset(u->m.get(), 0, u->nparams * sizeof(float)));
        GLK_HIP(hipMemset(u->v.get(), 0, u->nparams * sizeof(float)));
        u->adam_t = 0;
        unet_pack(u, nullptr);
        GLK_HIP(hipDeviceSynchronize());
    });
}

gl_status gl_unet_get_params(const gl_unet *u, float *host_params)
{
    return guarded([&] {
        if (!u || !host_params) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_get_params: NULL argument");
        GLK_HIP(hipDeviceSynchronize());
        GLK_HIP(hipMemcpy(host_params, u->theta.get(), u->nparams * sizeof(float), hipMemcpyDeviceToHost));
    });
}

gl_status gl_unet_predict(gl_unet *u, const gl_mesh *mesh, const void *psi, const void *psi_base, double mu,
                          double dmu, void *psi_out, gl_stream stream)
{
    return guarded([&] {
        if (!u || !mesh || !psi || !psi_base || !psi_out) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_predict: NULL argument");
        if (psi == psi_out || psi_base == psi_out) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_predict: output aliases an input");
        if (!(dmu != 0.0)) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_predict: dmu must be nonzero");
        check_grid(u, mesh);
        hipStream_t s = as_stream(stream);
        unet_alloc(u, mesh->g.N[0]);
        unet_forward(u, mesh, (const double2 *)psi, (const double2 *)psi_base, mu, dmu, s);
        const int P = mesh->g.n;
        k_predict<<<blocks_for(P), kBlock, 0, s>>>(P, (const double2 *)psi_base, u->o.get(), dmu, (double2 *)psi_out);
        GLK_CHECK_LAUNCH();
    });
}

gl_status gl_unet_loss_grad(gl_unet *u, const gl_mesh *mesh, const void *psi, const void *psi_base, double mu,
                            double dmu, const void *target, double *loss, float *host_grad, gl_stream stream)
{
    return guarded([&] {
        if (!u || !mesh || !psi || !psi_base || !target || !loss)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_loss_grad: NULL argument");
        if (!(dmu != 0.0)) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_loss_grad: dmu must be nonzero");
        check_grid(u, mesh);
        hipStream_t s = as_stream(stream);
        unet_alloc(u, mesh->g.N[0]);
        k_fill_f32<<<blocks_for((int64_t)u->nparams), kBlock, 0, s>>>((int)u->nparams, u->grad.get(), 0.0f);
        *loss = unet_loss(u, mesh, (const double2 *)psi, (const double2 *)psi_base, (const double2 *)target, mu, dmu,
                          1.0f, s);
        unet_backward(u, s);
        if (host_grad) {
            GLK_HIP(hipMemcpyAsync(host_grad, u->grad.get(), u->nparams * sizeof(float), hipMemcpyDeviceToHost, s));
            GLK_HIP(hipStreamSynchronize(s));
        }
    });
}

gl_status gl_unet_train_step(gl_unet *u, const gl_mesh *mesh, int count, const void *const *psi,
                             const void *const *psi_base, const double *mu, const double *dmu,
                             const void *const *target, const gl_adam_opts *opts, double *loss, gl_stream stream)
{
    return guarded([&] {
        if (!u || !mesh || !psi || !psi_base || !mu || !dmu || !target || !opts)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_train_step: NULL argument");
        if (count < 1) fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_train_step: count must be >= 1");
        if (!(opts->lr > 0.0) || !(opts->beta1 >= 0.0 && opts->beta1 < 1.0) || !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) ||
            !(opts->eps > 0.0))
            fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_train_step: invalid Adam options");
        check_grid(u, mesh);
        for (int k = 0; k < count; ++k)
            if (!psi[k] || !psi_base[k] || !target[k] || !(dmu[k] != 0.0))
                fail(GL_ERR_INVALID_ARGUMENT, "gl_unet_train_step: sample");
        hipStream_t s = as_stream(stream);
        unet_alloc(u, mesh->g.N[0]);
        k_fill_f32<<<blocks_for((int64_t)u->nparams), kBlock, 0, s>>>((int)u->nparams, u->grad.get(), 0.0f);
        double tot = 0.0;
        for (int k = 0; k < count; ++k) {
            tot += unet_loss(u, mesh, (const double2 *)psi[k], (const double2 *)psi_base[k], (const double2 *)target[k],
                             mu[k], dmu[k], 1.0f / count, s);
            unet_backward(u, s);
        }
        u->adam_t += 1;
        const double c1 = 1.0 - std::pow(opts->beta1, (double)u->adam_t);
        const double c2 = 1.0 - std::pow(opts->beta2, (double)u->adam_t);
        k_adam<<<blocks_for((int64_t)u->nparams), kBlock, 0, s>>>((int)u->nparams, u->theta.get(), u->m.get(),
                                                                  u->v.get(), u->grad.get(), (float)opts->lr,
                                                                  (float)opts->beta1, (float)opts->beta2,
                                                                  (float)opts->eps, (float)c1, (float)c2);
        unet_pack(u, s);
        GLK_CHECK_LAUNCH();
        GLK_HIP(hipStreamSynchronize(s));
        if (loss) *loss = tot / count;
    });
}

void gl_unet_destroy(gl_unet *u)
{
    if (u) (void)hipDeviceSynchronize();
    delete u;
}

}  // extern "C"
