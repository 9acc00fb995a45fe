// Learned near-interface correction of a 2x-coarsened membrane run: patch
// features from the lattice and the marker polygon, a four-layer 3 x 3
// convolutional network on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), its backward pass, Adam, training targets from a fine run,
// and the fused per-tile correction (the C ABI of include/ii_learned.h).
//
// Convolutions are implicit GEMMs: a wave owns 16 output channels (MFMA
// rows, the weights) by 16 output pixels (columns) and walks K = 9 taps x 32
// input channels in steps of 32, one tap per step, so that each lane's eight
// K values are eight consecutive channels of one pixel: one 16-byte LDS
// read.  Each lane ends with four consecutive output channels of one pixel,
// written back as one 8-byte store.  The weight fragments of a layer (at
// most 9 x 2) stay in registers for all of the wave's pixel tiles.
#include <math.h>

#include "common.hpp"
#include "../../include/ii_learned.h"

namespace iilbm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kPatch = 24, kOut = 16, kHalo = 4;
constexpr int kNP = II_CNN_NPARAM;
// map sizes of the input and of layers 1-4, channel counts
constexpr int HS[5] = {24, 22, 20, 18, 16};
constexpr int CI[4] = {4, 32, 32, 32};
constexpr int CO[4] = {32, 32, 32, 9};
// FP32 parameter offsets: W[dy][dx][ci][co] then b[co], layer by layer
constexpr int OFF_W[4] = {0, 1184, 10432, 19680};
constexpr int OFF_B[4] = {1152, 10400, 19648, 22272};
// Packed BF16 fragments (u16 elements): 512 per (k step, n tile).
// Forward: K = 9 * CI padded to 32-multiples, N = CO padded to 16-multiples.
constexpr int FKS[4] = {2, 9, 9, 9};
constexpr int FNT[4] = {2, 2, 2, 1};
constexpr int FOFF[4] = {0, 2048, 11264, 20480};
// Backward-data of layers 2-4: K = 9 taps x 32 output channels, N = 32.
constexpr int BOFF = 25088;
constexpr int BSIZE = 9 * 2 * 512;
constexpr int kPacked = BOFF + 3 * BSIZE;
// saved activations per patch: a1 | a2 | a3 (BF16, [pixel][32])
constexpr int SAVE_OFF[4] = {0, 0, 15488, 28288};
constexpr int kSave = 38656;
constexpr int kMaxCand = 256;    // candidate chords per patch
constexpr float kBand = 4.0f, kClip = 8.0f;

__device__ __forceinline__ u16 to_bf16(float f)
{
    // round to nearest even (finite inputs)
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(u16 h) { return __uint_as_float((unsigned)h << 16); }
// two floats to packed BF16 (lo in the low half), round to nearest even
// (v_cvt_pk_bf16_f32)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// ---------------------------------------------------------------------------
// Packing
// ---------------------------------------------------------------------------
__global__ void k_pack(const float* __restrict__ prm, u16* __restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kPacked) return;
    float v = 0.f;
    if (e < BOFF) {
        int l = 3;
        while (FOFF[l] > e) l--;
        const int r = e - FOFF[l], j = r & 7, lane = (r >> 3) & 63, idx = r >> 9;
        const int ks = idx / FNT[l], nt = idx % FNT[l];
        const int k = 32 * ks + 8 * (lane >> 4) + j, n = 16 * nt + (lane & 15);
        if (k < 9 * CI[l] && n < CO[l]) {
            const int t = k / CI[l], ci = k % CI[l];
            v = prm[OFF_W[l] + (t * CI[l] + ci) * CO[l] + n];
        }
    } else {
        const int r0 = e - BOFF, l = 1 + r0 / BSIZE, r = r0 % BSIZE;
        const int j = r & 7, lane = (r >> 3) & 63, idx = r >> 9;
        const int ks = idx >> 1, nt = idx & 1;
        const int k = 32 * ks + 8 * (lane >> 4) + j, ci = 16 * nt + (lane & 15);
        const int t = k >> 5, co = k & 31;
        if (co < CO[l]) v = prm[OFF_W[l] + (t * 32 + ci) * CO[l] + co];
    }
    out[e] = to_bf16(v);
}

// ---------------------------------------------------------------------------
// One convolution as an implicit GEMM on MFMA.
//   FULL = false: out[q] = sum_t src[q + d_t] W_t   (valid, map HSRC -> HSRC-2)
//   FULL = true:  out[q] = sum_t src[q - d_t] W'_t  (full, map HSRC -> HSRC+2,
//                 reads outside the source are zero)
// `src` is LDS [HSRC^2][CIN] BF16.  The weights are the MFMA's first operand
// (rows = output channels) and the pixels its second (columns), so that
// each lane ends with four consecutive channels of one pixel:
// epi(pixel, n0, v) gets channels n0 .. n0 + 3 of every output pixel.
// The layer's packed weight fragments are staged once per block in LDS `wl`
// (KS * NT * 512 elements) and then held in registers by every wave; the
// caller separates two uses of `wl` by a barrier.
// ---------------------------------------------------------------------------
constexpr int kWl = 9 * 2 * 512;

// `rows`: bit r set when output row r is needed; a pixel tile none of whose
// rows is needed is skipped (its outputs are left as they are).
// PS: elements between consecutive pixels of a 32-channel `src` (32 packed,
// or padded so that the lanes' 16-byte reads spread over the LDS banks).
template <int HSRC, int HDST, int CIN, int KS, int NT, bool FULL, class Epi, int PS = 32>
__device__ __forceinline__ void conv_mfma(const u16* src, const u16* __restrict__ frag, u16* wl,
                                          Epi epi, unsigned rows = ~0u)
{
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4;
    static_assert(KS * NT * 512 <= kWl, "fragment staging buffer");
    // per-lane LDS offsets (elements) of the two taps of the 4-channel input
    // layer: lane group g takes taps 8 ks + 2 g and + 1 (-1: past the 9 taps)
    int toff[CIN == 4 ? KS : 1][2];
    if (CIN == 4) {
#pragma unroll
        for (int ks = 0; ks < (CIN == 4 ? KS : 1); ks++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int t = 8 * ks + 2 * g + h;
                toff[ks][h] = t < 9 ? ((t / 3) * HSRC + t % 3) * 4 : -1;
            }
    }
    // wl == nullptr: `frag` already points into LDS
    const u16* fr = frag;
    if (wl) {
        for (int e = threadIdx.x; e < KS * NT * 64; e += blockDim.x)
            ((uint4*)wl)[e] = ((const uint4*)frag)[e];
        __syncthreads();
        fr = wl;
    }
    bf16x8 b[KS][NT];
#pragma unroll
    for (int ks = 0; ks < KS; ks++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
            b[ks][nt] = *(const bf16x8*)(fr + ((ks * NT + nt) * 64 + lane) * 8);
    constexpr int M = HDST * HDST, MT = (M + 15) / 16;
    static_assert(HDST <= 32, "row mask");
    rows = __builtin_amdgcn_readfirstlane(rows);   // the same in every lane
    for (int mt = wave; mt < MT; mt += nwave) {
        // rows of the tile's first and last pixel (at most two: HDST >= 16)
        const int r0 = (mt * 16) / HDST, r1 = min(mt * 16 + 15, M - 1) / HDST;
        if (!((rows >> r0) & ((2u << (r1 - r0)) - 1u))) continue;
        const int pix = mt * 16 + (lane & 15);
        const int p = min(pix, M - 1);
        const int py = p / HDST, px = p % HDST;
        // the pixel's own source position; taps add compile-time offsets
        const u16* sp = src + (py * HSRC + px) * (CIN == 32 ? PS : CIN) + (CIN == 32 ? 8 * g : 0);
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            bf16x8 a;
            if (CIN == 32) {
                const int dy = ks / 3, dx = ks % 3;
                int sy = 0, sx = 0;
                bool ok = true;
                if (FULL) {
                    sy = py - dy;
                    sx = px - dx;
                    ok = sy >= 0 && sy < HSRC && sx >= 0 && sx < HSRC;
                }
                if (!FULL) {
                    a = *(const bf16x8*)(sp + (dy * HSRC + dx) * PS);
                } else if (ok) {
                    a = *(const bf16x8*)(src + (sy * HSRC + sx) * PS + 8 * g);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) a[j] = (__bf16)0.0f;
                }
            } else {
                // four channels per tap
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    uint2 v = make_uint2(0u, 0u);
                    if (toff[CIN == 4 ? ks : 0][h] >= 0) v = *(const uint2*)(sp + toff[CIN == 4 ? ks : 0][h]);
                    a[4 * h + 0] = __builtin_bit_cast(__bf16, (u16)(v.x & 0xffffu));
                    a[4 * h + 1] = __builtin_bit_cast(__bf16, (u16)(v.x >> 16));
                    a[4 * h + 2] = __builtin_bit_cast(__bf16, (u16)(v.y & 0xffffu));
                    a[4 * h + 3] = __builtin_bit_cast(__bf16, (u16)(v.y >> 16));
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[ks][nt], a, acc[nt], 0, 0, 0);
        }
        if (pix < M) {
#pragma unroll
            for (int nt = 0; nt < NT; nt++) epi(pix, 16 * nt + 4 * g, acc[nt]);
        }
    }
}

// Forward layer l (0..3) of the network from LDS src to LDS dst (layers
// 0-2, ReLU, BF16) and, when `save` is set, to the saved activations.
// PSS / PSD: pixel strides (elements) of src and dst in LDS; the saved
// activations are always packed (32 per pixel).
template <int L, int PSS = 32, int PSD = 32>
__device__ __forceinline__ void hidden_layer(const u16* src, u16* dst, const u16* __restrict__ packed,
                                             const float* __restrict__ prm, u16* save, u16* wl,
                                             unsigned rows = ~0u)
{
    const float* bias = prm + OFF_B[L];
    auto epi = [&](int pix, int n0, f32x4 v) {
        const float4 bb = *(const float4*)(bias + n0);
        const uint2 h = make_uint2(pack_bf16(fmaxf(v[0] + bb.x, 0.f), fmaxf(v[1] + bb.y, 0.f)),
                                   pack_bf16(fmaxf(v[2] + bb.z, 0.f), fmaxf(v[3] + bb.w, 0.f)));
        *(uint2*)(dst + pix * PSD + n0) = h;
        if (save) *(uint2*)(save + pix * 32 + n0) = h;
    };
    conv_mfma<HS[L], HS[L + 1], CI[L], FKS[L], FNT[L], false, decltype(epi), PSS>(
        src, packed + FOFF[L], wl, epi, rows);
}

// ---------------------------------------------------------------------------
// Training forward: one block per patch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_forward(const float* __restrict__ prm,
                                                 const u16* __restrict__ packed,
                                                 const u16* __restrict__ in, float* __restrict__ out,
                                                 u16* __restrict__ save)
{
    __shared__ __align__(16) u16 bx[20 * 20 * 32];
    __shared__ __align__(16) u16 by[22 * 22 * 32];
    __shared__ __align__(16) u16 wl[kWl];
    const long long n = blockIdx.x;
    const u16* src = in + n * (kPatch * kPatch * 4);
    for (int e = threadIdx.x; e < kPatch * kPatch * 4 / 2; e += blockDim.x)
        ((unsigned*)bx)[e] = ((const unsigned*)src)[e];
    __syncthreads();
    u16* sv = save ? save + n * kSave : nullptr;
    hidden_layer<0>(bx, by, packed, prm, sv ? sv + SAVE_OFF[1] : nullptr, wl);
    __syncthreads();
    hidden_layer<1>(by, bx, packed, prm, sv ? sv + SAVE_OFF[2] : nullptr, wl);
    __syncthreads();
    hidden_layer<2>(bx, by, packed, prm, sv ? sv + SAVE_OFF[3] : nullptr, wl);
    __syncthreads();
    const float* b4 = prm + OFF_B[3];
    float* o = out + n * (kOut * kOut * 9);
    conv_mfma<18, 16, 32, 9, 1, false>(by, packed + FOFF[3], wl, [&](int pix, int n0, f32x4 v) {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (n0 + j < 9) o[pix * 9 + n0 + j] = v[j] + b4[n0 + j];
    });
}

// ---------------------------------------------------------------------------
// Backward: one block per patch; per-patch gradients go to a partial buffer
// that k_reduce sums over patches in a fixed order.
// ---------------------------------------------------------------------------
// Weight gradient of layer L: dW[(t, ci), co] = sum_p a[p + d_t, ci] dz[p, co]
// (MFMA rows (t, ci), columns co, K over the output pixels).
template <int L>
__device__ __forceinline__ void weight_grad(const u16* a, const u16* dz, float* part)
{
    constexpr int HA = HS[L], HD = HS[L + 1], CIN = CI[L], COUT = CO[L];
    constexpr int P = HD * HD, KS = (P + 31) / 32;
    constexpr int MT = (9 * CIN + 15) / 16, NT = (COUT + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int g = lane >> 4;
    for (int f = wave; f < MT * NT; f += nwave) {
        const int mt = f / NT, nt = f % NT;
        const int r = mt * 16 + (lane & 15);         // A row of this lane
        const int t = r / CIN, ci = r % CIN;
        const bool rok = r < 9 * CIN;
        const int dy = rok ? t / 3 : 0, dx = rok ? t % 3 : 0;
        const int co = nt * 16 + (lane & 15);        // B column of this lane
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < KS; ks++) {
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int p = 32 * ks + 8 * g + j;
                u16 ha = 0, hb = 0;
                if (p < P) {
                    const int py = p / HD, px = p % HD;
                    if (rok) ha = a[((py + dy) * HA + px + dx) * CIN + ci];
                    hb = dz[p * 32 + co];
                }
                av[j] = __builtin_bit_cast(__bf16, ha);
                bv[j] = __builtin_bit_cast(__bf16, hb);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int rr = mt * 16 + 4 * g + j;
            if (rr < 9 * CIN && co < COUT) {
                const int tt = rr / CIN, cc = rr % CIN;
                part[OFF_W[L] + (tt * CIN + cc) * COUT + co] = acc[j];
            }
        }
    }
    // bias: sum of dz over the pixels, one thread per channel in pixel order
    if ((int)threadIdx.x < COUT) {
        float s = 0.f;
        for (int p = 0; p < P; p++) s += from_bf16(dz[p * 32 + threadIdx.x]);
        part[OFF_B[L] + threadIdx.x] = s;
    }
}

// dz of the input of layer L (1..3): (sum_t dz_next[q - d_t] W_t^T) * (a[q] > 0)
template <int L>
__device__ __forceinline__ void data_grad(const u16* dz_next, const u16* a, u16* dz,
                                          const u16* __restrict__ packed, u16* wl)
{
    conv_mfma<HS[L + 1], HS[L], 32, 9, 2, true>(
        dz_next, packed + BOFF + (L - 1) * BSIZE, wl, [&](int pix, int n0, f32x4 v) {
            // ReLU'(z) from the saved activation: zero where a <= 0
            const uint2 av = *(const uint2*)(a + pix * 32 + n0);
            const unsigned ah[4] = {av.x & 0xffffu, av.x >> 16, av.y & 0xffffu, av.y >> 16};
            float w[4];
#pragma unroll
            for (int j = 0; j < 4; j++) w[j] = ah[j] != 0 && !(ah[j] & 0x8000u) ? v[j] : 0.f;
            *(uint2*)(dz + pix * 32 + n0) = make_uint2(pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]));
        });
}

template <int L>
__device__ __forceinline__ void load_act(u16* dst, const u16* __restrict__ src)
{
    constexpr int n = HS[L] * HS[L] * CI[L] / 2;
    for (int e = threadIdx.x; e < n; e += blockDim.x) ((unsigned*)dst)[e] = ((const unsigned*)src)[e];
}

__global__ void k_count(const uint8_t* __restrict__ mask, long long n, int* __restrict__ count)
{
    __shared__ int s[256];
    int c = 0;
    for (long long e = threadIdx.x; e < n; e += blockDim.x) c += mask[e] ? 1 : 0;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = s[0];
}

__global__ __launch_bounds__(256) void k_backward(
    const u16* __restrict__ packed, const u16* __restrict__ in, const u16* __restrict__ save,
    const float* __restrict__ out, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, const int* __restrict__ count, float* __restrict__ part)
{
    __shared__ __align__(16) u16 ba[22 * 22 * 32];
    __shared__ __align__(16) u16 bz0[22 * 22 * 32];
    __shared__ __align__(16) u16 bz1[22 * 22 * 32];
    __shared__ float red[256];
    __shared__ __align__(16) u16 wl[kWl];
    const long long n = blockIdx.x;
    float* pp = part + n * (kNP + 1);
    const float* o = out + n * (kOut * kOut * 9);
    const float* tg = target + n * (kOut * kOut * 9);
    const uint8_t* mk = mask + n * (kOut * kOut);
    const float scale = 2.f / (9.f * (float)max(*count, 1));
    // dz of the output: 2 m (out - target) / (9 sum m); channels 9..31 zero
    float ls = 0.f;
    for (int e = threadIdx.x; e < kOut * kOut * 32; e += blockDim.x) {
        const int p = e >> 5, c = e & 31;
        float v = 0.f;
        if (c < 9 && mk[p]) {
            const float d = o[p * 9 + c] - tg[p * 9 + c];
            v = scale * d;
            ls += d * d;
        }
        bz0[e] = to_bf16(v);
    }
    red[threadIdx.x] = ls;
    load_act<3>(ba, save + n * kSave + SAVE_OFF[3]);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) pp[kNP] = red[0];
    weight_grad<3>(ba, bz0, pp);
    data_grad<3>(bz0, ba, bz1, packed, wl);
    __syncthreads();
    load_act<2>(ba, save + n * kSave + SAVE_OFF[2]);
    __syncthreads();
    weight_grad<2>(ba, bz1, pp);
    data_grad<2>(bz1, ba, bz0, packed, wl);
    __syncthreads();
    load_act<1>(ba, save + n * kSave + SAVE_OFF[1]);
    __syncthreads();
    weight_grad<1>(ba, bz0, pp);
    data_grad<1>(bz0, ba, bz1, packed, wl);
    __syncthreads();
    load_act<0>(ba, in + n * (kPatch * kPatch * 4));
    __syncthreads();
    weight_grad<0>(ba, bz1, pp);
}

// grad[j] = sum over patches in order; loss = sum of squares / (9 count)
__global__ void k_reduce(const float* __restrict__ part, int n, const int* __restrict__ count,
                         float* __restrict__ grad, float* __restrict__ loss)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > kNP) return;
    float s = 0.f;
    for (int q = 0; q < n; q++) s += part[(long long)q * (kNP + 1) + j];
    if (j < kNP)
        grad[j] = s;
    else
        loss[0] = s / (9.f * (float)max(*count, 1));
}

__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ grad,
                       float* __restrict__ m, float* __restrict__ v, float lr, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kNP) return;
    const float g = grad[j];
    const float mj = 0.9f * m[j] + 0.1f * g;
    const float vj = 0.999f * v[j] + 0.001f * g * g;
    m[j] = mj;
    v[j] = vj;
    prm[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// Band tiles, features and the fused correction
// ---------------------------------------------------------------------------
// One block per instance: every chord marks the tiles that its box, grown
// by 4.5, meets (a tile is in the band when some chord does), then the marked
// tiles are listed in row-major order.
__global__ void k_band_tiles(const InstDev* __restrict__ insts, const double2* __restrict__ Xall,
                             int cap, int* __restrict__ tiles, int* __restrict__ count)
{
    const InstDev I = insts[blockIdx.x];
    __shared__ int flag[1024];
    __shared__ int base[1024];
    const int nt = I.tiles_x * I.tiles_y;
    const double2* X = Xall + I.mk_off;
    const int N = I.n_markers;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) flag[t] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double2 a = X[k], b = X[(k + 1) % N];
        // tile (tx, ty) covers nodes [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15]
        const int tx0 = max(0, (int)ceil((fmin(a.x, b.x) - 4.5 - 15.0) / kTile));
        const int tx1 = min(I.tiles_x - 1, (int)floor((fmax(a.x, b.x) + 4.5) / kTile));
        const int ty0 = max(0, (int)ceil((fmin(a.y, b.y) - 4.5 - 15.0) / kTile));
        const int ty1 = min(I.tiles_y - 1, (int)floor((fmax(a.y, b.y) + 4.5) / kTile));
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) flag[ty * I.tiles_x + tx] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int t = 0; t < nt; t++) {
            base[t] = c;
            c += flag[t];
        }
        count[blockIdx.x] = min(c, cap);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += blockDim.x)
        if (flag[t] && base[t] < cap)
            ((int2*)tiles)[(long long)blockIdx.x * cap + base[t]] =
                make_int2(t % I.tiles_x, t / I.tiles_x);
}

constexpr int kRowCap = 16;   // crossings of one patch row inside the patch

struct GeomShared {
    float4 cand[kMaxCand];        // chords (a, b - a) within 8 lu of the patch, relative,
                                  // sorted by min y
    float cinv[kMaxCand];         // 1 / |b - a|^2 (0 for a degenerate chord)
    float cmin[kMaxCand];         // their min y
    float4 tmp[kMaxCand];         // unsorted staging
    float tkey[kMaxCand];         // and its min y
    float rowx[kPatch][kRowCap];  // x of the crossings of each patch row inside the patch
    int rown[kPatch];             // their count
    int rowpar[kPatch];           // parity of the crossings right of the patch
    int ncand, overflow;
};
struct FlowShared {
    float raw[kPatch * kPatch][3];   // scaled rho - 1, u_x, u_y
    float red[16];
};
constexpr int kPatchThreads = 256;

// Features of the 24 x 24 patch around tile (tx, ty), in two parts: the
// geometry (from the markers alone) and the flow (from the lattice alone),
// so that the first can run before the lattice it pairs with exists.
// Geometry: the signed-distance channel of the BF16 input and the flags
// (bit 0 inside, bit 1 band).
//  - inside: the even-odd rule on the ray from the node towards +x, an
//    edge counting when it straddles the node's row (half-open in y) and
//    crosses it right of the node; every chord's crossing of every patch row
//    is found once per patch;
//  - distance: the nearest chord among those within 8 lu of the patch,
//    searched in a window of the chords sorted by their lowest y.
__device__ void patch_geom(const InstDev& I, const double2* __restrict__ X, int tx, int ty,
                           const ii_cnn_scales& sc, GeomShared& S, u16* in, uint8_t* flags,
                           int* err)
{
    const int N = I.n_markers;
    const int ox = tx * kTile - kHalo, oy = ty * kTile - kHalo;  // patch origin node
    for (int r = threadIdx.x; r < kPatch; r += blockDim.x) {
        S.rown[r] = 0;
        S.rowpar[r] = 0;
    }
    if (threadIdx.x == 0) {
        S.ncand = 0;
        S.overflow = 0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double2 a = X[k], b = X[(k + 1) % N];
        // rows y = oy + r that the edge straddles: (a.y > y) != (b.y > y)
        const double lo = fmin(a.y, b.y), hi = fmax(a.y, b.y);
        const int r0 = max(0, (int)ceil(lo) - oy), r1 = min(kPatch - 1, (int)ceil(hi) - 1 - oy);
        for (int r = r0; r <= r1; r++) {
            const double y = (double)(oy + r);
            if ((a.y > y) == (b.y > y)) continue;
            const double xc = a.x + (y - a.y) * (b.x - a.x) / (b.y - a.y);
            if (xc > (double)(ox + kPatch - 1)) {
                atomicXor(&S.rowpar[r], 1);
            } else if (xc > (double)ox) {
                const int c = atomicAdd(&S.rown[r], 1);
                if (c < kRowCap) S.rowx[r][c] = (float)(xc - ox);
                else S.overflow = 1;
            }
        }
        const double m = kClip;
        if (fmax(a.x, b.x) >= ox - m && fmin(a.x, b.x) <= ox + kPatch - 1 + m && hi >= oy - m &&
            lo <= oy + kPatch - 1 + m) {
            const int c = atomicAdd(&S.ncand, 1);
            if (c < kMaxCand) {
                const float ax = (float)(a.x - ox), ay = (float)(a.y - oy);
                const float bx = (float)(b.x - ox), by = (float)(b.y - oy);
                S.tmp[c] = make_float4(ax, ay, bx - ax, by - ay);
                S.tkey[c] = fminf(ay, by);
            } else {
                S.overflow = 1;
            }
        }
    }
    __syncthreads();
    const int nc = min(S.ncand, kMaxCand);
    // rank sort by the lowest y (ties by position in the staging list)
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const float4 v = S.tmp[c];
        const float key = S.tkey[c];
        int r = 0;
        for (int d = 0; d < nc; d++) {
            const float kd = S.tkey[d];
            r += (kd < key || (kd == key && d < c)) ? 1 : 0;
        }
        const float ll = v.z * v.z + v.w * v.w;
        S.cand[r] = v;
        S.cinv[r] = ll > 0.f ? 1.f / ll : 0.f;
        S.cmin[r] = key;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPatch * kPatch; q += blockDim.x) {
        const int py = q / kPatch, px = q % kPatch;
        const float fx = (float)px, fy = (float)py;
        // chords reach at most 2 lu, so those within 8 of the row have their
        // lowest y in [py - 10, py + 8]
        int lo = 0, hi = nc;
        {
            int a0 = 0, a1 = nc;
            while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (S.cmin[mid] < fy - (kClip + 2.f)) a0 = mid + 1; else a1 = mid;
            }
            lo = a0;
            a1 = nc;
            while (a0 < a1) {
                const int mid = (a0 + a1) >> 1;
                if (S.cmin[mid] <= fy + kClip) a0 = mid + 1; else a1 = mid;
            }
            hi = a0;
        }
        float d2 = kClip * kClip;
        for (int c = lo; c < hi; c++) {
            const float4 s = S.cand[c];
            float t = ((fx - s.x) * s.z + (fy - s.y) * s.w) * S.cinv[c];
            t = fminf(fmaxf(t, 0.f), 1.f);
            const float qx = s.x + t * s.z - fx, qy = s.y + t * s.w - fy;
            d2 = fminf(d2, qx * qx + qy * qy);
        }
        int ins = S.rowpar[py];
        const int nr = min(S.rown[py], kRowCap);
        for (int c = 0; c < nr; c++) ins ^= S.rowx[py][c] > fx ? 1 : 0;
        const float dist = sqrtf(d2);
        const float sd = ins ? -dist : dist;
        in[q * 4 + 3] = to_bf16(sd * sc.in_scale[3]);
        flags[q] = (uint8_t)(ins | (dist <= kBand ? 2 : 0));
    }
    // more chords near the patch than the lists hold: the features are
    // incomplete, which the handle reports as ECAPACITY
    if (threadIdx.x == 0 && S.overflow) atomicOr(err, (int)kErrCapacity);
}

// Flow: the three flow channels (rho - 1, u_x, u_y of the pulled
// distributions, u = sum_i e_i f_i, times their input scales), divided by the
// patch amplitude s = max(rms over the patch of their vector, 1e-6), which
// goes to *pscale: the network sees amplitude-free flow and its output is
// multiplied back by s.
template <typename T>
__device__ void patch_flow(const InstDev& I, const T* __restrict__ A, int tx, int ty,
                           const ii_cnn_scales& sc, FlowShared& S, u16* in, float* pscale)
{
    const int ox = tx * kTile - kHalo, oy = ty * kTile - kHalo;
    for (int q = threadIdx.x; q < kPatch * kPatch; q += blockDim.x) {
        int gx = (ox + q % kPatch) % I.nx, gy = (oy + q / kPatch) % I.ny;
        if (gx < 0) gx += I.nx;
        if (gy < 0) gy += I.ny;
        float d[9];
        pull<T, float>(I, A, gx, gy, d);
        float r, ux, uy;
        moments<float>(d, r, ux, uy);
        S.raw[q][0] = r * sc.in_scale[0];
        S.raw[q][1] = ux * sc.in_scale[1];
        S.raw[q][2] = uy * sc.in_scale[2];
    }
    __syncthreads();
    float ss = 0.f;
    for (int q = threadIdx.x; q < kPatch * kPatch; q += blockDim.x)
        ss += S.raw[q][0] * S.raw[q][0] + S.raw[q][1] * S.raw[q][1] + S.raw[q][2] * S.raw[q][2];
    // per-wave sums, then the waves' sums in order
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
    if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = ss;
    __syncthreads();
    float tot = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) tot += S.red[w];
    const float amp = fmaxf(sqrtf(tot / (float)(kPatch * kPatch)), 1e-6f);
    const float inv = 1.f / amp;
    for (int q = threadIdx.x; q < kPatch * kPatch; q += blockDim.x) {
        in[q * 4 + 0] = to_bf16(S.raw[q][0] * inv);
        in[q * 4 + 1] = to_bf16(S.raw[q][1] * inv);
        in[q * 4 + 2] = to_bf16(S.raw[q][2] * inv);
    }
    if (threadIdx.x == 0) *pscale = amp;
}

// Grid (n_inst, G): block y of instance x takes the instance's band tiles
// y, y + G, ... below its count, so that the launch does not depend on the
// counts, which only the device knows, and empty slots cost no block.
constexpr int kSlotStride = 64;

__global__ __launch_bounds__(kPatchThreads) void k_patch_geom(
    const InstDev* __restrict__ insts, const double2* __restrict__ Xall, ii_cnn_scales sc, int cap,
    const int* __restrict__ tiles, const int* __restrict__ count, u16* __restrict__ in,
    uint8_t* __restrict__ flags, int* __restrict__ err)
{
    const int inst = blockIdx.x, n = count[inst];
    if ((int)blockIdx.y >= n) return;
    const InstDev I = insts[inst];
    __shared__ GeomShared S;
    for (int r = blockIdx.y; r < n; r += gridDim.y) {
        if (r != (int)blockIdx.y) __syncthreads();   // the previous patch is done with S
        const long long slot = (long long)inst * cap + r;
        const int2 t = ((const int2*)tiles)[slot];
        patch_geom(I, Xall + I.mk_off, t.x, t.y, sc, S, in + slot * (kPatch * kPatch * 4),
                   flags + slot * (kPatch * kPatch), err + inst);
    }
}

template <typename T>
__global__ __launch_bounds__(kPatchThreads) void k_patch_flow(
    const InstDev* __restrict__ insts, const void* A0, ii_cnn_scales sc, int cap,
    const int* __restrict__ tiles, const int* __restrict__ count, u16* __restrict__ in,
    float* __restrict__ pscale)
{
    const int inst = blockIdx.x, n = count[inst];
    if ((int)blockIdx.y >= n) return;
    const InstDev I = insts[inst];
    __shared__ FlowShared S;
    for (int r = blockIdx.y; r < n; r += gridDim.y) {
        if (r != (int)blockIdx.y) __syncthreads();   // the previous patch is done with S
        const long long slot = (long long)inst * cap + r;
        const int2 t = ((const int2*)tiles)[slot];
        patch_flow<T>(I, (const T*)A0, t.x, t.y, sc, S, in + slot * (kPatch * kPatch * 4),
                      pscale + slot);
    }
}

// Targets: f^eq(rho_c, u_hat) - f^eq(rho_c, u_c) in network units (over the
// output scale and the patch amplitude), u_hat = 2 u_f at fine node (2x, 2y);
// the
// band mask of the output pixels from the patch flags.
template <typename TC, typename TF>
__global__ void k_targets(const InstDev* __restrict__ ic, const void* Ac,
                          const InstDev* __restrict__ iff, const void* Af, float inv_out, int cap,
                          const int* __restrict__ tiles, const int* __restrict__ count,
                          const uint8_t* __restrict__ flags, const float* __restrict__ pscale,
                          float* __restrict__ target, uint8_t* __restrict__ mask)
{
    const int inst = blockIdx.x / cap, r = blockIdx.x % cap;
    if (r >= count[inst]) return;
    const InstDev C = ic[inst], F = iff[inst];
    const int2 t = ((const int2*)tiles)[blockIdx.x];
    const long long slot = blockIdx.x;
    const int q = threadIdx.x;   // 256 output nodes
    const int oy = q / kOut, ox = q % kOut;
    const int x = t.x * kTile + ox, y = t.y * kTile + oy;
    double dc[9], df[9];
    pull<TC, double>(C, (const TC*)Ac, x, y, dc);
    pull<TF, double>(F, (const TF*)Af, 2 * x, 2 * y, df);
    double rc, uc, vc, rf, uf, vf;
    moments<double>(dc, rc, uc, vc);
    moments<double>(df, rf, uf, vf);
    // velocity target only: the density stays the coarse one
    rf = rc;
    uf *= 2.0;
    vf *= 2.0;
    // He-Luo equilibrium deviations w_i [drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u]
    float* tg = target + slot * (kOut * kOut * 9) + q * 9;
    const double inv = (double)inv_out / (double)pscale[slot];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const double ef = EX[i] * uf + EY[i] * vf, ec = EX[i] * uc + EY[i] * vc;
        const double a = WD[i] * (rf + 3.0 * ef + 4.5 * ef * ef - 1.5 * (uf * uf + vf * vf));
        const double b = WD[i] * (rc + 3.0 * ec + 4.5 * ec * ec - 1.5 * (uc * uc + vc * vc));
        tg[i] = (float)((a - b) * inv);
    }
    const uint8_t fl = flags[slot * (kPatch * kPatch) + (oy + kHalo) * kPatch + ox + kHalo];
    mask[slot * (kOut * kOut) + q] = (fl & 2) ? 1 : 0;
}

// The network and the masked add of one coarse step on the patches that
// k_patch_geom and k_patch_flow built from the state before any tile was corrected (a tile's
// halo overlaps its neighbours' nodes).  Persistent: one block of twelve
// waves per compute unit (LDS holds one block's buffers and fragments)
// stages every forward weight fragment in LDS once and
// then walks the band tiles of all instances, listed instance by instance,
// in a grid stride, so that the work is balanced and no layer waits on L2
// for its fragments.
constexpr int kMaxInstLds = 4096;   // instances whose tile offsets fit in LDS
constexpr int kFwdFrag = FOFF[3] + 9 * 512;
constexpr int kCorrThreads = 768;   // twelve waves: three per SIMD
constexpr int kPadPix = 40;         // LDS elements per activation pixel in k_correct

template <typename T>
__global__ __launch_bounds__(kCorrThreads) void k_correct(const InstDev* __restrict__ insts, int n_inst,
                                                 void* A0, const float* __restrict__ prm,
                                                 const u16* __restrict__ packed, ii_cnn_scales sc,
                                                 int cap, const int* __restrict__ tiles,
                                                 const int* __restrict__ count,
                                                 const u16* __restrict__ in,
                                                 const uint8_t* __restrict__ flags,
                                                 const float* __restrict__ pscale)
{
    // activations with each pixel's 32 channels padded to kPadPix elements
    // (80 bytes), so that the 16 pixels of an MFMA operand read, and the
    // epilogue's 8-byte stores, fall on distinct LDS banks
    __shared__ __align__(16) u16 bx[20 * 20 * kPadPix];
    __shared__ __align__(16) u16 by[22 * 22 * kPadPix];
    __shared__ __align__(16) u16 wf[kFwdFrag];
    __shared__ int first[kMaxInstLds + 1];   // first[j]: band tiles of instances < j
    __shared__ __align__(16) u16 pin[2][kPatch * kPatch * 4];   // input patches, double buffered
    __shared__ __align__(4) uint8_t pfl[2][kPatch * kPatch];     // and their flags
    __shared__ unsigned band_rows[4];
    for (int e = threadIdx.x; e < kFwdFrag / 8; e += blockDim.x)
        ((uint4*)wf)[e] = ((const uint4*)packed)[e];
    // exclusive scan of the counts, one block width at a time
    __shared__ int part[kCorrThreads];
    int carry = 0;
    for (int j0 = 0; j0 < n_inst; j0 += kCorrThreads) {
        const int j = j0 + threadIdx.x;
        const int c = j < n_inst ? min(count[j], cap) : 0;
        part[threadIdx.x] = c;
        __syncthreads();
        for (int o = 1; o < kCorrThreads; o <<= 1) {
            const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (j < n_inst) first[j + 1] = carry + part[threadIdx.x];
        carry += part[kCorrThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) first[0] = 0;
    __syncthreads();
    const int total = first[n_inst];
    // slot of the k-th band tile: its instance is the last j with first[j] <= k
    auto slot_of = [&](int k, int& inst) -> long long {
        int lo = 0, hi = n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (first[mid] <= k) lo = mid; else hi = mid;
        }
        inst = __builtin_amdgcn_readfirstlane(lo);
        return (long long)inst * cap + (k - first[inst]);
    };
    // a patch and its flags are 1152 + 144 dwords: two and at most one per thread
    constexpr int kInW = kPatch * kPatch * 2, kFlW = kPatch * kPatch / 4;
    static_assert(kInW <= 2 * kCorrThreads && kFlW <= kCorrThreads, "patch staging");
    unsigned r0 = 0, r1 = 0, rf = 0;
    auto fetch = [&](long long slot) {
        const unsigned* si = (const unsigned*)(in + slot * (kPatch * kPatch * 4));
        const unsigned* sf = (const unsigned*)(flags + slot * (kPatch * kPatch));
        r0 = si[threadIdx.x];
        if (threadIdx.x + kCorrThreads < kInW) r1 = si[threadIdx.x + kCorrThreads];
        if (threadIdx.x < kFlW) rf = sf[threadIdx.x];
    };
    auto stage = [&](int b) {
        ((unsigned*)pin[b])[threadIdx.x] = r0;
        if (threadIdx.x + kCorrThreads < kInW) ((unsigned*)pin[b])[threadIdx.x + kCorrThreads] = r1;
        if (threadIdx.x < kFlW) ((unsigned*)pfl[b])[threadIdx.x] = rf;
    };
    T* A = (T*)A0;
    int cur = 0;
    if ((int)blockIdx.x < total) {
        int inst;
        fetch(slot_of(blockIdx.x, inst));
        stage(0);
    }
    for (int k = blockIdx.x; k < total; k += gridDim.x) {
        __syncthreads();   // pin[cur] staged; the previous tile is done with every buffer
        int inst;
        const long long slot = slot_of(k, inst);
        const InstDev I = insts[inst];
        const int2 t = ((const int2*)tiles)[slot];
        const float os = sc.out_scale * pscale[slot];
        // the next tile's patch travels while this one is computed
        const int kn = k + gridDim.x;
        if (kn < total) {
            int in_n;
            fetch(slot_of(kn, in_n));
        }
        const uint8_t* fl = pfl[cur];
        // Output rows with a band node (the others get no correction), and
        // the rows of each hidden layer that feed them: a valid 3 x 3
        // convolution's output row r reads input rows r .. r + 2.  The first
        // four waves see four output rows each.
        if (threadIdx.x < kOut * kOut) {
            const int oy = threadIdx.x / kOut, ox = threadIdx.x % kOut;
            const unsigned long long b =
                __ballot((fl[(oy + kHalo) * kPatch + ox + kHalo] & 2) != 0);
            if ((threadIdx.x & 63) == 0) {
                unsigned m = 0;
                for (int r = 0; r < 4; r++)
                    if ((b >> (16 * r)) & 0xffffull) m |= 1u << r;
                band_rows[threadIdx.x >> 6] = m << (4 * (threadIdx.x >> 6));
            }
        }
        __syncthreads();
        const unsigned m4 = band_rows[0] | band_rows[1] | band_rows[2] | band_rows[3];
        const unsigned m3 = (m4 | m4 << 1 | m4 << 2) & 0x3ffffu;
        const unsigned m2 = (m3 | m3 << 1 | m3 << 2) & 0xfffffu;
        const unsigned m1 = (m2 | m2 << 1 | m2 << 2) & 0x3fffffu;
        if (m4) {
            hidden_layer<0, 32, kPadPix>(pin[cur], by, wf, prm, nullptr, nullptr, m1);
            __syncthreads();
            hidden_layer<1, kPadPix, kPadPix>(by, bx, wf, prm, nullptr, nullptr, m2);
            __syncthreads();
            hidden_layer<2, kPadPix, kPadPix>(bx, by, wf, prm, nullptr, nullptr, m3);
            __syncthreads();
            const float* b4 = prm + OFF_B[3];
            T* base = A + I.lat_off;
            auto epi4 = [&](int pix, int n0, f32x4 v) {
                if (n0 >= 9) return;
                const int oy = pix / kOut, ox = pix % kOut;
                const int q = (oy + kHalo) * kPatch + ox + kHalo;
                const uint8_t f = fl[q];
                if (!(f & 2)) return;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int c = n0 + j;
                    if (c >= 9) break;
                    if (c != 0) {
                        const uint8_t fs = fl[q - EY[c] * kPatch - EX[c]];
                        if ((fs & 1) != (f & 1)) continue;   // a link across the polygon
                    }
                    // pre-collision f_c(x) is the value stored at x - e_c (no
                    // other tile touches it)
                    int x = t.x * kTile + ox - EX[c], y = t.y * kTile + oy - EY[c];
                    x = x < 0 ? x + I.nx : (x >= I.nx ? x - I.nx : x);
                    y = y < 0 ? y + I.ny : (y >= I.ny ? y - I.ny : y);
                    T* p = base + c * I.plane + (long long)y * I.pitch + x;
                    Store<T>::st(p, Store<T>::ld(p, I.scale) + os * (v[j] + b4[c]), I.inv_scale);
                }
            };
            conv_mfma<18, 16, 32, 9, 1, false, decltype(epi4), kPadPix>(by, wf + FOFF[3], nullptr,
                                                                        epi4, m4);
        }
        if (kn < total) stage(cur ^ 1);
        cur ^= 1;
    }
}

// The masked add of given corrections (network units), one block per slot.
template <typename T>
__global__ void k_apply(const InstDev* __restrict__ insts, void* A0, float out_scale, int cap,
                        const int* __restrict__ tiles, const int* __restrict__ count,
                        const uint8_t* __restrict__ flags, const float* __restrict__ pscale,
                        const float* __restrict__ out)
{
    const int inst = blockIdx.x / cap, r = blockIdx.x % cap;
    if (r >= count[inst]) return;
    const InstDev I = insts[inst];
    const int2 t = ((const int2*)tiles)[blockIdx.x];
    const long long slot = blockIdx.x;
    const int oy = threadIdx.x / kOut, ox = threadIdx.x % kOut;
    const uint8_t* fl = flags + slot * (kPatch * kPatch);
    const int q = (oy + kHalo) * kPatch + ox + kHalo;
    const uint8_t f = fl[q];
    if (!(f & 2)) return;
    T* base = (T*)A0 + I.lat_off;
    for (int c = 0; c < 9; c++) {
        if (c != 0 && (fl[q - EY[c] * kPatch - EX[c]] & 1) != (f & 1)) continue;
        int x = t.x * kTile + ox - EX[c], y = t.y * kTile + oy - EY[c];
        x = x < 0 ? x + I.nx : (x >= I.nx ? x - I.nx : x);
        y = y < 0 ? y + I.ny : (y >= I.ny ? y - I.ny : y);
        T* p = base + c * I.plane + (long long)y * I.pitch + x;
        const float d = out_scale * pscale[slot] * out[slot * (kOut * kOut * 9) + threadIdx.x * 9 + c];
        Store<T>::st(p, Store<T>::ld(p, I.scale) + d, I.inv_scale);
    }
}

// Learned correction needs periodic membranes on 16-multiples (the patches
// wrap) and the same storage across instances.
int check_learned(const HandleView& v)
{
    if (v.failed) return II_LBM_ESTATE;
    for (int j = 0; j < v.n_inst; j++) {
        const InstDev& I = v.inst[j];
        if (I.iface != II_LBM_IF_MEMBRANE || I.bounded || I.nx % kTile || I.ny % kTile ||
            I.tiles_x * I.tiles_y > 1024 || I.storage != v.inst[0].storage)
            return II_LBM_EINVAL;
    }
    return II_LBM_OK;
}

int err(hipError_t e) { return e == hipSuccess ? II_LBM_OK : II_LBM_EDEVICE; }

dim3 slot_grid(const HandleView& v, const LearnedCfg& c)
{
    return dim3((unsigned)v.n_inst, (unsigned)std::min(c.cap, kSlotStride));
}

}  // namespace

int learned_validate(const HandleView& v, int cap)
{
    const int rc = check_learned(v);
    if (rc) return rc;
    if (v.n_inst > kMaxInstLds || cap < 1) return II_LBM_EINVAL;
    for (int j = 0; j < v.n_inst; j++)
        if (cap < v.inst[j].tiles_x * v.inst[j].tiles_y) return II_LBM_EINVAL;
    return II_LBM_OK;
}

hipError_t learned_band(const HandleView& v, const LearnedCfg& c)
{
    hipLaunchKernelGGL(k_band_tiles, dim3(v.n_inst), dim3(256), 0, v.stream, v.d_inst,
                       v.P.X[v.parity], c.cap, c.tiles, c.count);
    return hipGetLastError();
}

hipError_t learned_geom(const HandleView& v, const LearnedCfg& c)
{
    hipLaunchKernelGGL(k_patch_geom, slot_grid(v, c), dim3(kPatchThreads), 0, v.stream, v.d_inst,
                       v.P.X[v.parity], c.sc, c.cap, (const int*)c.tiles, (const int*)c.count,
                       (u16*)c.in, c.flags, v.P.err);
    return hipGetLastError();
}

hipError_t learned_flow(const HandleView& v, const LearnedCfg& c)
{
    if (v.inst[0].storage == II_LBM_FP16)
        hipLaunchKernelGGL(k_patch_flow<_Float16>, slot_grid(v, c), dim3(kPatchThreads), 0,
                           v.stream, v.d_inst, v.P.lat[v.parity], c.sc, c.cap,
                           (const int*)c.tiles, (const int*)c.count, (u16*)c.in, c.pscale);
    else
        hipLaunchKernelGGL(k_patch_flow<float>, slot_grid(v, c), dim3(kPatchThreads), 0,
                           v.stream, v.d_inst, v.P.lat[v.parity], c.sc, c.cap,
                           (const int*)c.tiles, (const int*)c.count, (u16*)c.in, c.pscale);
    return hipGetLastError();
}

hipError_t learned_infer(const HandleView& v, const LearnedCfg& c)
{
    const dim3 grid((unsigned)std::max(1, v.n_cu));
    if (v.inst[0].storage == II_LBM_FP16)
        hipLaunchKernelGGL(k_correct<_Float16>, grid, dim3(kCorrThreads), 0, v.stream, v.d_inst,
                           v.n_inst, v.P.lat[v.parity], c.params, (const u16*)c.packed, c.sc,
                           c.cap, (const int*)c.tiles, (const int*)c.count, (const u16*)c.in,
                           c.flags, c.pscale);
    else
        hipLaunchKernelGGL(k_correct<float>, grid, dim3(kCorrThreads), 0, v.stream, v.d_inst,
                           v.n_inst, v.P.lat[v.parity], c.params, (const u16*)c.packed, c.sc,
                           c.cap, (const int*)c.tiles, (const int*)c.count, (const u16*)c.in,
                           c.flags, c.pscale);
    return hipGetLastError();
}

}  // namespace iilbm

using namespace iilbm;

extern "C" {

size_t ii_cnn_packed_bytes(void) { return (size_t)kPacked * sizeof(u16); }
size_t ii_cnn_save_bytes(void) { return (size_t)kSave * sizeof(u16); }
size_t ii_cnn_work_bytes(int32_t n)
{
    return n < 1 ? 0 : (size_t)n * (kNP + 1) * sizeof(float) + 256;
}

int ii_cnn_pack(const float* params, void* packed, void* stream)
{
    if (!params || !packed) return II_LBM_EINVAL;
    hipLaunchKernelGGL(k_pack, dim3((kPacked + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, (u16*)packed);
    return err(hipGetLastError());
}

int ii_cnn_forward(const float* params, const void* packed, const uint16_t* in, int32_t n,
                   float* out, uint16_t* save, void* stream)
{
    if (!params || !packed || !in || !out || n < 0) return II_LBM_EINVAL;
    if (n == 0) return II_LBM_OK;
    hipLaunchKernelGGL(k_forward, dim3(n), dim3(256), 0, (hipStream_t)stream, params,
                       (const u16*)packed, (const u16*)in, out, (u16*)save);
    return err(hipGetLastError());
}

int ii_cnn_backward(const float* params, const void* packed, const uint16_t* in,
                    const uint16_t* save, const float* out, const float* target,
                    const uint8_t* mask, int32_t n, float* grad, float* loss, void* work,
                    void* stream)
{
    if (!params || !packed || !in || !save || !out || !target || !mask || !grad || !loss ||
        !work || n < 1)
        return II_LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int* count = (int*)work;
    float* part = (float*)((char*)work + 256);
    hipLaunchKernelGGL(k_count, dim3(1), dim3(256), 0, s, mask, (long long)n * kOut * kOut, count);
    hipLaunchKernelGGL(k_backward, dim3(n), dim3(256), 0, s, (const u16*)packed, (const u16*)in,
                       (const u16*)save, out, target, mask, count, part);
    hipLaunchKernelGGL(k_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, part, (int)n, count,
                       grad, loss);
    return err(hipGetLastError());
}

int ii_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t t, float lr,
                void* packed, void* stream)
{
    if (!params || !grad || !m || !v || t < 1 || !packed) return II_LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
    hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, params, grad, m, v, lr, c1,
                       c2);
    hipLaunchKernelGGL(k_pack, dim3((kPacked + 255) / 256), dim3(256), 0, s, params, (u16*)packed);
    return err(hipGetLastError());
}

int ii_lbm_learned_tiles(ii_lbm_handle* h, int32_t cap, int32_t* tiles, int32_t* count)
{
    HandleView v;
    int rc = handle_view(h, &v);
    if (rc) return rc;
    if ((rc = learned_validate(v, cap))) return rc;
    if (!tiles || !count) return II_LBM_EINVAL;
    LearnedCfg c;
    c.cap = cap;
    c.tiles = tiles;
    c.count = count;
    return err(learned_band(v, c));
}

int ii_lbm_learned_patches(ii_lbm_handle* h, const ii_cnn_scales* sc, int32_t cap,
                           const int32_t* tiles, const int32_t* count, uint16_t* in,
                           uint8_t* flags, float* pscale)
{
    HandleView v;
    int rc = handle_view(h, &v);
    if (rc) return rc;
    if ((rc = learned_validate(v, cap))) return rc;
    if (!sc || !tiles || !count || !in || !flags || !pscale) return II_LBM_EINVAL;
    LearnedCfg c;
    c.sc = *sc;
    c.cap = cap;
    c.tiles = (int*)tiles;
    c.count = (int*)count;
    c.in = in;
    c.flags = flags;
    c.pscale = pscale;
    hipError_t e = learned_geom(v, c);
    if (e == hipSuccess) e = learned_flow(v, c);
    return err(e);
}

int ii_lbm_learned_targets(ii_lbm_handle* hc, ii_lbm_handle* hf, const ii_cnn_scales* sc,
                           int32_t cap, const int32_t* tiles, const int32_t* count,
                           const uint8_t* flags, const float* pscale, float* target, uint8_t* mask)
{
    HandleView c, f;
    int rc = handle_view(hc, &c);
    if (rc) return rc;
    if ((rc = handle_view(hf, &f))) return rc;
    if ((rc = check_learned(c))) return rc;
    if ((rc = check_learned(f))) return rc;
    if (!sc || !tiles || !count || !flags || !pscale || !target || !mask || cap < 1 ||
        !(sc->out_scale > 0.f))
        return II_LBM_EINVAL;
    if (c.n_inst != f.n_inst) return II_LBM_EINVAL;
    for (int j = 0; j < c.n_inst; j++)
        if (f.inst[j].nx != 2 * c.inst[j].nx || f.inst[j].ny != 2 * c.inst[j].ny) return II_LBM_EINVAL;
    // the fine handle's queue must be done before the coarse stream reads it
    hipError_t e = hipStreamSynchronize(f.stream);
    if (e != hipSuccess) return II_LBM_EDEVICE;
    const dim3 grid((unsigned)(c.n_inst * cap));
    const float inv = 1.f / sc->out_scale;
    const bool c16 = c.inst[0].storage == II_LBM_FP16, f16 = f.inst[0].storage == II_LBM_FP16;
#define II_TARGETS(TC, TF)                                                                       \
    hipLaunchKernelGGL((k_targets<TC, TF>), grid, dim3(256), 0, c.stream, c.d_inst,              \
                       c.P.lat[c.parity], f.d_inst, f.P.lat[f.parity], inv, (int)cap,            \
                       (const int*)tiles, (const int*)count, flags, pscale, target, mask)
    if (c16 && f16) II_TARGETS(_Float16, _Float16);
    else if (c16) II_TARGETS(_Float16, float);
    else if (f16) II_TARGETS(float, _Float16);
    else II_TARGETS(float, float);
#undef II_TARGETS
    return err(hipGetLastError());
}

int ii_lbm_learned_apply(ii_lbm_handle* h, const ii_cnn_scales* sc, int32_t cap,
                         const int32_t* tiles, const int32_t* count, const uint8_t* flags,
                         const float* pscale, const float* out)
{
    HandleView v;
    int rc = handle_view(h, &v);
    if (rc) return rc;
    if ((rc = check_learned(v))) return rc;
    if (!sc || !tiles || !count || !flags || !pscale || !out || cap < 1) return II_LBM_EINVAL;
    const dim3 grid((unsigned)(v.n_inst * cap));
    if (v.inst[0].storage == II_LBM_FP16)
        hipLaunchKernelGGL(k_apply<_Float16>, grid, dim3(256), 0, v.stream, v.d_inst,
                           v.P.lat[v.parity], sc->out_scale, (int)cap, (const int*)tiles,
                           (const int*)count, flags, pscale, out);
    else
        hipLaunchKernelGGL(k_apply<float>, grid, dim3(256), 0, v.stream, v.d_inst,
                           v.P.lat[v.parity], sc->out_scale, (int)cap, (const int*)tiles,
                           (const int*)count, flags, pscale, out);
    return err(hipGetLastError());
}

int ii_lbm_learned_infer(ii_lbm_handle* h, const float* params, const void* packed,
                         const ii_cnn_scales* sc, int32_t cap, const int32_t* tiles,
                         const int32_t* count, const uint16_t* in, const uint8_t* flags,
                         const float* pscale)
{
    HandleView v;
    int rc = handle_view(h, &v);
    if (rc) return rc;
    if ((rc = learned_validate(v, cap))) return rc;
    if (!params || !packed || !sc || !tiles || !count || !in || !flags || !pscale)
        return II_LBM_EINVAL;
    LearnedCfg c;
    c.params = params;
    c.packed = packed;
    c.sc = *sc;
    c.cap = cap;
    c.tiles = (int*)tiles;
    c.count = (int*)count;
    c.in = (uint16_t*)in;
    c.flags = (uint8_t*)flags;
    c.pscale = (float*)pscale;
    return err(learned_infer(v, c));
}

int ii_lbm_learned_correct(ii_lbm_handle* h, const float* params, const void* packed,
                           const ii_cnn_scales* sc, int32_t cap, int32_t* tiles, int32_t* count,
                           uint16_t* in, uint8_t* flags, float* pscale)
{
    if (!params || !packed || !sc || !in || !flags || !pscale) return II_LBM_EINVAL;
    int rc = ii_lbm_learned_tiles(h, cap, tiles, count);
    if (rc) return rc;
    if ((rc = ii_lbm_learned_patches(h, sc, cap, tiles, count, in, flags, pscale))) return rc;
    return ii_lbm_learned_infer(h, params, packed, sc, cap, tiles, count, in, flags, pscale);
}

}  // extern "C"
