// swe_lc.hpp -- gfx950 kernels of the learned coarse-grid flux correction.
//
// A small convolutional network (four 3x3 valid convolutions, 6 -> 32 -> 32
// -> 32 -> 6 channels, tanh after the first three) reads the state of a
// coarse grid and predicts corrections of the stage III face fluxes (Sec. 2.3
// of arXiv 1705.00614; the learned part is an extension of the method, the
// paper has none).  The network runs on crops: for an active S x S tile the
// (S+9)^2 window round the tile and the cell row and column before it
// (mirrored at walls) gives the (S+1)^2 corrections of those cells, so that
// the tile's west and south boundary faces (east and north faces of the
// neighbours' cells) are always fresh.
//
// Layouts: activations bf16, [crop][y][x][C] with C = 16 (the 6 features,
// zero padded) or 32; weights bf16 as [tap][out][in] (forward) and
// [tap][in][out] (backward data), both padded to multiples of 16; FP32 master
// weights, gradients and Adam moments in the packed order (W[out][in][3][3],
// then b[out]) per layer.  Every contraction is a 16x16x16 bf16 MFMA with
// FP32 accumulation: a wave owns 16 consecutive pixels (M) of one crop and
// all output channels (N tiles of 16), the reduction (K) runs over the 9 taps
// times the input channels in chunks of 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {
namespace lc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NL = 4;                         // layers
constexpr int HALO = NL;                      // crop margin
constexpr int CIN[NL] = {16, 32, 32, 32};     // padded input channels
constexpr int COUT[NL] = {32, 32, 32, 16};    // padded output channels
constexpr int CIN_REAL[NL] = {6, 32, 32, 32};
constexpr int COUT_REAL[NL] = {32, 32, 32, 6};

// packed FP32 parameter offsets of layer l: W then b
__host__ __device__ constexpr int w_count(int l) { return COUT_REAL[l] * CIN_REAL[l] * 9; }
__host__ __device__ constexpr int p_off(int l) {
    return l == 0 ? 0 : p_off(l - 1) + w_count(l - 1) + COUT_REAL[l - 1];
}
constexpr int NPARAM = p_off(NL);
// bf16 weight copies: [tap][COUT][CIN] per layer
__host__ __device__ constexpr int wb_count(int l) { return 9 * COUT[l] * CIN[l]; }
__host__ __device__ constexpr int wb_off(int l) { return l == 0 ? 0 : wb_off(l - 1) + wb_count(l - 1); }
constexpr int NWB = wb_off(NL);

__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ bf16x4 load4(const unsigned short* p) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    bf16x4 r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

// Number of crops: from the device (active tiles of a grid) or the host.
__device__ __forceinline__ int crop_count(const int* dev, int host) { return dev ? *dev : host; }

// ------------------------------------------------------------------ forward
// y = act(conv3x3_valid(x) + b); x [n][Sin][Sin][CI] bf16, y [n][Sout][Sout][CO]
// (bf16 with tanh, or FP32 linear for the last layer).
//
// A wave keeps its B operands (the layer's weights for every tap and output
// tile) in registers for all its items, and loads the A operands of its next
// 16-pixel item while the MFMAs of the current one run.  With 32 input
// channels a tap is one 16x16x32 bf16 MFMA (lane group kq holds channels
// 8kq..8kq+7 of A and B, one 16-byte load each); with 16 input channels a
// tap is one 16x16x16 MFMA.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 as8(const uint4& q) { return __builtin_bit_cast(bf16x8, q); }

// tanh of the hidden activations (stored as bf16): an odd Taylor polynomial
// below 1/16, else 1 - 2 / (e^(2|x|) + 1) from the hardware base-2 exponential
// and reciprocal; relative error about 1e-6, far below the bf16 spacing.
__device__ __forceinline__ float tanh_act(float x) {
    const float ax = __builtin_fabsf(x), x2 = x * x;
    const float small = x * (1.f + x2 * (-0.333333343f + x2 * 0.133333340f));
    const float e = __builtin_amdgcn_exp2f(2.88539008f * ax);
    const float big = __builtin_copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), x);
    return ax < 0.0625f ? small : big;
}

template <int CI> struct AFrag;
template <> struct AFrag<16> { typedef uint2 Q; Q v[9]; };
template <> struct AFrag<32> { typedef uint4 Q; Q v[9]; };

__device__ __forceinline__ bf16x4 as4(const uint2& q) {
    bf16x4 r;
    r[0] = (short)(q.x & 0xFFFFu); r[1] = (short)(q.x >> 16); r[2] = (short)(q.y & 0xFFFFu); r[3] = (short)(q.y >> 16);
    return r;
}

template <int CI>
__device__ __forceinline__ void load_a(AFrag<CI>& f, const unsigned short* __restrict__ x, int item, int blocks,
                                       int Sin, int Sout, int P, int m, int kq) {
    const int c = item / blocks, p = min((item % blocks) * 16 + m, P - 1);
    const int oy = p / Sout, ox = p % Sout;
    const unsigned short* xc = x + (size_t)c * Sin * Sin * CI;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const unsigned short* xp = xc + ((oy + tap / 3) * Sin + ox + tap % 3) * CI;
        if constexpr (CI == 32) f.v[tap] = *reinterpret_cast<const uint4*>(xp + 8 * kq);
        else f.v[tap] = *reinterpret_cast<const uint2*>(xp + 4 * kq);
    }
}

template <int CI, int CO, bool LAST>
__global__ __launch_bounds__(256) void k_conv_fwd(const unsigned short* __restrict__ x, void* __restrict__ y,
                                                   const unsigned short* __restrict__ wf, const float* __restrict__ bias,
                                                   int cob, int Sin, const int* cnt_dev, int cnt_host) {
    static_assert(CI == 16 || CI == 32, "input channels");
    constexpr int NT = CO / 16;
    const int Sout = Sin - 2, P = Sout * Sout, blocks = (P + 15) / 16;
    const int n = crop_count(cnt_dev, cnt_host);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int total = n * blocks, stride = gridDim.x * 4;
    int item = blockIdx.x * 4 + wv;
    if (item >= total) return;
    // B operands: lane (m, kq) holds w[tap][t*16 + m][k] for its k of each
    // chunk, as A holds x[pixel m][k]
    typename AFrag<CI>::Q B[9][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            B[tap][t] = *reinterpret_cast<const typename AFrag<CI>::Q*>(wf + (tap * CO + t * 16 + m) * CI +
                                                                         (CI / 4) * kq);
    float bb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bb[t] = t * 16 + m < cob ? bias[t * 16 + m] : 0.f;
    AFrag<CI> cur, nxt;
    load_a<CI>(cur, x, item, blocks, Sin, Sout, P, m, kq);
    for (; item < total; item += stride) {
        const int item2 = item + stride;
        if (item2 < total) load_a<CI>(nxt, x, item2, blocks, Sin, Sout, P, m, kq);
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (CI == 32)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as8(cur.v[tap]), as8(B[tap][t]), acc[t], 0, 0, 0);
                else
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as4(cur.v[tap]), as4(B[tap][t]), acc[t], 0, 0, 0);
            }
        // lane holds rows (pixels) p0 + 4*kq + i, column (channel) t*16 + m
        const int c = item / blocks, p0 = (item % blocks) * 16;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int ch = t * 16 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pp = p0 + 4 * kq + i;
                if (pp >= P) continue;
                const float v = acc[t][i] + bb[t];
                const size_t o = ((size_t)c * P + pp) * CO + ch;
                if constexpr (LAST) static_cast<float*>(y)[o] = ch < cob ? v : 0.f;
                else static_cast<unsigned short*>(y)[o] = to_bf16(tanh_act(v));
            }
        }
        cur = nxt;
    }
}

// ------------------------------------------------------------------ fused inference
// All four layers of one T x T block of a crop's output in one workgroup, the
// intermediate activations in LDS: the block's (T+8)^2 input window comes in
// from HBM once and only the FP32 output goes out, so an inference costs one
// launch instead of four and no activation round trips through HBM.  The
// weights of every layer are staged in LDS once per workgroup; each layer is
// the same per-pixel MFMA sequence as k_conv_fwd (taps in order, one MFMA per
// tap and output tile, the same bias, tanh and bf16 rounding), so the output
// equals the layer-by-layer forward.  A crop of side So is covered by
// ceil(So / T) blocks per side, the last one shifted back to end at So (its
// overlap is recomputed and written with the same values).
template <int T>
struct alignas(16) NetLds {
    static constexpr int P16 = 24, P32 = 40;      // pixel strides (bf16): channels + 8 against bank conflicts
    // a hidden layer's output plane is padded to whole 16-pixel blocks, so
    // that the rows of a ragged last block are stored without a test (and
    // never read)
    static constexpr int blk16(int side) { return ((side * side + 15) / 16) * 16; }
    static constexpr int A = (T + 8) * (T + 8) * P16 > blk16(T + 4) * P32 ? (T + 8) * (T + 8) * P16
                                                                           : blk16(T + 4) * P32;
    static constexpr int B = blk16(T + 6) * P32;
    unsigned short w[NWB];                        // bf16 weights of all layers, [tap][CO][CI]
    float bias[NL][32];
    unsigned short a[A];                          // input window, then layer-1 output
    unsigned short b[B];                          // layer-0 output, then layer-2 output
};

// One layer over the LDS plane `in` (side Win, pixel stride PI) into `out`
// (LDS bf16 with tanh, stride PO) or, for the last layer, through the writer
// `wr(oy, ox, ch, v)` (block-local output pixel, channel, FP32 value).
struct NoWriter {
    __device__ __forceinline__ void operator()(int, int, int, float) const {}
};
template <int CI, int CO, bool LAST, int Win, int NTH, class Wr>
__device__ __forceinline__ void net_layer(const unsigned short* in, int PI, unsigned short* out, int PO,
                                          const unsigned short* w, const float* bias, int cob, const Wr& wr) {
    constexpr int NT = CO / 16, Wout = Win - 2, P = Wout * Wout, blocks = (P + 15) / 16, nw = NTH / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    if (wv >= blocks) return;
    typename AFrag<CI>::Q B[9][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            B[tap][t] = *reinterpret_cast<const typename AFrag<CI>::Q*>(w + (tap * CO + t * 16 + m) * CI + (CI / 4) * kq);
    float bb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bb[t] = t * 16 + m < cob ? bias[t * 16 + m] : 0.f;
    // two blocks per pass (blk and blk + nw): four independent MFMA chains
    // and sixteen independent activations per lane hide more latency at two
    // waves per SIMD; a missing second block (wave-uniform) is computed on
    // clamped pixels and not stored
    for (int blk = wv; blk < blocks; blk += 2 * nw) {
        const bool two = blk + nw < blocks;
        int oy[2], ox[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = min((blk + h * nw) * 16 + m, P - 1);
            oy[h] = p / Wout;
            ox[h] = p % Wout;
        }
        f32x4 acc[2][NT];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[h][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // block-major: block 0's activations can overlap block 1's MFMAs
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const unsigned short* ip = in + ((oy[h] + tap / 3) * Win + ox[h] + tap % 3) * PI + (CI / 4) * kq;
                const typename AFrag<CI>::Q av = *reinterpret_cast<const typename AFrag<CI>::Q*>(ip);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if constexpr (CI == 32)
                        acc[h][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as8(av), as8(B[tap][t]), acc[h][t], 0, 0, 0);
                    else
                        acc[h][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as4(av), as4(B[tap][t]), acc[h][t], 0, 0,
                                                                              0);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) break;
            const int p0 = (blk + h * nw) * 16;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int ch = t * 16 + m;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int pp = p0 + 4 * kq + i;
                    const float v = acc[h][t][i] + bb[t];
                    if constexpr (LAST) {
                        if (pp >= P) continue;
                        wr(pp / Wout, pp % Wout, ch, ch < cob ? v : 0.f);
                    } else {
                        out[pp * PO + ch] = to_bf16(tanh_act(v));   // pp < blocks * 16: inside the padded plane
                    }
                }
            }
        }
    }
}

// All units of n crops through the four layers.  The source `src` (a
// read-only descriptor; what it fetches is held in three 16-byte registers
// of the caller, plain locals so that they stay in VGPRs) provides the
// input windows and the output writers:
//   src.load(u, q0, q1, q2)    fetch unit u's input window,
//   src.store(lds, q0, q1, q2) put it into the LDS plane (pixel stride 24)
//                              and return this thread's vote to run the unit,
//   src.source_near(c, oy0, ox0) whether the unit must run whatever the votes,
//   src.writer(c, oy0, ox0) the last layer's writer for a block of crop c,
//   src.begin()                once per workgroup, before anything else,
//   src.claim(u)               (thread 0) the unit after u of this workgroup.
// A workgroup's first unit is its index; the next unit's window is fetched
// while the current one computes.
template <int T, int NTH, class Src>
__device__ __forceinline__ void net_run(const Src& src, NetLds<T>& L, const unsigned short* __restrict__ wf,
                                        const float* __restrict__ params, int So, int n) {
    using N = NetLds<T>;
    const int ns = (So + T - 1) / T, units = n * ns * ns;
    src.begin();
    if ((int)blockIdx.x >= units) return;
    const int tid = threadIdx.x;
    constexpr int W0 = T + 2 * HALO;
    // every global load of the weight staging is issued before the first
    // store (one memory round trip, not one per piece)
    {
        constexpr int NV = NWB / 8, J = (NV + NTH - 1) / NTH;
        uint4 v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = min(tid + j * NTH, NV - 1);   // clamped: the tail re-reads the last piece
            v[j] = reinterpret_cast<const uint4*>(wf)[k];
        }
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (tid + j * NTH < NV) reinterpret_cast<uint4*>(L.w)[tid + j * NTH] = v[j];
    }
    for (int k = tid; k < NL * 32; k += NTH) {
        const int l = k / 32, ch = k % 32;
        constexpr int b0 = p_off(0) + w_count(0), b1 = p_off(1) + w_count(1), b2 = p_off(2) + w_count(2),
                      b3 = p_off(3) + w_count(3);   // bias offsets, folded at compile time
        const int off = l == 0 ? b0 : l == 1 ? b1 : l == 2 ? b2 : b3;
        L.bias[l][ch] = ch < (l == NL - 1 ? COUT_REAL[NL - 1] : 32) ? params[off + ch] : 0.f;
    }
    uint4 q0, q1, q2;
    src.load(blockIdx.x, q0, q1, q2);
    // the next unit's index, by iteration parity: thread 0 writes one slot
    // before the vote's barrier while slow threads may still read the other
    __shared__ int s_next[2];
    for (int u = blockIdx.x, it = 0; u < units; ++it) {
        const int c = u / (ns * ns), sub = u % (ns * ns);
        const int oy0 = min((sub / ns) * T, So - T), ox0 = min((sub % ns) * T, So - T);
        // a unit whose outputs no face would take is skipped (grid source:
        // the block's cells and their face neighbours all at most the
        // correction depth and none of them a source cell); its corrections
        // keep older values, which the step never applies there
        const int deep = src.store(L.a, q0, q1, q2);
        if (tid == 0) s_next[it & 1] = src.claim(u);
        const bool run = __syncthreads_or(deep) || src.source_near(c, oy0, ox0);
        const int next = s_next[it & 1];
        if (next < units) src.load(next, q0, q1, q2);
        u = next;
        if (!run) continue;
        const NoWriter nw;
        net_layer<16, 32, false, W0, NTH>(L.a, N::P16, L.b, N::P32, L.w + wb_off(0), L.bias[0], 32, nw);
        __syncthreads();
        net_layer<32, 32, false, W0 - 2, NTH>(L.b, N::P32, L.a, N::P32, L.w + wb_off(1), L.bias[1], 32, nw);
        __syncthreads();
        net_layer<32, 32, false, W0 - 4, NTH>(L.a, N::P32, L.b, N::P32, L.w + wb_off(2), L.bias[2], 32, nw);
        __syncthreads();
        net_layer<32, 16, true, W0 - 6, NTH>(L.b, N::P32, nullptr, 0, L.w + wb_off(3), L.bias[3], COUT_REAL[3],
                                             src.writer(c, oy0, ox0));
        // the next unit's input goes to L.a, last read by layer 2 (before the
        // barrier above); layer 3 reads L.b, next written after the barrier
        // that follows the next input
    }
}

// Writer of the last layer into the FP32 crop output y [n][So][So][16].
struct CropWriter {
    float* y;
    int So, c, oy0, ox0;
    __device__ __forceinline__ void operator()(int oy, int ox, int ch, float v) const {
        y[(((size_t)c * So + oy0 + oy) * So + ox0 + ox) * 16 + ch] = v;
    }
};

// Source of crops already in HBM: x [n][So+8][So+8][16] bf16; each thread
// moves two 16-byte pieces (tid and tid + NTH) of the window.
template <int T, int NTH>
struct CropSource {
    static constexpr int W0 = T + 2 * HALO, XV = W0 * W0 * 2;
    static_assert(XV > NTH && XV <= 2 * NTH, "two 16-byte pieces of the input window per thread");
    const unsigned short* x;
    float* y;
    int So, ns, tid;
    __device__ __forceinline__ void load(int u, uint4& q0, uint4& q1, uint4&) const {
        const int Sin = So + 2 * HALO, c = u / (ns * ns), sub = u % (ns * ns);
        const int oy0 = min((sub / ns) * T, So - T), ox0 = min((sub % ns) * T, So - T);
        const unsigned short* xc = x + (size_t)c * Sin * Sin * 16;
        const int k0 = tid, k1 = tid + NTH;
        q0 = *reinterpret_cast<const uint4*>(xc + ((size_t)(oy0 + (k0 >> 1) / W0) * Sin + ox0 + (k0 >> 1) % W0) *
                                                        16 + 8 * (k0 & 1));
        if (k1 < XV)
            q1 = *reinterpret_cast<const uint4*>(xc + ((size_t)(oy0 + (k1 >> 1) / W0) * Sin + ox0 + (k1 >> 1) % W0) *
                                                          16 + 8 * (k1 & 1));
    }
    // returns 1: crops handed in are always run
    __device__ __forceinline__ int store(unsigned short* a, const uint4& q0, const uint4& q1, const uint4&) const {
        *reinterpret_cast<uint4*>(a + (tid >> 1) * NetLds<T>::P16 + 8 * (tid & 1)) = q0;
        if (tid + NTH < XV) *reinterpret_cast<uint4*>(a + ((tid + NTH) >> 1) * NetLds<T>::P16 + 8 * (tid & 1)) = q1;
        return 1;
    }
    __device__ __forceinline__ bool source_near(int, int, int) const { return true; }
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ int claim(int u) const { return u + (int)gridDim.x; }   // a fixed stride
    __device__ __forceinline__ CropWriter writer(int c, int oy0, int ox0) const { return CropWriter{y, So, c, oy0, ox0}; }
};

// x: crops [n][So+8][So+8][16] bf16; y: [n][So][So][16] FP32 (channels >= 6
// zero); wf: bf16 weights of all layers; params: packed FP32 parameters (the
// biases are read from there).  Requires So >= T; n from the device or host.
template <int T, int NTH>
__global__ __launch_bounds__(NTH) void k_net_fwd(const unsigned short* __restrict__ x, float* __restrict__ y,
                                                 const unsigned short* __restrict__ wf,
                                                 const float* __restrict__ params, int So, const int* cnt_dev,
                                                 int cnt_host) {
    __shared__ NetLds<T> L;
    const CropSource<T, NTH> src{x, y, So, (So + T - 1) / T, (int)threadIdx.x};
    net_run<T, NTH>(src, L, wf, params, So, crop_count(cnt_dev, cnt_host));
}

// ------------------------------------------------------------------ backward data
// g_in = bf16(dL/da_in * (1 - a_in^2)) from g = dL/dz of this layer:
// dL/da_in[q] = sum_{tap, co} g[q - tap][co] w[co][ci][tap] (zero outside the
// output plane).  a_in and g_in: [n][Sin][Sin][CI]; g: [n][Sout][Sout][CO].
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const unsigned short* __restrict__ g,
                                                        const unsigned short* __restrict__ a_in,
                                                        unsigned short* __restrict__ g_in,
                                                        const unsigned short* __restrict__ wb, int Sin, int n) {
    constexpr int NT = CI / 16;
    const int Sout = Sin - 2, P = Sin * Sin, blocks = (P + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    for (int item = blockIdx.x * 4 + wv; item < n * blocks; item += gridDim.x * 4) {
        const int c = item / blocks, p0 = (item % blocks) * 16;
        const int p = min(p0 + m, P - 1);
        const int qy = p / Sin, qx = p % Sin;
        const unsigned short* gc = g + (size_t)c * Sout * Sout * CO;
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int oy = qy - tap / 3, ox = qx - tap % 3;
            const bool in = oy >= 0 && oy < Sout && ox >= 0 && ox < Sout;
            const unsigned short* gp = gc + ((in ? oy : 0) * Sout + (in ? ox : 0)) * CO + 4 * kq;
#pragma unroll
            for (int c0 = 0; c0 < CO; c0 += 16) {
                bf16x4 a = load4(gp + c0);
                if (!in) a = bf16x4{0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const bf16x4 b = load4(wb + (tap * CI + t * 16 + m) * CO + c0 + 4 * kq);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int ch = t * 16 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pp = p0 + 4 * kq + i;
                if (pp >= P) continue;
                const size_t o = ((size_t)c * P + pp) * CI + ch;
                const float a = from_bf16(a_in[o]);
                g_in[o] = to_bf16(acc[t][i] * (1.f - a * a));
            }
        }
    }
}

// ------------------------------------------------------------------ backward weights
// Partial weight and bias gradients of one pixel chunk per block:
// dW[tap][co][ci] = sum_p g[p][co] a_in[p + tap][ci], db[co] = sum_p g[p][co].
// The 9 x (CO/16) x (CI/16) output tiles are dealt round-robin to the 4
// waves; part[block] holds [tap][CO][CI] then [CO] in FP32.
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const unsigned short* __restrict__ g,
                                                     const unsigned short* __restrict__ a_in,
                                                     float* __restrict__ part, int Sin, int n, int chunk) {
    constexpr int TCO = CO / 16, TCI = CI / 16, NTILE = 9 * TCO * TCI, PER = (NTILE + 3) / 4;
    const int Sout = Sin - 2, P = Sout * Sout, total = n * P;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int q0 = blockIdx.x * chunk, q1 = min(total, q0 + chunk);
    f32x4 acc[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = q0; k0 < q1; k0 += 16) {
        // K index: pixels k0 + 4*kq + i of the flattened (crop, pixel) range
        int cc[4], py[4], px[4];
        bool ok[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = k0 + 4 * kq + i;
            ok[i] = q < q1;
            const int qq = ok[i] ? q : q0;
            cc[i] = qq / P;
            const int p = qq % P;
            py[i] = p / Sout;
            px[i] = p % Sout;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int tile = wv + 4 * j;
            if (tile >= NTILE) break;
            const int tap = tile / (TCO * TCI), to = (tile / TCI) % TCO, ti = tile % TCI;
            const int dy = tap / 3, dx = tap % 3;
            bf16x4 a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const size_t go = (((size_t)cc[i] * Sout + py[i]) * Sout + px[i]) * CO + to * 16 + m;
                const size_t ao = (((size_t)cc[i] * Sin + py[i] + dy) * Sin + px[i] + dx) * CI + ti * 16 + m;
                a[i] = ok[i] ? (short)g[go] : (short)0;
                b[i] = ok[i] ? (short)a_in[ao] : (short)0;
            }
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
        }
    }
    float* out = part + (size_t)blockIdx.x * (9 * CO * CI + CO);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int tile = wv + 4 * j;
        if (tile >= NTILE) break;
        const int tap = tile / (TCO * TCI), to = (tile / TCI) % TCO, ti = tile % TCI;
        // lane holds rows (co) to*16 + 4*kq + i, column (ci) ti*16 + m
#pragma unroll
        for (int i = 0; i < 4; ++i) out[(tap * CO + to * 16 + 4 * kq + i) * CI + ti * 16 + m] = acc[j][i];
    }
    // bias: thread t < CO sums its channel over the chunk
    if (threadIdx.x < CO) {
        float s = 0.f;
        for (int q = q0; q < q1; ++q) s += from_bf16(g[(size_t)q * CO + threadIdx.x]);
        out[9 * CO * CI + threadIdx.x] = s;
    }
}

// Sum the block partials (fixed order) into the packed FP32 gradient of a layer.
template <int CI, int CO>
__global__ void k_reduce_w(const float* __restrict__ part, int nblk, float* __restrict__ grad, int ci_real, int co_real) {
    const int per = 9 * CO * CI + CO;
    const int wc = co_real * ci_real * 9;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < wc + co_real; k += gridDim.x * blockDim.x) {
        int src;
        if (k < wc) {
            const int co = k / (ci_real * 9), ci = (k / 9) % ci_real, tap = k % 9;
            src = (tap * CO + co) * CI + ci;
        } else {
            src = 9 * CO * CI + (k - wc);
        }
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * per + src];
        grad[k] = s;
    }
}

// ------------------------------------------------------------------ parameters
// bf16 copies of the packed FP32 weights in both layouts (zero padding).
__global__ void k_pack_weights(const float* __restrict__ params, unsigned short* __restrict__ wf,
                               unsigned short* __restrict__ wb) {
    for (int l = 0; l < NL; ++l) {
        const int ci_p = CIN[l], co_p = COUT[l], cir = CIN_REAL[l], cor = COUT_REAL[l];
        const float* W = params + p_off(l);
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 9 * co_p * ci_p; k += gridDim.x * blockDim.x) {
            const int tap = k / (co_p * ci_p), co = (k / ci_p) % co_p, ci = k % ci_p;
            const float v = (co < cor && ci < cir) ? W[(co * cir + ci) * 9 + tap] : 0.f;
            const unsigned short h = to_bf16(v);
            wf[wb_off(l) + (tap * co_p + co) * ci_p + ci] = h;
            wb[wb_off(l) + (tap * ci_p + ci) * co_p + co] = h;
        }
    }
}

// Adam (bias-corrected) on the packed FP32 parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.f - b1) * gk;
        const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    }
}

// ------------------------------------------------------------------ loss
// g = bf16(mask (out - y) / count) for the 6 real channels (zero padding to
// 16); per-block loss partials 1/2 sum mask (out - y)^2 / count.
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ y, const float* __restrict__ mask,
                       unsigned short* __restrict__ g, int npix, float inv_count, double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npix * 16; k += gridDim.x * blockDim.x) {
        const int p = k / 16, ch = k % 16;
        float gv = 0.f;
        if (ch < 6) {
            const float d = out[k] - y[p * 6 + ch];
            const float mk = mask[p * 6 + ch];
            gv = mk * d * inv_count;
            s += 0.5 * (double)(mk * d * d) * (double)inv_count;
        }
        g[k] = to_bf16(gv);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace lc
}  // namespace swe

// ------------------------------------------------------------------ coarse grid I/O
// These need the step kernel's argument block and tile list.
#include "swe_step.hpp"

namespace swe {
namespace lc {

// Crop p of the grid's current tile list (all tiles when the grid does not
// skip dry tiles).
template <typename real>
__device__ __forceinline__ int crop_tile(const Args<real>& a, int slot, int p) {
    return a.skip ? entry_tile(list_entry(a.ctrl, a.lists, a.ntiles, slot, p)) : p;
}

// Grid cell (mirrored at walls) of pixel (wx, wy) of a tile's (S+9)^2 input
// window, which starts HALO + 1 cells before the tile.
template <typename real>
__device__ __forceinline__ int crop_cell(const Args<real>& a, int tile, int S, int wx, int wy) {
    int fx = 0, fy = 0;
    const int gx = mirror((tile % a.ntx) * S - 1 - HALO + wx, a.nx, fx);
    const int gy = mirror((tile / a.ntx) * S - 1 - HALO + wy, a.ny, fy);
    return gy * a.nx + gx;
}

// The stored values of one cell and its six network features (depth,
// velocity, bed, sqrt(c_f / g) = Manning n, wet flag), divided by the input
// scales, as bf16.
template <typename real> struct CellIn { real H, qx, qy, b, cf; };
template <typename real>
__device__ __forceinline__ void features(const Args<real>& a, const CellIn<real>& v, const float* iscale,
                                         unsigned short (&o)[6]) {
    const bool w = v.H > a.eps;
    float f[6];
    f[0] = (float)v.H;
    f[1] = w ? (float)(v.qx / v.H) : 0.f;
    f[2] = w ? (float)(v.qy / v.H) : 0.f;
    f[3] = (float)v.b;
    f[4] = sqrtf((float)v.cf / (float)a.g_d);
    f[5] = w ? 1.f : 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) o[c] = to_bf16(f[c] / iscale[c]);
}

// Input crops of the active tiles: the six features of every cell of each
// (S+9)^2 window (mirrored at walls), divided by the input scales, as bf16.
template <typename real>
__global__ void k_gather(Args<real> a, int slot, int S, const float* __restrict__ iscale, unsigned short* __restrict__ x,
                         int* __restrict__ tiles_out) {
    const int Sin = S + 1 + 2 * HALO, P = Sin * Sin;
    const int n = a.skip ? a.ctrl->seg_off[slot][NSEG] : a.ntiles;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n * P; k += gridDim.x * blockDim.x) {
        const int p = k / P, q = k % P;
        const int tile = crop_tile(a, slot, p);
        if (tiles_out && q == 0) tiles_out[p] = tile;
        const int gi = crop_cell(a, tile, S, q % Sin, q / Sin);
        const CellIn<real> v{a.Hi[gi], a.Qxi[gi], a.Qyi[gi], a.bed[gi], a.cf[gi]};
        unsigned short f[6];
        features(a, v, iscale, f);
        unsigned short* o = x + (size_t)k * 16;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = f[c];
    }
}

// Corrections of the active tiles' cells and of the cell row and column
// before each tile, from the network output.  A cell shared by two active
// crops gets the same value from both (same inputs, same summation order).
template <typename real>
__global__ void k_scatter(Args<real> a, int slot, int S, const float* __restrict__ oscale, const float* __restrict__ out,
                          real* __restrict__ corrE, real* __restrict__ corrN) {
    const int So = S + 1, P = So * So, nc = a.nx * a.ny;
    const int n = a.skip ? a.ctrl->seg_off[slot][NSEG] : a.ntiles;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n * P; k += gridDim.x * blockDim.x) {
        const int p = k / P, q = k % P;
        const int tile = crop_tile(a, slot, p);
        const int gx = (tile % a.ntx) * S - 1 + q % So, gy = (tile / a.ntx) * S - 1 + q / So;
        if (gx < 0 || gy < 0 || gx >= a.nx || gy >= a.ny) continue;
        const int gi = gy * a.nx + gx;
        const float* o = out + (size_t)k * 16;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            corrE[c * nc + gi] = (real)(o[c] * oscale[c]);
            corrN[c * nc + gi] = (real)(o[3 + c] * oscale[3 + c]);
        }
    }
}

// Writer of the last layer straight into a grid's correction planes (what
// k_scatter does from the crop output): crop pixel (oy0 + oy, ox0 + ox) is
// grid cell (x0 + ox, y0 + oy), x0 = tile column * S - 1 + ox0.
template <typename real>
struct CorrWriter {
    real* corrE;
    real* corrN;
    const float* oscale;
    int nx, ny, x0, y0;
    __device__ __forceinline__ void operator()(int oy, int ox, int ch, float v) const {
        const int gx = x0 + ox, gy = y0 + oy;
        if (ch >= 6 || gx < 0 || gy < 0 || gx >= nx || gy >= ny) return;
        const size_t nc = (size_t)nx * ny, gi = (size_t)gy * nx + gx;
        if (ch < 3) corrE[ch * nc + gi] = (real)(v * oscale[ch]);
        else corrN[(ch - 3) * nc + gi] = (real)(v * oscale[ch]);
    }
};

// Source of the input windows straight from a grid's current layer (what
// k_gather does into HBM): thread tid < (T+8)^2 fetches the five stored
// values of one window pixel and turns them into its features at the store.
template <int T, int NTH, typename real>
struct GridSource {
    static constexpr int W0 = T + 2 * HALO;
    static_assert(W0 * W0 <= NTH, "one window pixel per thread");
    static_assert(5 * sizeof(real) <= 48, "five stored values in three 16-byte registers");
    const Args<real>* a;
    int slot, S, So, ns, tid;
    const float* iscale;
    real* corrE;
    real* corrN;
    const float* oscale;
    // units after the first are claimed from claims[slot] (workgroups that
    // run blocks take fewer); the pre-step of the next step, which uses the
    // other slot, finds that one cleared by this launch (both are zero when
    // the network is attached)
    int* claims;
    __device__ __forceinline__ void begin() const {
        if (blockIdx.x == 0 && tid == 0) claims[slot ^ 1] = 0;
    }
    __device__ __forceinline__ int claim(int) const { return atomicAdd(&claims[slot], 1) + (int)gridDim.x; }
    __device__ __forceinline__ int origin(int u, int& tile, int& oy0, int& ox0) const {
        const int c = u / (ns * ns), sub = u % (ns * ns);
        oy0 = min((sub / ns) * T, So - T);
        ox0 = min((sub % ns) * T, So - T);
        tile = crop_tile(*a, slot, c);
        return c;
    }
    __device__ __forceinline__ void load(int u, uint4& q0, uint4& q1, uint4& q2) const {
        if (tid >= W0 * W0) return;
        int tile, oy0, ox0;
        origin(u, tile, oy0, ox0);
        const int gi = crop_cell(*a, tile, S, ox0 + tid % W0, oy0 + tid / W0);
        real v[6] = {a->Hi[gi], a->Qxi[gi], a->Qyi[gi], a->bed[gi], a->cf[gi], real(0)};
        uint4 q[3];
        static_assert(sizeof v <= sizeof q, "fits");
        __builtin_memcpy(q, v, sizeof v);
        q0 = q[0]; q1 = q[1]; q2 = q[2];
    }
    // returns 1 if this window pixel is one of the block's output cells or
    // their face neighbours (pixels HALO-1 .. HALO+T of each axis) and deeper
    // than the correction depth: the step corrects a face only where its
    // cells are (the stored depth is the depth after the Lagrangian stage
    // except on source cells, which source_near covers)
    __device__ __forceinline__ int store(unsigned short* lds, const uint4& q0, const uint4& q1, const uint4& q2) const {
        if (tid >= W0 * W0) return 0;
        const uint4 q[3] = {q0, q1, q2};
        real v[6];
        __builtin_memcpy(v, q, sizeof v);
        unsigned short f[6];
        features(*a, CellIn<real>{v[0], v[1], v[2], v[3], v[4]}, iscale, f);
        const uint4 lo = {f[0] | ((unsigned)f[1] << 16), f[2] | ((unsigned)f[3] << 16), f[4] | ((unsigned)f[5] << 16), 0u};
        *reinterpret_cast<uint4*>(lds + tid * NetLds<T>::P16) = lo;
        *reinterpret_cast<uint4*>(lds + tid * NetLds<T>::P16 + 8) = uint4{0u, 0u, 0u, 0u};
        const int px = tid % W0, py = tid / W0;
        const bool near = px >= HALO - 1 && px <= HALO + T && py >= HALO - 1 && py <= HALO + T;
        return near && v[0] > a->corr_hmin;
    }
    // whether the block's cells or their face neighbours meet the inlet
    // rectangle (their depth after the Lagrangian stage includes the source)
    __device__ __forceinline__ bool source_near(int c, int oy0, int ox0) const {
        if (a->ni <= 0 || a->nj <= 0) return false;
        const int tile = crop_tile(*a, slot, c);
        const int x0 = (tile % a->ntx) * S - 2 + ox0, y0 = (tile / a->ntx) * S - 2 + oy0;   // first neighbour
        return x0 < a->i0 + a->ni && a->i0 < x0 + T + 2 && y0 < a->j0 + a->nj && a->j0 < y0 + T + 2;
    }
    __device__ __forceinline__ CorrWriter<real> writer(int c, int oy0, int ox0) const {
        const int tile = crop_tile(*a, slot, c);
        return CorrWriter<real>{corrE, corrN, oscale, a->nx, a->ny, (tile % a->ntx) * S - 1 + ox0,
                                (tile / a->ntx) * S - 1 + oy0};
    }
};

// Before a step of a grid with an attached network: crops of the active
// tiles of list `slot`, the four layers and the corrections of those tiles
// in one launch (the work of k_gather, the four forward layers and
// k_scatter, with the same arithmetic per value).  Requires S + 1 >= T.
template <int T, int NTH, typename real>
__global__ __launch_bounds__(NTH) void k_net_grid(Args<real> a, int slot, int S, const float* __restrict__ iscale,
                                                  const float* __restrict__ oscale, real* __restrict__ corrE,
                                                  real* __restrict__ corrN, const unsigned short* __restrict__ wf,
                                                  const float* __restrict__ params, int* __restrict__ claims) {
    __shared__ NetLds<T> L;
    const int So = S + 1;
    const GridSource<T, NTH, real> src{&a, slot, S, So, (So + T - 1) / T, (int)threadIdx.x, iscale, corrE, corrN,
                                       oscale, claims};
    const int n = a.skip ? a.ctrl->seg_off[slot][NSEG] : a.ntiles;
    net_run<T, NTH>(src, L, wf, params, So, n);
}

// Training labels of n crops (coarse tiles tiles[p], (S+1)^2 cells from the
// row and column before the tile): the correction that
// makes each coarse face carry the fine solution's flux over one coarse step,
// (mean of the r fine line taps through the face - the coarse tap) / tau_c,
// divided by the output scales; mask 1 on interior faces of in-domain cells.
// Fine taps: ftx [3][r*ny][nx+1], fty [3][ny+1][r*nx]; coarse taps (r = 1):
// ctx [3][ny][nx+1], cty [3][ny+1][nx] (planes mass, normal, tangential).
template <typename real>
__global__ void k_labels(const int* __restrict__ tiles, int n, int S, int ntx, int nx, int ny, int r,
                         const real* __restrict__ ftx, const real* __restrict__ fty, const real* __restrict__ ctx,
                         const real* __restrict__ cty, double inv_tau, const float* __restrict__ oscale,
                         float* __restrict__ y, float* __restrict__ mask, int* __restrict__ mcount) {
    const int So = S + 1, P = So * So;
    const size_t pfx = (size_t)r * ny * (nx + 1), pcx = (size_t)ny * (nx + 1);
    const size_t pfy = (size_t)(ny + 1) * r * nx, pcy = (size_t)(ny + 1) * nx;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n * P; k += gridDim.x * blockDim.x) {
        const int p = k / P, q = k % P, tile = tiles[p];
        const int gx = (tile % ntx) * S - 1 + q % So, gy = (tile / ntx) * S - 1 + q / So;
        float lab[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float msk[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (gx >= 0 && gy >= 0 && gx < nx && gy < ny) {
            if (gx + 1 < nx) {   // east face = x line I = gx + 1
                double f[3];
                for (int c = 0; c < 3; ++c) {
                    double sum = 0.0;
                    for (int j = 0; j < r; ++j) sum += (double)ftx[c * pfx + (size_t)(gy * r + j) * (nx + 1) + gx + 1];
                    f[c] = (sum / r - (double)ctx[c * pcx + (size_t)gy * (nx + 1) + gx + 1]) * inv_tau;
                }
                lab[0] = (float)f[0]; lab[1] = (float)f[1]; lab[2] = (float)f[2];
                msk[0] = msk[1] = msk[2] = 1.f;
            }
            if (gy + 1 < ny) {   // north face = y line J = gy + 1
                double f[3];
                for (int c = 0; c < 3; ++c) {
                    double sum = 0.0;
                    for (int i = 0; i < r; ++i) sum += (double)fty[c * pfy + (size_t)(gy + 1) * r * nx + gx * r + i];
                    f[c] = (sum / r - (double)cty[c * pcy + (size_t)(gy + 1) * nx + gx]) * inv_tau;
                }
                lab[3] = (float)f[0]; lab[4] = (float)f[2]; lab[5] = (float)f[1];   // world x, y momentum
                msk[3] = msk[4] = msk[5] = 1.f;
            }
        }
        int cnt = 0;
        for (int c = 0; c < 6; ++c) {
            y[(size_t)k * 6 + c] = lab[c] / oscale[c];
            mask[(size_t)k * 6 + c] = msk[c];
            cnt += msk[c] > 0.f;
        }
        if (cnt) atomicAdd(&mcount[p], cnt);
    }
}

// Minibatch: crops idx[b] of the data set into the network's input, label
// and mask buffers.
__global__ void k_batch_copy(const int* __restrict__ idx, int nb, int So, const unsigned short* __restrict__ X,
                             const float* __restrict__ Y, const float* __restrict__ M, unsigned short* __restrict__ x,
                             float* __restrict__ y, float* __restrict__ m) {
    const int Sin = So + 2 * HALO;
    const size_t px = (size_t)Sin * Sin * 16, py = (size_t)So * So * 6;
    const size_t total = (size_t)nb * (px + 2 * py);
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        if (k < (size_t)nb * px) {
            const size_t b = k / px, o = k % px;
            x[k] = X[(size_t)idx[b] * px + o];
        } else if (k < (size_t)nb * (px + py)) {
            const size_t kk = k - (size_t)nb * px, b = kk / py, o = kk % py;
            y[kk] = Y[(size_t)idx[b] * py + o];
        } else {
            const size_t kk = k - (size_t)nb * (px + py), b = kk / py, o = kk % py;
            m[kk] = M[(size_t)idx[b] * py + o];
        }
    }
}

// Labels of the data set re-expressed in new output scales: y *= old / new.
__global__ void k_rescale(float* __restrict__ y, size_t n, const float* __restrict__ ratio) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        y[k] *= ratio[k % 6];
}

}  // namespace lc
}  // namespace swe
