// Convolutional neural operator of the learned warm start: a five-level U-Net on NHWC bf16
// activations with FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), its backward pass and an Adam update, all hand-written.
//
// Topology (channels per level 32, 64, 128, 256, 256; 3x3 convolutions with ReLU):
//   encoder level l: conv(cin -> C_l), conv(C_l -> C_l) = s_l; 2x2 average pooling between levels
//   bottleneck:      conv(256 -> 256), conv(256 -> 256)
//   decoder level l: nearest 2x upsampling, concatenation [up, s_l], conv(. -> C_l), conv(C_l -> C_l)
//   head:            1x1 convolution 32 -> 4 (no activation), FP32 output.
// The network input has 4 planes, padded to 8 channels in memory (the padding channels are zero).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbmib_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr int CIN0 = 8;        // padded input channels
constexpr int NIN = 4;         // real input planes
constexpr int NOUT = 4;        // output planes
constexpr int LEVELS = 5;
constexpr int CH[LEVELS] = {32, 64, 128, 256, 256};

// ---------------------------------------------------------------------------------------------
// Convolution forward as an implicit GEMM: Y[p][co] = act(sum_k W[co][k] X^[k][p] + b[co]),
// k = tap * cin + ci, X^[k][p] = X[p shifted by tap][ci] (zero outside the image).
// One wavefront computes a (16 TM) x (16 TN) tile of (output channels) x (pixels); its operands
// are read straight from global memory as 8 consecutive channels per lane (16-byte loads):
// A lane l holds W[co][k .. k+7] with co = l % 16, k = 8 (l / 16) + 32 s; B lane l holds
// X[pixel l % 16][k .. k+7]; the result lane l holds rows 4 (l / 16) + r of column l % 16.
// X has pixel stride xstride; Y is written at Y[p ystride + yoff + co].
// gate: as in k_conv_fwd_lds. Requires cin, xstride % 8 == 0, cout % (16 TM) == 0, ystride, yoff % 4 == 0.
template <int TM, int TN>
__global__ void __launch_bounds__(256) k_conv_fwd(const __bf16* __restrict__ X, int cin, int xstride,
                                                  const __bf16* __restrict__ Wt, const float* __restrict__ bias, int cout,
                                                  int taps, int H, int Wd, long long P, int relu, __bf16* __restrict__ Y,
                                                  int ystride, int yoff, const __bf16* __restrict__ gate) {
    const int lane = threadIdx.x % WAVE;
    const long long wave = (long long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int co_tiles = cout / (16 * TM);
    const long long tiles = (long long)co_tiles * ((P + 16 * TN - 1) / (16 * TN));
    if (wave >= tiles) return;
    const int co0 = (int)(wave % co_tiles) * 16 * TM;
    const long long p0 = (wave / co_tiles) * 16 * TN;
    const int K = taps * cin;
    const int HW = H * Wd;
    int py[TN], px[TN];
    long long pb[TN];
    bool pv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const long long p = p0 + j * 16 + lane % 16;
        pv[j] = p < P;
        const long long n = p / HW;
        const int r = (int)(p - n * HW);
        py[j] = r / Wd;
        px[j] = r - py[j] * Wd;
        pb[j] = n * HW;
    }
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const int kk = k0 + (lane / 16) * 8;
        const bool kv = kk < K;
        const int tap = kv ? kk / cin : 0;
        const int ci = kk - tap * cin;
        const int dy = taps == 9 ? tap / 3 - 1 : 0;
        const int dx = taps == 9 ? tap % 3 - 1 : 0;
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            a[i] = kv ? *reinterpret_cast<const bf16x8*>(Wt + (long long)(co0 + i * 16 + lane % 16) * K + kk) : zero;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int y = py[j] + dy, x = px[j] + dx;
            const bool in = kv && pv[j] && y >= 0 && y < H && x >= 0 && x < Wd;
            b[j] = in ? *reinterpret_cast<const bf16x8*>(X + (pb[j] + (long long)y * Wd + x) * xstride + ci) : zero;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            if (!pv[j]) continue;
            const int cb = co0 + i * 16 + (lane / 16) * 4;
            const long long p = p0 + j * 16 + lane % 16;
            bf16x4 o, gv = {};
            if (gate) gv = *reinterpret_cast<const bf16x4*>(gate + p * ystride + yoff + cb);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[i][j][r] + (bias ? bias[cb + r] : 0.f);
                if (relu) v = v > 0.f ? v : 0.f;
                if (gate && !((float)gv[r] > 0.f)) v = 0.f;
                o[r] = (__bf16)v;
            }
            *reinterpret_cast<bf16x4*>(Y + p * ystride + yoff + cb) = o;
        }
}

// Convolution forward (3x3) with the input and the weights staged through LDS. A workgroup of 4
// wavefronts owns COB output channels x CONV_NPX (64 or 128) pixels, the pixels being a TH x TW
// block of one image (TW = min(64, W), TH = CONV_NPX / TW, rows beyond the image masked). Per chunk
// of 32 input channels it stages the (TH + 2) x (TW + 2) input block with its one-pixel halo (zero
// outside the image) and the chunk's weights of all nine taps ([tap][channel][32 + 8]) as 16-byte
// vectors into LDS, then runs the nine taps from there: the B operand of tap (dy, dx) for output
// pixel (ty, tx) is the staged pixel (ty + dy + 1, tx + dx + 1), so every input value and weight
// is read from memory once per chunk. The global loads of the next chunk are issued into
// registers before the MFMAs of the current one and stored into LDS after them. Wavefront w
// computes 32 channels x (CONV_NPX / WN) pixels with WM = COB / 32 wavefronts along the channels.
// With gate (same layout as Y), the output is zeroed where gate is not positive (the backward of
// a ReLU whose output gate is). Requires cin % 32 == 0, cout % COB == 0, xstride % 8 == 0,
// ystride, yoff % 4 == 0.
template <int COB, int CONV_NPX>
__global__ void __launch_bounds__(256) k_conv_fwd_lds(const __bf16* __restrict__ X, int cin, int xstride,
                                                      const __bf16* __restrict__ Wt, const float* __restrict__ bias,
                                                      int cout, int H, int Wd, int tw, int relu,
                                                      __bf16* __restrict__ Y, int ystride, int yoff,
                                                      const __bf16* __restrict__ gate) {
    constexpr int CK = 32, LDP = CK + 8;
    constexpr int MAXP = (CONV_NPX / 64 + 2) * 66;  // largest staged block: TW = 64
    constexpr int WM = COB / 32, WN = 4 / WM, TNW = CONV_NPX / (16 * WN);
    constexpr int PV = (MAXP * (CK / 8) + 255) / 256;        // input vectors per thread and chunk (bound)
    constexpr int NWV = 9 * COB * (CK / 8), WV = (NWV + 255) / 256;   // weight vectors
    __shared__ __bf16 patch[MAXP * LDP];
    __shared__ __bf16 wst[9 * COB * LDP];
    const int th = CONV_NPX / tw;
    const int pw = tw + 2, np = (th + 2) * pw, npv = np * (CK / 8);
    const int co_tiles = cout / COB;
    const int bx_tiles = Wd / tw, by_tiles = (H + th - 1) / th;
    long long b = blockIdx.x;
    const int cot = (int)(b % co_tiles);
    b /= co_tiles;
    const int bxt = (int)(b % bx_tiles);
    b /= bx_tiles;
    const int byt = (int)(b % by_tiles);
    const long long n = b / by_tiles;
    const int x0 = bxt * tw, y0 = byt * th;
    const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
    const int wm = wv / WN, wn = wv % WN;
    const int K = 9 * cin;
    const long long img = n * H * Wd;

    int tyj[TNW], txj[TNW];
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
        const int q = wn * (CONV_NPX / WN) + j * 16 + lane % 16;   // pixel of the block
        tyj[j] = q / tw;
        txj[j] = q % tw;
    }
    f32x4 acc[2][TNW];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    const int kg = 8 * (lane / 16);                 // this lane's 8-channel group within a k step

    bf16x8 pr[PV], wr[WV];
    auto fetch = [&](int ci0) {
#pragma unroll
        for (int r = 0; r < PV; ++r) {
            const int v = t + 256 * r;
            pr[r] = zero;
            if (v < npv) {
                const int pix = v / (CK / 8), g = v % (CK / 8);
                const int y = y0 - 1 + pix / pw, x = x0 - 1 + pix % pw;
                if (y >= 0 && y < H && x >= 0 && x < Wd)
                    pr[r] = *reinterpret_cast<const bf16x8*>(X + (img + (long long)y * Wd + x) * xstride + ci0 + 8 * g);
            }
        }
#pragma unroll
        for (int r = 0; r < WV; ++r) {
            const int v = t + 256 * r;
            wr[r] = zero;
            if (v < NWV) {
                const int g = v % (CK / 8), row = v / (CK / 8);      // row = tap * COB + channel
                const int tap = row / COB, co = row % COB;
                wr[r] = *reinterpret_cast<const bf16x8*>(Wt + (long long)(cot * COB + co) * K + (long long)tap * cin +
                                                         ci0 + 8 * g);
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int r = 0; r < PV; ++r) {
            const int v = t + 256 * r;
            if (v < npv) *reinterpret_cast<bf16x8*>(patch + (v / (CK / 8)) * LDP + 8 * (v % (CK / 8))) = pr[r];
        }
#pragma unroll
        for (int r = 0; r < WV; ++r) {
            const int v = t + 256 * r;
            if (v < NWV) *reinterpret_cast<bf16x8*>(wst + (v / (CK / 8)) * LDP + 8 * (v % (CK / 8))) = wr[r];
        }
    };

    fetch(0);
    for (int ci0 = 0; ci0 < cin; ci0 += CK) {
        __syncthreads();                            // the previous chunk's reads are done
        stash();
        __syncthreads();
        if (ci0 + CK < cin) fetch(ci0 + CK);        // in flight during this chunk's MFMAs
#pragma unroll 3
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;   // offsets + 1
            bf16x8 a[2], bv[TNW];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(wst + (tap * COB + wm * 32 + i * 16 + lane % 16) * LDP + kg);
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[j] = *reinterpret_cast<const bf16x8*>(patch + ((tyj[j] + dy) * pw + txj[j] + dx) * LDP + kg);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    const int co_w = cot * COB + wm * 32;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int y = y0 + tyj[j];
            if (y >= H) continue;
            const long long p = img + (long long)y * Wd + x0 + txj[j];
            const int cb = co_w + i * 16 + (lane / 16) * 4;
            bf16x4 o, gv = {};
            if (gate) gv = *reinterpret_cast<const bf16x4*>(gate + p * ystride + yoff + cb);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[i][j][r] + (bias ? bias[cb + r] : 0.f);
                if (relu) v = v > 0.f ? v : 0.f;
                if (gate && !((float)gv[r] > 0.f)) v = 0.f;
                o[r] = (__bf16)v;
            }
            *reinterpret_cast<bf16x4*>(Y + p * ystride + yoff + cb) = o;
        }
}

// Weight and bias gradients staged through LDS. A workgroup of 4 wavefronts owns a BM x BN tile of
// (output channel) x (k = tap cin + ci) and a range of pixels (one split). Per step of 32 pixels
// it reads dY [32 pixels][BM channels] and X^ [32 pixels][BN columns] as 16-byte vectors of 8
// channels, stores both transposed in LDS ([channel][pixel]) and runs one 16x16x32 MFMA per
// 16 x 16 sub-tile: lane l reads 8 consecutive pixels of row l % 16. Each wavefront owns 32 x 32.
// The workgroups of the first k tile also sum dY over their pixels (the bias gradient). Split s
// writes its partials to part[s][cout K + cout]: the weights [co][k], then the biases.
// Requires cout % BM == 0, cin % 8 == 0 and strides % 8 == 0.
template <int BM>
__global__ void __launch_bounds__(256) k_conv_wgrad_lds(const __bf16* __restrict__ dY, int cout, int dys,
                                                        const __bf16* __restrict__ X, int cin, int xs, int taps, int H,
                                                        int Wd, long long P, int split_len, int nsplit,
                                                        float* __restrict__ part) {
    constexpr int BN = 4096 / BM;
    constexpr int KP = 32, LD = KP + 8;
    __shared__ __bf16 As[BM][LD];
    __shared__ __bf16 Bs[BN][LD];
    __shared__ float bred[256 / (BM / 8)][BM];
    const int K = taps * cin;
    const int co_tiles = cout / BM, k_tiles = (K + BN - 1) / BN;
    const int b = blockIdx.x;
    const int cot = b % co_tiles, kt = (b / co_tiles) % k_tiles, s = b / (co_tiles * k_tiles);
    if (s >= nsplit) return;
    const int co0 = cot * BM, k0 = kt * BN;
    const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
    constexpr int WN = BN / 32;                    // wavefronts along k
    const int wm = wv / WN, wn = wv % WN;
    const int HW = H * Wd;
    const long long pbeg = (long long)s * split_len;
    const long long pend = pbeg + split_len < P ? pbeg + split_len : P;
    // staging roles: the pixel is the fastest index, so that the lanes of a wavefront store
    // consecutive pixels of one or two LDS rows (transposed stores free of bank conflicts)
    constexpr int AG = BM / 8;                     // 8-channel groups of dY per pixel
    const int a_pix = t % KP, a_g = t / KP;        // valid for t < 32 * AG
    const bool a_on = t < KP * AG;
    float bsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    // Software pipeline: the global loads of the next slice go into registers before the MFMA
    // of the current one, and are stored (transposed) into LDS after the barrier that ends it.
    constexpr int BR = (BN * KP / 8 + 255) / 256;   // X^ vectors per thread and slice
    bf16x8 va = zero, vb[BR];
    auto load = [&](long long q) {
        if (a_on) {
            const long long p = q + a_pix;
            va = p < pend ? *reinterpret_cast<const bf16x8*>(dY + p * dys + co0 + 8 * a_g) : zero;
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int v_ = t + 256 * r;
            vb[r] = zero;
            if (v_ < BN * KP / 8) {
                const int pix = v_ % KP, g = v_ / KP;
                const int k = k0 + 8 * g;
                const long long p = q + pix;
                if (k < K && p < pend) {
                    const int tap = k / cin, ci = k - tap * cin;
                    const int dy = taps == 9 ? tap / 3 - 1 : 0, dx = taps == 9 ? tap % 3 - 1 : 0;
                    const long long n = p / HW;
                    const int rr = (int)(p - n * HW);
                    const int y = rr / Wd + dy, x = rr % Wd + dx;
                    if (y >= 0 && y < H && x >= 0 && x < Wd)
                        vb[r] = *reinterpret_cast<const bf16x8*>(X + (n * HW + (long long)y * Wd + x) * xs + ci);
                }
            }
        }
    };
    auto store = [&]() {
        if (a_on) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                As[8 * a_g + e][a_pix] = va[e];
                bsum[e] += (float)va[e];
            }
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int v_ = t + 256 * r;
            if (v_ < BN * KP / 8) {
                const int pix = v_ % KP, g = v_ / KP;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[8 * g + e][pix] = vb[r][e];
            }
        }
    };
    if (pbeg < pend) load(pbeg);
    for (long long q = pbeg; q < pend; q += KP) {
        store();
        __syncthreads();
        if (q + KP < pend) load(q + KP);
        bf16x8 a[2], bb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + lane % 16][8 * (lane / 16)]);
#pragma unroll
        for (int j = 0; j < 2; ++j) bb[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + j * 16 + lane % 16][8 * (lane / 16)]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float* out = part + (long long)s * (cout * K + cout);   // split row: weights, then biases
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = k0 + wn * 32 + j * 16 + lane % 16;
            if (k >= K) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + wm * 32 + i * 16 + (lane / 16) * 4 + r;
                out[(long long)co * K + k] = acc[i][j][r];
            }
        }
    if (kt == 0) {
        if (a_on)
#pragma unroll
            for (int e = 0; e < 8; ++e) bred[a_pix][8 * a_g + e] = bsum[e];
        __syncthreads();
        if (t < BM) {
            float v = 0.f;
            for (int r = 0; r < KP; ++r) v += bred[r][t];
            out[(long long)cout * K + co0 + t] = v;
        }
    }
}

// Weight and bias gradients, deeper steps: as k_conv_wgrad_lds, but each barrier pair covers KP
// pixels (KP / 32 MFMA steps per 16 x 16 sub-tile) and every thread stages several 8-channel
// vectors of each operand. Requires KP to divide H W, W and KP to divide one another, and splits of
// a multiple of KP pixels. The bias gradient (row sums of dY over the pixels) comes from the
// same MFMA unit: the wavefronts of the first k tile multiply their dY rows by a ones operand.
template <int BM, int KP>
__global__ void __launch_bounds__(256) k_conv_wgrad_deep(const __bf16* __restrict__ dY, int cout, int dys,
                                                         const __bf16* __restrict__ X, int cin, int xs, int taps, int H,
                                                         int Wd, long long P, int split_len, int nsplit,
                                                         float* __restrict__ part) {
    constexpr int BN = 4096 / BM;
    constexpr int LD = KP + 8;
    constexpr int AV = BM * KP / 8, BV = BN * KP / 8;      // 8-channel vectors per step
    constexpr int AR = (AV + 255) / 256, BR = (BV + 255) / 256;
    __shared__ __bf16 As[BM][LD];
    __shared__ __bf16 Bs[BN][LD];
    const int K = taps * cin;
    const int co_tiles = cout / BM, k_tiles = (K + BN - 1) / BN;
    const int b = blockIdx.x;
    const int cot = b % co_tiles, kt = (b / co_tiles) % k_tiles, s = b / (co_tiles * k_tiles);
    if (s >= nsplit) return;
    const int co0 = cot * BM, k0 = kt * BN;
    const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
    constexpr int WN = BN / 32;                    // wavefronts along k
    const int wm = wv / WN, wn = wv % WN;
    const int HW = H * Wd;
    const long long pbeg = (long long)s * split_len;
    const long long pend = pbeg + split_len < P ? pbeg + split_len : P;
    const bool bias = kt == 0 && wn == 0;
    f32x4 acc[2][2], accb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bf16x8 zero = {};
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
    // A step of KP pixels starts at a multiple of KP, KP divides H W, and W and KP divide one
    // another: the step lies in one image, within one row (W >= KP) or over whole rows (W < KP),
    // so only the step's base is divided; the channel offsets, taps, shifts and row/column offsets
    // of each staged vector are fixed for the whole split.
    int b_ci[BR], b_dy[BR], b_dx[BR], b_pix[BR], b_row[BR], b_col[BR];
    bool b_on[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        const int v_ = t + 256 * r;
        const int g = v_ / KP, k = k0 + 8 * g;
        b_pix[r] = v_ % KP;
        b_row[r] = b_pix[r] / Wd;
        b_col[r] = b_pix[r] - b_row[r] * Wd;
        b_on[r] = v_ < BV && k < K;
        const int tap = k / cin;
        b_ci[r] = k - tap * cin;
        b_dy[r] = taps == 9 ? tap / 3 - 1 : 0;
        b_dx[r] = taps == 9 ? tap % 3 - 1 : 0;
    }
    bf16x8 va[AR], vb[BR];
    auto load = [&](long long q) {
        const long long n = q / HW;
        const int rr = (int)(q - n * HW);
        const int y0 = rr / Wd, x0 = rr - y0 * Wd;
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int v_ = t + 256 * r;
            va[r] = zero;
            if (v_ < AV) {
                const int pix = v_ % KP, g = v_ / KP;
                const long long p = q + pix;
                if (p < pend) va[r] = *reinterpret_cast<const bf16x8*>(dY + p * dys + co0 + 8 * g);
            }
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            vb[r] = zero;
            if (b_on[r] && q + b_pix[r] < pend) {
                const int y = y0 + b_row[r] + b_dy[r], x = x0 + b_col[r] + b_dx[r];
                if (y >= 0 && y < H && x >= 0 && x < Wd)
                    vb[r] = *reinterpret_cast<const bf16x8*>(X + (n * HW + (long long)y * Wd + x) * xs + b_ci[r]);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < AR; ++r) {
            const int v_ = t + 256 * r;
            if (v_ < AV) {
                const int pix = v_ % KP, g = v_ / KP;
#pragma unroll
                for (int e = 0; e < 8; ++e) As[8 * g + e][pix] = va[r][e];
            }
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            const int v_ = t + 256 * r;
            if (v_ < BV) {
                const int pix = v_ % KP, g = v_ / KP;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[8 * g + e][pix] = vb[r][e];
            }
        }
    };
    if (pbeg < pend) load(pbeg);
    for (long long q = pbeg; q < pend; q += KP) {
        store();
        __syncthreads();
        if (q + KP < pend) load(q + KP);
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks) {
            bf16x8 a[2], bb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + lane % 16][32 * ks + 8 * (lane / 16)]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bb[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + j * 16 + lane % 16][32 * ks + 8 * (lane / 16)]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
            if (bias)
#pragma unroll
                for (int i = 0; i < 2; ++i) accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], ones, accb[i], 0, 0, 0);
        }
        __syncthreads();
    }
    float* out = part + (long long)s * (cout * K + cout);   // split row: weights, then biases
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = k0 + wn * 32 + j * 16 + lane % 16;
            if (k >= K) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + wm * 32 + i * 16 + (lane / 16) * 4 + r;
                out[(long long)co * K + k] = acc[i][j][r];
            }
        }
    // every column of the ones product holds the row sums; column 0 is written
    if (bias && lane % 16 == 0)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(long long)cout * K + co0 + wm * 32 + i * 16 + (lane / 16) * 4 + r] = accb[i][r];
}

// Fixed-order sum of the split partials into the FP32 gradient.
// Rows r are summed into r % 8 partial sums (independent loads in flight), which are then added
// in order 0..7: a fixed order, so the result does not depend on the launch.
__device__ __forceinline__ float strided_sum8(const float* __restrict__ part, int rows, long long n, long long i) {
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int r = 0;
    for (; r + 8 <= rows; r += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(long long)(r + u) * n + i];
    for (int u = 0; r + u < rows; ++u) a[u] += part[(long long)(r + u) * n + i];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ void k_sum_splits(const float* __restrict__ part, int nsplit, long long n, float* __restrict__ g) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g[i] = strided_sum8(part, nsplit, n, i);
}

// W'[ci][8 - t][co] = W[co][t][ci] for every 3x3 layer at once (backward data is the forward
// convolution of dY with W'); the flipped copy of a layer sits at the layer's bf16 offset.
constexpr int FLIP_MAXL = 24;
struct FlipTab {
    int n;                              // layers (3x3, in offset order)
    long long total;                    // weights in all of them
    long long off[FLIP_MAXL];           // bf16 offset of each layer
    int cout[FLIP_MAXL], cin[FLIP_MAXL];
};
__global__ void k_flip_all(const __bf16* __restrict__ W, FlipTab tab, __bf16* __restrict__ Wf) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tab.total) return;
    int l = 0;
    while (l + 1 < tab.n && i >= tab.off[l + 1]) ++l;
    const long long o = i - tab.off[l];
    const int cin = tab.cin[l], cout = tab.cout[l];
    const int ci = (int)(o % cin);
    const int t = (int)((o / cin) % 9);
    const int co = (int)(o / (9LL * cin));
    Wf[tab.off[l] + ((long long)ci * 9 + (8 - t)) * cout + co] = W[i];
}

// 2x2 average pooling of a channel slice: out[n][y][x][c] = mean of in[n][2y+i][2x+j][off + c].
// One thread per output pixel and 8 channels (C, stride, off multiples of 8).
__global__ void k_pool(const __bf16* __restrict__ in, int stride, int off, int C, int B, int H, int Wd,
                       __bf16* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int h = H / 2, w = Wd / 2, G = C / 8;
    const long long n_out = (long long)B * h * w * G;
    if (i >= n_out) return;
    const int c = 8 * (int)(i % G);
    const long long q = i / G;
    const int x = (int)(q % w), y = (int)((q / w) % h);
    const long long n = q / ((long long)w * h);
    const long long b = ((n * H + 2 * y) * Wd + 2 * x) * stride + off + c;
    const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(in + b);
    const bf16x8 v1 = *reinterpret_cast<const bf16x8*>(in + b + stride);
    const bf16x8 v2 = *reinterpret_cast<const bf16x8*>(in + b + (long long)Wd * stride);
    const bf16x8 v3 = *reinterpret_cast<const bf16x8*>(in + b + (long long)Wd * stride + stride);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        o[k] = (__bf16)(0.25f * (((float)v0[k] + (float)v1[k]) + ((float)v2[k] + (float)v3[k])));
    *reinterpret_cast<bf16x8*>(out + q * C + c) = o;
}

// Adjoint of the pooling, accumulated: dIn[n][2y+i][2x+j][off + c] += dOut[n][y][x][c] / 4, then
// zeroed where gate (the ReLU output, same layout as dIn) is not positive.
__global__ void k_pool_bwd(const __bf16* __restrict__ dOut, int C, int B, int H, int Wd, __bf16* __restrict__ dIn,
                           int stride, int off, const __bf16* __restrict__ gate) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = C / 8;
    const long long n_in = (long long)B * H * Wd * G;
    if (i >= n_in) return;
    const int c = 8 * (int)(i % G);
    const long long q = i / G;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H);
    const long long n = q / ((long long)Wd * H);
    const bf16x8 g = *reinterpret_cast<const bf16x8*>(dOut + ((n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * C + c);
    const long long o = q * stride + off + c;
    bf16x8 d = *reinterpret_cast<const bf16x8*>(dIn + o);
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(gate + o);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        d[k] = (__bf16)((float)d[k] + 0.25f * (float)g[k]);
        if (!((float)a[k] > 0.f)) d[k] = (__bf16)0.f;
    }
    *reinterpret_cast<bf16x8*>(dIn + o) = d;
}

// Nearest 2x upsampling into a channel slice: out[n][y][x][off + c] = in[n][y/2][x/2][c].
__global__ void k_up(const __bf16* __restrict__ in, int C, int B, int H, int Wd, __bf16* __restrict__ out, int stride,
                     int off) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = C / 8;
    const long long n_out = (long long)B * H * Wd * G;
    if (i >= n_out) return;
    const int c = 8 * (int)(i % G);
    const long long q = i / G;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H);
    const long long n = q / ((long long)Wd * H);
    *reinterpret_cast<bf16x8*>(out + q * stride + off + c) =
        *reinterpret_cast<const bf16x8*>(in + ((n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * C + c);
}

// Adjoint of the upsampling: dIn[n][y][x][c] = sum of the four dOut[n][2y+i][2x+j][off + c],
// zeroed where gate (the ReLU output, layout of dIn) is not positive.
__global__ void k_up_bwd(const __bf16* __restrict__ dOut, int stride, int off, int C, int B, int H, int Wd,
                         __bf16* __restrict__ dIn, const __bf16* __restrict__ gate) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int h = H / 2, w = Wd / 2, G = C / 8;
    const long long n_in = (long long)B * h * w * G;
    if (i >= n_in) return;
    const int c = 8 * (int)(i % G);
    const long long q = i / G;
    const int x = (int)(q % w), y = (int)((q / w) % h);
    const long long n = q / ((long long)w * h);
    const long long b = ((n * H + 2 * y) * Wd + 2 * x) * stride + off + c;
    const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(dOut + b);
    const bf16x8 v1 = *reinterpret_cast<const bf16x8*>(dOut + b + stride);
    const bf16x8 v2 = *reinterpret_cast<const bf16x8*>(dOut + b + (long long)Wd * stride);
    const bf16x8 v3 = *reinterpret_cast<const bf16x8*>(dOut + b + (long long)Wd * stride + stride);
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(gate + q * C + c);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        o[k] = (__bf16)(((float)v0[k] + (float)v1[k]) + ((float)v2[k] + (float)v3[k]));
        if (!((float)a[k] > 0.f)) o[k] = (__bf16)0.f;
    }
    *reinterpret_cast<bf16x8*>(dIn + q * C + c) = o;
}

// FP32 input planes [P][4] -> bf16 [P][8] (channels 4..7 zero).
__global__ void k_pack_input(const float* __restrict__ in, long long P, __bf16* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * CIN0) return;
    const long long p = i / CIN0;
    const int c = (int)(i - p * CIN0);
    out[i] = (__bf16)(c < NIN ? in[p * NIN + c] : 0.f);
}

// Head: out[p][o] = sum_c Wh[o][c] A[p][c] + bh[o], 1x1, FP32 output.
__global__ void k_head_fwd(const __bf16* __restrict__ A, const float* __restrict__ Wh, const float* __restrict__ bh,
                           long long P, float* __restrict__ out) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float a[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) a[c] = (float)A[p * 32 + c];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 32; ++c) s += Wh[o * 32 + c] * a[c];
        out[p * NOUT + o] = s + bh[o];
    }
}

// Head backward, data: dA[p][c] = sum_o Wh[o][c] dOut[p][o] (bf16), zeroed where gate[p][c] (the
// ReLU output the head reads) is not positive.
__global__ void k_head_dgrad(const float* __restrict__ Wh, const float* __restrict__ dOut, long long P,
                             __bf16* __restrict__ dA, const __bf16* __restrict__ gate) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float g[NOUT];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) g[o] = dOut[p * NOUT + o];
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        float s = 0.f;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) s += Wh[o * 32 + c] * g[o];
        dA[p * 32 + c] = (float)gate[p * 32 + c] > 0.f ? (__bf16)s : (__bf16)0.f;
    }
}

// Head backward, parameters: per block of HEAD_PIX pixels the partial sums
// dWh[o][c] = sum_p dOut[p][o] A[p][c] (column 32 o + c) and dbh[o] = sum_p dOut[p][o] (column
// 128 + o), each thread over a quarter of the channels of every 64th pixel, then a fixed-order tree.
constexpr int HEAD_PIX = 256;
constexpr int HEAD_NP = NOUT * 32 + NOUT;
__global__ void __launch_bounds__(256) k_head_wgrad(const __bf16* __restrict__ A, const float* __restrict__ dOut,
                                                    long long P, float* __restrict__ part) {
    static_assert(NOUT == 4 && HEAD_PIX % 64 == 0, "head gradient layout");
    __shared__ float red[64][HEAD_NP + 1];
    // thread (g, j): channels 8 g .. 8 g + 7 of pixels j, j + 64, ... of the block (16-byte loads)
    const int t = threadIdx.x, g = t & 3, j = t >> 2;
    float s[NOUT][8], sb[NOUT];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        sb[o] = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) s[o][e] = 0.f;
    }
    const long long p0 = (long long)blockIdx.x * HEAD_PIX;
#pragma unroll
    for (int k = 0; k < HEAD_PIX / 64; ++k) {
        const long long p = p0 + j + 64 * k;
        if (p >= P) break;
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + p * 32 + 8 * g);
        const float4 d = *reinterpret_cast<const float4*>(dOut + p * NOUT);
        const float dv[NOUT] = {d.x, d.y, d.z, d.w};
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            sb[o] += dv[o];
#pragma unroll
            for (int e = 0; e < 8; ++e) s[o][e] += dv[o] * (float)a[e];
        }
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
#pragma unroll
        for (int e = 0; e < 8; ++e) red[j][o * 32 + 8 * g + e] = s[o][e];
        if (g == 0) red[j][NOUT * 32 + o] = sb[o];
    }
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {          // fixed-order tree over the 64 pixel lanes
        for (int idx = t; idx < w * HEAD_NP; idx += 256) {
            const int jj = idx / HEAD_NP, q = idx - jj * HEAD_NP;
            red[jj][q] += red[jj + w][q];
        }
        __syncthreads();
    }
    for (int q = t; q < HEAD_NP; q += 256) part[(long long)blockIdx.x * HEAD_NP + q] = red[0][q];
}

// Column sums of a [rows][n] FP32 array in fixed order: out[i] = sum_r part[r][i].
// One workgroup per column: thread t adds rows t, t + 256, ... in order, then a fixed-order
// tree in LDS (the result does not depend on the launch).
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ part, int rows, int n, float* __restrict__ out) {
    __shared__ float red[256];
    const int i = blockIdx.x;
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) acc += part[(long long)r * n + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

// Masked mean squared error over P pixels and 4 planes (mask NULL: all ones).
// Block partials of sum(mask err^2) and sum(mask), then the final sums in FP64.
constexpr int LOSS_PIX = 2048;
__global__ void __launch_bounds__(256) k_loss_part(const float* __restrict__ out, const float* __restrict__ tgt,
                                                   const float* __restrict__ mask, long long P, double* __restrict__ part) {
    const long long p0 = (long long)blockIdx.x * LOSS_PIX;
    __shared__ double r1[256], r2[256];
    double s1 = 0, s2 = 0;
    for (long long p = p0 + threadIdx.x; p < p0 + LOSS_PIX && p < P; p += 256) {
        const double m = mask ? mask[p] : 1.0;
        double e2 = 0;
        for (int o = 0; o < NOUT; ++o) {
            const double d = (double)out[p * NOUT + o] - (double)tgt[p * NOUT + o];
            e2 += d * d;
        }
        s1 += m * e2;
        s2 += m;
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r1[0];
        part[2 * blockIdx.x + 1] = r2[0];
    }
}

// loss[0] = sum(mask err^2) / (4 sum(mask)), loss[1] = 4 sum(mask).
__global__ void __launch_bounds__(256) k_loss_final(const double* __restrict__ part, int nparts, double* __restrict__ loss) {
    __shared__ double r1[256], r2[256];
    double s1 = 0, s2 = 0;
    for (int k = threadIdx.x; k < nparts; k += 256) {
        s1 += part[2 * k];
        s2 += part[2 * k + 1];
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double cnt = NOUT * r2[0];
        loss[0] = cnt > 0 ? r1[0] / cnt : 0.0;
        loss[1] = cnt;
    }
}

// dOut = 2 mask (out - tgt) / count.
__global__ void k_loss_grad(const float* __restrict__ out, const float* __restrict__ tgt, const float* __restrict__ mask,
                            long long P, const double* __restrict__ loss, float* __restrict__ g) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * NOUT) return;
    const double cnt = loss[1];
    const float m = mask ? mask[i / NOUT] : 1.f;
    g[i] = cnt > 0 ? (float)(2.0 * m * ((double)out[i] - (double)tgt[i]) / cnt) : 0.f;
}

// Adam on the FP32 master parameters; the bf16 copy of each conv weight is refreshed.
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2, float wd,
                       const long long* __restrict__ bf_map, __bf16* __restrict__ bf) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float t = theta[i] - lr * (mh / (sqrtf(vh) + eps) + wd * theta[i]);
    theta[i] = t;
    const long long b = bf_map[i];
    if (b >= 0) bf[b] = (__bf16)t;
}

// Global L2 norm of the gradient and its clipping: NORM_BLOCKS block partials of sum g^2 in FP64
// (grid-stride, then a fixed-order tree in the block), one block that adds the partials in order
// and turns the norm into the scale min(1, max_norm / norm), and an in-place scaling that reads
// the scale from device memory (no host synchronisation).
constexpr int NORM_BLOCKS = 512;
__global__ void __launch_bounds__(256) k_sqnorm_part(const float* __restrict__ g, long long n, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)NORM_BLOCKS * 256)
        s += (double)g[i] * (double)g[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_clip_scale(const double* __restrict__ part, double max_norm, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < NORM_BLOCKS; ++b) s += part[b];
    const double norm = sqrt(s);
    out[0] = norm;
    out[1] = norm > max_norm ? max_norm / norm : 1.0;
}

__global__ void k_scale_grads(float* __restrict__ g, long long n, const double* __restrict__ scale) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = scale[1];
    if (c != 1.0) g[i] = (float)((double)g[i] * c);
}

// FP32 master -> bf16 copies (after set_params).
__global__ void k_to_bf(const float* __restrict__ theta, long long n, const long long* __restrict__ bf_map,
                        __bf16* __restrict__ bf) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long b = bf_map[i];
    if (b >= 0) bf[b] = (__bf16)theta[i];
}

inline unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------------------------
// Host side: topology, buffers, and the forward / backward / update sequences.

namespace {

struct Layer {
    int cin, cout, taps;
    long long w_off, b_off;     // offsets in the flat FP32 parameter vector
    long long bf_off;           // offset of the bf16 weight copy
};

struct Act {                    // one activation buffer (and its gradient) at one level
    __bf16* a;
    __bf16* g;
    int c;
};

std::vector<Layer> topology() {
    std::vector<Layer> L;
    auto add = [&](int ci, int co, int taps) { L.push_back({ci, co, taps, 0, 0, 0}); };
    int c = CIN0;
    for (int l = 0; l < LEVELS; ++l) {          // encoder + bottleneck: 2 convs per level
        add(c, CH[l], 9);
        add(CH[l], CH[l], 9);
        c = CH[l];
    }
    for (int l = LEVELS - 2; l >= 0; --l) {     // decoder: input = [up (channels of level l+1 output), s_l]
        const int up = CH[l + 1];
        add(up + CH[l], CH[l], 9);
        add(CH[l], CH[l], 9);
    }
    add(CH[0], NOUT, 1);                        // head
    long long off = 0, bf = 0;
    for (auto& x : L) {
        x.w_off = off;
        off += (long long)x.cout * x.taps * x.cin;
        x.b_off = off;
        off += x.cout;
        x.bf_off = bf;
        bf += (long long)x.cout * x.taps * x.cin;
    }
    return L;
}

long long param_count() {
    const auto L = topology();
    return L.back().b_off + L.back().cout;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

struct nn_unet {
    int B = 0, H = 0, W = 0;
    hipStream_t stream = nullptr;
    std::vector<Layer> L;
    long long np = 0, nbf = 0;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    __bf16* wbf = nullptr;          // bf16 weights, concatenated per layer
    __bf16* wflip = nullptr;        // flipped bf16 weights of every 3x3 layer (backward data), as wbf
    FlipTab ftab{};
    long long* bf_map = nullptr;    // parameter index -> bf16 index or -1
    float* split = nullptr;         // weight-gradient split partials
    size_t split_floats = 0;
    float* small = nullptr;         // bias / head partials
    size_t small_floats = 0;
    double* lossp = nullptr;        // loss partials
    double* loss = nullptr;         // [2]
    __bf16* in0 = nullptr;          // [P0][8]
    Act enc_a[LEVELS]{}, pool[LEVELS]{}, cat[LEVELS - 1]{}, dec_a[LEVELS - 1]{}, dec_b[LEVELS - 1]{};
    Act bott_b{};                   // bottleneck second conv output
    float* out = nullptr;           // [P0][4] FP32 head output
    float* dout = nullptr;          // [P0][4]
    int last_b = 0;                 // batch of the last forward
    std::string err;
};

namespace {

thread_local std::string g_nn_error;

int nfail(nn_unet* u, int code, const std::string& msg) {
    if (u)
        u->err = msg;
    else
        g_nn_error = msg;
    return code;
}

#define NCHK(u, call)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return nfail((u), NN_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t layout(nn_unet* u, int B, int H, int W, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = align_up(off);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const auto L = topology();
    const long long np = L.back().b_off + L.back().cout;
    long long nbf = 0;
    for (auto& x : L) nbf += (long long)x.cout * x.taps * x.cin;
    const long long P0 = (long long)B * H * W;
    float* theta = (float*)take(np * 4);
    float* m = (float*)take(np * 4);
    float* v = (float*)take(np * 4);
    float* grad = (float*)take(np * 4);
    __bf16* wbf = (__bf16*)take(nbf * 2);
    long long maxw = 0;
    for (auto& x : L) maxw = std::max(maxw, (long long)x.cout * x.taps * x.cin);
    __bf16* wflip = (__bf16*)take(nbf * 2);
    long long* bf_map = (long long*)take(np * 8);
    // split partials: at most 64 splits of the largest weight
    const size_t split_floats = (size_t)64 * maxw;
    float* split = (float*)take(split_floats * 4);
    const size_t small_floats = (size_t)std::max<long long>((P0 + HEAD_PIX - 1) / HEAD_PIX * HEAD_NP, 256 * 256);
    float* small = (float*)take(small_floats * 4);
    double* lossp = (double*)take(((P0 + LOSS_PIX - 1) / LOSS_PIX) * 2 * 8);
    double* loss = (double*)take(2 * 8);
    __bf16* in0 = (__bf16*)take(P0 * CIN0 * 2);
    Act enc_a[LEVELS]{}, pool[LEVELS]{}, cat[LEVELS - 1]{}, dec_a[LEVELS - 1]{}, dec_b[LEVELS - 1]{}, bott{};
    auto act = [&](long long P, int c) {
        Act a;
        a.c = c;
        a.a = (__bf16*)take(P * c * 2);
        a.g = (__bf16*)take(P * c * 2);
        return a;
    };
    for (int l = 0; l < LEVELS; ++l) {
        const long long P = (long long)B * (H >> l) * (W >> l);
        enc_a[l] = act(P, CH[l]);
        if (l > 0) pool[l] = act(P, CH[l - 1]);
        if (l < LEVELS - 1) {
            cat[l] = act(P, CH[l + 1] + CH[l]);
            dec_a[l] = act(P, CH[l]);
            dec_b[l] = act(P, CH[l]);
        } else {
            bott = act(P, CH[l]);
        }
    }
    float* out = (float*)take(P0 * NOUT * 4);
    float* dout = (float*)take(P0 * NOUT * 4);
    if (u) {
        u->L = L;
        u->np = np;
        u->nbf = nbf;
        u->theta = theta;
        u->m = m;
        u->v = v;
        u->grad = grad;
        u->wbf = wbf;
        u->wflip = wflip;
        u->bf_map = bf_map;
        u->split = split;
        u->split_floats = split_floats;
        u->small = small;
        u->small_floats = small_floats;
        u->lossp = lossp;
        u->loss = loss;
        u->in0 = in0;
        for (int l = 0; l < LEVELS; ++l) {
            u->enc_a[l] = enc_a[l];
            u->pool[l] = pool[l];
        }
        for (int l = 0; l < LEVELS - 1; ++l) {
            u->cat[l] = cat[l];
            u->dec_a[l] = dec_a[l];
            u->dec_b[l] = dec_b[l];
        }
        u->bott_b = bott;
        u->out = out;
        u->dout = dout;
    }
    return align_up(off);
}

// Layer indices in topology order.
int enc_conv(int l, int k) { return 2 * l + k; }                        // k = 0, 1
int dec_conv(int l, int k) { return 2 * LEVELS + 2 * (LEVELS - 2 - l) + k; }
int head_layer() { return 2 * LEVELS + 2 * (LEVELS - 1); }

hipError_t conv_fwd(nn_unet* u, const Layer& ly, const __bf16* X, int xstride, const __bf16* Wt, const float* bias,
                    int relu, int B, int H, int W, __bf16* Y, int ystride, int yoff, const __bf16* gate = nullptr) {
    const long long P = (long long)B * H * W;
    // 3x3 layers with 32-channel multiples and power-of-two widths: input staged through LDS
    if (ly.taps == 9 && ly.cin % 32 == 0 && ly.cout % 32 == 0 && xstride % 8 == 0 && ystride % 4 == 0 &&
        yoff % 4 == 0 && W >= 8 && (W & (W - 1)) == 0) {      // W >= 8: the staged block fits MAXP
        const int tw = W < 64 ? W : 64;
        const int cob = ly.cout % 64 == 0 ? 64 : 32;
        // 128 pixels per workgroup unless that leaves fewer than two workgroups per CU
        const long long blk128 = (long long)B * ((H + 128 / tw - 1) / (128 / tw)) * (W / tw) * (ly.cout / cob);
        const int npx = blk128 >= 512 ? 128 : 64;
        const int th = npx / tw;
        const unsigned nblk = (unsigned)((long long)B * ((H + th - 1) / th) * (W / tw) * (ly.cout / cob));
        if (cob == 64 && npx == 128)
            hipLaunchKernelGGL((k_conv_fwd_lds<64, 128>), dim3(nblk), dim3(256), 0, u->stream, X, ly.cin, xstride, Wt,
                               bias, ly.cout, H, W, tw, relu, Y, ystride, yoff, gate);
        else if (cob == 64)
            hipLaunchKernelGGL((k_conv_fwd_lds<64, 64>), dim3(nblk), dim3(256), 0, u->stream, X, ly.cin, xstride, Wt,
                               bias, ly.cout, H, W, tw, relu, Y, ystride, yoff, gate);
        else if (npx == 128)
            hipLaunchKernelGGL((k_conv_fwd_lds<32, 128>), dim3(nblk), dim3(256), 0, u->stream, X, ly.cin, xstride, Wt,
                               bias, ly.cout, H, W, tw, relu, Y, ystride, yoff, gate);
        else
            hipLaunchKernelGGL((k_conv_fwd_lds<32, 64>), dim3(nblk), dim3(256), 0, u->stream, X, ly.cin, xstride, Wt,
                               bias, ly.cout, H, W, tw, relu, Y, ystride, yoff, gate);
        return hipGetLastError();
    }
    constexpr int TM = 2, TN = 4;
    if (ly.cout % (16 * TM) || ly.cin % 8 || xstride % 8 || ystride % 4 || yoff % 4) return hipErrorInvalidValue;
    const long long tiles = (long long)(ly.cout / (16 * TM)) * ((P + 16 * TN - 1) / (16 * TN));
    hipLaunchKernelGGL((k_conv_fwd<TM, TN>), dim3(blocks(tiles, 4)), dim3(256), 0, u->stream, X, ly.cin, xstride, Wt,
                       bias, ly.cout, ly.taps, H, W, P, relu, Y, ystride, yoff, gate);
    return hipGetLastError();
}

// Pixels per staging step of the weight gradient: 128 when such a step lies in one image (within a
// row, or over whole rows of a narrower level) and each split keeps at least two of them
// (LBMIB_WGRAD_KP=32 selects the shallow kernel, for comparison), else 32.
int wgrad_kp(long long P, long long nsplit, int H, int W) {
    static const int forced = [] {
        const char* v = std::getenv("LBMIB_WGRAD_KP");
        return v ? std::atoi(v) : 0;
    }();
    if (forced == 32) return 32;
    // W and H W are powers of two here: a 128-pixel step fits one image once H W >= 128
    return ((long long)H * W % 128 == 0 && (W % 128 == 0 || 128 % W == 0) && P / nsplit >= 256) ? 128 : 32;
}

// dW (into grad at w_off) and db (at b_off) of a 3x3 layer from dY [P] (stride dys) and its input X.
hipError_t conv_wgrad(nn_unet* u, const Layer& ly, const __bf16* dY, int dys, const __bf16* X, int xs, int B, int H,
                      int W) {
    const long long P = (long long)B * H * W;
    const int K = ly.taps * ly.cin;
    const int BM = ly.cout % 64 == 0 ? 64 : 32;
    const int BN = 4096 / BM;
    if (ly.cout % BM || ly.cin % 8 || dys % 8 || xs % 8) return hipErrorInvalidValue;
    const long long wsz = (long long)ly.cout * K;
    if (ly.b_off != ly.w_off + wsz) return hipErrorInvalidValue;
    const long long tiles = (long long)(ly.cout / BM) * ((K + BN - 1) / BN);
    // splits: enough workgroups to fill the chip, at least 256 pixels each, within the partial buffer
    long long nsplit = std::max<long long>(1, std::min<long long>(P / 256, (2048 + tiles - 1) / tiles));
    nsplit = std::min<long long>(nsplit, 256);
    while ((size_t)nsplit * (wsz + ly.cout) > u->split_floats && nsplit > 1) --nsplit;
    // deeper steps (KP pixels per barrier pair) while every split still holds two of them
    const int KP = wgrad_kp(P, nsplit, H, W);
    long long split_len = (P + nsplit - 1) / nsplit;
    split_len = (split_len + KP - 1) / KP * KP;
    nsplit = (P + split_len - 1) / split_len;
    const dim3 grid((unsigned)(tiles * nsplit));
    if (KP == 128 && BM == 64)
        hipLaunchKernelGGL((k_conv_wgrad_deep<64, 128>), grid, dim3(256), 0, u->stream, dY, ly.cout, dys, X, ly.cin, xs,
                           ly.taps, H, W, P, (int)split_len, (int)nsplit, u->split);
    else if (KP == 128)
        hipLaunchKernelGGL((k_conv_wgrad_deep<32, 128>), grid, dim3(256), 0, u->stream, dY, ly.cout, dys, X, ly.cin, xs,
                           ly.taps, H, W, P, (int)split_len, (int)nsplit, u->split);
    else if (BM == 64)
        hipLaunchKernelGGL(k_conv_wgrad_lds<64>, grid, dim3(256), 0, u->stream, dY, ly.cout, dys, X, ly.cin, xs, ly.taps,
                           H, W, P, (int)split_len, (int)nsplit, u->split);
    else
        hipLaunchKernelGGL(k_conv_wgrad_lds<32>, grid, dim3(256), 0, u->stream, dY, ly.cout, dys, X, ly.cin, xs, ly.taps,
                           H, W, P, (int)split_len, (int)nsplit, u->split);
    // weights and biases are adjacent in the parameter vector, as in each split row
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks(wsz + ly.cout)), dim3(256), 0, u->stream, (const float*)u->split,
                       (int)nsplit, wsz + ly.cout, u->grad + ly.w_off);
    return hipGetLastError();
}

// dX [P][cin] (stride dxs) of a 3x3 layer from dY (stride dys): forward convolution with the
// flipped weights.
hipError_t conv_dgrad(nn_unet* u, const Layer& ly, const __bf16* dY, int dys, int B, int H, int W, __bf16* dX, int dxs,
                      const __bf16* gate = nullptr) {
    Layer t{ly.cout, ly.cin, 9, 0, 0, 0};
    return conv_fwd(u, t, dY, dys, u->wflip + ly.bf_off, nullptr, 0, B, H, W, dX, dxs, 0, gate);
}

// Refresh the flipped weights after the bf16 copy changed (set_params, Adam).
hipError_t flip_weights(nn_unet* u) {
    hipLaunchKernelGGL(k_flip_all, dim3(blocks(u->ftab.total)), dim3(256), 0, u->stream, (const __bf16*)u->wbf, u->ftab,
                       u->wflip);
    return hipGetLastError();
}

int forward(nn_unet* u, int B, const float* d_in, float* d_out) {
    const int H = u->H, W = u->W;
    const long long P0 = (long long)B * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(blocks(P0 * CIN0)), dim3(256), 0, u->stream, d_in, P0, u->in0);
    NCHK(u, hipGetLastError());
    const __bf16* x = u->in0;
    int xs = CIN0;
    for (int l = 0; l < LEVELS; ++l) {
        const int h = H >> l, w = W >> l;
        const Layer& c0 = u->L[enc_conv(l, 0)];
        const Layer& c1 = u->L[enc_conv(l, 1)];
        if (l > 0) {
            // pooled s_{l-1}: the skip slice of cat[l-1]
            const Act& src = u->cat[l - 1];
            const long long n = (long long)B * h * w * CH[l - 1];
            hipLaunchKernelGGL(k_pool, dim3(blocks(n / 8)), dim3(256), 0, u->stream, (const __bf16*)src.a, src.c, CH[l],
                               CH[l - 1], B, 2 * h, 2 * w, u->pool[l].a);
            NCHK(u, hipGetLastError());
            x = u->pool[l].a;
            xs = CH[l - 1];
        }
        NCHK(u, conv_fwd(u, c0, x, xs, u->wbf + c0.bf_off, u->theta + c0.b_off, 1, B, h, w, u->enc_a[l].a, CH[l], 0));
        if (l < LEVELS - 1)
            NCHK(u, conv_fwd(u, c1, u->enc_a[l].a, CH[l], u->wbf + c1.bf_off, u->theta + c1.b_off, 1, B, h, w,
                             u->cat[l].a, u->cat[l].c, CH[l + 1]));
        else
            NCHK(u, conv_fwd(u, c1, u->enc_a[l].a, CH[l], u->wbf + c1.bf_off, u->theta + c1.b_off, 1, B, h, w,
                             u->bott_b.a, CH[l], 0));
    }
    const __bf16* below = u->bott_b.a;      // output of the level below (l + 1)
    for (int l = LEVELS - 2; l >= 0; --l) {
        const int h = H >> l, w = W >> l;
        const long long n = (long long)B * h * w * CH[l + 1];
        hipLaunchKernelGGL(k_up, dim3(blocks(n / 8)), dim3(256), 0, u->stream, below, CH[l + 1], B, h, w, u->cat[l].a,
                           u->cat[l].c, 0);
        NCHK(u, hipGetLastError());
        const Layer& d0 = u->L[dec_conv(l, 0)];
        const Layer& d1 = u->L[dec_conv(l, 1)];
        NCHK(u, conv_fwd(u, d0, u->cat[l].a, u->cat[l].c, u->wbf + d0.bf_off, u->theta + d0.b_off, 1, B, h, w,
                         u->dec_a[l].a, CH[l], 0));
        NCHK(u, conv_fwd(u, d1, u->dec_a[l].a, CH[l], u->wbf + d1.bf_off, u->theta + d1.b_off, 1, B, h, w,
                         u->dec_b[l].a, CH[l], 0));
        below = u->dec_b[l].a;
    }
    const Layer& hd = u->L[head_layer()];
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks(P0)), dim3(256), 0, u->stream, (const __bf16*)u->dec_b[0].a,
                       (const float*)(u->theta + hd.w_off), (const float*)(u->theta + hd.b_off), P0, u->out);
    NCHK(u, hipGetLastError());
    if (d_out) NCHK(u, hipMemcpyAsync(d_out, u->out, P0 * NOUT * 4, hipMemcpyDeviceToDevice, u->stream));
    u->last_b = B;
    return NN_OK;
}

int backward(nn_unet* u, const float* d_tgt, const float* d_mask, double* d_loss_out) {
    const int B = u->last_b, H = u->H, W = u->W;
    const long long P0 = (long long)B * H * W;
    const int nl = (int)((P0 + LOSS_PIX - 1) / LOSS_PIX);
    hipLaunchKernelGGL(k_loss_part, dim3(nl), dim3(256), 0, u->stream, (const float*)u->out, d_tgt, d_mask, P0, u->lossp);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, u->stream, (const double*)u->lossp, nl, u->loss);
    hipLaunchKernelGGL(k_loss_grad, dim3(blocks(P0 * NOUT)), dim3(256), 0, u->stream, (const float*)u->out, d_tgt, d_mask,
                       P0, (const double*)u->loss, u->dout);
    NCHK(u, hipGetLastError());
    if (d_loss_out) NCHK(u, hipMemcpyAsync(d_loss_out, u->loss, 2 * 8, hipMemcpyDeviceToDevice, u->stream));
    // head
    const Layer& hd = u->L[head_layer()];
    const int nh = (int)((P0 + HEAD_PIX - 1) / HEAD_PIX);
    hipLaunchKernelGGL(k_head_dgrad, dim3(blocks(P0)), dim3(256), 0, u->stream, (const float*)(u->theta + hd.w_off),
                       (const float*)u->dout, P0, u->dec_b[0].g, (const __bf16*)u->dec_b[0].a);
    hipLaunchKernelGGL(k_head_wgrad, dim3(nh), dim3(256), 0, u->stream, (const __bf16*)u->dec_b[0].a,
                       (const float*)u->dout, P0, u->small);
    hipLaunchKernelGGL(k_colsum, dim3(HEAD_NP), dim3(256), 0, u->stream, (const float*)u->small, nh, HEAD_NP,
                       u->grad + hd.w_off);
    NCHK(u, hipGetLastError());
    // decoder, top level first
    for (int l = 0; l < LEVELS - 1; ++l) {
        const int h = H >> l, w = W >> l;
        const long long P = (long long)B * h * w;
        const Layer& d0 = u->L[dec_conv(l, 0)];
        const Layer& d1 = u->L[dec_conv(l, 1)];
        // the gradients of ReLU outputs arrive gated by their producers (head, upsampling adjoint,
        // backward-data epilogue, pooling adjoint)
        NCHK(u, conv_wgrad(u, d1, u->dec_b[l].g, CH[l], u->dec_a[l].a, CH[l], B, h, w));
        NCHK(u, conv_dgrad(u, d1, u->dec_b[l].g, CH[l], B, h, w, u->dec_a[l].g, CH[l], u->dec_a[l].a));
        NCHK(u, conv_wgrad(u, d0, u->dec_a[l].g, CH[l], u->cat[l].a, u->cat[l].c, B, h, w));
        NCHK(u, conv_dgrad(u, d0, u->dec_a[l].g, CH[l], B, h, w, u->cat[l].g, u->cat[l].c));
        // the upsampled part of the concatenation goes to the output of the level below
        __bf16* gbelow = l + 1 < LEVELS - 1 ? u->dec_b[l + 1].g : u->bott_b.g;
        const __bf16* abelow = l + 1 < LEVELS - 1 ? u->dec_b[l + 1].a : u->bott_b.a;
        const long long n = (long long)B * (h / 2) * (w / 2) * CH[l + 1];
        hipLaunchKernelGGL(k_up_bwd, dim3(blocks(n / 8)), dim3(256), 0, u->stream, (const __bf16*)u->cat[l].g, u->cat[l].c, 0,
                           CH[l + 1], B, h, w, gbelow, abelow);
        NCHK(u, hipGetLastError());
    }
    // bottleneck and encoder, deepest level first
    for (int l = LEVELS - 1; l >= 0; --l) {
        const int h = H >> l, w = W >> l;
        const long long P = (long long)B * h * w;
        const Layer& c0 = u->L[enc_conv(l, 0)];
        const Layer& c1 = u->L[enc_conv(l, 1)];
        __bf16 *ga, *aa;
        int stride, off;
        if (l == LEVELS - 1) {
            ga = u->bott_b.g;
            aa = u->bott_b.a;
            stride = CH[l];
            off = 0;
        } else {
            // skip slice of cat[l]: the decoder's part is there, the pooling path adds its part
            ga = u->cat[l].g;
            aa = u->cat[l].a;
            stride = u->cat[l].c;
            off = CH[l + 1];
            const long long n = P * CH[l];
            hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(n / 8)), dim3(256), 0, u->stream, (const __bf16*)u->pool[l + 1].g,
                               CH[l], B, h, w, ga, stride, off, (const __bf16*)aa);
            NCHK(u, hipGetLastError());
        }
        NCHK(u, conv_wgrad(u, c1, ga + off, stride, u->enc_a[l].a, CH[l], B, h, w));
        NCHK(u, conv_dgrad(u, c1, ga + off, stride, B, h, w, u->enc_a[l].g, CH[l], u->enc_a[l].a));
        const __bf16* xin = l > 0 ? u->pool[l].a : u->in0;
        const int xs = l > 0 ? CH[l - 1] : CIN0;
        NCHK(u, conv_wgrad(u, c0, u->enc_a[l].g, CH[l], xin, xs, B, h, w));
        if (l > 0) NCHK(u, conv_dgrad(u, c0, u->enc_a[l].g, CH[l], B, h, w, u->pool[l].g, CH[l - 1]));
    }
    return NN_OK;
}

}  // namespace

extern "C" {

long long nn_unet_param_count(void) { return param_count(); }

size_t nn_unet_workspace_bytes(int batch, int H, int W) {
    if (batch < 1 || H < 16 || W < 128 || H % 16 || W % 128) return 0;
    return layout(nullptr, batch, H, W, nullptr);
}

int nn_unet_create(int batch, int H, int W, void* ws, size_t bytes, void* stream, nn_unet** out) {
    if (!out) return nfail(nullptr, NN_E_INVAL, "out is NULL");
    *out = nullptr;
    if (batch < 1 || H < 16 || W < 128 || H % 16 || W % 128)
        return nfail(nullptr, NN_E_INVAL, "need batch >= 1, H a multiple of 16 and W a multiple of 128");
    const size_t need = layout(nullptr, batch, H, W, nullptr);
    if (!ws || bytes < need) return nfail(nullptr, NN_E_NOMEM, "workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(ws) % 256) return nfail(nullptr, NN_E_INVAL, "workspace not 256-byte aligned");
    nn_unet* u = new (std::nothrow) nn_unet();
    if (!u) return nfail(nullptr, NN_E_NOMEM, "host allocation failed");
    u->B = batch;
    u->H = H;
    u->W = W;
    u->stream = (hipStream_t)stream;
    layout(u, batch, H, W, (char*)ws);
    std::vector<long long> map(u->np, -1);
    for (size_t i = 0; i + 1 < u->L.size(); ++i) {      // the head stays FP32
        const Layer& x = u->L[i];
        const long long n = (long long)x.cout * x.taps * x.cin;
        for (long long k = 0; k < n; ++k) map[x.w_off + k] = x.bf_off + k;
    }
    u->ftab.n = 0;
    for (size_t i = 0; i < u->L.size(); ++i) {
        const Layer& x = u->L[i];
        if (x.taps != 9) continue;
        if (u->ftab.n == FLIP_MAXL) {
            delete u;
            return nfail(nullptr, NN_E_INVAL, "too many layers for the flip table");
        }
        u->ftab.off[u->ftab.n] = x.bf_off;
        u->ftab.cout[u->ftab.n] = x.cout;
        u->ftab.cin[u->ftab.n] = x.cin;
        u->ftab.total = x.bf_off + (long long)x.cout * 9 * x.cin;   // the 3x3 layers come first and are contiguous
        ++u->ftab.n;
    }
    hipError_t e = hipMemcpy(u->bf_map, map.data(), map.size() * 8, hipMemcpyHostToDevice);
    for (float* a : {u->theta, u->m, u->v, u->grad})
        if (e == hipSuccess) e = hipMemsetAsync(a, 0, u->np * 4, u->stream);
    if (e == hipSuccess) e = hipMemsetAsync(u->wbf, 0, u->nbf * 2, u->stream);
    if (e == hipSuccess) e = hipMemsetAsync(u->wflip, 0, u->nbf * 2, u->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(u->stream);
    if (e != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete u;
        return nfail(nullptr, NN_E_HIP, "create: " + m);
    }
    *out = u;
    return NN_OK;
}

int nn_unet_set_params(nn_unet* u, const float* params, int on_device) {
    if (!u || !params) return NN_E_INVAL;
    NCHK(u, hipMemcpyAsync(u->theta, params, u->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           u->stream));
    NCHK(u, hipMemsetAsync(u->m, 0, u->np * 4, u->stream));
    NCHK(u, hipMemsetAsync(u->v, 0, u->np * 4, u->stream));
    hipLaunchKernelGGL(k_to_bf, dim3(blocks(u->np)), dim3(256), 0, u->stream, (const float*)u->theta, u->np,
                       (const long long*)u->bf_map, u->wbf);
    NCHK(u, hipGetLastError());
    NCHK(u, flip_weights(u));
    if (!on_device) NCHK(u, hipStreamSynchronize(u->stream));
    return NN_OK;
}

int nn_unet_get_params(nn_unet* u, float* params, int on_device) {
    if (!u || !params) return NN_E_INVAL;
    NCHK(u, hipMemcpyAsync(params, u->theta, u->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           u->stream));
    if (!on_device) NCHK(u, hipStreamSynchronize(u->stream));
    return NN_OK;
}

int nn_unet_get_grads(nn_unet* u, float* grads, int on_device) {
    if (!u || !grads) return NN_E_INVAL;
    NCHK(u, hipMemcpyAsync(grads, u->grad, u->np * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           u->stream));
    if (!on_device) NCHK(u, hipStreamSynchronize(u->stream));
    return NN_OK;
}

int nn_unet_forward(nn_unet* u, int b, const float* d_in, float* d_out) {
    if (!u || !d_in) return NN_E_INVAL;
    if (b < 1 || b > u->B) return nfail(u, NN_E_INVAL, "batch outside [1, capacity]");
    return forward(u, b, d_in, d_out);
}

int nn_unet_backward(nn_unet* u, const float* d_target, const float* d_mask, double* d_loss) {
    if (!u || !d_target) return NN_E_INVAL;
    if (u->last_b < 1) return nfail(u, NN_E_STATE, "no forward pass");
    return backward(u, d_target, d_mask, d_loss);
}

int nn_unet_adam(nn_unet* u, double lr, double beta1, double beta2, double eps, int t, double weight_decay) {
    if (!u || t < 1) return NN_E_INVAL;
    const float c1 = (float)(1.0 - std::pow(beta1, t)), c2 = (float)(1.0 - std::pow(beta2, t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(u->np)), dim3(256), 0, u->stream, u->theta, u->m, u->v, (const float*)u->grad,
                       u->np, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2, (float)weight_decay,
                       (const long long*)u->bf_map, u->wbf);
    NCHK(u, hipGetLastError());
    NCHK(u, flip_weights(u));
    return NN_OK;
}

int nn_unet_clip_grad_norm(nn_unet* u, double max_norm, double* d_norm) {
    if (!u || !(max_norm > 0.0)) return NN_E_INVAL;
    if (u->small_floats < 2 * (NORM_BLOCKS + 2)) return NN_E_INVAL;
    // the bias / head partial buffer is free between backward passes
    double* part = reinterpret_cast<double*>(u->small);
    double* out = part + NORM_BLOCKS;
    hipLaunchKernelGGL(k_sqnorm_part, dim3(NORM_BLOCKS), dim3(256), 0, u->stream, (const float*)u->grad, u->np, part);
    NCHK(u, hipGetLastError());
    hipLaunchKernelGGL(k_clip_scale, dim3(1), dim3(64), 0, u->stream, (const double*)part, max_norm, out);
    NCHK(u, hipGetLastError());
    hipLaunchKernelGGL(k_scale_grads, dim3(blocks(u->np)), dim3(256), 0, u->stream, u->grad, u->np,
                       (const double*)out);
    NCHK(u, hipGetLastError());
    if (d_norm) NCHK(u, hipMemcpyAsync(d_norm, out, 2 * sizeof(double), hipMemcpyDeviceToDevice, u->stream));
    return NN_OK;
}

void nn_unet_destroy(nn_unet* u) { delete u; }

const char* nn_unet_last_error(nn_unet* u) { return u ? u->err.c_str() : g_nn_error.c_str(); }

}  // extern "C"
