// Learned CG pair force: inference of f(r) = s * taper(r) * [W3 . silu(W2 silu(W1 x + b1) + b2) + b3],
// x = r / rc, on gfx950 matrix cores.  It stands in for F^CG of Eq. (1) (Sec. 2.2:
// a force between centres of mass); below r_min the cubic CG table is used instead.
//
// One wavefront evaluates a tile of 32 pairs, layer 2 computed transposed
// (Z2^T = W2 H1^T, output units x pairs) so that every result a lane holds belongs to
// its own pair:
//   * layer 1 (rank one in x) in VALU: lane l computes, for pair l % 32, the 32 hidden
//     units 16 kb + 8 (l / 32) + j (kb = 0..3, j = 0..7), applies silu and writes them
//     as BF16 straight into the B operands (column = pair) of four MFMA K-blocks;
//   * layer 2 (64 x 64 x 32) on v_mfma_f32_32x32x16_bf16 with FP32 accumulation; W2
//     (row = output unit, BF16) is held in registers as the A operands for the whole
//     kernel (lane l: row 32 mb + l % 32 of M-block mb, K columns 16 kb + 8 (l / 32) .. +7);
//   * layer 3: lane l holds, for pair l % 32, output units 32 mb + 8 (v / 4) + 4 (l / 32)
//     + v % 4 (v = 0..15), multiplies silu(z2) by W3 and adds the two half-wavefronts'
//     sums with one exchange.
// Operand and result lane layouts were checked on the device with a known product.
#include <algorithm>

#include "adres_mlp.h"

namespace adres {
namespace {

constexpr int kTile = 32;
constexpr int kWaves = 4;
constexpr int kBlockM = 64 * kWaves;
constexpr int kQueue = kTile + 64;   // queued pairs per wave: a partial tile plus one window

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// taper(r) = 1 below rc - tw, cos^2 ramp to 0 at rc (same shape as the resolution function)
__device__ __forceinline__ float taper_f(float r, float rc, float tw)
{
    float u = (r - (rc - tw)) / tw;
    if (u <= 0.0f) return 1.0f;
    if (u >= 1.0f) return 0.0f;
    float c = __cosf(1.5707963267948966f * u);
    return c * c;
}

// r of pair p: input distances, or a pair of Morton slots whose centres are read.
struct PairSource {
    const double *r;        // non-null: distances
    const int2 *pairs;      // else: (t, u) slot pairs
    const double4 *Rw;
    int64_t n;              // pair count; with n_dev: the capacity, the count read from n_dev
    const int *n_dev;
};

__device__ __forceinline__ double pair_r(const PairSource &src, const DevParams &P, int64_t p)
{
    if (src.r) return src.r[p];
    const int2 tu = src.pairs[p];
    const double4 a = src.Rw[tu.x], b = src.Rw[tu.y];
    const double d0 = mi(a.x - b.x, P.box[0], P.inv_box[0]);
    const double d1 = mi(a.y - b.y, P.box[1], P.inv_box[1]);
    const double d2 = mi(a.z - b.z, P.box[2], P.inv_box[2]);
    return sqrt(dist2_exact(d0, d1, d2));
}

template <bool FP8>
__global__ __launch_bounds__(kBlockM) void k_mlp_forward(MlpDev M, DevParams P, PairSource src, float *__restrict__ out,
                                                        Ctrl *ctrl, int check_halt, int step)
{
    if (check_halt && step > ctrl->halt) return;
    if (src.n_dev) src.n = min((int64_t)*src.n_dev, src.n);   // src.n holds the buffer capacity here
    // silu(z) = z / (1 + 2^t) with t = -log2(e) z.  The constants are folded so that each
    // layer works on t directly: layer 1 forms t1 = (-log2e W1) x + (-log2e b1) and hands
    // g1 = t1 / (1 + 2^t1) = silu(z1) / (-ln 2) to the matrix cores, whose product with W2
    // plus (-log2e b2) is then t2 = -log2e z2 (log2e ln 2 = 1); layer 3 adds
    // (-ln 2 W3) t2 / (1 + 2^t2) = W3 silu(z2).
    __shared__ float sW1[kHidden], sB1[kHidden];
    __shared__ float sW3[kHidden];
    constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
    for (int i = threadIdx.x; i < kHidden; i += kBlockM) {
        sW1[i] = -kLog2e * M.w1[i];
        sB1[i] = -kLog2e * M.b1[i];
        sW3[i] = -kLn2 * M.w3[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    // A operands: W2 rows (output units) 32 mb + col; BF16: K columns 16 kb + 8 half .. +7;
    // FP8 (32x32x64, one K-block): K columns 32 half .. +31
    bf16x8 Wop[2][4];
    int32x8 Wq[2];
    float dq = 1.0f, inv_sg = 1.0f, inv_dq = 1.0f;
    if constexpr (FP8) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            Wq[mb] = *reinterpret_cast<const int32x8 *>(M.w2_fp8 + (32 * mb + col) * (kHidden / 4) + 8 * half);
        dq = M.fp8_scale[0];
        inv_sg = M.fp8_scale[1];
        inv_dq = M.fp8_scale[2];
    } else {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                Wop[mb][kb] =
                    *reinterpret_cast<const bf16x8 *>(M.w2_bf16 + (32 * mb + col) * kHidden + 16 * kb + 8 * half);
    }
    // -log2e b2 of the output units of this lane's result rows (32 mb + 8 (v / 4) + 4 half
    // + v % 4): the accumulator's initial value (FP8: in units of the product's scale)
    floatx16 c2[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) c2[mb][v] = -kLog2e * M.b2[32 * mb + 8 * (v >> 2) + 4 * half + (v & 3)] * inv_dq;
    const float b3 = M.w3[kHidden], inv_rc = 1.0f / (float)M.rc, rcf = (float)M.rc, twf = (float)M.tw, sc = (float)M.scale;

    // Pairs are read in windows of 64 (one per lane).  A pair below r_min takes the table
    // and one at or beyond rc is zero, both written at once by its lane; the others are
    // appended to a per-wave queue in LDS (ballot + prefix count), and the network runs on
    // full tiles of 32 queued pairs, plus one partial tile at the end.
    __shared__ double qr[kWaves][kQueue];
    __shared__ int qp[kWaves][kQueue];
    const int wv = threadIdx.x >> 6;
    int q_head = 0, q_len = 0;   // wave-uniform ring-buffer state

    auto run_tile = [&](int count) {
        // lane col takes queued pair col (both half-wavefronts the same pair)
        const int slot = (q_head + (col < count ? col : 0)) % kQueue;
        const double r = col < count ? qr[wv][slot] : M.rc;
        const int p = qp[wv][slot];
        const float x = (float)r * inv_rc;
        bf16x8 H[4];
        int32x8 Hq;
        if constexpr (FP8) {
            // g1 / s_g of input units 32 half + 4 w + e, rounded to E4M3 (nearest even), four per word
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                float g[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int u = 32 * half + 4 * w + e;
                    const float t = fmaf(sW1[u], x, sB1[u]);
                    g[e] = t * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)) * inv_sg;
                }
                int pk = __builtin_amdgcn_cvt_pk_fp8_f32(g[0], g[1], 0, false);
                Hq[w] = __builtin_amdgcn_cvt_pk_fp8_f32(g[2], g[3], pk, true);
            }
        } else {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int u = 16 * kb + 8 * half + j;
                    const float t = fmaf(sW1[u], x, sB1[u]);
                    H[kb][j] = (__bf16)(t * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)));
                }
        }
        float y = 0.0f;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            floatx16 acc = c2[mb];
            if constexpr (FP8) {
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(Wq[mb], Hq, acc, 0, 0, 0, 0, 0, 0);
            } else {
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wop[mb][kb], H[kb], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float t = acc[v] * dq;
                const float w = sW3[32 * mb + 8 * (v >> 2) + 4 * half + (v & 3)];
                y = fmaf(w * t, __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)), y);
            }
        }
        y += __shfl_xor(y, 32, 64);
        if (half == 0 && col < count) out[p] = sc * taper_f((float)r, rcf, twf) * (y + b3);
        q_head = (q_head + count) % kQueue;
        q_len -= count;
    };

    const int64_t n_win = (src.n + 63) / 64;
    const int64_t wave_id = (int64_t)blockIdx.x * kWaves + wv;
    const int64_t n_waves = (int64_t)gridDim.x * kWaves;
    for (int64_t win = wave_id; win < n_win; win += n_waves) {
        const int64_t p = win * 64 + lane;
        const bool ok = p < src.n;
        const double r = ok ? pair_r(src, P, p) : M.rc;
        bool net = false;
        if (ok) {
            if (r < M.r_min && P.tab) {
                double u = (r - P.tab_lo) / P.tab_h;
                if (r < P.tab_lo) atomicOr(&ctrl->err, kErrTableRange);
                double kf = floor(u);
                kf = kf >= 0.0 ? kf : 0.0;
                kf = kf > (double)(P.tab_n - 2) ? (double)(P.tab_n - 2) : kf;
                const float t = (float)(u - kf);
                const float4 c = P.tab[(int)kf];
                out[p] = ((c.w * t + c.z) * t + c.y) * t + c.x;
            } else if (r >= M.rc) {
                out[p] = 0.0f;
            } else {
                net = true;
            }
        }
        const uint64_t mask = __ballot(net);
        if (net) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            const int slot = (q_head + q_len + rank) % kQueue;
            qr[wv][slot] = r;
            qp[wv][slot] = (int)p;
        }
        wave_lds_sync();
        q_len += __popcll(mask);
        while (q_len >= kTile) {
            run_tile(kTile);
            wave_lds_sync();
        }
    }
    if (q_len > 0) run_tile(q_len);
}

}  // namespace

void launch_mlp_forward_r(hipStream_t s, const MlpDev &M, const DevParams &P, const double *r, float *f, int64_t n,
                          Ctrl *ctrl)
{
    PairSource src{r, nullptr, nullptr, n, nullptr};
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int blocks = (int)std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
    if (M.fp8) k_mlp_forward<true><<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, 0, 0);
    else k_mlp_forward<false><<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, 0, 0);
}

void launch_mlp_forward_pairs(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs,
                              const double4 *Rw, float *f, const int *n_dev, int64_t n_cap, Ctrl *ctrl,
                              int check_halt, int step)
{
    PairSource src{nullptr, pairs, Rw, n_cap, n_dev};
    const int64_t tiles = (n_cap + kTile - 1) / kTile;
    const int blocks = (int)std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
    if (M.fp8) k_mlp_forward<true><<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, check_halt, step);
    else k_mlp_forward<false><<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, check_halt, step);
}

}  // namespace adres

namespace adres {
namespace {
__global__ void k_mlp_convert(const float *__restrict__ params, __bf16 *__restrict__ w2, __bf16 *__restrict__ w2t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kHidden * kHidden) return;
    const __bf16 b = (__bf16)params[2 * kHidden + i];
    w2[i] = b;
    w2t[(i % kHidden) * kHidden + i / kHidden] = b;
}
}  // namespace

// FP8 variant: s_w = max |W2| / 448 and s_g = G / 448 with G = 1.01 max(0.2785,
// max_u |silu(b1_u)|, max_u |silu(W1_u + b1_u)|) / ln 2, a bound on |h1| / ln 2 for inputs
// x = r / rc in [0, 1] (silu is monotone above its minimum -0.27846); W2 / s_w rounded to
// E4M3 (nearest even), row-major, four values per word.  One workgroup.
__global__ __launch_bounds__(256) void k_mlp_fp8_prepare(const float *__restrict__ params, int *__restrict__ w2q,
                                                        float *__restrict__ scale)
{
    __shared__ float red_w[256], red_g[256];
    const float *W1 = params, *b1 = params + kHidden, *W2 = params + 2 * kHidden;
    float wm = 0.0f, gm = 0.0f;
    for (int i = threadIdx.x; i < kHidden * kHidden; i += 256) wm = fmaxf(wm, fabsf(W2[i]));
    if (threadIdx.x < kHidden) {
        const int u = threadIdx.x;
        const float z0 = b1[u], z1 = W1[u] + b1[u];
        gm = fmaxf(fabsf(z0 / (1.0f + expf(-z0))), fabsf(z1 / (1.0f + expf(-z1))));
    }
    red_w[threadIdx.x] = wm;
    red_g[threadIdx.x] = gm;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) {
            red_w[threadIdx.x] = fmaxf(red_w[threadIdx.x], red_w[threadIdx.x + h]);
            red_g[threadIdx.x] = fmaxf(red_g[threadIdx.x], red_g[threadIdx.x + h]);
        }
        __syncthreads();
    }
    const float s_w = red_w[0] > 0.0f ? red_w[0] / 448.0f : 1.0f;
    const float G = 1.01f * fmaxf(0.2785f, red_g[0]) / 0.6931471805599453f;
    const float s_g = G / 448.0f;
    const float inv_sw = 1.0f / s_w;
    for (int k = threadIdx.x; k < kHidden * kHidden / 4; k += 256) {
        const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(W2[4 * k] * inv_sw, W2[4 * k + 1] * inv_sw, 0, false);
        w2q[k] = __builtin_amdgcn_cvt_pk_fp8_f32(W2[4 * k + 2] * inv_sw, W2[4 * k + 3] * inv_sw, pk, true);
    }
    if (threadIdx.x == 0) {
        scale[0] = s_w * s_g;
        scale[1] = 1.0f / s_g;
        scale[2] = 1.0f / (s_w * s_g);
    }
}

void launch_mlp_fp8_prepare(hipStream_t s, const float *params, int *w2_fp8, float *scale)
{
    k_mlp_fp8_prepare<<<1, 256, 0, s>>>(params, w2_fp8, scale);
}

void launch_mlp_convert(hipStream_t s, const float *params, __bf16 *w2_bf16, __bf16 *w2t_bf16)
{
    k_mlp_convert<<<(kHidden * kHidden + 255) / 256, 256, 0, s>>>(params, w2_bf16, w2t_bf16);
}
}  // namespace adres
