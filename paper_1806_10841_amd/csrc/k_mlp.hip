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
    int64_t n;              // pair count, or read from n_dev when that is non-null
    const int *n_dev;
};

__device__ __forceinline__ double pair_r(const PairSource &src, const DevParams &P, int64_t p)
{
    if (src.r) return src.r[p];
    const int2 tu = src.pairs[p];
    const double4 a = src.Rw[tu.x], b = src.Rw[tu.y];
    const double d0 = mi(a.x - b.x, P.box[0], P.half[0]);
    const double d1 = mi(a.y - b.y, P.box[1], P.half[1]);
    const double d2 = mi(a.z - b.z, P.box[2], P.half[2]);
    return sqrt(dist2_exact(d0, d1, d2));
}

__global__ __launch_bounds__(kBlockM) void k_mlp_forward(MlpDev M, DevParams P, PairSource src, float *__restrict__ out,
                                                        Ctrl *ctrl, int check_halt, int step)
{
    if (check_halt && step > ctrl->halt) return;
    if (src.n_dev) src.n = *src.n_dev;
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
    // A operands: W2 rows (output units) 32 mb + col, K columns 16 kb + 8 half .. +7
    bf16x8 Wop[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            Wop[mb][kb] = *reinterpret_cast<const bf16x8 *>(M.w2_bf16 + (32 * mb + col) * kHidden + 16 * kb + 8 * half);
    // -log2e b2 of the output units of this lane's result rows (32 mb + 8 (v / 4) + 4 half
    // + v % 4): the accumulator's initial value
    floatx16 c2[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) c2[mb][v] = -kLog2e * M.b2[32 * mb + 8 * (v >> 2) + 4 * half + (v & 3)];
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
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = 16 * kb + 8 * half + j;
                const float t = fmaf(sW1[u], x, sB1[u]);
                H[kb][j] = (__bf16)(t * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)));
            }
        float y = 0.0f;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            floatx16 acc = c2[mb];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wop[mb][kb], H[kb], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float t = acc[v];
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
    k_mlp_forward<<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, 0, 0);
}

void launch_mlp_forward_pairs(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs,
                              const double4 *Rw, float *f, const int *n_dev, int64_t n_cap, Ctrl *ctrl,
                              int check_halt, int step)
{
    PairSource src{nullptr, pairs, Rw, 0, n_dev};
    const int64_t tiles = (n_cap + kTile - 1) / kTile;
    const int blocks = (int)std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
    k_mlp_forward<<<std::max(blocks, 1), kBlockM, 0, s>>>(M, P, src, f, ctrl, check_halt, step);
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

void launch_mlp_convert(hipStream_t s, const float *params, __bf16 *w2_bf16, __bf16 *w2t_bf16)
{
    k_mlp_convert<<<(kHidden * kHidden + 255) / 256, 256, 0, s>>>(params, w2_bf16, w2t_bf16);
}
}  // namespace adres
