// Learned CG pair force: inference of f(r) = s * taper(r) * [W3 . silu(W2 silu(W1 x + b1) + b2) + b3],
// x = r / rc, on gfx950 matrix cores.  It stands in for F^CG of Eq. (1) (Sec. 2.2:
// a force between centres of mass); below r_min the cubic CG table is used instead.
//
// One wavefront evaluates a tile of 32 pairs:
//   * layer 1 (rank one in x) in VALU: lane l computes, for pair l % 32, the 32 hidden
//     units 16 kb + 8 (l / 32) + j (kb = 0..3, j = 0..7), applies silu and writes them
//     as BF16 straight into the A operands of four MFMA K-blocks;
//   * layer 2 (32 x 64 x 64) on v_mfma_f32_32x32x16_bf16 with FP32 accumulation; W2
//     (row = output unit, BF16) is held in registers as the B operands for the whole
//     kernel (lane l: column l % 32 of N-block nb, K rows 8 (l / 32) .. +7);
//   * layer 3: lane l owns output unit 32 nb + l % 32 of rows 8 (v / 4) + 4 (l / 32) + v % 4,
//     multiplies silu(z2) by W3 and the 32 lanes of a half-wavefront add their
//     products with butterfly shuffles.
// Operand and result lane layouts were checked on the device with a known product.
#include <algorithm>

#include "adres_mlp.h"

namespace adres {
namespace {

constexpr int kTile = 32;
constexpr int kWaves = 4;
constexpr int kBlockM = 64 * kWaves;

__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

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
    __shared__ float sW1[kHidden], sB1[kHidden];
    for (int i = threadIdx.x; i < kHidden; i += kBlockM) {
        sW1[i] = M.w1[i];
        sB1[i] = M.b1[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    // B operands: W2 rows (output units) 32 nb + col, K columns 16 kb + 8 half .. +7
    bf16x8 Bop[2][4];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            Bop[nb][kb] = *reinterpret_cast<const bf16x8 *>(M.w2_bf16 + (32 * nb + col) * kHidden + 16 * kb + 8 * half);
    const float b2u[2] = {M.b2[col], M.b2[32 + col]};
    const float w3u[2] = {M.w3[col], M.w3[32 + col]};
    const float b3 = M.w3[kHidden], inv_rc = 1.0f / (float)M.rc, rcf = (float)M.rc, twf = (float)M.tw, sc = (float)M.scale;

    const int64_t n_tiles = (src.n + kTile - 1) / kTile;
    const int64_t wave_id = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * kWaves;
    for (int64_t tile = wave_id; tile < n_tiles; tile += n_waves) {
        const int64_t p = tile * kTile + col;
        const bool ok = p < src.n;
        const double r = ok ? pair_r(src, P, p) : M.rc;
        const float x = (float)r * inv_rc;
        bf16x8 A[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = 16 * kb + 8 * half + j;
                A[kb][j] = (__bf16)silu_f(fmaf(sW1[u], x, sB1[u]));
            }
        float part[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) part[v] = 0.0f;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = {};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kb], Bop[nb][kb], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) part[v] += w3u[nb] * silu_f(acc[v] + b2u[nb]);
        }
        // sum over the 32 output units held by the 32 lanes of this half-wavefront
#pragma unroll
        for (int v = 0; v < 16; ++v)
#pragma unroll
            for (int off = 1; off < 32; off <<= 1) part[v] += __shfl_xor(part[v], off, 32);
        // lane with col < 16 writes row 8 (col / 4) + 4 half + col % 4
        float y = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v)
            if (v == col) y = part[v];
        const int row = 8 * (col >> 2) + 4 * half + (col & 3);
        const double rr = __shfl(r, row, 64);
        if (col < 16) {
            const int64_t q = tile * kTile + row;
            if (q < src.n) {
                float f;
                if (rr < M.r_min && P.tab) {
                    double u = (rr - P.tab_lo) / P.tab_h;
                    if (rr < P.tab_lo) atomicOr(&ctrl->err, kErrTableRange);
                    double kf = floor(u);
                    kf = kf >= 0.0 ? kf : 0.0;
                    kf = kf > (double)(P.tab_n - 2) ? (double)(P.tab_n - 2) : kf;
                    const float t = (float)(u - kf);
                    const float4 c = P.tab[(int)kf];
                    f = ((c.w * t + c.z) * t + c.y) * t + c.x;
                } else if (rr >= M.rc) {
                    f = 0.0f;
                } else {
                    f = sc * taper_f((float)rr, rcf, twf) * (y + b3);
                }
                out[q] = f;
            }
        }
    }
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
