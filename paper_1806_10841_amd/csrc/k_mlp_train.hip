// Force-matching training of the learned CG force on gfx950 matrix cores.
//
// For a frame of CG sites with centres R_I and mapped forces F^map_I (the summed
// atomistic non-bonded forces of molecule I; multiscale coarse-graining / force
// matching, Izvekov & Voth 2005), the prediction is F_I = sum_J f(r_IJ) R_hat_IJ
// (the CG part of Eq. (1) with w = 0), the loss chi2 = c sum_I |F_I - F^map_I|^2
// with c = 1 / (3 N_frames N), and for an unordered pair the loss gradient w.r.t.
// f(r_IJ) is g_IJ = 2 c (e_I - e_J) . R_hat_IJ, e = F - F^map.
//
// k_mlp_backward takes tiles of 32 pairs per wavefront (the layout of the
// inference kernel), recomputes the forward pass and back-propagates:
//   dy_p = g_p s taper(r_p);  dW3 += dy h2;  dz2 = dy W3 silu'(z2);
//   dW2 += dz2^T h1      (64 x 64 x 32 pairs: v_mfma_f32_32x32x16_bf16, accumulated in
//                         registers over all the wave's tiles);
//   dh1  = dz2 W2        (32 x 64 x 64: v_mfma_f32_32x32x16_bf16);
//   dz1 = dh1 silu'(z1); dW1 += dz1 x;  db1 += dz1.
// h1 and dz2 are staged per wave in LDS to move between the MFMA result layout
// (lane = column) and the operand layouts (lane = row, 8 K values).  Each wave
// writes its partial gradient; k_grad_reduce sums the waves in a fixed order, so
// gradients are bit-reproducible.  k_adam applies Adam (Kingma & Ba 2015).
#include <algorithm>

#include "adres_mlp.h"

namespace adres {
namespace {

constexpr int kTile = 32;
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kPad = 8;   // bf16 padding per LDS row (breaks power-of-two strides)

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float taper_f(float r, float rc, float tw)
{
    float u = (r - (rc - tw)) / tw;
    if (u <= 0.0f) return 1.0f;
    if (u >= 1.0f) return 0.0f;
    float c = __cosf(1.5707963267948966f * u);
    return c * c;
}

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// e = F - F^map per Morton slot (F in Morton order, F^map in caller order), and the
// per-block sum of |e|^2.
__global__ __launch_bounds__(256) void k_fm_residual(int n, const int *__restrict__ perm, const double *__restrict__ F,
                                                     const double *__restrict__ fmap, double *__restrict__ e,
                                                     double *__restrict__ part)
{
    __shared__ double red[256];
    const int t = blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (t < n) {
        const int a = perm[t];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = F[(int64_t)d * n + t] - fmap[(int64_t)d * n + a];
            e[(int64_t)d * n + t] = v;
            s += v * v;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss += c * sum(part), one workgroup, fixed order
__global__ __launch_bounds__(256) void k_loss_accumulate(const double *__restrict__ part, int n_part, double c,
                                                         double *__restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss += c * red[0];
}

__global__ __launch_bounds__(kThreads) void k_mlp_backward(MlpDev M, DevParams P, const int2 *__restrict__ pairs,
                                                          const int *__restrict__ n_dev, const double4 *__restrict__ Rw,
                                                          const double *__restrict__ e, double c2,
                                                          float *__restrict__ gpart)
{
    __shared__ float sW1[kHidden], sB1[kHidden];
    __shared__ __attribute__((aligned(16))) __bf16 h1s[kWaves][kTile][kHidden + kPad];
    __shared__ __attribute__((aligned(16))) __bf16 dz2s[kWaves][kTile][kHidden + kPad];
    for (int i = threadIdx.x; i < kHidden; i += kThreads) {
        sW1[i] = M.w1[i];
        sB1[i] = M.b1[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31, wave = threadIdx.x >> 6;
    const int n = P.n_mol;

    // B operands of the forward product (B[k][n] = W2[n][k]) and of dh1 = dz2 W2 (B[n][k] = W2[n][k])
    bf16x8 Bf[2][4], Bb[2][4];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            Bf[nb][kb] = *reinterpret_cast<const bf16x8 *>(M.w2_bf16 + (32 * nb + col) * kHidden + 16 * kb + 8 * half);
            Bb[nb][kb] = *reinterpret_cast<const bf16x8 *>(M.w2t_bf16 + (32 * nb + col) * kHidden + 16 * kb + 8 * half);
        }
    float w1u[2], b1u[2], b2u[2], w3u[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        w1u[nb] = M.w1[32 * nb + col];
        b1u[nb] = M.b1[32 * nb + col];
        b2u[nb] = M.b2[32 * nb + col];
        w3u[nb] = M.w3[32 * nb + col];
    }
    const float inv_rc = 1.0f / (float)M.rc, rcf = (float)M.rc, twf = (float)M.tw, sc = (float)M.scale;

    float gW1[2] = {0.f, 0.f}, gB1[2] = {0.f, 0.f}, gB2[2] = {0.f, 0.f}, gW3[2] = {0.f, 0.f}, gB3 = 0.f;
    floatx16 accW2[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) accW2[mb][nb] = floatx16{};

    const int64_t n_pairs = *n_dev;
    const int64_t n_tiles = (n_pairs + kTile - 1) / kTile;
    const int64_t wave_id = (int64_t)blockIdx.x * kWaves + wave;
    const int64_t n_waves = (int64_t)gridDim.x * kWaves;
    for (int64_t tile = wave_id; tile < n_tiles; tile += n_waves) {
        const int64_t p = tile * kTile + col;
        float x = 0.0f, dy = 0.0f;
        if (p < n_pairs) {
            const int2 tu = pairs[p];
            const double4 a = Rw[tu.x], b = Rw[tu.y];
            const double d0 = mi(a.x - b.x, P.box[0], P.inv_box[0]);
            const double d1 = mi(a.y - b.y, P.box[1], P.inv_box[1]);
            const double d2 = mi(a.z - b.z, P.box[2], P.inv_box[2]);
            const double r = sqrt(dist2_exact(d0, d1, d2));
            x = (float)r * inv_rc;
            if (r < M.rc && r >= M.r_min) {
                const double g = c2 * ((e[tu.x] - e[tu.y]) * d0 + (e[n + tu.x] - e[n + tu.y]) * d1 +
                                       (e[2 * n + tu.x] - e[2 * n + tu.y]) * d2) / r;
                dy = (float)g * sc * taper_f((float)r, rcf, twf);
            }
        }
        if (half == 0) gB3 += dy;

        // forward layer 1 into A operands and LDS (row = pair, column = unit)
        bf16x8 A[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = 16 * kb + 8 * half + j;
                const float z = fmaf(sW1[u], x, sB1[u]);
                A[kb][j] = (__bf16)(z * sigm(z));
            }
            *reinterpret_cast<bf16x8 *>(&h1s[wave][col][16 * kb + 8 * half]) = A[kb];
        }
        // rows of this lane in the 32x32 result layout, and their dy and x
        float dyr[16], xr[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = 8 * (v >> 2) + 4 * half + (v & 3);
            dyr[v] = __shfl(dy, row, 64);
            xr[v] = __shfl(x, row, 64);
        }
        // forward layer 2, layer-3 gradients, dz2 into LDS (row = pair, column = unit)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 acc = {};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kb], Bf[nb][kb], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 8 * (v >> 2) + 4 * half + (v & 3);
                const float z2 = acc[v] + b2u[nb];
                const float s = sigm(z2);
                gW3[nb] += dyr[v] * (z2 * s);
                const float dz2 = dyr[v] * w3u[nb] * (s * (1.0f + z2 * (1.0f - s)));
                gB2[nb] += dz2;
                dz2s[wave][row][32 * nb + col] = (__bf16)dz2;
            }
        }
        wave_lds_sync();
        // dW2[n][k] += sum_pairs dz2[pair][n] h1[pair][k]   (rows n: A = dz2^T, cols k: B = h1)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            bf16x8 At[2], Bt[2];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int pr = 16 * kb + 8 * half + j;
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    At[mb][j] = dz2s[wave][pr][32 * mb + col];
                    Bt[mb][j] = h1s[wave][pr][32 * mb + col];
                }
            }
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    accW2[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(At[mb], Bt[nb], accW2[mb][nb], 0, 0, 0);
        }
        // dh1[pair][k] = sum_n dz2[pair][n] W2[n][k]; dz1 = dh1 silu'(z1)
        bf16x8 Ad[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) Ad[kb] = *reinterpret_cast<const bf16x8 *>(&dz2s[wave][col][16 * kb + 8 * half]);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            floatx16 dh = {};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) dh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ad[kb], Bb[nb][kb], dh, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float z1 = fmaf(w1u[nb], xr[v], b1u[nb]);
                const float s = sigm(z1);
                const float dz1 = dh[v] * (s * (1.0f + z1 * (1.0f - s)));
                gW1[nb] += dz1 * xr[v];
                gB1[nb] += dz1;
            }
        }
        wave_lds_sync();   // LDS tiles are rewritten by the next tile
    }

    // per-wave partial gradient: per-unit sums over the two half-wavefronts
    float *g = gpart + wave_id * kMlpParams;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const float a1 = gW1[nb] + __shfl_xor(gW1[nb], 32, 64);
        const float a2 = gB1[nb] + __shfl_xor(gB1[nb], 32, 64);
        const float a3 = gB2[nb] + __shfl_xor(gB2[nb], 32, 64);
        const float a4 = gW3[nb] + __shfl_xor(gW3[nb], 32, 64);
        if (half == 0) {
            const int u = 32 * nb + col;
            g[u] = a1;
            g[kHidden + u] = a2;
            g[2 * kHidden + kHidden * kHidden + u] = a3;
            g[3 * kHidden + kHidden * kHidden + u] = a4;
        }
    }
    float b3s = gB3;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) b3s += __shfl_xor(b3s, off, 64);
    if (lane == 0) g[kMlpParams - 1] = b3s;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 32 * mb + 8 * (v >> 2) + 4 * half + (v & 3);   // output unit n
                const int cc = 32 * nb + col;                                  // input unit k
                g[2 * kHidden + row * kHidden + cc] = accW2[mb][nb][v];
            }
}

// grad[i] += sum over waves of gpart[w][i] (FP64) in a fixed order: chunks of
// kReduceChunk consecutive waves are summed in wave order (k_grad_chunks, one thread per
// parameter and chunk), then the chunk sums in chunk order (k_grad_finish).
constexpr int kReduceChunk = 32;

__global__ __launch_bounds__(256) void k_grad_chunks(const float *__restrict__ gpart, int n_waves,
                                                     double *__restrict__ gred)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    const int w0 = blockIdx.y * kReduceChunk;
    const int w1 = min(w0 + kReduceChunk, n_waves);
    double s = 0.0;
    for (int w = w0; w < w1; ++w) s += (double)gpart[(int64_t)w * kMlpParams + i];
    gred[(int64_t)blockIdx.y * kMlpParams + i] = s;
}

__global__ __launch_bounds__(256) void k_grad_finish(const double *__restrict__ gred, int n_chunks,
                                                     double *__restrict__ grad)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += gred[(int64_t)c * kMlpParams + i];
    grad[i] += s;
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ a, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters; bias corrections from the host.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
                                              const double *__restrict__ grad, float lr, float b1, float b2,
                                              float bc1, float bc2, float eps)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    const float g = (float)grad[i];
    const float mi_ = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi_;
    v[i] = vi;
    params[i] -= lr * (mi_ / bc1) / (sqrtf(vi / bc2) + eps);
}

constexpr int kBackwardBlocks = 256;

}  // namespace

int mlp_backward_waves() { return kBackwardBlocks * kWaves; }
int mlp_reduce_chunks() { return (kBackwardBlocks * kWaves + kReduceChunk - 1) / kReduceChunk; }

void launch_fm_residual(hipStream_t s, int n, const int *perm, const double *F, const double *fmap, double *e,
                        double *part, int *n_part)
{
    *n_part = (n + 255) / 256;
    k_fm_residual<<<*n_part, 256, 0, s>>>(n, perm, F, fmap, e, part);
}

void launch_loss_accumulate(hipStream_t s, const double *part, int n_part, double c, double *loss)
{
    k_loss_accumulate<<<1, 256, 0, s>>>(part, n_part, c, loss);
}

void launch_mlp_backward(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs, const int *n_dev,
                         const double4 *Rw, const double *e, double c2, float *gpart, double *gred, double *grad)
{
    k_mlp_backward<<<kBackwardBlocks, kThreads, 0, s>>>(M, P, pairs, n_dev, Rw, e, c2, gpart);
    const int n_waves = kBackwardBlocks * kWaves;
    const dim3 grid((kMlpParams + 255) / 256, mlp_reduce_chunks());
    k_grad_chunks<<<grid, 256, 0, s>>>(gpart, n_waves, gred);
    k_grad_finish<<<(kMlpParams + 255) / 256, 256, 0, s>>>(gred, mlp_reduce_chunks(), grad);
}

void launch_zero(hipStream_t s, double *a, int n) { k_fill_zero<<<(n + 255) / 256, 256, 0, s>>>(a, n); }

void launch_adam(hipStream_t s, float *params, float *m, float *v, const double *grad, double lr, double b1,
                 double b2, double bc1, double bc2, double eps)
{
    k_adam<<<(kMlpParams + 255) / 256, 256, 0, s>>>(params, m, v, grad, (float)lr, (float)b1, (float)b2, (float)bc1,
                                                   (float)bc2, (float)eps);
}

}  // namespace adres
