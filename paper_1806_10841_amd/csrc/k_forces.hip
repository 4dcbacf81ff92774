// Force-interpolation kernel, Eq. (1) of Sec. 2.2:
//   F_ab = ww F^AT_ab + (1 - ww) F^CG_ab,  ww = w_a w_b,
// with F^AT the sum of atom-atom WCA forces between the two molecules and F^CG a
// force between their centres of mass, shared among a molecule's sites by mass
// fraction; plus the bonded terms, which are not interpolated (Sec. 2.2, last
// paragraph).
//
// Work mapping (gfx950, wave64): four lanes per home molecule.  Lane q of the
// group walks neighbour-list entries q, q+4, q+8, ... of its molecule (full list:
// every pair is seen from both sides, so no atomics and a fixed summation order)
// and accumulates, in FP64, the force on every site of the home molecule.  The
// four partial sums are then combined with two butterfly shuffles, after which
// lane q owns site q: it adds the bonded force, writes F and optionally applies
// the closing half-kick of velocity Verlet.  A 256-thread workgroup covers 64
// consecutive Morton slots, i.e. a compact cluster of cells, so neighbour gathers
// hit the same cache lines across the workgroup.
//
// Pair arithmetic in PT (double or float).  In the float variant the displacement
// is formed in FP64 (minimum image of FP64 coordinates) and rounded once to FP32;
// everything after that is FP32, and the accumulation is FP64.  Cutoff decisions
// of the CG part use the FP64 centre distance.  An atom tile is skipped when the
// centres are farther apart than rc_at + rho_a + rho_b (rho: largest site distance
// from the centre), which no interacting atom pair can be (triangle inequality).
#include "adres_internal.h"

namespace adres {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 4;   // lanes per home molecule

template <typename PT>
__device__ __forceinline__ PT wca_f_over_r(PT r2, PT sig2, PT eps, PT &u, bool want_u)
{
    PT inv = PT(1) / r2;
    PT s = sig2 * inv;
    PT s6 = s * s * s;
    if (want_u) u = PT(4) * eps * s6 * (s6 - PT(1)) + eps;
    return PT(24) * eps * s6 * (PT(2) * s6 - PT(1)) * inv;
}

// Cubic table of the CG force magnitude; interval and fraction located in FP64.
template <typename PT>
__device__ __forceinline__ PT table_f(const DevParams &P, double r, Ctrl *ctrl)
{
    double u = (r - P.tab_lo) / P.tab_h;
    if (r < P.tab_lo) atomicOr(&ctrl->err, kErrTableRange);
    double kf = floor(u);
    kf = kf >= 0.0 ? kf : 0.0;   // also maps NaN to interval 0
    kf = kf > (double)(P.tab_n - 2) ? (double)(P.tab_n - 2) : kf;
    PT t = (PT)(u - kf);
    float4 c = P.tab[(int)kf];
    return ((PT(c.w) * t + PT(c.z)) * t + PT(c.y)) * t + PT(c.x);
}

// Closing half-kick of velocity Verlet, v += F dt / (2m), in the oracle's operation order.
__device__ __forceinline__ void half_kick(double *v, int64_t ns, int64_t site, const double F[3], double dt,
                                          double m)
{
#pragma clang fp contract(off)
    for (int d = 0; d < 3; ++d) v[d * ns + site] = v[d * ns + site] + F[d] * dt / (2.0 * m);
}

template <int SPM, typename PT, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_forces(ForceArgs a)
{
    const DevParams &P = a.P;
    if (a.check_halt && a.step >= a.ctrl->halt) return;
    const int n = P.n_mol;
    const int64_t ns = P.n_sites;
    const int gid = blockIdx.x * kBlock + threadIdx.x;
    const int t = gid / kLanes, q = gid % kLanes;
    const bool valid = t < n;
    const int tt = valid ? t : n - 1;

    double xi[SPM][3];
#pragma unroll
    for (int i = 0; i < SPM; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) xi[i][d] = a.x[d * ns + (int64_t)tt * SPM + i];
    const double Ra0 = a.R[tt], Ra1 = a.R[n + tt], Ra2 = a.R[2 * n + tt];
    const double wa = a.w[tt], rha = a.rho[tt];

    double acc[SPM][3];
#pragma unroll
    for (int i = 0; i < SPM; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
    double uat = 0.0, ucg = 0.0, ubond = 0.0;

    const PT sig2A = (PT)P.sig2_at, epsA = (PT)P.eps_at, rcA2 = (PT)P.rcA2;
    const PT sig2C = (PT)P.sig2_cg, epsC = (PT)P.eps_cg;
    const int cnt = valid ? min(a.cnt[tt], a.cap) : 0;

    for (int k = q; k < cnt; k += kLanes) {
        const int u = a.nbr[(int64_t)k * n + tt];
        const double ww = wa * a.w[u];
        const double D0 = mi(Ra0 - a.R[u], P.box[0], P.half[0]);
        const double D1 = mi(Ra1 - a.R[n + u], P.box[1], P.half[1]);
        const double D2 = mi(Ra2 - a.R[2 * n + u], P.box[2], P.half[2]);
        const double r2c = dist2_exact(D0, D1, D2);
        if (ww > 0.0) {
            const double bound = P.rc_at + rha + a.rho[u] + 1e-9;
            if (r2c < bound * bound) {
                const PT pww = (PT)ww;
#pragma unroll
                for (int j = 0; j < SPM; ++j) {
                    const double xj0 = a.x[(int64_t)u * SPM + j];
                    const double xj1 = a.x[ns + (int64_t)u * SPM + j];
                    const double xj2 = a.x[2 * ns + (int64_t)u * SPM + j];
#pragma unroll
                    for (int i = 0; i < SPM; ++i) {
                        const PT dx = (PT)mi(xi[i][0] - xj0, P.box[0], P.half[0]);
                        const PT dy = (PT)mi(xi[i][1] - xj1, P.box[1], P.half[1]);
                        const PT dz = (PT)mi(xi[i][2] - xj2, P.box[2], P.half[2]);
                        const PT r2 = (dx * dx + dy * dy) + dz * dz;
                        if (r2 < rcA2) {
                            PT uu = PT(0);
                            const PT c = pww * wca_f_over_r<PT>(r2, sig2A, epsA, uu, ENERGY);
                            acc[i][0] += (double)(c * dx);
                            acc[i][1] += (double)(c * dy);
                            acc[i][2] += (double)(c * dz);
                            if (ENERGY) uat += 0.5 * ww * (double)uu;
                        }
                    }
                }
            }
        }
        if (ww < 1.0 && r2c < P.rcC2) {
            PT uu = PT(0);
            PT fr;
            if (P.cg_kind == ADRES_CG_WCA) {
                fr = wca_f_over_r<PT>((PT)r2c, sig2C, epsC, uu, ENERGY);
            } else {
                const double r = sqrt(r2c);
                fr = table_f<PT>(P, r, a.ctrl) / (PT)r;
            }
            const PT sc = (PT)(1.0 - ww) * fr;
            const PT d0 = (PT)D0, d1 = (PT)D1, d2 = (PT)D2;
#pragma unroll
            for (int i = 0; i < SPM; ++i) {
                const PT s = (PT)P.mfrac[i] * sc;
                acc[i][0] += (double)(s * d0);
                acc[i][1] += (double)(s * d1);
                acc[i][2] += (double)(s * d2);
            }
            if (ENERGY) ucg += 0.5 * (1.0 - ww) * (double)uu;
        }
    }

    // combine the four lanes' partial sums (every lane ends with the same bits)
#pragma unroll
    for (int i = 0; i < SPM; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = acc[i][d];
            v += __shfl_xor(v, 1, kLanes);
            v += __shfl_xor(v, 2, kLanes);
            acc[i][d] = v;
        }

    double F[3] = {0.0, 0.0, 0.0};
    double xq[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < SPM; ++i)
        if (i == q) {
            F[0] = acc[i][0]; F[1] = acc[i][1]; F[2] = acc[i][2];
            xq[0] = xi[i][0]; xq[1] = xi[i][1]; xq[2] = xi[i][2];
        }

    if (valid && q < SPM) {
        if (P.bond_kind == ADRES_BOND_HARMONIC) {
#pragma unroll
            for (int k = 0; k < SPM; ++k) {
                if (k == q) continue;
                const double d0 = mi(xq[0] - xi[k][0], P.box[0], P.half[0]);
                const double d1 = mi(xq[1] - xi[k][1], P.box[1], P.half[1]);
                const double d2 = mi(xq[2] - xi[k][2], P.box[2], P.half[2]);
                const double r = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
                const double fr = -P.k_bond * (r - P.r0_bond) / r;
                F[0] += fr * d0; F[1] += fr * d1; F[2] += fr * d2;
                if (ENERGY && k > q) ubond += 0.5 * P.k_bond * (r - P.r0_bond) * (r - P.r0_bond);
            }
        } else if (P.bond_kind == ADRES_BOND_FENE) {
            const int ca = a.perm[t];
            const int chain = ca / P.chain_len;
            for (int side = -1; side <= 1; side += 2) {
                const int cb = ca + side;
                if (cb < 0 || cb >= n || cb / P.chain_len != chain) continue;
                const int ub = a.inv_perm[cb];
                const double d0 = mi(xq[0] - a.x[(int64_t)ub * SPM], P.box[0], P.half[0]);
                const double d1 = mi(xq[1] - a.x[ns + (int64_t)ub * SPM], P.box[1], P.half[1]);
                const double d2 = mi(xq[2] - a.x[2 * ns + (int64_t)ub * SPM], P.box[2], P.half[2]);
                const double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
                if (r2 >= P.R02) {
                    atomicOr(&a.ctrl->err, kErrFene);
                    continue;
                }
                const double fr = -P.k_bond / (1.0 - r2 / P.R02);
                F[0] += fr * d0; F[1] += fr * d1; F[2] += fr * d2;
                if (ENERGY) ubond += 0.5 * (-0.5 * P.k_bond * P.R02 * log(1.0 - r2 / P.R02));
            }
        }
        if (!(isfinite(F[0]) && isfinite(F[1]) && isfinite(F[2]))) atomicOr(&a.ctrl->err, kErrNonFinite);
        const int64_t site = (int64_t)(a.out_perm ? a.out_perm[t] : t) * SPM + q;
        a.f[site] = F[0];
        a.f[ns + site] = F[1];
        a.f[2 * ns + site] = F[2];
        if (a.v) half_kick(a.v, ns, (int64_t)t * SPM + q, F, a.dt, P.mass[q]);
    }

    if (ENERGY) {
        // block reduction in a fixed order: wavefront butterflies, then 4 waves in LDS
        __shared__ double red[kBlock / 64][3];
        double e[3] = {uat, ucg, ubond};
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) e[c] += __shfl_xor(e[c], off, 64);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) {
            red[wave][0] = e[0]; red[wave][1] = e[1]; red[wave][2] = e[2];
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
            a.epart[blockIdx.x * 3 + threadIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(256) void k_energy_reduce(const double *__restrict__ epart, int n_blocks,
                                                       double *__restrict__ energy)
{
    __shared__ double red[256][3];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n_blocks; b += 256)
        for (int c = 0; c < 3; ++c) s[c] += epart[b * 3 + c];
    for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = s[c];
    __syncthreads();
    for (int half = 128; half >= 1; half >>= 1) {
        if (threadIdx.x < half)
            for (int c = 0; c < 3; ++c) red[threadIdx.x][c] += red[threadIdx.x + half][c];
        __syncthreads();
    }
    if (threadIdx.x < 3) energy[threadIdx.x] = red[0][threadIdx.x];
    if (threadIdx.x == 3) energy[3] = 0.0;
}

template <int SPM, typename PT>
void dispatch_energy(hipStream_t s, const ForceArgs &a, int blocks)
{
    if (a.epart)
        k_forces<SPM, PT, true><<<blocks, kBlock, 0, s>>>(a);
    else
        k_forces<SPM, PT, false><<<blocks, kBlock, 0, s>>>(a);
}

template <typename PT>
void dispatch_spm(hipStream_t s, const ForceArgs &a, int blocks)
{
    switch (a.P.spm) {
    case 1: dispatch_energy<1, PT>(s, a, blocks); break;
    case 2: dispatch_energy<2, PT>(s, a, blocks); break;
    case 3: dispatch_energy<3, PT>(s, a, blocks); break;
    default: dispatch_energy<4, PT>(s, a, blocks); break;
    }
}

}  // namespace

int launch_forces(hipStream_t s, const ForceArgs &a, int pair_precision)
{
    const int blocks = (int)(((int64_t)a.P.n_mol * kLanes + kBlock - 1) / kBlock);
    if (pair_precision == 32)
        dispatch_spm<float>(s, a, blocks);
    else
        dispatch_spm<double>(s, a, blocks);
    return blocks;
}

void launch_energy_reduce(hipStream_t s, const double *epart, int n_blocks, double *energy)
{
    k_energy_reduce<<<1, 256, 0, s>>>(epart, n_blocks, energy);
}

}  // namespace adres
