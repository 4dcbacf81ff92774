// Per-molecule streaming kernels: centres of mass and resolution weights
// (Sec. 2.2), gathers into / scatters out of the Morton-ordered state, and the
// velocity-Verlet kick-drift half step.  One thread per molecule; a molecule's
// sites are contiguous in each SoA row, so a wavefront touches 64 * s * 8 bytes
// of one row per access.
#include "adres_internal.h"

#include <climits>

namespace adres {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n, int per_block = kBlock) { return (int)((n + per_block - 1) / per_block); }

template <int SPM>
__device__ __forceinline__ void load_sites(const double *x, int64_t ns, int mol, double (&p)[SPM][3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < SPM; ++k) p[k][d] = x[d * ns + (int64_t)mol * SPM + k];
}

template <int SPM>
__device__ __forceinline__ void store_sites(double *x, int64_t ns, int mol, const double (&p)[SPM][3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < SPM; ++k) x[d * ns + (int64_t)mol * SPM + k] = p[k][d];
}

template <int SPM>
__device__ __forceinline__ bool all_finite(const double (&p)[SPM][3])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < SPM; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) ok = ok && isfinite(p[k][d]);
    return ok;
}

// Weight, stretch and displacement bookkeeping of one molecule at slot t.
template <int SPM>
__device__ __forceinline__ void finish_molecule(const DevParams &P, const double (&p)[SPM][3], int t,
                                                double *R, double *w, double *rho, const double *R_ref,
                                                Ctrl *ctrl, int halt_value)
{
    const int n = P.n_mol;
    double Rm[3], rh;
    mol_com<SPM>(P, p, Rm, rh);
    R[t] = Rm[0];
    R[n + t] = Rm[1];
    R[2 * n + t] = Rm[2];
    w[t] = res_weight(P, Rm);
    rho[t] = rh;
    if (SPM > 1 && rh > P.rho_max) atomicOr(&ctrl->err, kErrStretch);
    if (!all_finite<SPM>(p)) atomicOr(&ctrl->err, kErrNonFinite);
    if (R_ref) {
        double q0 = mi(Rm[0] - R_ref[t], P.box[0], P.half[0]);
        double q1 = mi(Rm[1] - R_ref[n + t], P.box[1], P.half[1]);
        double q2 = mi(Rm[2] - R_ref[2 * n + t], P.box[2], P.half[2]);
        if (dist2_exact(q0, q1, q2) > P.half_skin2) atomicMin(&ctrl->halt, halt_value);
    }
}

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_weights_caller(DevParams P, const double *__restrict__ x,
                                                           double *__restrict__ com, double *__restrict__ w,
                                                           Ctrl *ctrl)
{
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= P.n_mol) return;
    double p[SPM][3];
    load_sites<SPM>(x, P.n_sites, a, p);
    double R[3], rh;
    mol_com<SPM>(P, p, R, rh);
    com[a] = R[0];
    com[P.n_mol + a] = R[1];
    com[2 * P.n_mol + a] = R[2];
    w[a] = res_weight(P, R);
    if (SPM > 1 && rh > P.rho_max) atomicOr(&ctrl->err, kErrStretch);
    if (!all_finite<SPM>(p)) atomicOr(&ctrl->err, kErrNonFinite);
}

// Caller-order x (and v) -> Morton-ordered state through perm; centres of mass,
// weights; optional displacement check against R_ref (sets halt = 0).
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_gather(DevParams P, const double *__restrict__ xc,
                                                   const double *__restrict__ vc, StateBufs S,
                                                   const double *__restrict__ R_ref, Ctrl *ctrl)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    int a = S.perm[t];
    double p[SPM][3];
    load_sites<SPM>(xc, P.n_sites, a, p);
    store_sites<SPM>(S.x, P.n_sites, t, p);
    if (vc) {
        double q[SPM][3];
        load_sites<SPM>(vc, P.n_sites, a, q);
        store_sites<SPM>(S.v, P.n_sites, t, q);
    }
    finish_molecule<SPM>(P, p, t, S.R, S.w, S.rho, R_ref, ctrl, 0);
}

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_scatter_out(DevParams P, StateBufs S, double *__restrict__ xc,
                                                        double *__restrict__ vc, double *__restrict__ fc)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    int a = S.perm[t];
    double p[SPM][3];
    if (xc) {
        load_sites<SPM>(S.x, P.n_sites, t, p);
        store_sites<SPM>(xc, P.n_sites, a, p);
    }
    if (vc) {
        load_sites<SPM>(S.v, P.n_sites, t, p);
        store_sites<SPM>(vc, P.n_sites, a, p);
    }
    if (fc) {
        load_sites<SPM>(S.f, P.n_sites, t, p);
        store_sites<SPM>(fc, P.n_sites, a, p);
    }
}

// ---------------------------------------------------------------- Langevin noise
// Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
// SC'11), keyed by the seed, counter = (step, site, component block).
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Two standard normal deviates from two 32-bit words (Box-Muller).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &n0, double &n1)
{
    double u1 = ((double)a + 1.0) * (1.0 / 4294967296.0);   // (0, 1]
    double u2 = (double)b * (1.0 / 4294967296.0);
    double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    n0 = r * c;
    n1 = r * s;
}

// First half of a velocity-Verlet step on the Morton-ordered state:
//   v += F dt / 2m; x += v dt; fold; new centre of mass, weight, displacement check.
// With gamma > 0 the drift is split around an exact Ornstein-Uhlenbeck step
// (BAOAB splitting, Leimkuhler & Matthews 2013):
//   x += v dt/2;  v = c v + sqrt((1 - c^2) kT / m) N(0,1), c = exp(-gamma dt);  x += v dt/2.
// Skipped entirely when an earlier step of this chunk requested a list rebuild.
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_kick_drift(DevParams P, StateBufs S,
                                                       const double *__restrict__ R_ref, Ctrl *ctrl,
                                                       int step, double dt, double gamma, double kT,
                                                       uint64_t seed, uint64_t step_abs)
{
#pragma clang fp contract(off)
    if (step > ctrl->halt) return;
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    const int64_t ns = P.n_sites;
    double p[SPM][3];
    double c_ou = 0.0, s_ou[SPM];
    if (gamma > 0.0) {
        c_ou = exp(-gamma * dt);
#pragma unroll
        for (int k = 0; k < SPM; ++k) s_ou[k] = sqrt((1.0 - c_ou * c_ou) * kT / P.mass[k]);
    }
#pragma unroll
    for (int k = 0; k < SPM; ++k) {
        double g[3] = {0.0, 0.0, 0.0};
        if (gamma > 0.0) {
            int caller_site = S.perm[t] * SPM + k;
            U4 r = philox4x32_10(U4{(uint32_t)step_abs, (uint32_t)(step_abs >> 32), (uint32_t)caller_site, 0u},
                                 (uint32_t)seed, (uint32_t)(seed >> 32));
            double n3;
            box_muller(r.x, r.y, g[0], g[1]);
            box_muller(r.z, r.w, g[2], n3);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int64_t i = d * ns + (int64_t)t * SPM + k;
            double v = S.v[i] + S.f[i] * dt / (2.0 * P.mass[k]);
            double y;
            if (gamma > 0.0) {
                y = S.x[i] + v * (0.5 * dt);
                v = c_ou * v + s_ou[k] * g[d];
                y = fold(y + v * (0.5 * dt), P.box[d]);
            } else {
                y = fold(S.x[i] + v * dt, P.box[d]);
            }
            S.v[i] = v;
            S.x[i] = y;
            p[k][d] = y;
        }
    }
    finish_molecule<SPM>(P, p, t, S.R, S.w, S.rho, R_ref, ctrl, step);
}

__global__ void k_reset_halt(Ctrl *ctrl)
{
    if (threadIdx.x == 0) ctrl->halt = INT_MAX;
}

}  // namespace

#define ADRES_SPM_DISPATCH(spm, CALL) \
    switch (spm) {                    \
    case 1: { constexpr int S_ = 1; CALL; } break; \
    case 2: { constexpr int S_ = 2; CALL; } break; \
    case 3: { constexpr int S_ = 3; CALL; } break; \
    default: { constexpr int S_ = 4; CALL; } break; \
    }

void launch_weights_caller(hipStream_t s, const DevParams &P, const double *x, double *com, double *w,
                           Ctrl *ctrl)
{
    ADRES_SPM_DISPATCH(P.spm, (k_weights_caller<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x, com, w, ctrl)));
}

void launch_gather(hipStream_t s, const DevParams &P, const double *x_caller, const double *v_caller,
                   const StateBufs &S, const double *R_ref, Ctrl *ctrl)
{
    ADRES_SPM_DISPATCH(P.spm, (k_gather<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x_caller, v_caller, S, R_ref, ctrl)));
}

void launch_scatter_out(hipStream_t s, const DevParams &P, const StateBufs &S, double *x_caller,
                        double *v_caller, double *f_caller)
{
    ADRES_SPM_DISPATCH(P.spm, (k_scatter_out<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, S, x_caller, v_caller, f_caller)));
}

void launch_kick_drift(hipStream_t s, const DevParams &P, const StateBufs &S, const double *R_ref,
                       Ctrl *ctrl, int step, double dt, double gamma, double kT, uint64_t seed,
                       uint64_t step_abs)
{
    ADRES_SPM_DISPATCH(P.spm, (k_kick_drift<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, S, R_ref, ctrl, step, dt, gamma, kT, seed, step_abs)));
}

void launch_reset_halt(hipStream_t s, Ctrl *ctrl) { k_reset_halt<<<1, 64, 0, s>>>(ctrl); }

}  // namespace adres
