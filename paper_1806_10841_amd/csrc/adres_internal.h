// Internal definitions of libadres: parameter block passed to kernels, device
// helpers and host-side launch wrappers.  gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stddef.h>
#include <stdint.h>

#include "adres.h"

namespace adres {

constexpr int kMaxSites = ADRES_MAX_SITES;

// Bits of the device error word (latched until read by a synchronising call).
enum : int {
    kErrStretch = 1,
    kErrFene = 2,
    kErrTableRange = 4,
    kErrNonFinite = 8,
};

// Device control block: step-halt index for speculative step chunks, error bits,
// neighbour-list overflow.
struct Ctrl {
    int halt;       // first step (within the current chunk) that requested a list rebuild
    int err;        // kErr* bits
    int overflow;   // bit 0: a neighbour-list row longer than its capacity; bit 1: a tile's
                    // neighbour halo larger than its capacity
    int max_count;  // longest neighbour-list row seen by the last build
    int max_halo;   // largest tile halo seen by the last halo build (on overflow)
    // set by the publication that ends a step chunk: go = a drift asked for a rebuild (the
    // rebuild enqueued behind the chunk runs; else its kernels return at once); fix = the
    // positions sit in the other buffer than the one the host assumed, because an odd
    // number of the chunk's drifts did not run (the rebuild's kernels then exchange the two
    // position buffers; a guarded kernel finds fix right after go)
    int go, fix;
};
static_assert(offsetof(Ctrl, fix) == offsetof(Ctrl, go) + sizeof(int), "fix follows go");

// Copy of the control block in host-mapped pinned memory, published after the work it
// reports on (by a one-thread kernel, or by the first kernel of a rebuild: ChainHead); the
// host polls it instead of synchronising the stream.  Each word holds the publication's
// sequence number (high half) with one field (low half) and is written with one 8-byte
// store, so that the host takes the fields once every word carries the sequence number it
// waits for: no fence orders the stores.
enum CtrlPubField : int { kPubHalt, kPubErr, kPubOverflow, kPubMaxCount, kPubMaxHalo, kPubFields };
struct CtrlPub {
    unsigned long long w[8];
};

// The publication of a step chunk, taken by the first kernel of the guarded rebuild that
// is enqueued behind the chunk (one launch less per chunk).  ctrl == nullptr: none.
struct ChainHead {
    Ctrl *ctrl;
    CtrlPub *pub;
    unsigned seq;
    int len_drift;   // the chunk's drifting kernels
};

// In that first kernel: every workgroup derives go and fix from the halt index (which no
// kernel of the rebuild writes before the next one clears it); workgroup 0 publishes the
// fields and stores go and fix for the later kernels of the rebuild.  Without a head, go
// and fix are read from where the publication stored them (go == nullptr: an unguarded
// launch).  Returns go.
__device__ __forceinline__ bool chain_go(const ChainHead &head, const int *go, bool &fix)
{
    if (head.ctrl) {
        Ctrl *c = head.ctrl;
        const int h = c->halt;
        // the chunk's drifts that ran: all, none (a list overflow stopped the chunk), or up
        // to and including the one that asked for the rebuild
        const int ran = h == INT_MAX ? head.len_drift : (h < 0 ? 0 : min(h + 1, head.len_drift));
        const int g = (h >= 0 && h != INT_MAX) ? 1 : 0;
        const int f = (head.len_drift - ran) & 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int v[kPubFields] = {h, c->err, c->overflow, c->max_count, c->max_halo};
#pragma unroll
            for (int i = 0; i < kPubFields; ++i)
                __hip_atomic_store(&head.pub->w[i], ((unsigned long long)head.seq << 32) | (unsigned)v[i],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            c->go = g;
            c->fix = f;
        }
        fix = f != 0;
        return g != 0;
    }
    fix = go && go[1] != 0;
    return !go || go[0] != 0;
}

// Parameters in the form the kernels use (passed by value).
struct DevParams {
    int n_mol, spm;
    int64_t n_sites;
    double box[3], half[3], inv_box[3];
    double mass[kMaxSites], mfrac[kMaxSites], inv_2m[kMaxSites], M;
    double inv_M;    // 1 / M, exact when M is a power of two (then M_pow2 = 1)
    int M_pow2;
    int region;
    double center[3], d_at, d_hy, d_end;
    double eps_at, sig2_at, rcA2, rc_at;
    double eps_cg, sig2_cg, rcC2;
    int cg_kind, bond_kind;
    int scheme;      // ADRES_SCHEME_*
    double k_bond, r0_bond, R02;
    int chain_len;
    // the list reach assumes every site within rho_max of its centre and leaves at least
    // r_skin/2 per molecule for motion; a site farther out spends part of that budget
    // (list_stale), up to rho_lim = rho_max + r_skin/2, the largest distance any list can
    // cover (0 for single-site molecules)
    double rho_max, rho_lim;
    double half_skin;
    // How far a molecule's centre may move from where the list was built (list_stale): a pair
    // stays listed while neither molecule exceeds its budget.  cg_half = (r_list - r_c,CG)/2
    // keeps the CG cutoff between centres covered; at_half = rho_max + r_skin/2, less the
    // molecule's current extent, keeps its atom pairs covered (each is 1e300 where the model
    // has no such part).  With force interpolation and a static region (w0_cg) a molecule of
    // weight zero at the step being checked has no atom pairs and takes cg_half alone.
    double cg_half, at_half;
    int w0_cg;
    // cubic CG table
    const float4 *tab;
    int tab_n;
    double tab_lo, tab_h, tab_inv_h;
    // correction force along the resolution coordinate: td_n values at the bin centres
    // of [td_lo, td_hi) (bin width td_h) and the integrals of the interpolated force from
    // td_lo to each centre (td_u, for its potential); td_n = 0: none
    const double *td;
    const double *td_u;
    int td_n;
    double td_lo, td_hi, td_h;
    // self-adjusting region: caller indices of the anchor molecules
    const int *anchors;
    int n_anchors;
};

// Cell grid over the box.
struct Grid {
    int n[3];
    double inv_len[3];
    int n_cells;
    int off_lo[3];   // stencil offsets per dimension: [off_lo, off_hi]
    int off_hi[3];
};

// ---------------------------------------------------------------- device helpers
// The helpers below fix the floating-point operation order (no contraction) so
// that centres of mass, weights and list distances are reproducible bit for bit.

// Minimum image of a coordinate difference |d| < 1.5 L as d - L rint(d / L) (one multiply,
// one rounding, one fused multiply-add): the single rounding of d -+ L, i.e. the value of
// adding or subtracting L when |d| > L / 2 and d itself otherwise, except within rounding of
// |d| = L / 2, where both images are equally near (no cutoff reaches that far: the box is
// at least twice the list radius).
__device__ __forceinline__ double mi(double d, double L, double invL)
{
    return fma(-L, rint(d * invL), d);
}

__device__ __forceinline__ double fold(double r, double L)
{
    if (r >= L) r -= L;
    else if (r < 0.0) r += L;
    return r;
}

__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

// Centre of mass of one molecule from its site coordinates p[k][d]:
// R = x0 + ((m1 d1 + m2 d2) + m3 d3) / M, folded into [0, L).  Also the largest
// site distance from R.
// One coordinate of the centre of mass from the sites' coordinate d.
template <int SPM>
__device__ __forceinline__ double com_dim(const DevParams &P, const double (&c)[SPM], int d)
{
#pragma clang fp contract(off)
    const double x0 = c[0];
    if constexpr (SPM == 1) return fold(x0 + 0.0, P.box[d]);   // x0 + 0 / M without the division
    double acc = 0.0;
#pragma unroll
    for (int k = 1; k < SPM; ++k) acc = acc + P.mass[k] * mi(c[k] - x0, P.box[d], P.inv_box[d]);
    // a product with 1 / M is the quotient itself when M is a power of two
    return fold(x0 + (P.M_pow2 ? acc * P.inv_M : acc / P.M), P.box[d]);
}

template <int SPM>
__device__ __forceinline__ void mol_com(const DevParams &P, const double (&p)[SPM][3], double R[3],
                                        double &rho)
{
#pragma clang fp contract(off)
    for (int d = 0; d < 3; ++d) {
        double c[SPM];
#pragma unroll
        for (int k = 0; k < SPM; ++k) c[k] = p[k][d];
        R[d] = com_dim<SPM>(P, c, d);
    }
    double rmax2 = 0.0;
#pragma unroll
    for (int k = 0; k < SPM; ++k) {
        double q0 = mi(p[k][0] - R[0], P.box[0], P.inv_box[0]);
        double q1 = mi(p[k][1] - R[1], P.box[1], P.inv_box[1]);
        double q2 = mi(p[k][2] - R[2], P.box[2], P.inv_box[2]);
        double r2 = dist2_exact(q0, q1, q2);
        rmax2 = r2 > rmax2 ? r2 : rmax2;
    }
    rho = sqrt(rmax2);
}

// Gradient of the resolution weight with respect to the centre of mass (the drift force of
// Eq. (2)): dw/dd = -(pi / (2 d_hy)) sin(pi (d - d_at) / d_hy) inside the hybrid layer,
// times the gradient of the distance (sign of the x offset for a slab, the unit offset for
// a sphere); 0 outside the layer.
__device__ __forceinline__ void weight_gradient(const DevParams &P, const double4 &R, double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    if (P.region != ADRES_REGION_SLAB_X && P.region != ADRES_REGION_SPHERE) return;
    double q0 = mi(R.x - P.center[0], P.box[0], P.inv_box[0]);
    double d;
    double q1 = 0.0, q2 = 0.0;
    if (P.region == ADRES_REGION_SLAB_X) {
        d = fabs(q0);
    } else {
        q1 = mi(R.y - P.center[1], P.box[1], P.inv_box[1]);
        q2 = mi(R.z - P.center[2], P.box[2], P.inv_box[2]);
        d = sqrt(dist2_exact(q0, q1, q2));
    }
    if (d <= P.d_at || d >= P.d_end) return;
    const double dw = -(M_PI / (2.0 * P.d_hy)) * sin(M_PI * (d - P.d_at) / P.d_hy);
    if (P.region == ADRES_REGION_SLAB_X) {
        g[0] = q0 > 0.0 ? dw : -dw;
    } else {
        g[0] = dw * q0 / d;
        g[1] = dw * q1 / d;
        g[2] = dw * q2 / d;
    }
}

// Distance of a centre of mass from the AT region's centre (slab: |x offset|; sphere:
// Euclidean), minimum image; q receives the offset (slab: x only).
__device__ __forceinline__ double res_distance(const DevParams &P, const double R[3], double q[3])
{
#pragma clang fp contract(off)
    q[0] = mi(R[0] - P.center[0], P.box[0], P.inv_box[0]);
    if (P.region == ADRES_REGION_SLAB_X) {
        q[1] = q[2] = 0.0;
        return fabs(q[0]);
    }
    q[1] = mi(R[1] - P.center[1], P.box[1], P.inv_box[1]);
    q[2] = mi(R[2] - P.center[2], P.box[2], P.inv_box[2]);
    return sqrt(dist2_exact(q[0], q[1], q[2]));
}

// Correction force on a centre of mass along the resolution coordinate: its value F(d)
// from the table (linear between bin centres, the end values held out to td_lo and
// td_hi, 0 outside [td_lo, td_hi)), its unit direction (the gradient of d) in dir, and
// with ENERGY its potential -integral of F from td_lo to min(d, td_hi) in u.
// The same from a distance d and the offset q it was measured along (slab: x only).
template <bool ENERGY>
__device__ __forceinline__ double corr_force_dq(const DevParams &P, double d, const double q[3], double dir[3],
                                                double &u)
{
    dir[0] = dir[1] = dir[2] = 0.0;
    u = 0.0;
    if (!(d >= P.td_lo)) return 0.0;
    const int n = P.td_n;
    const double t = (d - P.td_lo) / P.td_h - 0.5;   // in bin widths from the first centre
    double f;
    if (d >= P.td_hi) {
        if (ENERGY) u = -(P.td_u[n - 1] + P.td[n - 1] * (0.5 * P.td_h));
        return 0.0;
    } else if (t <= 0.0) {
        f = P.td[0];
        if (ENERGY) u = -(P.td[0] * (d - P.td_lo));
    } else if (t >= (double)(n - 1)) {
        f = P.td[n - 1];
        if (ENERGY) u = -(P.td_u[n - 1] + P.td[n - 1] * ((t - (double)(n - 1)) * P.td_h));
    } else {
        const int k = (int)t;
        const double s = t - (double)k;
        const double f0 = P.td[k], f1 = P.td[k + 1];
        f = f0 * (1.0 - s) + f1 * s;
        if (ENERGY) u = -(P.td_u[k] + P.td_h * s * (f0 + 0.5 * (f1 - f0) * s));
    }
    if (d > 0.0) {
        if (P.region == ADRES_REGION_SLAB_X) {
            dir[0] = q[0] > 0.0 ? 1.0 : -1.0;
        } else {
            dir[0] = q[0] / d;
            dir[1] = q[1] / d;
            dir[2] = q[2] / d;
        }
    }
    return f;
}

template <bool ENERGY>
__device__ __forceinline__ double corr_force(const DevParams &P, const double R[3], double dir[3], double &u)
{
    double q[3];
    const double d = res_distance(P, R, q);
    return corr_force_dq<ENERGY>(P, d, q, dir, u);
}

// Resolution weight of a distance from the AT centre (1 up to d_at, cos^2 ramp across
// the hybrid layer, 0 beyond).
__device__ __forceinline__ double weight_of_distance(const DevParams &P, double d)
{
#pragma clang fp contract(off)
    if (d <= P.d_at) return 1.0;
    if (d >= P.d_end) return 0.0;
    double c = cos(M_PI * (d - P.d_at) / (2.0 * P.d_hy));
    return c * c;
}

// Resolution weight of a centre of mass (1 in AT, cos^2 ramp in HY, 0 in CG).  The
// self-adjusting region's weights need every anchor's centre: they are written by a
// separate pass (launch_anchor_weights) and this returns a placeholder 0.
__device__ __forceinline__ double res_weight(const DevParams &P, const double R[3])
{
#pragma clang fp contract(off)
    if (P.region == ADRES_REGION_ALL_AT) return 1.0;
    if (P.region == ADRES_REGION_ALL_CG || P.region == ADRES_REGION_SPHERES) return 0.0;
    double q[3];
    const double d = res_distance(P, R, q);
    if (d <= P.d_at) return 1.0;
    if (d >= P.d_end) return 0.0;
    double c = cos(M_PI * (d - P.d_at) / (2.0 * P.d_hy));
    return c * c;
}

// Cell index along one dimension; NaN or out-of-range input lands in a valid cell
// (the error word reports non-finite positions separately).
__device__ __forceinline__ int cell_coord(double r, double inv_len, int n)
{
    double s = r * inv_len;
    if (!(s >= 0.0)) return 0;
    return s < (double)(n - 1) ? (int)s : n - 1;
}

// ---------------------------------------------------------------- lane exchanges
// Exchanges inside groups of four consecutive lanes by DPP quad permutations (a VALU
// move, no LDS round trip).  CTRL is the quad_perm selector: lane i of a quad reads lane
// ((CTRL >> 2 i) & 3) of the same quad.  Every lane of the quad must be active.
constexpr int kQuadXor1 = 0xB1;   // [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;   // [2, 3, 0, 1]
template <int K>
constexpr int kQuadBcast = 0x55 * K;   // [K, K, K, K]

template <int CTRL>
__device__ __forceinline__ double quad_perm(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the four lanes of a quad; every lane ends with the same bits
// ((a + b) + (c + d) with the pairs formed the same way on every lane).
__device__ __forceinline__ double quad_sum(double v)
{
    v += quad_perm<kQuadXor1>(v);
    return v + quad_perm<kQuadXor2>(v);
}

// 1/sqrt(x) for x > 0 to FP64 precision: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * (1.5 - hx * y * y);
    y = y * (1.5 - hx * y * y);
    return y;
}

// ---------------------------------------------------------------- integrator helpers
// Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): counter = (step, caller site), key = seed.
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
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    n0 = r * cs;
    n1 = r * sn;
}

// Opening half of a velocity-Verlet step for one site: v += F dt / 2m, then the
// drift x += v dt folded into [0, L).  With gamma > 0 the drift is split around an
// exact Ornstein-Uhlenbeck step (BAOAB, Leimkuhler & Matthews 2013):
//   x += v dt/2;  v = c v + sqrt((1 - c^2) kT / m) N(0,1), c = exp(-gamma dt);  x += v dt/2.
// inv_2m = 1 / (2m), precomputed per site (the same bits as 0.5 / m).  Operation order as
// in the oracle's integrator (no contraction).
__device__ __forceinline__ void open_and_drift(const DevParams &P, double m, double inv_2m, int caller_site, double x[3],
                                               double v[3], const double F[3], double dt, double gamma,
                                               double kT, uint64_t seed, uint64_t step_abs)
{
#pragma clang fp contract(off)
    double g[3] = {0.0, 0.0, 0.0};
    double c_ou = 0.0, s_ou = 0.0;
    if (gamma > 0.0) {
        U4 r = philox4x32_10(U4{(uint32_t)step_abs, (uint32_t)(step_abs >> 32), (uint32_t)caller_site, 0u},
                             (uint32_t)seed, (uint32_t)(seed >> 32));
        double n3;
        box_muller(r.x, r.y, g[0], g[1]);
        box_muller(r.z, r.w, g[2], n3);
        c_ou = exp(-gamma * dt);
        s_ou = sqrt((1.0 - c_ou * c_ou) * kT / m);
    }
    for (int d = 0; d < 3; ++d) {
        double vv = v[d] + F[d] * dt * inv_2m;
        double y;
        if (gamma > 0.0) {
            y = x[d] + vv * (0.5 * dt);
            vv = c_ou * vv + s_ou * g[d];
            y = fold(y + vv * (0.5 * dt), P.box[d]);
        } else {
            y = fold(x[d] + vv * dt, P.box[d]);
        }
        v[d] = vv;
        x[d] = y;
    }
}

// Closing half-kick v += F dt / 2m, as (F dt) * (1 / 2m) (the oracle's value for
// power-of-two masses).
__device__ __forceinline__ void close_kick(double v[3], const double F[3], double dt, double inv_2m)
{
#pragma clang fp contract(off)
    for (int d = 0; d < 3; ++d) v[d] = v[d] + F[d] * dt * inv_2m;
}

// Whether a molecule's list entries may no longer hold every pair in reach: its centre
// lies sqrt(d2) from where the list was built and its farthest site rh from its centre.
// An unlisted pair started at least r_list apart, so its centres are now at least r_list
// minus the two displacements apart, and its sites that less the two extents: the CG part
// is out of reach while each displacement is within cg_half, the atom pairs while each
// displacement plus extent is within at_half (r_list >= r_c,AT + 2 rho_max + r_skin).  A
// compact molecule (extent below rho_max) thus moves further than r_skin/2, one with a
// site beyond rho_max less far.
__device__ __forceinline__ bool list_stale(const DevParams &P, double d2, double rh)
{
    const double b = fmin(P.cg_half, P.at_half - rh);
    return !(b >= 0.0) || d2 > b * b;
}

// Centre and weight of a molecule at slot t into Rw, with the stretch / non-finite
// checks and the displacement check against R_ref (which lowers ctrl->halt to
// halt_value).
template <int SPM>
__device__ __forceinline__ void store_molecule(const DevParams &P, const double (&p)[SPM][3], int t,
                                               double4 *Rw, const double4 *R_ref, Ctrl *ctrl, int halt_value)
{
    double R[3], rh;
    mol_com<SPM>(P, p, R, rh);
    const double w = res_weight(P, R);
    Rw[t] = make_double4(R[0], R[1], R[2], w);
    bool finite = true;
#pragma unroll
    for (int k = 0; k < SPM; ++k) finite = finite && isfinite(p[k][0]) && isfinite(p[k][1]) && isfinite(p[k][2]);
    if (!finite) atomicOr(&ctrl->err, kErrNonFinite);
    if (SPM > 1 && rh > P.rho_lim) atomicOr(&ctrl->err, kErrStretch);
    if (R_ref) {
        const double4 r0 = R_ref[t];
        double q0 = mi(R[0] - r0.x, P.box[0], P.inv_box[0]);
        double q1 = mi(R[1] - r0.y, P.box[1], P.inv_box[1]);
        double q2 = mi(R[2] - r0.z, P.box[2], P.inv_box[2]);
        if (list_stale(P, dist2_exact(q0, q1, q2), SPM > 1 ? rh : 0.0)) atomicMin(&ctrl->halt, halt_value);
    }
}

// ---------------------------------------------------------------- launch wrappers
// All launches are asynchronous on `s`.  Arrays in "sorted" order are indexed by
// Morton slot; "caller" arrays by the caller's molecule/site index.

// Morton-ordered state of one configuration: positions, packed centre + weight,
// velocities and the order itself.  The centres are current after a gather, a reorder, the
// first drift of a step loop and the centres pass; the fused step kernel refreshes them
// only when something reads them between list builds (the network's pair pre-pass, the
// weights of a self-adjusting region), since it derives every centre it needs from x.
struct StateBufs {
    double *x;        // [3][n_sites]
    double *v;        // [3][n_sites]
    double4 *Rw;      // [n_mol] {Rx, Ry, Rz, w}
    int *perm;        // slot -> caller molecule
    int *key;         // slot -> Morton rank of its cell
};

void launch_weights_caller(hipStream_t s, const DevParams &P, const double *x, double *com, double *w,
                           Ctrl *ctrl);
// caller x (and v) -> sorted state through S.perm; centres, weights, rho; optional
// displacement check against R_ref (sets halt = 0)
void launch_gather(hipStream_t s, const DevParams &P, const double *x_caller, const double *v_caller,
                   const StateBufs &S, const double4 *R_ref, Ctrl *ctrl);
void launch_scatter_out(hipStream_t s, const DevParams &P, const int *perm, const double *x, const double *v,
                        const double *f, double *x_caller, double *v_caller, double *f_caller);
// opening half-kick + drift of one step from x_in to x_out (new Rw/rho, displacement check)
struct StepArgs {
    double dt, gamma, kT;
    uint64_t seed, step_abs;
};
void launch_kick_drift(hipStream_t s, const DevParams &P, const double *x_in, double *v, const double *f,
                       double *x_out, double4 *Rw_out, const double4 *R_ref, const int *perm, Ctrl *ctrl, int step,
                       const StepArgs &st);
// centres and weights of the sorted state from its positions (before a reorder, when the
// step kernels have not kept them) and the cell keys of launch_cell_keys, in one pass
// (head: the step chunk's publication, see ChainHead)
void launch_centres_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank, const double *x,
                         double4 *Rw, int *key, int *count, const int *go = nullptr, const double *x_alt = nullptr,
                         double4 *Rw_alt = nullptr, const ChainHead &head = ChainHead{});
void launch_reset_halt(hipStream_t s, Ctrl *ctrl);
// the control block's fields into host-mapped memory, tagged with seq (see CtrlPub)
void launch_publish(hipStream_t s, Ctrl *ctrl, CtrlPub *pub, unsigned seq);
void launch_map_cg(hipStream_t s, const DevParams &P, const double *x, const double *f, double *com, double *fmap);

// cell list
void launch_cell_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank,
                      const double4 *Rw, int *key, int *count, const int *go = nullptr,
                      const double4 *Rw_alt = nullptr, const ChainHead &head = ChainHead{});
// exclusive scan of count[0..n) into start[0..n] (start[n] = total); resets count (and
// fill if non-null); tiles: scratch of at least n / 1024 + 1 ints; n <= scan_max_elements()
void launch_scan_cells(hipStream_t s, int *count, int n, int *start, int *fill, int *tiles, const int *go = nullptr);
int scan_max_elements();
// the cell sort after the keys pass: counts (in place) scanned per tile of 1024 cells, the
// cells' starts start[0..n_cells] and every molecule's slot in new_from (cell order, arbitrary
// within a cell); fill cleared here; tiles: scratch of at least n_cells / 1024 + 1 ints;
// n_cells <= scan_max_elements().  reset: a control block whose halt index and list reports
// are cleared (whether or not go is set), after a chain head published them.
void launch_scatter_slots(hipStream_t s, int n_mol, int n_cells, const int *key, int *count, int *start, int *fill,
                          int *tiles, int *new_from, const int *go = nullptr, Ctrl *reset = nullptr);
// caller order within each cell, then the state gathered into the new slot order; clears
// the counts for the next build
void launch_sort_permute(hipStream_t s, const DevParams &P, int n_cells, const int *start, int *new_from,
                         int *count, const StateBufs &src, const StateBufs &dst, int *inv_perm, double4 *R_ref,
                         bool with_v, const int *go = nullptr);

// Verlet list: ELL, row-major nbr[slot * cap + k]; each row is padded with the
// row's own slot up to a multiple of 4 entries (cap is a multiple of 4).
// stencil: rank-major [n_cells][27] neighbour cell ranks, -1 = skipped (fixed at set-up)
void launch_list_build(hipStream_t s, const DevParams &P, const Grid &G, const int *stencil, const int *start,
                       const double4 *Rw, double rl2, int *nbr, int *cnt, int cap, unsigned *mcost, Ctrl *ctrl,
                       const int *go = nullptr, const double4 *Rw_alt = nullptr);

// Neighbour halo of every force-kernel tile (64 consecutive slots), stored at the tile's
// dispatch position p = tile_pos[tile] (launch_tile_order), so that the force kernel's
// workgroup p finds it without first reading which tile it runs: hid[p * hcap + l] lists
// the slots the tile reads, its own 64 first (l < 64, the tile's slot order), then every
// other slot of its molecules' rows once; hn[p] is the count.  tperm[p * 64 + j] is the
// tile's j-th molecule by falling cost (mcost from the list build; ties and the empty tail
// of a short last tile in slot order): the force kernel's thread group j takes it, so each
// wavefront's sixteen molecules have similar row work.  Row j of the dispatch-ordered rows
// (r = p * 64 + j) is that molecule's: hcnt[r] its length (0 for the empty tail) and lnbr
// its entries as local halo indices (uint16), entry k at r * lcap + (k % 4) * (lcap / 4) +
// k / 4, so that lane q of the quad finds its entries q, q + 4, ... contiguous.  A halo
// larger than hcap sets overflow bit 1, max_halo and halt = -1.
constexpr int kHaloTile = 64;
void launch_halo_build(hipStream_t s, int n_mol, const int *nbr, const int *cnt, int cap, int hcap, int lcap,
                       const unsigned *mcost, const int *tile_pos, int *hid, int *hn, int *hcnt, uint16_t *lnbr,
                       uint8_t *tperm, Ctrl *ctrl, const int *go = nullptr);
// LDS bytes of the force kernel's halo staging per halo molecule, and the largest halo
// capacity that fits a workgroup's LDS
int halo_stride_bytes(int spm, int pair_precision);
int halo_capacity_limit(int spm, int pair_precision);

// half list (t < u pairs) + per-entry pair ids; up_off receives n + 1 offsets
void launch_half_list(hipStream_t s, int n, int *nbr, const int *cnt, int cap, int *cnt_up, int *up_off,
                      int *scratch, int2 *pairs, int64_t pairs_cap, int *pid, const int *go = nullptr);

// forces
enum ForceMode : int {
    kModeForce = 0,   // F(x) only
    kModeStep = 1,    // F(x_n), closing half-kick of step n, opening half-kick + drift of step n+1
    kModeClose = 2,   // F(x_n) and the closing half-kick of the last step
};
struct ForceArgs {
    DevParams P;
    const double *x;        // step-n positions (sorted)
    const double4 *Rw;      // step-n weights of a self-adjusting region (w only)
    int cap;                // row capacity of the slot-indexed list (pair ids)
    // tile halos, cost order and rows as local halo indices, all at the dispatch position
    // (launch_halo_build)
    const int *hid, *hn;
    int hcap;
    const int *hcnt;
    const uint16_t *lnbr;
    int lcap;
    const uint8_t *tperm;
    const int *perm, *inv_perm;   // slot -> caller, caller -> slot
    int mode;
    double *f;                    // kModeForce / kModeClose: output forces
    const int *out_perm;          // non-null: write f in caller order via perm
    double *v;                    // kModeStep / kModeClose: velocities (in place)
    double *x_out;                // kModeStep: step n+1 positions
    double4 *Rw_out;              //   and, if non-null, their centres and weights
    const double4 *R_ref;
    StepArgs st;
    Ctrl *ctrl;
    int step, check_halt;
    double *epart;                // non-null: per-block energy partials [blocks][4]
    const int *pid;               // learned CG force: pair id of every list entry
    const float *f_pair;          //   and the network's f(r) per pair
    // multiple time stepping: the slow part (CG pair part, the CG share of the drift, the
    // correction force) enters the force with this factor; 0 skips it (inner steps)
    double slow_scale;
    // dispatch order of the workgroups (launch_tile_order): the tile workgroup p runs
    const int *tile_order;
    // self-adjusting region: offset from the nearest anchor centre and its length per slot
    const double4 *near;
};
// returns the block count; e0/e1 (optional) are recorded at the kernel's start and end;
// the launch takes hcap * halo_stride_bytes() bytes of dynamic LDS
int launch_forces(hipStream_t s, const ForceArgs &a, int pair_precision, hipEvent_t e0 = nullptr,
                  hipEvent_t e1 = nullptr);
int force_blocks(int n_mol);
void launch_energy_reduce(hipStream_t s, const double *epart, int n_blocks, double *energy);

// workgroup dispatch order of the force kernel, rebuilt with the list (k_cells.hip):
// order[p] is the tile dispatched as workgroup p, pos[tile] its inverse
void launch_tile_order(hipStream_t s, const DevParams &P, const unsigned *mcost, int n_tiles, int *order, int *pos, const int *go = nullptr);

// correction force (k_state.hip)
constexpr int kTdMaxBins = 4096;
// cen: anchor centres [K][3] for ADRES_REGION_SPHERES (else null)
void launch_density_profile(hipStream_t s, const DevParams &P, const double *x, const double *cen,
                            unsigned long long *counts);
void launch_anchor_centres(hipStream_t s, const DevParams &P, const double *x, double *cen);
void launch_region_volumes(hipStream_t s, const DevParams &P, const double *cen, long long n_samples,
                           unsigned long long seed, unsigned long long *counts);
// vol: sampled bin volumes (counts over n_vol points) or null for the closed forms
void launch_td_update(hipStream_t s, const DevParams &P, double *td, double *td_u, const long long *counts,
                      long long n_frames, double prefactor, const long long *vol, long long n_vol);

// self-adjusting region (k_state.hip): weights from the nearest anchor centre, for the
// Morton-ordered state (Rw in place, and the offset from the nearest anchor with its
// length into near; anchors located through inv_perm; skipped like the step kernels once
// a chunk has halted) or for caller-order centres (com [3][n] -> w)
constexpr int kMaxAnchors = 1024;
constexpr int kAnchorGrid = 16;                                       // anchor cells per axis, at most
constexpr int kAnchorCells = kAnchorGrid * kAnchorGrid * kAnchorGrid;
// aslot [n_anchors]: the anchors' slots, refreshed from inv_perm when refresh is set (after
// every reorder), read otherwise
void launch_anchor_weights(hipStream_t s, const DevParams &P, double4 *Rw, const int *inv_perm, int *aslot,
                           int refresh, Ctrl *ctrl, int step, int check_halt, double4 *near, const int *go = nullptr,
                           double4 *Rw_alt = nullptr);
void launch_anchor_weights_caller(hipStream_t s, const DevParams &P, const double *com, double *w);

}  // namespace adres
