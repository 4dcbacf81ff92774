// Force-interpolation kernel, Eq. (1) of Sec. 2.2:
//   F_ab = ww F^AT_ab + (1 - ww) F^CG_ab,  ww = w_a w_b,
// with F^AT the sum of atom-atom WCA forces between the two molecules and F^CG a
// force between their centres of mass, shared among a molecule's sites by mass
// fraction; plus the bonded terms, which are not interpolated (Sec. 2.2, last
// paragraph).  In its step mode the same kernel also finishes velocity Verlet
// for step n (closing half-kick) and starts step n+1 (opening half-kick, drift,
// new centre of mass and weight, list-displacement check), so one MD step is one
// launch.
//
// Work mapping (gfx950, wave64): four lanes per home molecule, 16 molecules per
// wavefront, consecutive Morton slots (a compact cluster of cells) per workgroup.
// Lane q takes the molecule's list entries in blocks of kPre (entries kPre q ..,
// then 4 kPre further on): one vector load fetches the block's neighbour slots and
// their 32-byte {R, w} gathers are issued back to back before any arithmetic, so
// each lane keeps kPre independent memory chains in flight (the kernel is bound by
// gather latency, not by arithmetic).  Every lane accumulates, in FP64, the
// atom-tile forces on all sites of its molecule and the molecule's total CG force;
// two butterfly shuffles combine the four lanes; lane q then owns site q.
//
// Full (two-sided) list: no atomics, fixed summation order, bit-reproducible.
// Pair arithmetic in PT (double or float).  In the float variant an atom-pair
// displacement is the FP64 centre difference rounded once to FP32 plus the two
// sites' FP32 offsets from their centres (|offset| < rho_max), which keeps it within
// a few 1e-7 of the FP64 value without FP64 work per atom pair; the CG cutoff is
// decided on the FP64 centre distance.  The FP64 variant forms every displacement
// from FP64 coordinates.
//
// Workgroups are mapped XCD by XCD: the hardware deals workgroup b to XCD b mod 8,
// so logical block ranges are assigned per XCD and every XCD's L2 serves one
// contiguous stretch of Morton slots (a compact region of space).  An atom tile is skipped when the centres are farther apart
// than rc_at + rho_a + rho_b (rho: largest site distance from the centre), which
// no interacting atom pair can be (triangle inequality).
#include <hip/hip_ext.h>

#include "adres_internal.h"

namespace adres {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 4;   // lanes per home molecule
constexpr int kPre = 2;     // list entries a lane fetches and gathers together
constexpr int kXcds = 8;

// logical block of this workgroup: XCD k (= blockIdx mod 8) takes a contiguous range
__device__ __forceinline__ int xcd_block()
{
    const int B = gridDim.x, b = blockIdx.x;
    const int q = B / kXcds, r = B % kXcds, x = b % kXcds, i = b / kXcds;
    return x * q + (x < r ? x : r) + i;
}

template <typename PT>
__device__ __forceinline__ PT recip(PT x) { return PT(1) / x; }
template <>
__device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }   // 1 ulp

template <typename PT>
__device__ __forceinline__ PT wca_f_over_r(PT r2, PT sig2, PT eps, PT &u, bool want_u)
{
    PT inv = recip<PT>(r2);
    PT s = sig2 * inv;
    PT s6 = s * s * s;
    if (want_u) u = PT(4) * eps * s6 * (s6 - PT(1)) + eps;
    return PT(24) * eps * s6 * (PT(2) * s6 - PT(1)) * inv;
}

// Cubic table of the CG force magnitude; interval and fraction located in FP64 (by a
// multiplication with the reciprocal knot spacing: within an ulp of the quotient).
template <typename PT>
__device__ __forceinline__ PT table_f(const DevParams &P, double r, Ctrl *ctrl)
{
    double u = (r - P.tab_lo) * P.tab_inv_h;
    if (r < P.tab_lo) atomicOr(&ctrl->err, kErrTableRange);
    double kf = floor(u);
    kf = kf >= 0.0 ? kf : 0.0;   // also maps NaN to interval 0
    kf = kf > (double)(P.tab_n - 2) ? (double)(P.tab_n - 2) : kf;
    PT t = (PT)(u - kf);
    float4 c = P.tab[(int)kf];
    return ((PT(c.w) * t + PT(c.z)) * t + PT(c.y)) * t + PT(c.x);
}

// At most 128 VGPRs (4 waves per SIMD): 4 lanes x 64k molecules is ~4000 wavefronts,
// which then fit the 1024 SIMDs in a single round.
// Variants (VAR): kVarForce, force interpolation, Eq. (1); kVarHam, potential energy
// interpolation, Eq. (2): pair weights (w_a + w_b) / 2, the molecule's single-molecule
// potentials V^AT, V^CG (half of each of its pair potentials) accumulated on hybrid
// molecules, and their drift force -(V^AT - V^CG) grad w shared by mass fraction;
// kVarNear, force interpolation with a correction field around the nearest anchor of a
// self-adjusting region (its own instantiation, so that the extra load does not weigh on
// the common kernels' registers).
enum : int { kVarForce = 0, kVarHam = 1, kVarNear = 2 };

template <int SPM, typename PT, int MODE, bool ENERGY, int VAR>
__global__ __launch_bounds__(kBlock, 4) void k_forces(ForceArgs a)
{
    constexpr bool HAM = VAR == kVarHam;
    const DevParams &P = a.P;
    const int halt = a.ctrl->halt;
    const int n = P.n_mol;
    const int64_t ns = P.n_sites;
    const int slot = xcd_block();
    const int blk = a.tile_order ? a.tile_order[slot] : slot;
    const int gid = blk * kBlock + threadIdx.x;
    const int t = gid / kLanes, q = gid % kLanes;
    const bool valid = t < n;
    const int tt = valid ? t : n - 1;

    // home sites of the workgroup's 64 molecules, staged in LDS (read by every lane of a
    // quad in the atom tiles, the bonds and the drift)
    __shared__ double sx[kBlock / kLanes][SPM][3];
    // velocities and reference centres are only needed after the force loop; staging them
    // here lets their loads overlap the prologue instead of adding a wait at the end
    __shared__ double sv[MODE == kModeForce ? 1 : kBlock / kLanes][SPM][3];
    __shared__ double4 sref[MODE == kModeStep ? kBlock / kLanes : 1];
    const int ml = threadIdx.x / kLanes;
    // every load of the molecule's own data (and the halt index) is issued before the
    // first wait, so that the prologue costs one memory round trip
    double lx[3] = {0.0, 0.0, 0.0}, lv[3] = {0.0, 0.0, 0.0};
    if (q < SPM) {
#pragma unroll
        for (int d = 0; d < 3; ++d) lx[d] = a.x[d * ns + (int64_t)tt * SPM + q];
        if (MODE != kModeForce)
#pragma unroll
            for (int d = 0; d < 3; ++d) lv[d] = a.v[d * ns + (int64_t)tt * SPM + q];
    }
    double4 lref = make_double4(0.0, 0.0, 0.0, 0.0);
    if (MODE == kModeStep) lref = a.R_ref[tt];
    const double4 me = a.Rw[tt];
    const double rha = (double)a.rho[tt];
    constexpr bool kOff = sizeof(PT) == 4;   // FP32 displacements from site offsets
    // (a single-site molecule's offset from its centre is exactly zero: no loads or stores)
    float hoff[SPM][3] = {};
    if (kOff && SPM > 1) {
#pragma unroll
        for (int i = 0; i < SPM; ++i)
#pragma unroll
            for (int d = 0; d < 3; ++d) hoff[i][d] = a.off[(int64_t)tt * (3 * SPM) + 3 * i + d];
    }
    const int cnt = valid ? a.cnt[tt] : 0;
    // the same decision in every wave: only an earlier launch can set halt below this step
    // (this one sets it to its own step at the lowest), so no workgroup stops at the barrier
    if (a.check_halt && a.step > halt) return;
    if (q < SPM) {
#pragma unroll
        for (int d = 0; d < 3; ++d) sx[ml][q][d] = lx[d];
        if (MODE != kModeForce)
#pragma unroll
            for (int d = 0; d < 3; ++d) sv[ml][q][d] = lv[d];
    }
    if (MODE == kModeStep && q == 0) sref[ml] = lref;
    __syncthreads();
#define XI(i, d) sx[ml][(i)][(d)]

    double acc[SPM][3];
#pragma unroll
    for (int i = 0; i < SPM; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
    double cg0 = 0.0, cg1 = 0.0, cg2 = 0.0;
    double uat = 0.0, ucg = 0.0, ubond = 0.0;
    // Eq. (2): a molecule on which the weight gradient is non-zero needs V^AT and V^CG
    // (inside the hybrid layer, where the weight gradient is non-zero; the gradient itself
    // is formed after the pair loop so that it takes no registers there)
    bool hy_home = false;
    if (HAM && (P.region == ADRES_REGION_SLAB_X || P.region == ADRES_REGION_SPHERE)) {
        const double Rm[3] = {me.x, me.y, me.z};
        double qh[3];
        const double dh = res_distance(P, Rm, qh);
        hy_home = dh > P.d_at && dh < P.d_end;
    }
    double vat = 0.0, vcg = 0.0;

    const PT sig2A = (PT)P.sig2_at, epsA = (PT)P.eps_at, rcA2 = (PT)P.rcA2;
    const PT sig2C = (PT)P.sig2_cg, epsC = (PT)P.eps_cg;
    const int *row = a.nbr + (int64_t)tt * a.cap;
    const bool with_slow = a.slow_scale != 0.0;

    for (int k0 = kPre * q; k0 < cnt; k0 += kPre * kLanes) {
        int us[kPre];
        if (kPre == 4) {
            const int4 id4 = *reinterpret_cast<const int4 *>(row + k0);
            us[0] = id4.x; us[1] = id4.y; us[kPre > 2 ? 2 : 0] = id4.z; us[kPre > 3 ? 3 : 0] = id4.w;
        } else {
            const int2 id2 = *reinterpret_cast<const int2 *>(row + k0);
            us[0] = id2.x; us[1] = id2.y;
        }
        double4 nb[kPre];
#pragma unroll
        for (int j = 0; j < kPre; ++j) nb[j] = a.Rw[us[j]];   // padding entries are valid slots
        // CG sites: the learned CG force of each entry's pair, requested with the centres
        // (pair ids exist for the row's real entries only)
        float fp[kPre] = {0.0f, 0.0f};
        if (SPM == 1 && P.cg_kind >= ADRES_CG_MLP) {
            const int2 pid2 = *reinterpret_cast<const int2 *>(a.pid + (int64_t)tt * a.cap + k0);
            fp[0] = a.f_pair[pid2.x];
            if (k0 + 1 < cnt) fp[1] = a.f_pair[pid2.y];
        }
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            if (k0 + j >= cnt) break;
            const int u = us[j];
            const double4 o = nb[j];
            const double ww = HAM ? 0.5 * (me.w + o.w) : me.w * o.w;   // weight of the AT part
            const double D0 = mi(me.x - o.x, P.box[0], P.half[0]);
            const double D1 = mi(me.y - o.y, P.box[1], P.half[1]);
            const double D2 = mi(me.z - o.z, P.box[2], P.half[2]);
            const double r2c = dist2_exact(D0, D1, D2);
            if (ww > 0.0) {
                // no atom pair of the tile can be within the cutoff beyond this centre
                // distance (every site lies within rho_max of its centre, a checked invariant)
                const double bound = P.rc_at + rha + P.rho_max + 1e-6;
                if (r2c < bound * bound) {
                    const PT pww = (PT)ww;
                    if constexpr (kOff) {
                        float no[3 * SPM];
                        if constexpr (SPM == 4) {   // 48 bytes, 16-byte aligned: three vector loads
                            const float4 *q4 = reinterpret_cast<const float4 *>(a.off + (int64_t)u * 12);
                            const float4 o0 = q4[0], o1 = q4[1], o2 = q4[2];
                            no[0] = o0.x; no[1] = o0.y; no[2] = o0.z; no[3] = o0.w;
                            no[4] = o1.x; no[5] = o1.y; no[6] = o1.z; no[7] = o1.w;
                            no[8] = o2.x; no[9] = o2.y; no[10] = o2.z; no[11] = o2.w;
                        } else {
#pragma unroll
                            for (int j2 = 0; j2 < 3 * SPM; ++j2)
                                no[j2] = SPM > 1 ? a.off[(int64_t)u * (3 * SPM) + j2] : 0.0f;
                        }
                        // D + (off_i - off_jj): the same bits with opposite sign from the
                        // other molecule's side, so pair forces cancel exactly (Newton's third law)
                        const float Df0 = (float)D0, Df1 = (float)D1, Df2 = (float)D2;
#pragma unroll
                        for (int i = 0; i < SPM; ++i) {
                            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                            for (int jj = 0; jj < SPM; ++jj) {
                                const float dx = Df0 + (hoff[i][0] - no[3 * jj]);
                                const float dy = Df1 + (hoff[i][1] - no[3 * jj + 1]);
                                const float dz = Df2 + (hoff[i][2] - no[3 * jj + 2]);
                                const float r2 = (dx * dx + dy * dy) + dz * dz;
                                if (r2 < (float)rcA2) {
                                    PT uu = PT(0);
                                    const PT c = pww * wca_f_over_r<PT>((PT)r2, sig2A, epsA, uu, ENERGY || hy_home);
                                    s0 += (double)(c * dx);
                                    s1 += (double)(c * dy);
                                    s2 += (double)(c * dz);
                                    if (ENERGY) uat += 0.5 * (HAM ? me.w : ww) * (double)uu;
                                    if (HAM) vat += 0.5 * (double)uu;
                                }
                            }
                            acc[i][0] += s0; acc[i][1] += s1; acc[i][2] += s2;
                        }
                    } else {
#pragma unroll 1
                    for (int jj = 0; jj < SPM; ++jj) {
                        const double xj0 = a.x[(int64_t)u * SPM + jj];
                        const double xj1 = a.x[ns + (int64_t)u * SPM + jj];
                        const double xj2 = a.x[2 * ns + (int64_t)u * SPM + jj];
#pragma unroll
                        for (int i = 0; i < SPM; ++i) {
                            const PT dx = (PT)mi(XI(i, 0) - xj0, P.box[0], P.half[0]);
                            const PT dy = (PT)mi(XI(i, 1) - xj1, P.box[1], P.half[1]);
                            const PT dz = (PT)mi(XI(i, 2) - xj2, P.box[2], P.half[2]);
                            const PT r2 = (dx * dx + dy * dy) + dz * dz;
                            if (r2 < rcA2) {
                                PT uu = PT(0);
                                const PT c = pww * wca_f_over_r<PT>(r2, sig2A, epsA, uu, ENERGY || hy_home);
                                acc[i][0] += (double)(c * dx);
                                acc[i][1] += (double)(c * dy);
                                acc[i][2] += (double)(c * dz);
                                if (ENERGY) uat += 0.5 * (HAM ? me.w : ww) * (double)uu;
                                if (HAM) vat += 0.5 * (double)uu;
                            }
                        }
                    }
                    }
                }
            }
            if (with_slow && ww < 1.0 && r2c < P.rcC2) {
                PT uu = PT(0);
                PT fr;
                if (P.cg_kind == ADRES_CG_WCA) {
                    fr = wca_f_over_r<PT>((PT)r2c, sig2C, epsC, uu, ENERGY || hy_home);
                } else if (P.cg_kind >= ADRES_CG_MLP) {
                    // the same bits from both sides of the pair (same r2c, same network value)
                    const float fv = SPM == 1 ? fp[j] : a.f_pair[a.pid[(int64_t)tt * a.cap + k0 + j]];
                    fr = (PT)fv * (PT)__builtin_amdgcn_rsqf((float)r2c);
                } else {
                    // r and 1/r from one refined reciprocal square root: no FP64 square
                    // root or division on the table path
                    const double ir = rsqrt_refined(r2c);
                    fr = table_f<PT>(P, r2c * ir, a.ctrl) * (PT)ir;
                }
                const PT sc = (PT)(1.0 - ww) * fr;
                cg0 += (double)(sc * (PT)D0);
                cg1 += (double)(sc * (PT)D1);
                cg2 += (double)(sc * (PT)D2);
                if (ENERGY) ucg += 0.5 * (HAM ? 1.0 - me.w : 1.0 - ww) * (double)uu;
                if (HAM) vcg += 0.5 * (double)uu;
            }
        }
    }

    // combine the four lanes' partial sums (every lane ends with the same bits)
    static_assert(kLanes == 4, "the quad exchanges below assume four lanes per molecule");
#pragma unroll
    for (int i = 0; i < SPM; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[i][d] = quad_sum(acc[i][d]);
    if (HAM) {
        vat = quad_sum(vat);
        vcg = quad_sum(vcg);
    }
    cg0 = quad_sum(cg0);
    cg1 = quad_sum(cg1);
    cg2 = quad_sum(cg2);

    double ucorr = 0.0;   // the correction field's potential (energy only)

    // lane q owns site q
    double F[3] = {0.0, 0.0, 0.0}, xq[3] = {0.0, 0.0, 0.0};
    double mfq = 0.0;   // the lane's site mass fraction
    double mq = 1.0, iq = 0.5;
#pragma unroll
    for (int i = 0; i < SPM; ++i)
        if (i == q) {
            const double mf = P.mfrac[i];
            const double ss = a.slow_scale;
            F[0] = acc[i][0] + mf * (ss * cg0);
            F[1] = acc[i][1] + mf * (ss * cg1);
            F[2] = acc[i][2] + mf * (ss * cg2);
            if (HAM && hy_home) {
                double gw[3];
                weight_gradient(P, me, gw);
                // drift force of Eq. (2): -(V^AT - V^CG) grad w(R), grad_x R = m_i / M
                const double dv = -(vat - ss * vcg) * mf;
                F[0] += dv * gw[0];
                F[1] += dv * gw[1];
                F[2] += dv * gw[2];
            }
            mfq = mf;
            xq[0] = XI(i, 0); xq[1] = XI(i, 1); xq[2] = XI(i, 2);
            mq = P.mass[i];
            iq = P.inv_2m[i];
        }
    const bool owner = valid && q < SPM;
    if (P.td_n > 0 && with_slow && q < SPM) {
        // correction force on the centre of mass along the resolution coordinate (Sec. 2.4),
        // shared by mass fraction (evaluated here, after the pair loop, to keep its values
        // out of the loop's registers)
        double qd[3], dd;
        if constexpr (VAR == kVarNear) {   // along the offset from the nearest anchor
            const double4 nr = a.near[tt];
            qd[0] = nr.x; qd[1] = nr.y; qd[2] = nr.z;
            dd = nr.w;
        } else {
            const double Rm[3] = {me.x, me.y, me.z};
            dd = res_distance(P, Rm, qd);
        }
        double tdir[3];
        const double ftd = corr_force_dq<ENERGY>(P, dd, qd, tdir, ucorr);
        const double ft = mfq * (a.slow_scale * ftd);
        F[0] += ft * tdir[0];
        F[1] += ft * tdir[1];
        F[2] += ft * tdir[2];
    }
    if (owner) {
        if (P.bond_kind == ADRES_BOND_HARMONIC) {
#pragma unroll
            for (int k = 0; k < SPM; ++k) {
                if (k == q) continue;
                const double d0 = mi(xq[0] - XI(k, 0), P.box[0], P.half[0]);
                const double d1 = mi(xq[1] - XI(k, 1), P.box[1], P.half[1]);
                const double d2 = mi(xq[2] - XI(k, 2), P.box[2], P.half[2]);
                const double r2b = (d0 * d0 + d1 * d1) + d2 * d2;
                const double ir = rsqrt_refined(r2b);
                const double r = r2b * ir;
                const double fr = -P.k_bond * (r - P.r0_bond) * ir;
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
    }

    const int64_t site = (int64_t)t * SPM + q;
    if (MODE == kModeForce) {
        if (owner) {
            const int64_t os = a.out_perm ? (int64_t)a.out_perm[t] * SPM + q : site;
            a.f[os] = F[0];
            a.f[ns + os] = F[1];
            a.f[2 * ns + os] = F[2];
        }
    } else if (MODE == kModeClose) {
        if (owner) {
            double v[3] = {sv[ml][q][0], sv[ml][q][1], sv[ml][q][2]};
            close_kick(v, F, a.st.dt, iq);
            a.v[site] = v[0]; a.v[ns + site] = v[1]; a.v[2 * ns + site] = v[2];
            a.f[site] = F[0]; a.f[ns + site] = F[1]; a.f[2 * ns + site] = F[2];
        }
    } else {   // kModeStep
        double xn[3] = {xq[0], xq[1], xq[2]};
        if (owner) {
            double v[3] = {sv[ml][q][0], sv[ml][q][1], sv[ml][q][2]};
            close_kick(v, F, a.st.dt, iq);
            const int caller_site = a.st.gamma > 0.0 ? a.perm[t] * SPM + q : 0;
            open_and_drift(P, mq, iq, caller_site, xn, v, F, a.st.dt, a.st.gamma, a.st.kT, a.st.seed, a.st.step_abs);
            a.v[site] = v[0]; a.v[ns + site] = v[1]; a.v[2 * ns + site] = v[2];
            a.x_out[site] = xn[0]; a.x_out[ns + site] = xn[1]; a.x_out[2 * ns + site] = xn[2];
        }
        // new centre, weight, rho and offsets, spread over the quad: lane d < 3 forms
        // coordinate d of the centre (the operation order of mol_com), lane q < SPM its
        // own site's offset and distance
        double col[SPM];
        const int dd = q < 3 ? q : 0;
        {
            double b[3][4];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                b[d][0] = quad_perm<kQuadBcast<0>>(xn[d]);
                b[d][1] = quad_perm<kQuadBcast<1>>(xn[d]);
                b[d][2] = quad_perm<kQuadBcast<2>>(xn[d]);
                b[d][3] = quad_perm<kQuadBcast<3>>(xn[d]);
            }
#pragma unroll
            for (int k = 0; k < SPM; ++k) col[k] = dd == 0 ? b[0][k] : (dd == 1 ? b[1][k] : b[2][k]);
        }
        const double Rd = com_dim<SPM>(P, col, dd);
        const double R0 = quad_perm<kQuadBcast<0>>(Rd), R1 = quad_perm<kQuadBcast<1>>(Rd),
                     R2 = quad_perm<kQuadBcast<2>>(Rd);
        double r2 = 0.0;
        if (owner) {
            const double o0 = mi(xn[0] - R0, P.box[0], P.half[0]);
            const double o1 = mi(xn[1] - R1, P.box[1], P.half[1]);
            const double o2 = mi(xn[2] - R2, P.box[2], P.half[2]);
            r2 = dist2_exact(o0, o1, o2);
            if (SPM > 1) {
                float *of = a.off_out + (int64_t)t * (3 * SPM) + 3 * q;
                of[0] = (float)o0; of[1] = (float)o1; of[2] = (float)o2;
            }
        }
        double m2 = r2;
        {
            const double y1 = quad_perm<kQuadXor1>(m2);
            m2 = y1 > m2 ? y1 : m2;
            const double y2 = quad_perm<kQuadXor2>(m2);
            m2 = y2 > m2 ? y2 : m2;
        }
        if (valid && q == 0) {
            const double R[3] = {R0, R1, R2};
            const double rh = sqrt(m2);
            a.Rw_out[t] = make_double4(R0, R1, R2, res_weight(P, R));
            a.rho_out[t] = (float)rh;
            if (!(isfinite(R0) && isfinite(R1) && isfinite(R2))) atomicOr(&a.ctrl->err, kErrNonFinite);
            if (SPM > 1 && rh > P.rho_max) atomicOr(&a.ctrl->err, kErrStretch);
            const double4 rr = sref[ml];
            const double q0 = mi(R0 - rr.x, P.box[0], P.half[0]);
            const double q1 = mi(R1 - rr.y, P.box[1], P.half[1]);
            const double q2 = mi(R2 - rr.z, P.box[2], P.half[2]);
            if (dist2_exact(q0, q1, q2) > P.half_skin2) atomicMin(&a.ctrl->halt, a.step);
        }
    }

#undef XI
    if (ENERGY) {
        // block reduction in a fixed order: wavefront butterflies, then 4 waves in LDS
        __shared__ double red[kBlock / 64][4];
        double e[4] = {uat, ucg, ubond, valid && q == 0 ? ucorr : 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) e[c] += __shfl_xor(e[c], off, 64);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) {
            red[wave][0] = e[0]; red[wave][1] = e[1]; red[wave][2] = e[2]; red[wave][3] = e[3];
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
            a.epart[blk * 4 + threadIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(256) void k_energy_reduce(const double *__restrict__ epart, int n_blocks,
                                                       double *__restrict__ energy)
{
    __shared__ double red[256][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n_blocks; b += 256)
        for (int c = 0; c < 4; ++c) s[c] += epart[b * 4 + c];
    for (int c = 0; c < 4; ++c) red[threadIdx.x][c] = s[c];
    __syncthreads();
    for (int half = 128; half >= 1; half >>= 1) {
        if (threadIdx.x < half)
            for (int c = 0; c < 4; ++c) red[threadIdx.x][c] += red[threadIdx.x + half][c];
        __syncthreads();
    }
    if (threadIdx.x < 4) energy[threadIdx.x] = red[0][threadIdx.x];
}

// Launch; with events, hipExtLaunchKernelGGL records them at the kernel's own start
// and end (the duration excludes launch gaps, as a profiler's kernel trace does).
template <typename K>
void launch_k(K kernel, hipStream_t s, const ForceArgs &a, int blocks, hipEvent_t e0, hipEvent_t e1)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlock), 0, s, e0, e1, 0, a);
    else
        kernel<<<blocks, kBlock, 0, s>>>(a);
}

template <int SPM, typename PT, int VAR>
void dispatch_mode(hipStream_t s, const ForceArgs &a, int blocks, hipEvent_t e0, hipEvent_t e1)
{
    switch (a.mode) {
    case kModeStep: launch_k(k_forces<SPM, PT, kModeStep, false, VAR>, s, a, blocks, e0, e1); break;
    case kModeClose: launch_k(k_forces<SPM, PT, kModeClose, false, VAR>, s, a, blocks, e0, e1); break;
    default:
        if (a.epart)
            launch_k(k_forces<SPM, PT, kModeForce, true, VAR>, s, a, blocks, e0, e1);
        else
            launch_k(k_forces<SPM, PT, kModeForce, false, VAR>, s, a, blocks, e0, e1);
    }
}

template <int SPM, typename PT>
void dispatch_scheme(hipStream_t s, const ForceArgs &a, int blocks, hipEvent_t e0, hipEvent_t e1)
{
    if (a.P.scheme == ADRES_SCHEME_HAMILTONIAN)
        dispatch_mode<SPM, PT, kVarHam>(s, a, blocks, e0, e1);
    else if (a.P.region == ADRES_REGION_SPHERES && a.P.td_n > 0)
        dispatch_mode<SPM, PT, kVarNear>(s, a, blocks, e0, e1);
    else
        dispatch_mode<SPM, PT, kVarForce>(s, a, blocks, e0, e1);
}

template <typename PT>
void dispatch_spm(hipStream_t s, const ForceArgs &a, int blocks, hipEvent_t e0, hipEvent_t e1)
{
    switch (a.P.spm) {
    case 1: dispatch_scheme<1, PT>(s, a, blocks, e0, e1); break;
    case 2: dispatch_scheme<2, PT>(s, a, blocks, e0, e1); break;
    case 3: dispatch_scheme<3, PT>(s, a, blocks, e0, e1); break;
    default: dispatch_scheme<4, PT>(s, a, blocks, e0, e1); break;
    }
}

}  // namespace

int force_blocks(int n_mol) { return (int)(((int64_t)n_mol * kLanes + kBlock - 1) / kBlock); }

int launch_forces(hipStream_t s, const ForceArgs &a, int pair_precision, hipEvent_t e0, hipEvent_t e1)
{
    const int blocks = force_blocks(a.P.n_mol);
    if (pair_precision == 32)
        dispatch_spm<float>(s, a, blocks, e0, e1);
    else
        dispatch_spm<double>(s, a, blocks, e0, e1);
    return blocks;
}

void launch_energy_reduce(hipStream_t s, const double *epart, int n_blocks, double *energy)
{
    k_energy_reduce<<<1, 256, 0, s>>>(epart, n_blocks, energy);
}

}  // namespace adres
