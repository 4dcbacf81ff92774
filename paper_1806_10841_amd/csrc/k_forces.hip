// Force-interpolation kernel, Eq. (1) of Sec. 2.2:
//   F_ab = ww F^AT_ab + (1 - ww) F^CG_ab,  ww = w_a w_b,
// with F^AT the sum of atom-atom WCA forces between the two molecules and F^CG a
// force between their centres of mass, shared among a molecule's sites by mass
// fraction; plus the bonded terms, which are not interpolated (Sec. 2.2, last
// paragraph).  In its step mode the same kernel also finishes velocity Verlet
// for step n (closing half-kick) and starts step n+1 (opening half-kick, drift,
// new centre of mass and the list-displacement check), so one MD step is one launch.
//
// Work mapping (gfx950, wave64): a workgroup is a tile of 64 consecutive Morton slots
// (a compact cluster of cells), four lanes per home molecule.  The tile's neighbour
// halo -- every molecule its rows reference, its own molecules first -- is staged in
// LDS: the raw FP64 site coordinates are copied in with coalesced 16-byte (or 8-byte)
// loads from the positions of step n, then one thread per halo molecule forms its
// centre of mass, weight, largest site distance and (for FP32 pairs) FP32 site offsets
// in place.  The pair loop then reads neighbours from LDS only, through rows of local
// halo indices: a kernel launch has two dependent rounds of global loads (own data and
// row heads, then the halo) instead of a gather chain per list entry, and no derived
// per-molecule array is written to or read from memory.  Lane q takes the molecule's
// entries q, q + 4, ...; every lane accumulates, in FP64, the atom-tile forces on all
// sites of its molecule and the molecule's total CG force; two butterfly shuffles
// combine the four lanes; lane q then owns site q.
//
// Full (two-sided) list: no atomics, fixed summation order, bit-reproducible (the order
// of the halo in LDS does not enter any sum).  Pair arithmetic in PT (double or float).
// In the float variant an atom-pair displacement is the FP64 centre difference rounded
// once to FP32 plus the two sites' FP32 offsets from their centres (|offset| < rho_max),
// which keeps it within a few 1e-7 of the FP64 value without FP64 work per atom pair;
// the CG cutoff is decided on the FP64 centre distance.  The FP64 variant forms every
// displacement from FP64 coordinates.
//
// Workgroups are mapped XCD by XCD: the hardware deals workgroup b to XCD b mod 8,
// so logical block ranges are assigned per XCD and every XCD's L2 serves one
// contiguous stretch of Morton slots (a compact region of space), where neighbouring
// tiles' halos overlap.  An atom tile is skipped when the centres are farther apart
// than rc_at + rho_a + rho_max (rho: largest site distance from the centre), which
// no interacting atom pair can be (triangle inequality).
#include <hip/hip_ext.h>

#include "adres_internal.h"

namespace adres {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 4;   // lanes per home molecule
constexpr int kXcds = 8;
static_assert(kBlock / kLanes == kHaloTile, "a workgroup is one halo tile");

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

// LDS layout of the staged halo, per halo molecule l at hs + l * kStride:
//   FP32 pairs: double4 {R, w} at 0, FP32 site offsets from R (float [SPM][3]) at 32;
//   FP64 pairs: double4 {R, w} at 0, raw FP64 site coordinates ([3][SPM]) at 32, kept for
//     the atom pairs.
// The largest site distance from the centre (rho) is kept for the tile's own molecules only
// (the atom-tile bound takes the neighbour's from rho_max).
template <int SPM, typename PT>
struct Stage {
    static constexpr bool kF32 = sizeof(PT) == 4;
    static constexpr int r16(int b) { return (b + 15) / 16 * 16; }
    static constexpr int kRawOff = 32;
    static constexpr int kOffOff = 32;
    static constexpr int kStride = kF32 ? r16(32 + 12 * SPM) : r16(32 + 24 * SPM);
};

// One molecule's FP64 site coordinates p[k][d] from the SoA rows (16-byte loads when the
// molecule's sites are 16-byte aligned in a row, i.e. an even number of sites).
template <int SPM>
__device__ __forceinline__ void load_molecule(const double *__restrict__ x, int64_t ns, int64_t u,
                                              double (&p)[SPM][3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *row = x + d * ns + u * SPM;
        if constexpr (SPM % 2 == 0) {
#pragma unroll
            for (int k = 0; k < SPM; k += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(row + k);
                p[k][d] = v.x;
                p[k + 1][d] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < SPM; ++k) p[k][d] = row[k];
        }
    }
}

// Whether a molecule with this centre can take part in an atom pair (only then are its FP32
// site offsets needed): with force interpolation both molecules of the pair have a non-zero
// weight, so its distance from the AT centre is below d_at + d_hy; with Eq. (2) one of them
// does, so it lies within that plus the largest centre distance of an atom tile.  A
// self-adjusting region's weights are not known here: always.
__device__ __forceinline__ bool maybe_atomistic(const DevParams &P, const double R[3])
{
    if (P.region == ADRES_REGION_ALL_CG) return false;
    if (P.region != ADRES_REGION_SLAB_X && P.region != ADRES_REGION_SPHERE) return true;
    const double reach = P.scheme == ADRES_SCHEME_HAMILTONIAN ? P.rc_at + 2.0 * P.rho_lim + 1e-6 : 0.0;
    double q[3];
    return res_distance(P, R, q) < P.d_end + reach;
}

// Centre of mass and (FP32 pairs) the FP32 site offsets, or (FP64 pairs) the raw site
// coordinates, of one halo molecule into its LDS record; the weight follows later.  With
// HOME, also rho (the tile's own molecules: the atom-tile bound takes rho_max for the
// neighbour).
template <int SPM, typename PT>
__device__ __forceinline__ double stage_molecule(const DevParams &P, unsigned char *mrec, const double (&p)[SPM][3],
                                                 bool home)
{
    using St = Stage<SPM, PT>;
    double R[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double c[SPM];
#pragma unroll
        for (int k = 0; k < SPM; ++k) c[k] = p[k][d];
        R[d] = com_dim<SPM>(P, c, d);
    }
    double rh = 0.0;
    if (home) {   // the operation order of mol_com
        double rmax2 = 0.0;
#pragma unroll
        for (int k = 0; k < SPM; ++k) {
            const double q0 = mi(p[k][0] - R[0], P.box[0], P.inv_box[0]);
            const double q1 = mi(p[k][1] - R[1], P.box[1], P.inv_box[1]);
            const double q2 = mi(p[k][2] - R[2], P.box[2], P.inv_box[2]);
            const double r2 = dist2_exact(q0, q1, q2);
            rmax2 = r2 > rmax2 ? r2 : rmax2;
        }
        rh = sqrt(rmax2);
    }
    if constexpr (St::kF32) {
        if (SPM > 1 && maybe_atomistic(P, R)) {
            float *od = reinterpret_cast<float *>(mrec + St::kOffOff);
#pragma unroll
            for (int k = 0; k < SPM; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) od[3 * k + d] = (float)mi(p[k][d] - R[d], P.box[d], P.inv_box[d]);
        }
    } else {
        double *raw = reinterpret_cast<double *>(mrec + St::kRawOff);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int k = 0; k < SPM; ++k) raw[d * SPM + k] = p[k][d];
    }
    double *rw = reinterpret_cast<double *>(mrec);
    rw[0] = R[0];
    rw[1] = R[1];
    rw[2] = R[2];
    return rh;
}

// Static LDS beside the halo: home sites, home rho and the energy partials.
constexpr int kStaticLds = (kBlock / kLanes) * kMaxSites * 3 * 8 + (kBlock / kLanes) * 4 + 256;

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
    using St = Stage<SPM, PT>;
    constexpr bool HAM = VAR == kVarHam;
    extern __shared__ __align__(16) unsigned char hs[];   // the tile's staged halo
    const DevParams &P = a.P;
    const int halt = a.ctrl->halt;
    const int n = P.n_mol;
    const int64_t ns = P.n_sites;
    const int slot = xcd_block();   // the dispatch position: the tile's halo, rows and cost order
    const int blk = a.tile_order[slot];   // the tile (its molecules' slots)
    const int q = threadIdx.x % kLanes;
    // the tile's molecules by falling cost: each wavefront's sixteen have similar row work
    // (ml: the molecule's place in the tile, its LDS record and its slot's offset; its row
    // is the thread group's row of the dispatch-ordered rows)
    const int64_t row = (int64_t)slot * kHaloTile + threadIdx.x / kLanes;
    const int ml = a.tperm[row];
    const int t = blk * kHaloTile + ml;
    const bool valid = t < n;
    const int tt = valid ? t : n - 1;

    // the home sites (FP64) for the bonds and the integration, and the home molecules' rho
    __shared__ double sx[kBlock / kLanes][SPM][3];
    __shared__ float srho[kBlock / kLanes];
    // every load that does not depend on another (the tile, the halo count and the first
    // halo ids, each molecule's row length and first local-row entries, the halt index: all
    // stored at the dispatch position) is issued before the first wait; the second round
    // brings the halo's sites (the tile's own molecules first, whose sites also fill sx).
    // Velocities and the reference centre are requested after the pair loop, which keeps
    // the workgroup's LDS within a quarter of the compute unit's (four workgroups per
    // compute unit)
    const int hn = min(a.hn[slot], a.hcap);
    const int *hid = a.hid + (int64_t)slot * a.hcap;
    const int la = threadIdx.x, lb = la + kBlock;
    const int ida = hid[min(la, a.hcap - 1)], idb = hid[min(lb, a.hcap - 1)];
    // (a row longer than cap exists only after an overflow, which stops every launch; the
    // empty tail of a short last tile has length 0)
    const int cnt = min(a.hcnt[row], a.cap);
    const int nq = cnt > q ? (cnt - q + 3) >> 2 : 0;   // this lane's entries k = q + 4 i
    const uint16_t *lrow = a.lnbr + row * a.lcap + q * (a.lcap >> 2);
    uint4 ch = make_uint4(0u, 0u, 0u, 0u);
    if (nq > 0) ch = *reinterpret_cast<const uint4 *>(lrow);
    // the same decision in every wave: only an earlier launch can set halt below this step
    // (this one sets it to its own step at the lowest), so no workgroup stops at a barrier
    if (a.check_halt && a.step > halt) return;

    // stage A: one thread per halo molecule (the tile's own molecules first), two molecules
    // per thread with all their sites requested before the first use: the halo arrives in
    // the second dependent round; then the thread forms the molecule's centre of mass and
    // rho (and the FP32 site offsets) with the operation order of mol_com, so that every
    // tile derives the same bits for a molecule, and stores them in LDS
    {
        // entries at or past the halo count are not written by the halo build: slot 0 instead
        const int64_t ua = la < hn ? ida : 0, ub = lb < hn ? idb : 0;
        double pa[SPM][3], pb[SPM][3];
        load_molecule<SPM>(a.x, ns, ua, pa);
        if (lb < hn) load_molecule<SPM>(a.x, ns, ub, pb);
        if (la < kHaloTile) {   // one of the tile's own molecules (record la, slot base + la)
#pragma unroll
            for (int k = 0; k < SPM; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) sx[la][k][d] = pa[k][d];
        }
        if (la < hn) {
            const double rh = stage_molecule<SPM, PT>(P, hs + la * St::kStride, pa, la < kHaloTile);
            if (la < kHaloTile) srho[la] = (float)rh;
        }
        if (lb < hn) stage_molecule<SPM, PT>(P, hs + lb * St::kStride, pb, false);
    }
    for (int l = 2 * kBlock + threadIdx.x; l < hn; l += kBlock) {   // halos over 512 molecules
        double pc[SPM][3];
        load_molecule<SPM>(a.x, ns, hid[l], pc);
        stage_molecule<SPM, PT>(P, hs + l * St::kStride, pc, false);
    }
    // the weights in a pass of their own, by the thread that staged the molecule, so that
    // the FP64 cosine's registers do not add to those of the centre computation (a
    // self-adjusting region's weights come from the anchor pass)
    for (int l = threadIdx.x; l < hn; l += kBlock) {
        double *rw = reinterpret_cast<double *>(hs + l * St::kStride);
        const double R[3] = {rw[0], rw[1], rw[2]};
        rw[3] = P.region == ADRES_REGION_SPHERES ? a.Rw[hid[l]].w : res_weight(P, R);
    }
    __syncthreads();

    const unsigned char *mine = hs + ml * St::kStride;
    const double4 me = *reinterpret_cast<const double4 *>(mine);
    const double rha = (double)srho[ml];
    constexpr bool kOff = St::kF32;   // FP32 displacements from site offsets
    float hoff[SPM][3] = {};   // (a single site's offset from its centre is exactly zero)
    if constexpr (kOff && SPM > 1) {
        const float *od = reinterpret_cast<const float *>(mine + St::kOffOff);
#pragma unroll
        for (int i = 0; i < SPM; ++i)
#pragma unroll
            for (int d = 0; d < 3; ++d) hoff[i][d] = od[3 * i + d];
    }
#define XI(i, d) (reinterpret_cast<const double *>(mine + St::kRawOff)[(d) * SPM + (i)])

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
    const bool with_slow = a.slow_scale != 0.0;

    for (int i = 0; i < nq; ++i) {
        const int j8 = i & 7;
        if (j8 == 0 && i > 0) ch = *reinterpret_cast<const uint4 *>(lrow + i);   // rows over 32 entries
        const unsigned wd = j8 < 2 ? ch.x : (j8 < 4 ? ch.y : (j8 < 6 ? ch.z : ch.w));
        const int l = (int)((wd >> (16 * (j8 & 1))) & 0xffffu);
        const int k = q + 4 * i;   // the entry's position in the row
        const unsigned char *nrec = hs + l * St::kStride;
        const double4 o = *reinterpret_cast<const double4 *>(nrec);
        const double ww = HAM ? 0.5 * (me.w + o.w) : me.w * o.w;   // weight of the AT part
        const double D0 = mi(me.x - o.x, P.box[0], P.inv_box[0]);
        const double D1 = mi(me.y - o.y, P.box[1], P.inv_box[1]);
        const double D2 = mi(me.z - o.z, P.box[2], P.inv_box[2]);
        const double r2c = dist2_exact(D0, D1, D2);
        if (ww > 0.0) {
            // no atom pair of the tile can be within the cutoff beyond this centre
            // distance (every site lies within rho_lim of its centre, a checked invariant)
            const double bound = P.rc_at + rha + P.rho_lim + 1e-6;
            if (r2c < bound * bound) {
                const PT pww = (PT)ww;
                if constexpr (kOff) {
                    const float *od = reinterpret_cast<const float *>(nrec + St::kOffOff);
                    // a neighbour site's FP32 offset (zero for single-site molecules, not stored)
                    auto nof = [od](int j) { return SPM > 1 ? od[j] : 0.0f; };
                    // D + (off_i - off_jj): the same bits with opposite sign from the
                    // other molecule's side, so pair forces cancel exactly (Newton's third law)
                    const float Df0 = (float)D0, Df1 = (float)D1, Df2 = (float)D2;
                    const float rcf = (float)rcA2;
                    // first pass: which of the tile's SPM x SPM atom pairs may be inside the
                    // cutoff (bit SPM ii + jj); few are, and the lanes of a wavefront disagree.
                    // The displacement is regrouped as (D - off_jj) + off_i (one subtraction per
                    // neighbour site) and tested against a cutoff padded by 2^-16 of r^2, far
                    // more than the few-ulp difference of the two groupings: a superset of the
                    // pairs inside, which the second pass tests exactly
                    const float rct = rcf * (1.0f + 1.0f / 65536.0f);
                    unsigned inside = 0u;
#pragma unroll
                    for (int jj = 0; jj < SPM; ++jj) {
                        const float e0 = Df0 - nof(3 * jj), e1 = Df1 - nof(3 * jj + 1),
                                    e2 = Df2 - nof(3 * jj + 2);
#pragma unroll
                        for (int ii = 0; ii < SPM; ++ii) {
                            const float dx = e0 + hoff[ii][0];
                            const float dy = e1 + hoff[ii][1];
                            const float dz = e2 + hoff[ii][2];
                            const float r2 = (dx * dx + dy * dy) + dz * dz;
                            inside |= (r2 < rct ? 1u : 0u) << (SPM * ii + jj);
                        }
                    }
                    // second pass: the exact test and the WCA force for the pairs the mask
                    // kept, in one loop over them (a wavefront runs it as often as its
                    // busiest lane has pairs), each term added to its site's FP64 sum; my
                    // site's offset is read from my LDS record by index
                    const float *myo = reinterpret_cast<const float *>(mine + St::kOffOff);
                    auto hof = [myo](int j) { return SPM > 1 ? myo[j] : 0.0f; };   // (single site: 0)
                    unsigned m = inside;
                    while (m) {
                        const int b = __builtin_ctz(m);
                        m &= m - 1u;
                        const int ii = b / SPM, jj = b % SPM;
                        const float dx = Df0 + (hof(3 * ii) - nof(3 * jj));
                        const float dy = Df1 + (hof(3 * ii + 1) - nof(3 * jj + 1));
                        const float dz = Df2 + (hof(3 * ii + 2) - nof(3 * jj + 2));
                        const float r2 = (dx * dx + dy * dy) + dz * dz;
                        if (!(r2 < rcf)) continue;
                        PT uu = PT(0);
                        const PT c = pww * wca_f_over_r<PT>((PT)r2, sig2A, epsA, uu, ENERGY || hy_home);
                        const double vx = (double)(c * dx), vy = (double)(c * dy), vz = (double)(c * dz);
#pragma unroll
                        for (int k2 = 0; k2 < SPM; ++k2)
                            if (k2 == ii) {
                                acc[k2][0] += vx;
                                acc[k2][1] += vy;
                                acc[k2][2] += vz;
                            }
                        if (ENERGY) uat += 0.5 * (HAM ? me.w : ww) * (double)uu;
                        if (HAM) vat += 0.5 * (double)uu;
                    }
                } else {
                    const double *xj = reinterpret_cast<const double *>(nrec + St::kRawOff);
#pragma unroll 1
                    for (int jj = 0; jj < SPM; ++jj) {
                        const double xj0 = xj[jj], xj1 = xj[SPM + jj], xj2 = xj[2 * SPM + jj];
#pragma unroll
                        for (int ii = 0; ii < SPM; ++ii) {
                            const PT dx = (PT)mi(XI(ii, 0) - xj0, P.box[0], P.inv_box[0]);
                            const PT dy = (PT)mi(XI(ii, 1) - xj1, P.box[1], P.inv_box[1]);
                            const PT dz = (PT)mi(XI(ii, 2) - xj2, P.box[2], P.inv_box[2]);
                            const PT r2 = (dx * dx + dy * dy) + dz * dz;
                            if (r2 < rcA2) {
                                PT uu = PT(0);
                                const PT c = pww * wca_f_over_r<PT>(r2, sig2A, epsA, uu, ENERGY || hy_home);
                                acc[ii][0] += (double)(c * dx);
                                acc[ii][1] += (double)(c * dy);
                                acc[ii][2] += (double)(c * dz);
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
                const float fv = a.f_pair[a.pid[(int64_t)tt * a.cap + k]];
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
#undef XI

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

    // the velocity and the reference centre, requested before the bonds and the correction
    // field so that their arithmetic covers the load
    double lv[3] = {0.0, 0.0, 0.0};
    if (MODE != kModeForce && q < SPM)
#pragma unroll
        for (int d = 0; d < 3; ++d) lv[d] = a.v[d * ns + (int64_t)tt * SPM + q];
    double4 lref = make_double4(0.0, 0.0, 0.0, 0.0);
    if (MODE == kModeStep && q == 0) lref = a.R_ref[tt];

#define XS(k, d) sx[ml][(k)][(d)]

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
            xq[0] = XS(i, 0); xq[1] = XS(i, 1); xq[2] = XS(i, 2);
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
                const double d0 = mi(xq[0] - XS(k, 0), P.box[0], P.inv_box[0]);
                const double d1 = mi(xq[1] - XS(k, 1), P.box[1], P.inv_box[1]);
                const double d2 = mi(xq[2] - XS(k, 2), P.box[2], P.inv_box[2]);
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
                const double d0 = mi(xq[0] - a.x[(int64_t)ub * SPM], P.box[0], P.inv_box[0]);
                const double d1 = mi(xq[1] - a.x[ns + (int64_t)ub * SPM], P.box[1], P.inv_box[1]);
                const double d2 = mi(xq[2] - a.x[2 * ns + (int64_t)ub * SPM], P.box[2], P.inv_box[2]);
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
            double v[3] = {lv[0], lv[1], lv[2]};
            close_kick(v, F, a.st.dt, iq);
            a.v[site] = v[0]; a.v[ns + site] = v[1]; a.v[2 * ns + site] = v[2];
            a.f[site] = F[0]; a.f[ns + site] = F[1]; a.f[2 * ns + site] = F[2];
        }
    } else {   // kModeStep
        double xn[3] = {xq[0], xq[1], xq[2]};
        if (owner) {
            double v[3] = {lv[0], lv[1], lv[2]};
            close_kick(v, F, a.st.dt, iq);
            const int caller_site = a.st.gamma > 0.0 ? a.perm[t] * SPM + q : 0;
            open_and_drift(P, mq, iq, caller_site, xn, v, F, a.st.dt, a.st.gamma, a.st.kT, a.st.seed, a.st.step_abs);
            a.v[site] = v[0]; a.v[ns + site] = v[1]; a.v[2 * ns + site] = v[2];
            a.x_out[site] = xn[0]; a.x_out[ns + site] = xn[1]; a.x_out[2 * ns + site] = xn[2];
        }
        // new centre (for the displacement check, and stored when something reads it before
        // the next list build) and rho (for the stretch check), spread over the quad: lane
        // d < 3 forms coordinate d of the centre (the operation order of mol_com), lane
        // q < SPM its own site's distance
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
            const double o0 = mi(xn[0] - R0, P.box[0], P.inv_box[0]);
            const double o1 = mi(xn[1] - R1, P.box[1], P.inv_box[1]);
            const double o2 = mi(xn[2] - R2, P.box[2], P.inv_box[2]);
            r2 = dist2_exact(o0, o1, o2);
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
            if (a.Rw_out) a.Rw_out[t] = make_double4(R0, R1, R2, res_weight(P, R));
            if (!(isfinite(R0) && isfinite(R1) && isfinite(R2))) atomicOr(&a.ctrl->err, kErrNonFinite);
            if (SPM > 1 && rh > P.rho_lim) atomicOr(&a.ctrl->err, kErrStretch);
            const double4 rr = lref;
            const double q0 = mi(R0 - rr.x, P.box[0], P.inv_box[0]);
            const double q1 = mi(R1 - rr.y, P.box[1], P.inv_box[1]);
            const double q2 = mi(R2 - rr.z, P.box[2], P.inv_box[2]);
            const double d2 = dist2_exact(q0, q1, q2);
            bool stale = list_stale(P, d2, SPM > 1 ? rh : 0.0);
            // (rare) a molecule that the next evaluation gives weight zero (its distance from
            // the AT region past the hybrid layer's end, with a margin far above the last
            // bits) has the CG cutoff's budget alone, which is at least list_stale's
            if (stale && P.w0_cg) {
                double qd[3];
                if (res_distance(P, R, qd) > P.d_end + 1e-9) stale = d2 > P.cg_half * P.cg_half;
            }
            if (stale) atomicMin(&a.ctrl->halt, a.step);
        }
    }

#undef XS
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
void launch_k(K kernel, hipStream_t s, const ForceArgs &a, int blocks, size_t lds, hipEvent_t e0, hipEvent_t e1)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlock), lds, s, e0, e1, 0, a);
    else
        kernel<<<blocks, kBlock, lds, s>>>(a);
}

template <int SPM, typename PT, int VAR>
void dispatch_mode(hipStream_t s, const ForceArgs &a, int blocks, hipEvent_t e0, hipEvent_t e1)
{
    const size_t lds = (size_t)a.hcap * Stage<SPM, PT>::kStride;
    switch (a.mode) {
    case kModeStep: launch_k(k_forces<SPM, PT, kModeStep, false, VAR>, s, a, blocks, lds, e0, e1); break;
    case kModeClose: launch_k(k_forces<SPM, PT, kModeClose, false, VAR>, s, a, blocks, lds, e0, e1); break;
    default:
        if (a.epart)
            launch_k(k_forces<SPM, PT, kModeForce, true, VAR>, s, a, blocks, lds, e0, e1);
        else
            launch_k(k_forces<SPM, PT, kModeForce, false, VAR>, s, a, blocks, lds, e0, e1);
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

namespace {
template <typename PT>
int stride_of(int spm)
{
    switch (spm) {
    case 1: return Stage<1, PT>::kStride;
    case 2: return Stage<2, PT>::kStride;
    case 3: return Stage<3, PT>::kStride;
    default: return Stage<4, PT>::kStride;
    }
}
}  // namespace

int halo_stride_bytes(int spm, int pair_precision)
{
    return pair_precision == 32 ? stride_of<float>(spm) : stride_of<double>(spm);
}

// a workgroup's LDS is 64 KiB: the static part and the staged halo share it
int halo_capacity_limit(int spm, int pair_precision)
{
    return (65536 - kStaticLds) / halo_stride_bytes(spm, pair_precision);
}

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
