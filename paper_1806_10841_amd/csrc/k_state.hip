// Per-molecule streaming kernels: centres of mass and resolution weights
// (Sec. 2.2), gathers into / scatters out of the Morton-ordered state, and the
// opening half of the first velocity-Verlet step.  One thread per molecule; a
// molecule's sites are contiguous in each SoA row, so a wavefront touches
// 64 * s * 8 consecutive bytes of a row per access.
#include "adres_internal.h"

#include <algorithm>
#include <climits>

namespace adres {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

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
    bool finite = true;
#pragma unroll
    for (int k = 0; k < SPM; ++k) finite = finite && isfinite(p[k][0]) && isfinite(p[k][1]) && isfinite(p[k][2]);
    if (!finite) atomicOr(&ctrl->err, kErrNonFinite);
    if (SPM > 1 && rh > P.rho_lim) atomicOr(&ctrl->err, kErrStretch);
}

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_gather(DevParams P, const double *__restrict__ xc,
                                                   const double *__restrict__ vc, StateBufs S,
                                                   const double4 *__restrict__ R_ref, Ctrl *ctrl)
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
    store_molecule<SPM>(P, p, t, S.Rw, R_ref, ctrl, 0);
}

// Centres and weights of the sorted state from its positions (no checks: the step kernel
// that wrote the positions made them), fused with the cell keys of the reorder that
// follows (what k_cell_keys derives from Rw): one pass over the positions instead of two.
// The weight of a self-adjusting region is written by its own pass and kept.
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_centres_keys(const int *__restrict__ go, DevParams P, Grid G, const int *__restrict__ cell_rank,
                                                         const double *__restrict__ x, double4 *__restrict__ Rw,
                                                         int *__restrict__ key, int *__restrict__ count,
                                                         const double *__restrict__ x_alt, double4 *__restrict__ Rw_alt,
                                                         ChainHead head)
{
    bool sw;   // the chunk's positions sit in the other buffer
    if (!chain_go(head, go, sw)) return;   // a guarded rebuild that was not asked for
    if (sw) {
        x = x_alt;
        Rw = Rw_alt;
    }
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    double p[SPM][3];
    load_sites<SPM>(x, P.n_sites, t, p);
    double R[3], rh;
    mol_com<SPM>(P, p, R, rh);
    const double w = P.region == ADRES_REGION_SPHERES ? Rw[t].w : res_weight(P, R);
    Rw[t] = make_double4(R[0], R[1], R[2], w);
    const int cx = cell_coord(R[0], G.inv_len[0], G.n[0]);
    const int cy = cell_coord(R[1], G.inv_len[1], G.n[1]);
    const int cz = cell_coord(R[2], G.inv_len[2], G.n[2]);
    const int k = cell_rank[cx + G.n[0] * (cy + G.n[1] * cz)];
    key[t] = k;
    atomicAdd(&count[k], 1);
}

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_scatter_out(DevParams P, const int *__restrict__ perm,
                                                        const double *__restrict__ x, const double *__restrict__ v,
                                                        const double *__restrict__ f, double *__restrict__ xc,
                                                        double *__restrict__ vc, double *__restrict__ fc)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    int a = perm[t];
    double p[SPM][3];
    if (xc) {
        load_sites<SPM>(x, P.n_sites, t, p);
        store_sites<SPM>(xc, P.n_sites, a, p);
    }
    if (vc) {
        load_sites<SPM>(v, P.n_sites, t, p);
        store_sites<SPM>(vc, P.n_sites, a, p);
    }
    if (fc) {
        load_sites<SPM>(f, P.n_sites, t, p);
        store_sites<SPM>(fc, P.n_sites, a, p);
    }
}

// Opening half of a step (kick with F(x_in), drift) for every site of a molecule,
// then its new centre, weight and rho; skipped once an earlier step of the chunk
// asked for a list rebuild.
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_kick_drift(DevParams P, const double *__restrict__ x_in,
                                                       double *__restrict__ v, const double *__restrict__ f,
                                                       double *__restrict__ x_out, double4 *__restrict__ Rw_out,
                                                       const double4 *__restrict__ R_ref,
                                                       const int *__restrict__ perm, Ctrl *ctrl, int step,
                                                       StepArgs st)
{
    if (step > ctrl->halt) return;
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    const int64_t ns = P.n_sites;
    double p[SPM][3];
    const int caller0 = st.gamma > 0.0 ? perm[t] * SPM : 0;
#pragma unroll
    for (int k = 0; k < SPM; ++k) {
        const int64_t i = (int64_t)t * SPM + k;
        double xx[3] = {x_in[i], x_in[ns + i], x_in[2 * ns + i]};
        double vv[3] = {v[i], v[ns + i], v[2 * ns + i]};
        const double F[3] = {f[i], f[ns + i], f[2 * ns + i]};
        open_and_drift(P, P.mass[k], P.inv_2m[k], caller0 + k, xx, vv, F, st.dt, st.gamma, st.kT, st.seed, st.step_abs);
        for (int d = 0; d < 3; ++d) {
            v[d * ns + i] = vv[d];
            x_out[d * ns + i] = xx[d];
            p[k][d] = xx[d];
        }
    }
    store_molecule<SPM>(P, p, t, Rw_out, R_ref, ctrl, step);
}

// Centre of mass and summed force of every molecule (caller order): the mapping of
// site forces onto the CG sites used as force-matching targets.
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_map_cg(DevParams P, const double *__restrict__ x,
                                                   const double *__restrict__ f, double *__restrict__ com,
                                                   double *__restrict__ fmap)
{
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= P.n_mol) return;
    double p[SPM][3], q[SPM][3];
    load_sites<SPM>(x, P.n_sites, a, p);
    load_sites<SPM>(f, P.n_sites, a, q);
    double R[3], rh;
    mol_com<SPM>(P, p, R, rh);
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < SPM; ++k) s += q[k][d];
        com[(int64_t)d * P.n_mol + a] = R[d];
        fmap[(int64_t)d * P.n_mol + a] = s;
    }
}

// Density profile along the resolution coordinate (Sec. 2.4), in the bins of the
// installed correction table: centre of mass (the operation order of the weights), its
// distance d from the AT centre, bin floor((d - lo) / h) (the top bin also takes a d that
// rounds to n below hi), counted per workgroup in LDS and added to the int64 totals.
// Bin index of a resolution distance in the correction table's bins, or -1 outside them.
__device__ __forceinline__ int td_bin(const DevParams &P, double d)
{
    if (!(d >= P.td_lo && d < P.td_hi)) return -1;
    const double u = floor((d - P.td_lo) / P.td_h);
    return u < (double)(P.td_n - 1) ? (int)u : P.td_n - 1;
}

// Distance from the nearest of the K anchor centres staged in LDS (the first of equally
// near ones).
__device__ __forceinline__ double nearest_anchor(const DevParams &P, const double (*cen)[3], int K, const double R[3])
{
#pragma clang fp contract(off)
    double best = INFINITY;
    for (int k = 0; k < K; ++k) {
        const double q0 = mi(R[0] - cen[k][0], P.box[0], P.inv_box[0]);
        const double q1 = mi(R[1] - cen[k][1], P.box[1], P.inv_box[1]);
        const double q2 = mi(R[2] - cen[k][2], P.box[2], P.inv_box[2]);
        const double r2 = dist2_exact(q0, q1, q2);
        best = r2 < best ? r2 : best;
    }
    return sqrt(best);
}

// Density profile along the resolution coordinate (Sec. 2.4), in the bins of the
// installed correction table: centre of mass (the operation order of the weights), its
// distance d from the AT centre (for anchor spheres: from the nearest anchor centre, given
// in cen [K][3]), bin floor((d - lo) / h) (the top bin also takes a d that rounds to n
// below hi), counted per workgroup in LDS and added to the int64 totals.
template <int SPM>
__global__ __launch_bounds__(kBlock) void k_density_profile(DevParams P, const double *__restrict__ x,
                                                            const double *__restrict__ cen,
                                                            unsigned long long *__restrict__ counts)
{
    __shared__ unsigned hist[kTdMaxBins];
    __shared__ double scen[kMaxAnchors][3];
    const int nb = P.td_n;
    const int K = cen ? P.n_anchors : 0;
    for (int b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0u;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        scen[k][0] = cen[3 * k];
        scen[k][1] = cen[3 * k + 1];
        scen[k][2] = cen[3 * k + 2];
    }
    __syncthreads();
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a < P.n_mol) {
        double p[SPM][3];
        load_sites<SPM>(x, P.n_sites, a, p);
        double R[3], rh, q[3];
        mol_com<SPM>(P, p, R, rh);
        const double d = cen ? nearest_anchor(P, scen, K, R) : res_distance(P, R, q);
        const int k = td_bin(P, d);
        if (k >= 0) atomicAdd(&hist[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kBlock)
        if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

// Centres of mass of the anchor molecules of a caller-order configuration: cen [K][3].
template <int SPM>
__global__ void k_anchor_centres(DevParams P, const double *__restrict__ x, double *__restrict__ cen)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_anchors) return;
    double p[SPM][3];
    load_sites<SPM>(x, P.n_sites, P.anchors[k], p);
    double R[3], rh;
    mol_com<SPM>(P, p, R, rh);
    cen[3 * k] = R[0];
    cen[3 * k + 1] = R[1];
    cen[3 * k + 2] = R[2];
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the finaliser applied to
// s + (k + 1) * 0x9E3779B97F4A7C15, the output for counter value k of stream key s.
__device__ __forceinline__ uint64_t splitmix64(uint64_t s, uint64_t k)
{
    uint64_t z = s + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Bin volumes by sampling (for bins without closed-form volumes, e.g. a union of moving
// spheres): point i has coordinate c = L_c * (top 53 bits of SplitMix64(seed, 3 i + c)) / 2^53,
// binned by its resolution distance like a centre of mass.  Grid-stride over the points,
// LDS histogram per workgroup, int64 totals.
__global__ __launch_bounds__(kBlock) void k_region_volumes(DevParams P, const double *__restrict__ cen,
                                                           long long n_samples, unsigned long long seed,
                                                           unsigned long long *__restrict__ counts)
{
#pragma clang fp contract(off)
    __shared__ unsigned hist[kTdMaxBins];
    __shared__ double scen[kMaxAnchors][3];
    const int nb = P.td_n;
    const int K = cen ? P.n_anchors : 0;
    for (int b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0u;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        scen[k][0] = cen[3 * k];
        scen[k][1] = cen[3 * k + 1];
        scen[k][2] = cen[3 * k + 2];
    }
    __syncthreads();
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n_samples;
         i += (long long)gridDim.x * kBlock) {
        double pnt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint64_t z = splitmix64(seed, 3ull * (uint64_t)i + (uint64_t)c);
            pnt[c] = P.box[c] * ((double)(z >> 11) * 0x1.0p-53);
        }
        double q[3];
        const double d = cen ? nearest_anchor(P, scen, K, pnt) : res_distance(P, pnt, q);
        const int k = td_bin(P, d);
        if (k >= 0) atomicAdd(&hist[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kBlock)
        if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

// One refinement of the correction force from accumulated counts (Sec. 2.4): number
// density per bin (counts / (n_frames V_k), V_k the slab pair of bins 2 h L_y L_z or the
// spherical shell 4/3 pi (r_k+1^3 - r_k^3)), its central-difference slope (one-sided at
// the end bins), F_k -= prefactor * slope_k; then the integrals of the interpolated force
// from lo to each bin centre for the potential.  counts == nullptr only recomputes the
// integrals.  One workgroup; n <= kTdMaxBins.
__global__ __launch_bounds__(kBlock) void k_td_update(DevParams P, double *__restrict__ td, double *__restrict__ td_u,
                                                      const long long *__restrict__ counts, long long n_frames,
                                                      double prefactor, const long long *__restrict__ vol,
                                                      long long n_vol)
{
#pragma clang fp contract(off)
    __shared__ double rho[kTdMaxBins];
    const int n = P.td_n;
    const double h = P.td_h, lo = P.td_lo;
    if (counts) {
        for (int k = threadIdx.x; k < n; k += kBlock) {
            double V;
            if (vol) {   // sampled volumes; an unsampled bin counts as empty
                V = ((double)vol[k] / (double)n_vol) * ((P.box[0] * P.box[1]) * P.box[2]);
                if (vol[k] == 0) {
                    rho[k] = 0.0;
                    continue;
                }
            } else if (P.region == ADRES_REGION_SLAB_X) {
                V = 2.0 * h * P.box[1] * P.box[2];
            } else {
                const double r0 = lo + k * h, r1 = lo + (k + 1) * h;
                V = (4.0 / 3.0) * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
            }
            rho[k] = (double)counts[k] / ((double)n_frames * V);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < n; k += kBlock) {
            double slope;
            if (n == 1) slope = 0.0;
            else if (k == 0) slope = (rho[1] - rho[0]) / h;
            else if (k == n - 1) slope = (rho[n - 1] - rho[n - 2]) / h;
            else slope = (rho[k + 1] - rho[k - 1]) / (2.0 * h);
            td[k] = td[k] - prefactor * slope;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // integral from lo to the first centre (the held end value), then trapezoids
        double acc = td[0] * (0.5 * h);
        td_u[0] = acc;
        for (int k = 0; k + 1 < n; ++k) {
            acc = acc + 0.5 * (td[k] + td[k + 1]) * h;
            td_u[k + 1] = acc;
        }
    }
}

// Self-adjusting AT region (Sec. 2.5): each molecule's weight from the minimum-image
// distance to the nearest anchor centre, d = min_k |R - A_k|.  Only distances up to reach
// (the end of the hybrid shell, or of the correction table if that is longer) change a
// result: beyond it the weight is 0, the correction force 0 and its potential the table's
// held value.  Every workgroup bins the anchors' centres in LDS on a grid of cells at least
// reach wide (nc[d] per axis, at most kAnchorGrid), a counting sort by cell; a molecule
// then visits the cells within one of its own (all of them along an axis of fewer than
// three cells), which hold every anchor within reach of it: nine rows of cells, each as
// at most two runs of consecutive cells, shared by the molecule's four lanes and merged by
// a quad reduction.  Equally near anchors resolve to the lowest anchor index, so within
// reach the result is the same, bit for bit, as a search over all anchors in index order;
// beyond it the distance found is only known to exceed reach (infinite if no anchor was
// visited).  Morton-ordered state: the anchors' slots (aslot) change only when the state is
// reordered; a launch with refresh takes them from inv_perm and workgroup 0 stores them
// for the launches that follow.  Only the w component of Rw is written (centres are read as
// three scalars, so the stores never overlap a read).  Dynamic LDS: anchor_lds_bytes.
__device__ __forceinline__ int anchor_cell(double r, double L, double inv_L, int nc)
{
    const double u = r - L * floor(r * inv_L);   // wrapped into [0, L] (the cell only has to be
    const int c = (int)(u * (nc * inv_L));        // the same function for both sides)
    return c < 0 ? 0 : (c < nc ? c : nc - 1);
}

constexpr int kAnchorLanes = 4;
constexpr int kAnchorMols = kBlock / kAnchorLanes;

__host__ __device__ inline size_t anchor_lds_bytes(int K, int n_cells)
{
    return (size_t)K * 24 + (size_t)(2 * n_cells + 1) * 4 + (size_t)K * 4 + 16;
}

__global__ __launch_bounds__(kBlock) void k_anchor_weights(const int *__restrict__ go, DevParams P, double4 *Rw, const int *__restrict__ inv_perm,
                                                           int *aslot, int refresh, Ctrl *ctrl, int step,
                                                           int check_halt, double4 *__restrict__ near, int3 nc,
                                                           double4 *Rw_alt)
{
#pragma clang fp contract(off)
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    // (go points at Ctrl::go, followed by Ctrl::fix: the chunk's positions sit in the other buffer)
    const bool sw = go && go[1] != 0;
    if (sw) Rw = Rw_alt;
    extern __shared__ __align__(16) unsigned char als[];
    __shared__ int wsum[kBlock / 64];
    const int K = P.n_anchors;
    const int n_cells = nc.x * nc.y * nc.z;
    double(*cen)[3] = reinterpret_cast<double(*)[3]>(als);
    int *ccount = reinterpret_cast<int *>(als + (size_t)K * 24);
    int *cstart = ccount + n_cells;
    unsigned short *sorted = reinterpret_cast<unsigned short *>(cstart + n_cells + 1);
    unsigned short *cell_of = sorted + K;
    const int q = threadIdx.x & (kAnchorLanes - 1);
    const int t = blockIdx.x * kAnchorMols + threadIdx.x / kAnchorLanes;
    const bool active = t < P.n_mol;
    double *me = reinterpret_cast<double *>(Rw + (active ? t : 0));
    const double R0 = me[0], R1 = me[1], R2 = me[2];
    const int halt = check_halt ? ctrl->halt : INT_MAX;
    for (int c = threadIdx.x; c < n_cells; c += kBlock) ccount[c] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
        const int sl = refresh ? inv_perm[P.anchors[k]] : aslot[k];
        if (refresh && blockIdx.x == 0) aslot[k] = sl;
        const double *r = reinterpret_cast<const double *>(Rw + sl);
        const double a0 = r[0], a1 = r[1], a2 = r[2];
        cen[k][0] = a0;
        cen[k][1] = a1;
        cen[k][2] = a2;
        const int c = (anchor_cell(a2, P.box[2], P.inv_box[2], nc.z) * nc.y +
                       anchor_cell(a1, P.box[1], P.inv_box[1], nc.y)) * nc.x +
                      anchor_cell(a0, P.box[0], P.inv_box[0], nc.x);
        cell_of[k] = (unsigned short)c;
        atomicAdd(&ccount[c], 1);
    }
    // the same decision in every workgroup, before a barrier it would skip: only an
    // earlier launch sets halt
    if (step > halt) return;
    __syncthreads();
    // exclusive scan of the counts: each thread sums a run of consecutive cells
    {
        const int run = (n_cells + kBlock - 1) / kBlock;
        const int c0 = threadIdx.x * run;
        int s = 0;
        for (int i = 0; i < run; ++i) s += c0 + i < n_cells ? ccount[c0 + i] : 0;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        int incl = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int before = incl - s;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        for (int i = 0; i < run && c0 + i < n_cells; ++i) {
            cstart[c0 + i] = before;
            before += ccount[c0 + i];
        }
        if (threadIdx.x == 0) cstart[n_cells] = K;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
        const int c = cell_of[k];
        sorted[cstart[c] + atomicSub(&ccount[c], 1) - 1] = (unsigned short)k;
    }
    __syncthreads();
    // the cells to visit along each axis: c-1, c, c+1 (periodic), or all of a short axis;
    // along x as at most two runs of consecutive cells
    const int cx = anchor_cell(R0, P.box[0], P.inv_box[0], nc.x);
    const int cy = anchor_cell(R1, P.box[1], P.inv_box[1], nc.y);
    const int cz = anchor_cell(R2, P.box[2], P.inv_box[2], nc.z);
    int xa, xb, xc = 0, xd = 0;
    if (nc.x < 3) { xa = 0; xb = nc.x; }
    else if (cx == 0) { xa = 0; xb = 2; xc = nc.x - 1; xd = nc.x; }
    else if (cx == nc.x - 1) { xa = nc.x - 2; xb = nc.x; xc = 0; xd = 1; }
    else { xa = cx - 1; xb = cx + 2; }
    const int ny = nc.y < 3 ? nc.y : 3, nz = nc.z < 3 ? nc.z : 3;
    auto nb = [](int c, int n, int i) {   // the i-th visited cell along an axis
        if (n < 3) return i;
        const int v = c - 1 + i;
        return v < 0 ? v + n : (v >= n ? v - n : v);
    };
    double best = INFINITY, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    int bk = INT_MAX;
    if (active) {
        for (int r = q; r < 9; r += kAnchorLanes) {   // this lane's rows of the nine
            const int iz = r / 3, iy = r - 3 * iz;
            if (iz >= nz || iy >= ny) continue;
            const int row = (nb(cz, nc.z, iz) * nc.y + nb(cy, nc.y, iy)) * nc.x;
            for (int h = 0; h < 2; ++h) {
                if (h && xc == xd) break;
                const int j0 = cstart[row + (h ? xc : xa)], j1 = cstart[row + (h ? xd : xb)];
                for (int j = j0; j < j1; ++j) {
                    const int k = sorted[j];
                    const double q0 = mi(R0 - cen[k][0], P.box[0], P.inv_box[0]);
                    const double q1 = mi(R1 - cen[k][1], P.box[1], P.inv_box[1]);
                    const double q2 = mi(R2 - cen[k][2], P.box[2], P.inv_box[2]);
                    const double r2 = dist2_exact(q0, q1, q2);
                    if (r2 < best || (r2 == best && k < bk)) {   // the first of equally near
                        best = r2;
                        bk = k;
                        b0 = q0; b1 = q1; b2 = q2;
                    }
                }
            }
        }
    }
    // the least (r2, k) of the quad's four lanes, in every lane
#pragma unroll
    for (int m = 1; m < kAnchorLanes; m <<= 1) {
        const double ob = __shfl_xor(best, m), o0 = __shfl_xor(b0, m), o1 = __shfl_xor(b1, m),
                     o2 = __shfl_xor(b2, m);
        const int ok = __shfl_xor(bk, m);
        if (ob < best || (ob == best && ok < bk)) {
            best = ob;
            bk = ok;
            b0 = o0; b1 = o1; b2 = o2;
        }
    }
    if (!active || q != 0) return;
    const double d = sqrt(best);
    me[3] = weight_of_distance(P, d);
    if (near) near[t] = make_double4(b0, b1, b2, d);
}

// The same for caller-order centres com [3][n_mol] into w [n_mol].
__global__ __launch_bounds__(kBlock) void k_anchor_weights_caller(DevParams P, const double *__restrict__ com,
                                                                  double *__restrict__ w)
{
#pragma clang fp contract(off)
    __shared__ double cen[kMaxAnchors][3];
    const int K = P.n_anchors;
    const int64_t n = P.n_mol;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        const int b = P.anchors[k];
        cen[k][0] = com[b];
        cen[k][1] = com[n + b];
        cen[k][2] = com[2 * n + b];
    }
    __syncthreads();
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= P.n_mol) return;
    const double R0 = com[a], R1 = com[n + a], R2 = com[2 * n + a];
    double best = INFINITY;
    for (int k = 0; k < K; ++k) {
        const double q0 = mi(R0 - cen[k][0], P.box[0], P.inv_box[0]);
        const double q1 = mi(R1 - cen[k][1], P.box[1], P.inv_box[1]);
        const double q2 = mi(R2 - cen[k][2], P.box[2], P.inv_box[2]);
        const double r2 = dist2_exact(q0, q1, q2);
        best = r2 < best ? r2 : best;
    }
    w[a] = weight_of_distance(P, sqrt(best));
}

__global__ void k_publish(Ctrl *__restrict__ ctrl, CtrlPub *pub, unsigned seq)
{
    if (threadIdx.x != 0) return;
    const int v[kPubFields] = {ctrl->halt, ctrl->err, ctrl->overflow, ctrl->max_count, ctrl->max_halo};
#pragma unroll
    for (int i = 0; i < kPubFields; ++i)
        __hip_atomic_store(&pub->w[i], ((unsigned long long)seq << 32) | (unsigned)v[i], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}


// clears the halt index and the list-overflow report (a fill kernel, so that no
// memset node is needed between the launches of a step loop)
__global__ void k_reset_halt(Ctrl *ctrl)
{
    if (threadIdx.x == 0) {
        ctrl->halt = INT_MAX;
        ctrl->overflow = 0;
        ctrl->max_count = 0;
        ctrl->max_halo = 0;
    }
}

}  // namespace

#define ADRES_SPM_DISPATCH(spm, CALL)                  \
    switch (spm) {                                     \
    case 1: { constexpr int S_ = 1; CALL; } break;     \
    case 2: { constexpr int S_ = 2; CALL; } break;     \
    case 3: { constexpr int S_ = 3; CALL; } break;     \
    default: { constexpr int S_ = 4; CALL; } break;    \
    }

void launch_weights_caller(hipStream_t s, const DevParams &P, const double *x, double *com, double *w,
                           Ctrl *ctrl)
{
    ADRES_SPM_DISPATCH(P.spm, (k_weights_caller<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x, com, w, ctrl)));
}

void launch_gather(hipStream_t s, const DevParams &P, const double *x_caller, const double *v_caller,
                   const StateBufs &S, const double4 *R_ref, Ctrl *ctrl)
{
    ADRES_SPM_DISPATCH(P.spm,
                       (k_gather<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x_caller, v_caller, S, R_ref, ctrl)));
}

void launch_scatter_out(hipStream_t s, const DevParams &P, const int *perm, const double *x, const double *v,
                        const double *f, double *x_caller, double *v_caller, double *f_caller)
{
    ADRES_SPM_DISPATCH(P.spm, (k_scatter_out<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(
                                  P, perm, x, v, f, x_caller, v_caller, f_caller)));
}

void launch_kick_drift(hipStream_t s, const DevParams &P, const double *x_in, double *v, const double *f,
                       double *x_out, double4 *Rw_out, const double4 *R_ref,
                       const int *perm, Ctrl *ctrl, int step, const StepArgs &st)
{
    ADRES_SPM_DISPATCH(P.spm, (k_kick_drift<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(
                                  P, x_in, v, f, x_out, Rw_out, R_ref, perm, ctrl, step, st)));
}

void launch_centres_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank, const double *x,
                         double4 *Rw, int *key, int *count, const int *go, const double *x_alt, double4 *Rw_alt,
                         const ChainHead &head)
{
    ADRES_SPM_DISPATCH(P.spm, (k_centres_keys<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(go, P, G, cell_rank, x, Rw,
                                                                                         key, count, x_alt, Rw_alt,
                                                                                         head)));
}


void launch_reset_halt(hipStream_t s, Ctrl *ctrl) { k_reset_halt<<<1, 64, 0, s>>>(ctrl); }

void launch_publish(hipStream_t s, Ctrl *ctrl, CtrlPub *pub, unsigned seq)
{
    k_publish<<<1, 64, 0, s>>>(ctrl, pub, seq);
}

void launch_map_cg(hipStream_t s, const DevParams &P, const double *x, const double *f, double *com, double *fmap)
{
    ADRES_SPM_DISPATCH(P.spm, (k_map_cg<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x, f, com, fmap)));
}

void launch_density_profile(hipStream_t s, const DevParams &P, const double *x, const double *cen,
                            unsigned long long *counts)
{
    ADRES_SPM_DISPATCH(P.spm, (k_density_profile<S_><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, x, cen, counts)));
}

void launch_anchor_centres(hipStream_t s, const DevParams &P, const double *x, double *cen)
{
    ADRES_SPM_DISPATCH(P.spm, (k_anchor_centres<S_><<<(P.n_anchors + 63) / 64, 64, 0, s>>>(P, x, cen)));
}

void launch_region_volumes(hipStream_t s, const DevParams &P, const double *cen, long long n_samples,
                           unsigned long long seed, unsigned long long *counts)
{
    const long long want = (n_samples + kBlock - 1) / kBlock;
    const int blocks = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    k_region_volumes<<<blocks, kBlock, 0, s>>>(P, cen, n_samples, seed, counts);
}

void launch_td_update(hipStream_t s, const DevParams &P, double *td, double *td_u, const long long *counts,
                      long long n_frames, double prefactor, const long long *vol, long long n_vol)
{
    k_td_update<<<1, kBlock, 0, s>>>(P, td, td_u, counts, n_frames, prefactor, vol, n_vol);
}

void launch_anchor_weights(hipStream_t s, const DevParams &P, double4 *Rw, const int *inv_perm, int *aslot,
                           int refresh, Ctrl *ctrl, int step, int check_halt, double4 *near, const int *go,
                           double4 *Rw_alt)
{
    // reach: where the weight and the correction force stop changing (the table's end
    // only while one is installed), padded by 2^-20 of itself; cells at least that wide
    double reach = P.d_end;
    if (P.td_n > 0) reach = std::max(reach, P.td_hi);
    reach *= 1.0 + 0x1p-20;
    int g[3];
    for (int d = 0; d < 3; ++d) g[d] = std::max(1, std::min(kAnchorGrid, (int)std::floor(P.box[d] / reach)));
    const int blocks = (P.n_mol + kAnchorMols - 1) / kAnchorMols;
    k_anchor_weights<<<blocks, kBlock, anchor_lds_bytes(P.n_anchors, g[0] * g[1] * g[2]), s>>>(
        go, P, Rw, inv_perm, aslot, refresh, ctrl, step, check_halt, near, make_int3(g[0], g[1], g[2]), Rw_alt);
}

void launch_anchor_weights_caller(hipStream_t s, const DevParams &P, const double *com, double *w)
{
    k_anchor_weights_caller<<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, com, w);
}

}  // namespace adres
