// Internal definitions of libadres: parameter block passed to kernels, device
// helpers and host-side launch wrappers.  gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
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
    int overflow;   // neighbour list row longer than capacity
    int max_count;  // longest neighbour-list row seen by the last build
};

// Parameters in the form the kernels use (passed by value).
struct DevParams {
    int n_mol, spm;
    int64_t n_sites;
    double box[3], half[3];
    double mass[kMaxSites], mfrac[kMaxSites], inv_2m[kMaxSites], M;
    int region;
    double center[3], d_at, d_hy, d_end;
    double eps_at, sig2_at, rcA2, rc_at;
    double eps_cg, sig2_cg, rcC2;
    int cg_kind, bond_kind;
    double k_bond, r0_bond, R02;
    int chain_len;
    double rho_max;
    double half_skin2;
    // cubic CG table
    const float4 *tab;
    int tab_n;
    double tab_lo, tab_h;
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

__device__ __forceinline__ double mi(double d, double L, double half)
{
    if (d > half) d -= L;
    else if (d < -half) d += L;
    return d;
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
template <int SPM>
__device__ __forceinline__ void mol_com(const DevParams &P, const double (&p)[SPM][3], double R[3],
                                        double &rho)
{
#pragma clang fp contract(off)
    for (int d = 0; d < 3; ++d) {
        double x0 = p[0][d];
        double acc = 0.0;
#pragma unroll
        for (int k = 1; k < SPM; ++k) acc = acc + P.mass[k] * mi(p[k][d] - x0, P.box[d], P.half[d]);
        R[d] = fold(x0 + acc / P.M, P.box[d]);
    }
    double rmax2 = 0.0;
#pragma unroll
    for (int k = 0; k < SPM; ++k) {
        double q0 = mi(p[k][0] - R[0], P.box[0], P.half[0]);
        double q1 = mi(p[k][1] - R[1], P.box[1], P.half[1]);
        double q2 = mi(p[k][2] - R[2], P.box[2], P.half[2]);
        double r2 = dist2_exact(q0, q1, q2);
        rmax2 = r2 > rmax2 ? r2 : rmax2;
    }
    rho = sqrt(rmax2);
}

// Resolution weight of a centre of mass (1 in AT, cos^2 ramp in HY, 0 in CG).
__device__ __forceinline__ double res_weight(const DevParams &P, const double R[3])
{
#pragma clang fp contract(off)
    if (P.region == ADRES_REGION_ALL_AT) return 1.0;
    if (P.region == ADRES_REGION_ALL_CG) return 0.0;
    double d;
    if (P.region == ADRES_REGION_SLAB_X) {
        d = fabs(mi(R[0] - P.center[0], P.box[0], P.half[0]));
    } else {
        double q0 = mi(R[0] - P.center[0], P.box[0], P.half[0]);
        double q1 = mi(R[1] - P.center[1], P.box[1], P.half[1]);
        double q2 = mi(R[2] - P.center[2], P.box[2], P.half[2]);
        d = sqrt(dist2_exact(q0, q1, q2));
    }
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

// ---------------------------------------------------------------- launch wrappers
// All launches are asynchronous on `s`.  Arrays in "sorted" order are indexed by
// Morton slot; "caller" arrays by the caller's molecule/site index.

struct StateBufs {   // sorted-order state (device)
    double *x, *v, *f;       // [3][n_sites]
    double *R;               // [3][n_mol]
    double *w, *rho;         // [n_mol]
    int *perm;               // slot -> caller molecule
    int *key;                // slot -> Morton rank of its cell
};

void launch_weights_caller(hipStream_t s, const DevParams &P, const double *x, double *com, double *w,
                           Ctrl *ctrl);
void launch_gather(hipStream_t s, const DevParams &P, const double *x_caller, const double *v_caller,
                   const StateBufs &S, const double *R_ref, Ctrl *ctrl);
void launch_scatter_out(hipStream_t s, const DevParams &P, const StateBufs &S, double *x_caller,
                        double *v_caller, double *f_caller);
void launch_kick_drift(hipStream_t s, const DevParams &P, const StateBufs &S, const double *R_ref,
                       Ctrl *ctrl, int step, double dt, double gamma, double kT, uint64_t seed,
                       uint64_t step_abs);
void launch_reset_halt(hipStream_t s, Ctrl *ctrl);

// cell list
void launch_cell_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank,
                      const StateBufs &S, int *count);
void launch_scan_cells(hipStream_t s, const int *count, int n_cells, int *start, int *fill);
void launch_scatter_slots(hipStream_t s, int n_mol, const int *key, const int *start, int *fill,
                          int *new_from);
void launch_sort_within_cells(hipStream_t s, int n_cells, const int *start, const int *perm_old,
                              int *new_from);
void launch_permute(hipStream_t s, const DevParams &P, const int *new_from, const StateBufs &src,
                    const StateBufs &dst, int *inv_perm, double *R_ref, bool with_v);

// Verlet list (ELL, column-major: nbr[k * n_mol + slot])
void launch_list_build(hipStream_t s, const DevParams &P, const Grid &G, const int *rank_cell,
                       const int *cell_rank, const int *start, const StateBufs &S, double rl2, int *nbr,
                       int *cnt, int cap, Ctrl *ctrl);

// forces
struct ForceArgs {
    DevParams P;
    const double *x, *R, *w, *rho;
    const int *nbr, *cnt;
    int cap;
    const int *perm, *inv_perm;   // slot -> caller, caller -> slot
    double *f;                    // output forces
    const int *out_perm;          // non-null: write f in caller order via perm
    double *v;                    // non-null: second half-kick v += f dt / 2m (sorted)
    double dt;
    Ctrl *ctrl;
    int step, check_halt;
    double *epart;                // non-null: per-block energy partials [blocks][3]
};
int launch_forces(hipStream_t s, const ForceArgs &a, int pair_precision);   // returns block count
void launch_energy_reduce(hipStream_t s, const double *epart, int n_blocks, double *energy);

}  // namespace adres
