/*
 * adres.h -- C ABI of the MI355X (gfx950) adaptive-resolution force-interpolation
 * library libadres.so.
 *
 * The method is the force-interpolation Adaptive Resolution Scheme (AdResS) as
 * stated in "ESPResSo++ 2.0: Advanced methods for multiscale molecular
 * simulation", Sec. 2 ("Adaptive resolution simulations"):
 *   - each molecule alpha carries a resolution value lambda(R_alpha) of its centre
 *     of mass R_alpha: 1 in the atomistic (AT) region, 0 in the coarse-grained (CG)
 *     region, smooth across the hybrid (HY) region (Sec. 2.2), a squared cosine
 *     (Sec. 2.3);
 *   - the non-bonded force between molecules alpha and beta is Eq. (1):
 *       F_ab = l_a l_b F^AT_ab + (1 - l_a l_b) F^CG_ab,
 *     F^AT the sum of atom-atom forces, F^CG a force between centres of mass;
 *   - intramolecular bonds are not interpolated (Sec. 2.2) and are integrated
 *     everywhere (Sec. 2.3);
 *   - neighbours are found with a linked-cell list (Sec. 5, introduction).
 * Beyond Eq. (1) the library offers potential energy interpolation, Eq. (2) (H-AdResS,
 * Sec. 2.3: adres_params.scheme), a correction field along the resolution coordinate with
 * its density profile and refinement (thermodynamic force, Sec. 2.4: adres_set_tdforce),
 * self-adjusting AT regions made of spheres around moving anchor molecules (Sec. 2.5:
 * ADRES_REGION_SPHERES) and RESPA multiple time stepping (Sec. 2.6:
 * adres_integrate_respa).
 *
 * Conventions for every call:
 *   - Units: lengths in sigma (atom diameter), energies in epsilon, masses in atom
 *     masses.  Box orthorhombic and periodic, coordinates in [0, L).
 *   - Arrays named x, v, f are DEVICE pointers to float64 structure-of-arrays of
 *     shape [3][N_s] (row 0 = x components, row 1 = y, row 2 = z), N_s = n_mol *
 *     sites_per_mol; molecule a owns sites a*s .. a*s+s-1.  com is [3][n_mol], w is
 *     [n_mol].  The caller owns these arrays; the library never frees them.
 *   - The library owns all other state (cell list, neighbour list, Morton-ordered
 *     copies, tables, network weights, optimiser state).  The caller's site order is
 *     preserved at the boundary; the Morton order is internal.
 *   - Work is enqueued on the stream given to adres_create and returns at once,
 *     except where a call is documented to synchronise (it then waits for that
 *     stream only).  One context per stream; a context is not thread-safe.
 *   - Errors: every call returns an adres_status.  Conditions detected on the
 *     device (non-finite values, a stretched molecule, a broken FENE bond, a table
 *     lookup below its range) are latched in a device flag word and reported by the
 *     next synchronising call; adres_last_error gives a message.
 */
#ifndef ADRES_H
#define ADRES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adres_ctx adres_ctx;

typedef enum {
    ADRES_OK = 0,
    ADRES_E_ARG = -1,          /* invalid argument or parameter */
    ADRES_E_NOMEM = -2,        /* device or host allocation failed */
    ADRES_E_HIP = -3,          /* a HIP runtime call failed */
    ADRES_E_BOX = -4,          /* box shorter than twice the list radius, or over 2^20 cells */
    ADRES_E_CAPACITY = -5,     /* neighbour list could not be grown */
    ADRES_E_STRETCH = -6,      /* a site is farther than rho_max + r_skin/2 from its centre
                                  of mass (no neighbour list can cover it) */
    ADRES_E_NONFINITE = -7,    /* a force or position is NaN or infinite */
    ADRES_E_FENE = -8,         /* a FENE bond reached its maximum extension R0 */
    ADRES_E_TABLE_RANGE = -9,  /* a CG table lookup below the table's first knot */
    ADRES_E_STATE = -10        /* call out of order (e.g. MLP kind without weights) */
} adres_status;

/* ADRES_REGION_SPHERES: a self-adjusting AT region (Sec. 2.5), the union of spheres of radius
 * d_at (hybrid shell d_hy) around the current centres of mass of anchor molecules chosen with
 * adres_set_anchors; the region moves with them.  Force interpolation only; a correction
 * field (adres_set_tdforce) acts around the nearest anchor. */
enum { ADRES_REGION_ALL_AT = 0, ADRES_REGION_SLAB_X = 1, ADRES_REGION_SPHERE = 2, ADRES_REGION_ALL_CG = 3,
       ADRES_REGION_SPHERES = 4 };
/* CG force between centres of mass: analytic WCA, cubic table, learned network with layer 2
 * on BF16 matrix cores, or its FP8 variant (inference only; see adres_mlp_set). */
enum { ADRES_CG_WCA = 0, ADRES_CG_TABLE = 1, ADRES_CG_MLP = 2, ADRES_CG_MLP_FP8 = 3 };
enum { ADRES_BOND_NONE = 0, ADRES_BOND_HARMONIC = 1, ADRES_BOND_FENE = 2 };
/* Coupling scheme: force interpolation, Eq. (1) (Sec. 2.2), or potential energy
 * interpolation, Eq. (2) (H-AdResS, Sec. 2.3). */
enum { ADRES_SCHEME_FORCE = 0, ADRES_SCHEME_HAMILTONIAN = 1 };

#define ADRES_MAX_SITES 4

typedef struct {
    int32_t n_mol;              /* molecules (>= 1) */
    int32_t sites_per_mol;      /* 1 .. ADRES_MAX_SITES */
    double  box[3];             /* periodic box lengths */
    double  site_mass[ADRES_MAX_SITES];
    int32_t region;             /* ADRES_REGION_*: where the AT region is (Sec. 2.2, 2.5) */
    double  center[3];          /* AT region centre (slab: only center[0] is used) */
    double  d_at, d_hy;         /* AT half-width / radius (of each sphere) and hybrid width */
    double  eps_at, sig_at, rc_at;   /* atom-atom WCA */
    double  eps_cg, sig_cg, rc_cg;   /* CG centre-of-mass force: WCA parameters and cutoff */
    int32_t cg_kind;            /* ADRES_CG_*: the CG force between centres of mass */
    int32_t bond_kind;          /* ADRES_BOND_* */
    double  k_bond, r0_bond;    /* harmonic: K, b0;  FENE: k, R0 */
    int32_t chain_len;          /* FENE: beads per chain (runs of consecutive molecules) */
    double  r_skin;             /* Verlet skin; the list is rebuilt when a centre of mass
                                   has moved further than its budget since the last build:
                                   min((r_list - rc_cg)/2, rho_max + r_skin/2 - the
                                   molecule's current extent; in the step loop the CG
                                   part alone for a molecule of weight zero with force
                                   interpolation and a static region), at least r_skin/2
                                   for a molecule within rho_max */
    double  rho_max;            /* bound on a site's distance from its centre of mass that
                                   the list radius assumes; a site farther out (thermal
                                   bond stretch) spends its excess from the molecule's
                                   motion budget, so the list is rebuilt earlier;
                                   beyond rho_max + r_skin/2: ADRES_E_STRETCH */
    int32_t pair_precision;     /* 64: FP64 pair arithmetic; 32: FP32 pair arithmetic on
                                   FP64-formed displacements, FP64 sums */
    int32_t scheme;             /* ADRES_SCHEME_FORCE: pair forces w_a w_b F^AT +
                                   (1 - w_a w_b) F^CG (Eq. (1)).  ADRES_SCHEME_HAMILTONIAN:
                                   forces of H = K + sum_a [w_a V^AT_a + (1 - w_a) V^CG_a]
                                   (Eq. (2)), V_a half of molecule a's intermolecular pair
                                   potentials: pair weights (w_a + w_b) / 2 and, on hybrid
                                   molecules, the drift force -(V^AT_a - V^CG_a) grad w_a
                                   shared by mass fraction; needs cg_kind ADRES_CG_WCA (the
                                   CG potential).  Energies (adres_forces) are then
                                   sum_a w_a V^AT_a and sum_a (1 - w_a) V^CG_a. */
} adres_params;

/* Create a context for one system on the current HIP device.  hip_stream is a
 * hipStream_t (NULL = default stream).  Validates the parameters (ADRES_E_ARG),
 * derives the list radius r_list = max(rc_cg, rc_at + 2 rho_max) + r_skin and the
 * cell grid (ADRES_E_BOX if any box length is below 2 r_list or the grid has more than
 * 2^20 cells), and allocates the
 * context's device state.  *out is set only on success. */
adres_status adres_create(const adres_params *params, void *hip_stream, adres_ctx **out);

/* Release everything the context owns.  Synchronises its stream first.  NULL is a no-op. */
void adres_destroy(adres_ctx *ctx);

/* Centres of mass and resolution weights (Sec. 2.2, 2.3): com [3][n_mol] and w [n_mol],
 * device, caller order.  R = x0 + ((m1 d1 + m2 d2) + m3 d3) / M with d_k the
 * minimum-image offsets of site k from site 0, folded into [0, L); w = 1 for d <= d_at,
 * cos^2(pi (d - d_at) / (2 d_hy)) inside the hybrid layer, 0 beyond, d the distance of R
 * from the AT centre (slab: along x).  Asynchronous. */
adres_status adres_weights(adres_ctx *ctx, const double *x, double *com, double *w);

/* Linked-cell list of the molecules' centres of mass (Sec. 5): cells of edge >= r_list,
 * ordered along a Morton curve; molecules counted per cell, exclusive-scanned and
 * scattered, ties inside a cell ordered by caller index.  Reorders the context's
 * internal copy of the state.  Asynchronous. */
adres_status adres_build_cells(adres_ctx *ctx, const double *x);

/* Rebuild the cell list for x, then the Verlet list of molecule pairs whose
 * minimum-image centre-of-mass distance is strictly below r_list.  n_pairs (host,
 * optional) receives the number of unordered pairs; passing it synchronises.
 * Synchronises once to check the list capacity (grown and refilled on overflow;
 * ADRES_E_CAPACITY if growth fails). */
adres_status adres_build_verlet(adres_ctx *ctx, const double *x, int64_t *n_pairs);

/* Forces of Eq. (1) plus the non-interpolated bonded terms, written to f (device,
 * caller order).  The atomistic part (ww = w_a w_b > 0) sums WCA over atom pairs with
 * r < rc_at and weights it by ww; the CG part (ww < 1) is (1 - ww) times the CG force
 * between centres of mass (r < rc_cg), shared among a molecule's sites by mass
 * fraction.  energy (device [4], optional): U_AT (ww-weighted), U_CG ((1 - ww)-weighted,
 * analytic CG only), U_bond, U_corr (the correction force's potential, see
 * adres_set_tdforce; 0 without one).  Builds the lists if none exist and rebuilds them if a
 * centre of mass moved further than its budget (see r_skin) since the last build; to decide, it
 * synchronises once before the force kernel is enqueued. */
adres_status adres_forces(adres_ctx *ctx, const double *x, double *f, double *energy);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): adres_forces with the same arguments and
 * results, which itself allocates nothing.  Its energy partials go to a static device array
 * of the library (one per GPU, 8192 workgroup slots, 256 KiB: at most 524,288 molecules;
 * larger contexts give ADRES_E_CAPACITY); where adres_forces would grow the neighbour list, a
 * tile halo or the network's half list, it returns ADRES_E_CAPACITY instead (a call of
 * adres_forces or adres_build_verlet beforehand sizes them).  Every call on one GPU shares
 * that array, and calls that overlap on one GPU (other streams or threads) race on it. */
adres_status adres_forces_noalloc(adres_ctx *ctx, const double *x, double *f, double *energy);

/* n_steps of velocity Verlet (v += F dt/2m; x += v dt; fold; F = F(x); v += F dt/2m)
 * on x, v (device, caller order, updated in place); f receives F(x_final).  The lists
 * are rebuilt whenever a centre of mass has moved further than its budget (see r_skin).
 * gamma > 0 adds a
 * Langevin thermostat at temperature kT with counter-based normal deviates keyed by
 * (seed, step, site); gamma = 0 is plain NVE.  n_rebuilds (host, optional) receives
 * the number of list rebuilds.  Synchronises at every rebuild and at the end. */
adres_status adres_integrate(adres_ctx *ctx, double *x, double *v, double *f, double dt,
                             int32_t n_steps, double gamma, double kT, uint64_t seed,
                             int32_t *n_rebuilds);

/* Multiple time stepping (Sec. 2.6): reversible RESPA (Tuckerman, Berne & Martyna 1992)
 * with n_outer outer steps of Dt = n_inner dt.  The slow part -- the CG pair part of the
 * coupling, the CG share +V^CG grad w of the Hamiltonian scheme's drift and the correction
 * force -- acts on the outer step; the fast part -- the atomistic pair part, the share
 * -V^AT grad w of the drift and the bonds -- on the inner step dt.  One outer step:
 * v += F_slow Dt/2m; n_inner times {v += F_fast dt/2m; x += v dt; fold; v += F_fast(x) dt/2m};
 * v += F_slow(x) Dt/2m.  The slow part is evaluated once per outer step (the CG pair work
 * and, for a learned CG force, the network are skipped on the other inner steps).
 * n_inner = 1 is adres_integrate.  x, v (device, caller order) are updated in place; f
 * receives the total force at the final positions.  gamma > 0 applies the Langevin
 * thermostat of adres_integrate at every inner step.  n_rebuilds as for adres_integrate.
 * ADRES_E_ARG unless n_inner >= 1, n_outer >= 0, n_inner n_outer < 2^31, dt > 0.
 * Synchronises at every list rebuild and at the end. */
adres_status adres_integrate_respa(adres_ctx *ctx, double *x, double *v, double *f, double dt,
                                   int32_t n_inner, int32_t n_outer, double gamma, double kT,
                                   uint64_t seed, int32_t *n_rebuilds);

/* Copy out the current Verlet list as unordered caller-index pairs (a < b), sorted
 * lexicographically, into pairs_host (host, [cap][2] int32).  *n receives the pair
 * count even when it exceeds cap.  Synchronises. */
adres_status adres_get_pairs(adres_ctx *ctx, int32_t *pairs_host, int64_t cap, int64_t *n);

/* Copy out the cell list: cell_start_host [n_cells + 1] (Morton-ordered cells) and
 * perm_host [n_mol] (caller index of each Morton-ordered slot).  Either may be NULL.
 * *n_cells receives the cell count.  Synchronises. */
adres_status adres_get_cells(adres_ctx *ctx, int32_t *cell_start_host, int32_t *perm_host,
                             int32_t *n_cells);

/* Install a cubic table of the CG force magnitude f(r) (positive = repulsive) on
 * n_knots equally spaced knots over [r_lo, r_hi]: coef4 (host, float32, [n_knots-1][4])
 * holds {c0, c1, c2, c3} of interval k, evaluated as ((c3 t + c2) t + c1) t + c0 with
 * t = (r - r_lo)/h - k.  Copied; used when cg_kind is ADRES_CG_TABLE and as the MLP's
 * fallback below its r_min.  2 <= n_knots <= 4096. */
adres_status adres_set_cg_table(adres_ctx *ctx, const float *coef4, int32_t n_knots,
                                double r_lo, double r_hi);

/* Correction force along the resolution coordinate: the thermodynamic force or free-energy
 * correction of Sec. 2.4, a field over the hybrid region that flattens the density
 * profile across it.  It acts on each molecule's centre of mass along the direction in
 * which the distance d from the AT centre grows (slab: sign of the minimum-image x
 * offset; sphere: the unit offset; anchor spheres: the unit offset from the nearest anchor
 * centre, the first of equally near ones, with no reaction on the anchors; none at d = 0)
 * and reaches the sites by mass fraction,
 * in every later force evaluation (adres_forces, adres_integrate, adres_map_cg).
 * table (host, float64 [n]) holds its value F_k at the bin centres
 * d_k = d_lo + (k + 1/2) h, h = (d_hi - d_lo) / n; F(d) is linear between neighbouring
 * centres, holds F_0 from d_lo to d_0 and F_{n-1} from d_{n-1} to d_hi, and is 0 outside
 * [d_lo, d_hi).  Its potential -integral of F from d_lo to min(d, d_hi) is reported as
 * U_corr.  Needs region ADRES_REGION_SLAB_X, ADRES_REGION_SPHERE or ADRES_REGION_SPHERES
 * (for the last the table is that of a single sphere, e.g. refined with region
 * ADRES_REGION_SPHERE and the same d_at, d_hy); 1 <= n <= 4096,
 * 0 <= d_lo < d_hi, finite values (ADRES_E_ARG otherwise).  n = 0 removes the correction.
 * Copied; synchronises. */
adres_status adres_set_tdforce(adres_ctx *ctx, const double *table, int32_t n, double d_lo, double d_hi);

/* Copy the installed correction values (e.g. after adres_tdforce_update) to table_host
 * (host, float64 [n], n the installed length).  ADRES_E_STATE without a table.
 * Synchronises. */
adres_status adres_get_tdforce(adres_ctx *ctx, double *table_host, int32_t n);

/* Density profile along the resolution coordinate (Sec. 2.4), in the bins of the installed
 * correction table: adds to counts (device, int64 [n], caller-initialised) the number of
 * molecules of x (device, caller order) whose centre-of-mass distance d from the AT
 * centre lies in bin floor((d - d_lo) / h) of [d_lo, d_hi); for ADRES_REGION_SPHERES d is
 * the distance from the nearest anchor centre of x.  Call once per sampled frame.
 * ADRES_E_STATE without a table (or without anchors).  Asynchronous. */
adres_status adres_density_profile(adres_ctx *ctx, const double *x, int64_t *counts);

/* Bin volumes by sampling, for regions whose bins have no closed-form volume (a union of
 * moving anchor spheres, Sec. 2.5 with Sec. 2.4): adds to vol_counts (device, int64 [n],
 * caller-initialised) the bins of n_samples points uniform in the box, binned by their
 * resolution distance like centres of mass (anchor spheres: from the nearest anchor centre
 * of x, device caller order; x may be NULL for the other regions).  Point i has
 * coordinate c = L_c * (SplitMix64(seed, 3 i + c) >> 11) * 2^-53, SplitMix64(s, k) the
 * SplitMix64 finaliser (Steele, Lea and Flood 2014) of s + (k + 1) * 0x9E3779B97F4A7C15.
 * The volume of bin k is vol_counts_k / n_samples times the box volume.  ADRES_E_STATE
 * without a table; n_samples >= 1.  Asynchronous. */
adres_status adres_region_volumes(adres_ctx *ctx, const double *x, int64_t n_samples, uint64_t seed,
                                  int64_t *vol_counts);

/* One refinement of the correction force from a density profile (Sec. 2.4: the
 * thermodynamic force is built from the distorted profile and refined iteratively):
 * rho_k = counts_k / (n_frames V_k), V_k the volume of bin k (slab: both sides of the
 * mid-plane, 2 h L_y L_z; sphere: the shell 4/3 pi (r_{k+1}^3 - r_k^3), r_k = d_lo + k h),
 * then F_k <- F_k - prefactor * (drho/dd)_k with the slope by central differences of the
 * neighbouring bins (one-sided at the two end bins, 0 for a single bin).  The usual
 * prefactor is M / (rho_0^2 kappa_T).  counts: device int64 [n], n_frames >= 1; not for
 * ADRES_REGION_SPHERES (ADRES_E_ARG: use adres_tdforce_update_sampled).  Asynchronous. */
adres_status adres_tdforce_update(adres_ctx *ctx, const int64_t *counts, int64_t n_frames, double prefactor);

/* The same refinement with sampled bin volumes (adres_region_volumes): V_k = vol_counts_k /
 * n_vol_samples times the box volume, n_vol_samples the points behind vol_counts in total; a
 * bin no sample fell in counts as empty.  Any region.  counts, vol_counts: device int64 [n].
 * Asynchronous. */
adres_status adres_tdforce_update_sampled(adres_ctx *ctx, const int64_t *counts, int64_t n_frames,
                                          const int64_t *vol_counts, int64_t n_vol_samples, double prefactor);

/* Anchors of a self-adjusting AT region (region ADRES_REGION_SPHERES, Sec. 2.5): mols (host,
 * int32 [k]) are caller molecule indices; each anchor's current centre of mass is the centre
 * of a sphere, and a molecule's resolution distance is its minimum-image distance to the
 * nearest anchor centre, d = min_k |R - R_k| (so w is the largest single-sphere weight).
 * The weights follow the anchors at every step.  1 <= k <= 1024 and 0 <= mols[i] < n_mol
 * (ADRES_E_ARG otherwise, and for other regions); weights, forces and integration return
 * ADRES_E_STATE until anchors are set.  Copied; synchronises. */
adres_status adres_set_anchors(adres_ctx *ctx, const int32_t *mols, int32_t k);

/* Learned CG force (replaces F^CG of Eq. (1) when cg_kind is ADRES_CG_MLP):
 *   f(r) = scale * taper(r) * [W3 . silu(W2 silu(W1 x + b1) + b2) + b3],  x = r / rc,
 * silu(z) = z / (1 + e^-z), taper = 1 below rc - taper_width and a cos^2 ramp to 0 at rc,
 * positive f = repulsive along R_ab / r.  Below r_min the installed cubic table is used
 * (the fallback).  Hidden width 64: params (host, float32, 4353 values) are
 * W1[64], b1[64], W2[64*64] (row = output unit), b2[64], W3[64], b3.  Layer 2 runs on
 * BF16 matrix cores with FP32 accumulation; layers 1 and 3 in FP32.  With cg_kind
 * ADRES_CG_MLP_FP8 layer 2 runs on FP8 E4M3 (OCP) matrix cores instead: W2 / s_w and
 * h1 / (s_g ln 2) rounded to E4M3 (nearest even) with per-tensor scales s_w = max|W2| / 448
 * and s_g = G / 448, G = 1.01 max(0.2785, max_u |silu(b1_u)|, max_u |silu(W1_u + b1_u)|)
 * / ln 2 (a bound on |h1| / ln 2 for r / rc in [0, 1]), FP32 accumulation; each result
 * then carries the E4M3 rounding of two factors (relative 2^-4 each).  The values are
 * copied; n_params must be 4353. */
adres_status adres_mlp_set(adres_ctx *ctx, const float *params, int32_t n_params, double rc, double scale,
                           double taper_width, double r_min);

/* Copy the network's current FP32 parameters (e.g. after training) to params (host,
 * 4353 floats).  Synchronises. */
adres_status adres_mlp_get(adres_ctx *ctx, float *params, int32_t n_params);

/* Evaluate the installed network (with its taper, cutoff and table fallback) at n
 * distances: r (device, float64 [n]) -> f (device, float32 [n]).  Asynchronous. */
adres_status adres_mlp_eval(adres_ctx *ctx, const double *r, float *f, int64_t n);

/* Mapped forces for force matching: the Eq. (1) forces at x (into f, device [3][N_s],
 * caller order; with region ADRES_REGION_ALL_AT these are the atomistic forces), then
 * per molecule its centre of mass com [3][n_mol] and the sum of its site forces
 * f_map [3][n_mol] (intramolecular bond forces cancel in the sum).  Synchronises as
 * adres_forces does. */
adres_status adres_map_cg(adres_ctx *ctx, const double *x, double *f, double *com, double *f_map);

/* Force matching of the learned CG force (multiscale coarse-graining, Izvekov & Voth
 * 2005; the training counterpart of F^CG in Eq. (1)).  The context must describe CG
 * sites: sites_per_mol = 1, region ADRES_REGION_ALL_CG, cg_kind ADRES_CG_MLP, a network
 * installed.  com and f_map (device, float64) hold n_frames frames, each [3][n_mol] in
 * caller order: centres R_I and mapped forces F^map_I.  The prediction is
 * F_I = sum_J f(r_IJ) (R_I - R_J) / r_IJ over r_IJ < rc (table below r_min), the loss
 * chi2 = sum_frames sum_I |F_I - F^map_I|^2 / (3 n_frames n_mol).
 * adres_mlp_fm_grad: loss (host, optional) and its gradient w.r.t. the 4353 parameters
 * (host float64, optional) at the current parameters; synchronises.
 * adres_mlp_train_step: the same gradient followed by one Adam step (beta1 0.9, beta2
 * 0.999, eps 1e-8, learning rate lr > 0) on the FP32 parameters; loss (host, optional)
 * is the loss before the step; synchronises.  Both rebuild the context's lists per frame. */
adres_status adres_mlp_fm_grad(adres_ctx *ctx, const double *com, const double *f_map, int32_t n_frames,
                               double *grad, double *loss);
adres_status adres_mlp_train_step(adres_ctx *ctx, const double *com, const double *f_map, int32_t n_frames,
                                  double lr, double *loss);

/* Diagnostic: device time of the kernels enqueued since the last call, measured with
 * HIP events on the context's stream.  enable selects what the following calls record:
 * 0 nothing, 1 the force kernel (Eq. (1) with its fused integrator stages), 2 the learned
 * CG force's pair pre-pass (contexts with a network CG kind; one per force
 * evaluation); every >= 1 records only every every-th such launch (events slow the
 * launch stream down, so sampling keeps the timed run close to an untimed one).  Other
 * values give ADRES_E_ARG.  ms (host) receives the summed duration of the launches
 * recorded before this call and launches (host) their number; a launch of adres_integrate
 * that returned at once, because an earlier kernel of its step chunk asked for a list
 * rebuild (or a list overflow stopped the chunk), is not counted.  Synchronises. */
adres_status adres_kernel_timing(adres_ctx *ctx, int32_t enable, int32_t every, double *ms, int64_t *launches);

/* Message describing the last error of this context (never NULL). */
const char *adres_last_error(const adres_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADRES_H */
