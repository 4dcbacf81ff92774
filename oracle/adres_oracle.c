/*
 * FP64 CPU oracle for the force-interpolation adaptive resolution scheme (AdResS).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header or constant generator with the HIP
 * library.  It is deliberately plain: every result is the written-out definition,
 * summed over *all* other molecules (no neighbour list, no cells, no blocking),
 * in IEEE double precision, compiled with -ffp-contract=off.
 *
 * Paper: "ESPResSo++ 2.0: Advanced methods for multiscale molecular simulation".
 *   - resolution function lambda(R_alpha): 1 in the atomistic (AT) region, 0 in the
 *     coarse-grained (CG) region, a smooth squared cosine across the hybrid (HY)
 *     region, evaluated at each molecule's centre of mass
 *     (Sec. 2.2 "Force interpolation"; Sec. 2.3 names the squared cosine);
 *   - Eq. (1): F_ab = l_a l_b F^AT_ab + (1 - l_a l_b) F^CG_ab, with F^AT the sum of
 *     atom-atom forces between the two molecules and F^CG a force between their
 *     centres of mass (Sec. 2.2, text following Eq. (1));
 *   - intramolecular bond terms are not interpolated (Sec. 2.2, last paragraph) and
 *     are integrated everywhere (Sec. 2.3);
 *   - force interpolation obeys Newton's third law and has no conserved energy
 *     (Sec. 2.3, paragraph after Eq. (2));
 *   - potential energy interpolation, Eq. (2) (H-AdResS, Sec. 2.3): the Hamiltonian
 *     sum_alpha [l_a V^AT_a + (1 - l_a) V^CG_a] plus kinetic (and bond) energy; its forces
 *     carry the drift term -(V^AT_a - V^CG_a) grad l_a and conserve the energy.  Reading:
 *     V_a is half of each intermolecular pair potential of molecule a (so that the
 *     molecules' V add up to the total potential), with the CG potential analytic WCA;
 *   - a correction force on the centres of mass along the direction of resolution
 *     change, to flatten the density profile across the hybrid region: the
 *     thermodynamic force, built from the density profile and refined iteratively
 *     (Sec. 2.4).  Readings at orc_td_force and orc_tdforce_update;
 *   - multiple time stepping: the softer CG forces on a longer time step than the
 *     atomistic ones, by RESPA (Sec. 2.6).  Reading at orc_respa;
 *   - self-adjusting AT regions: spheres around moving anchors whose overlap is the AT
 *     region (Sec. 2.5), with force interpolation.  Reading at orc_anchor_distance.
 * Potentials (WCA, FENE, harmonic bonds), sizes and time steps are those of the
 * synthetic workloads; the readings taken where the paper is silent are listed
 * at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_SITES 8

enum { ORC_OK = 0, ORC_STRETCH = 1, ORC_FENE = 2, ORC_TABLE_RANGE = 4, ORC_NONFINITE = 8 };
enum { ORC_REGION_AT = 0, ORC_REGION_SLAB = 1, ORC_REGION_SPHERE = 2, ORC_REGION_CG = 3, ORC_REGION_SPHERES = 4 };
enum { ORC_CG_WCA = 0, ORC_CG_TABLE = 1, ORC_CG_MLP = 2 };
enum { ORC_BOND_NONE = 0, ORC_BOND_HARMONIC = 1, ORC_BOND_FENE = 2 };
enum { ORC_SCHEME_FORCE = 0, ORC_SCHEME_HAMILTONIAN = 1 };
enum { ORC_PART_ALL = 0, ORC_PART_FAST = 1, ORC_PART_SLOW = 2 };

typedef struct {
    int32_t n_mol, spm;
    double box[3];
    double mass[ORC_MAX_SITES];
    int32_t region;
    double center[3], d_at, d_hy;
    double eps_at, sig_at, rc_at, eps_cg, sig_cg, rc_cg;
    int32_t cg_kind, bond_kind;
    double k_bond, r0_bond;
    int32_t chain_len;
    double rho_max;
    /* cubic table of the CG force magnitude: n_knots-1 intervals x {c0,c1,c2,c3} */
    const float *tab;
    int32_t tab_n;
    double tab_lo, tab_hi;
    /* MLP CG force (FP64 weights, layout W1[H] b1[H] W2[H*H] b2[H] W3[H] b3) */
    const double *mlp;
    int32_t mlp_hidden;
    double mlp_rc, mlp_scale, mlp_taper, mlp_rmin;
    /* ORC_SCHEME_FORCE: force interpolation, Eq. (1); ORC_SCHEME_HAMILTONIAN: potential
     * energy interpolation, Eq. (2) (H-AdResS) */
    int32_t scheme;
    /* correction force along the resolution coordinate (Sec. 2.4): td_n values at the
     * bin centres of [td_lo, td_hi); td_n = 0 means none */
    const double *td;
    int32_t td_n;
    double td_lo, td_hi;
    /* ORC_REGION_SPHERES: the AT region is the union of spheres of radius d_at (hybrid
     * shell d_hy) around the centres of mass of these molecules (Sec. 2.5) */
    const int32_t *anchors;
    int32_t n_anchors;
} orc_params;

/* Minimum image of one coordinate difference (periodic orthorhombic box).
 * Valid for |d| < 1.5 L, which holds for differences of wrapped coordinates. */
static double orc_mi(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

static double orc_sx(const orc_params *P, const double *x, int dim, int64_t site)
{
    int64_t ns = (int64_t)P->n_mol * P->spm;
    return x[dim * ns + site];
}

/* Total mass of a molecule, summed left to right over its sites. */
static double orc_mol_mass(const orc_params *P)
{
    double M = 0.0;
    for (int k = 0; k < P->spm; ++k) M = M + P->mass[k];
    return M;
}

/* Centre of mass R_alpha of molecule a (Sec. 2.2: lambda is evaluated at the centre
 * of mass).  Reading: mass-weighted mean of the minimum-image offsets from site 0,
 *   R = x0 + ((m1 d1 + m2 d2) + m3 d3) / M,
 * accumulated left to right, then folded once into [0, L).
 * Also returns the largest site distance from R (for the stretch check). */
static void orc_com(const orc_params *P, const double *x, int64_t a, double R[3], double *rho)
{
    double M = orc_mol_mass(P);
    int64_t s0 = a * P->spm;
    for (int d = 0; d < 3; ++d) {
        double L = P->box[d];
        double x0 = orc_sx(P, x, d, s0);
        double acc = 0.0;
        for (int k = 1; k < P->spm; ++k)
            acc = acc + P->mass[k] * orc_mi(orc_sx(P, x, d, s0 + k) - x0, L);
        double r = x0 + acc / M;
        if (r >= L) r -= L;
        else if (r < 0.0) r += L;
        R[d] = r;
    }
    double rmax2 = 0.0;
    for (int k = 0; k < P->spm; ++k) {
        double q[3];
        for (int d = 0; d < 3; ++d) q[d] = orc_mi(orc_sx(P, x, d, s0 + k) - R[d], P->box[d]);
        double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
        if (r2 > rmax2) rmax2 = r2;
    }
    *rho = sqrt(rmax2);
}

/* Resolution function of the distance d from the centre of the AT region
 * (Sec. 2.2: 1 inside the AT region, 0 in the CG region, smooth in between; Sec. 2.3:
 * squared cosine).  Reading: w = cos^2(pi (d - d_at) / (2 d_hy)) on d_at < d < d_at + d_hy,
 * exactly 1 for d <= d_at and exactly 0 for d >= d_at + d_hy. */
double orc_weight_of_distance(double d, double d_at, double d_hy)
{
    if (d <= d_at) return 1.0;
    if (d >= d_at + d_hy) return 0.0;
    double c = cos(M_PI * (d - d_at) / (2.0 * d_hy));
    return c * c;
}

/* Distance of a centre of mass from the AT region's centre.  Reading: for a slab,
 * |minimum-image x offset| from the slab's mid-plane; for a sphere, the Euclidean
 * minimum-image distance from its centre. */
static double orc_region_distance(const orc_params *P, const double R[3])
{
    if (P->region == ORC_REGION_SLAB)
        return fabs(orc_mi(R[0] - P->center[0], P->box[0]));
    double q[3];
    for (int d = 0; d < 3; ++d) q[d] = orc_mi(R[d] - P->center[d], P->box[d]);
    return sqrt((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
}

/* Gradient of the weight with respect to the centre of mass (Eq. (2)'s drift needs it):
 * dw/dd = -(pi / (2 d_hy)) sin(pi (d - d_at) / d_hy) inside the hybrid layer, 0 outside;
 * grad d = sign of the minimum-image x offset along x (slab) or the unit minimum-image
 * offset (sphere). */
static void orc_weight_gradient(const orc_params *P, const double R[3], double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    if (P->region != ORC_REGION_SLAB && P->region != ORC_REGION_SPHERE) return;
    double d = orc_region_distance(P, R);
    if (d <= P->d_at || d >= P->d_at + P->d_hy) return;
    double dw = -(M_PI / (2.0 * P->d_hy)) * sin(M_PI * (d - P->d_at) / P->d_hy);
    if (P->region == ORC_REGION_SLAB) {
        double q = orc_mi(R[0] - P->center[0], P->box[0]);
        g[0] = q > 0.0 ? dw : -dw;
        return;
    }
    for (int k = 0; k < 3; ++k) g[k] = dw * orc_mi(R[k] - P->center[k], P->box[k]) / d;
}

/* Correction force on a centre of mass (Sec. 2.4) and its potential.  Readings: the
 * force acts along the gradient of the resolution distance d (slab: the sign of the
 * minimum-image x offset; sphere: the unit offset from the centre; none at d = 0) with
 * magnitude F(d) taken from td_n values F_k given at the bin centres
 * d_k = lo + (k + 1/2) h, h = (hi - lo) / td_n: linear between neighbouring centres, the
 * end value held from lo to d_0 and from d_{n-1} to hi, zero outside [lo, hi).  Its
 * potential is U(d) = -integral of F from lo to min(d, hi) (0 below lo), integrated here
 * piece by piece.  dir receives the unit direction, *u the potential, *scale the sum of
 * the magnitudes of the table values F depends on (the term scale of the force).  com
 * holds all centres of mass (the anchors' for a self-adjusting region). */
static double orc_td_force(const orc_params *P, const double *com, const double R[3], double dir[3],
                           double *u, double *scale)
{
    dir[0] = dir[1] = dir[2] = 0.0;
    *u = 0.0;
    *scale = 0.0;
    if (P->td_n <= 0 ||
        (P->region != ORC_REGION_SLAB && P->region != ORC_REGION_SPHERE && P->region != ORC_REGION_SPHERES))
        return 0.0;
    double d;
    if (P->region == ORC_REGION_SPHERES) {
        /* self-adjusting region (Sec. 2.5 with Sec. 2.4).  Reading: the field acts along the
         * offset from the nearest anchor centre (the first of equally near ones), with the
         * table of a single sphere; the anchors feel no reaction (an external field) */
        int64_t n = P->n_mol;
        double best = INFINITY, qb[3] = {0.0, 0.0, 0.0};
        for (int32_t k = 0; k < P->n_anchors; ++k) {
            int64_t b = P->anchors[k];
            double q[3];
            for (int c = 0; c < 3; ++c) q[c] = orc_mi(R[c] - com[c * n + b], P->box[c]);
            double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
            if (r2 < best) {
                best = r2;
                qb[0] = q[0]; qb[1] = q[1]; qb[2] = q[2];
            }
        }
        d = sqrt(best);
        if (d > 0.0)
            for (int k = 0; k < 3; ++k) dir[k] = qb[k] / d;
    } else {
        d = orc_region_distance(P, R);
        if (d > 0.0) {
            if (P->region == ORC_REGION_SLAB) {
                dir[0] = orc_mi(R[0] - P->center[0], P->box[0]) > 0.0 ? 1.0 : -1.0;
            } else {
                for (int k = 0; k < 3; ++k) dir[k] = orc_mi(R[k] - P->center[k], P->box[k]) / d;
            }
        }
    }
    int n = P->td_n;
    double lo = P->td_lo, hi = P->td_hi, h = (hi - lo) / n;
    const double *F = P->td;
    if (d < lo) return 0.0;
    /* potential: the pieces [lo, d_0], [d_k, d_k+1] for each k, [d_n-1, hi] clipped at d */
    double top = d < hi ? d : hi;
    double integral = 0.0;
    double c0 = lo + 0.5 * h;
    integral += F[0] * ((top < c0 ? top : c0) - lo);
    for (int k = 0; k + 1 < n; ++k) {
        double a = lo + (k + 0.5) * h, b = lo + (k + 1.5) * h;
        if (top <= a) break;
        double e = top < b ? top : b;
        /* integral of the line through (a, F_k), (b, F_k+1) from a to e */
        double fa_ = F[k], fe = F[k] + (F[k + 1] - F[k]) * (e - a) / h;
        integral += 0.5 * (fa_ + fe) * (e - a);
    }
    double cn = lo + (n - 0.5) * h;
    if (top > cn) integral += F[n - 1] * (top - cn);
    *u = -integral;
    if (d >= hi) return 0.0;
    /* force value at d */
    double t = (d - lo) / h - 0.5;   /* position in units of h from the first centre */
    if (t <= 0.0) { *scale = fabs(F[0]); return F[0]; }
    if (t >= n - 1) { *scale = fabs(F[n - 1]); return F[n - 1]; }
    int k = (int)floor(t);
    double s = t - k;
    *scale = fabs(F[k]) + fabs(F[k + 1]);
    return F[k] * (1.0 - s) + F[k + 1] * s;
}

static double orc_weight(const orc_params *P, const double R[3])
{
    if (P->region == ORC_REGION_AT) return 1.0;
    if (P->region == ORC_REGION_CG) return 0.0;
    return orc_weight_of_distance(orc_region_distance(P, R), P->d_at, P->d_hy);
}

/* Centres of mass (3 x n_mol, SoA), weights (n_mol) and the stretch flag. */
/* Self-adjusting AT region (Sec. 2.5): spheres around the current centres of mass of the
 * anchor molecules, whose overlap forms the AT region.  Reading: a molecule's resolution
 * distance is its minimum-image distance to the nearest anchor centre, d = min_k |R - R_k|,
 * and w = w(d); since w falls with d this is the largest of the single-sphere weights (the
 * union of the spheres).  The anchors move with the simulation, so the region follows. */
static double orc_anchor_distance(const orc_params *P, const double *com, int64_t a)
{
    int64_t n = P->n_mol;
    double best = INFINITY;
    for (int32_t k = 0; k < P->n_anchors; ++k) {
        int64_t b = P->anchors[k];
        double q[3];
        for (int d = 0; d < 3; ++d) q[d] = orc_mi(com[d * n + a] - com[d * n + b], P->box[d]);
        double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
        if (r2 < best) best = r2;
    }
    return sqrt(best);
}

int orc_weights(const orc_params *P, const double *x, double *com, double *w, double *rho_out)
{
    int status = 0;
    int64_t n = P->n_mol;
#pragma omp parallel for schedule(static) reduction(| : status)
    for (int64_t a = 0; a < n; ++a) {
        double R[3], rho;
        orc_com(P, x, a, R, &rho);
        for (int d = 0; d < 3; ++d) com[d * n + a] = R[d];
        if (P->region != ORC_REGION_SPHERES) w[a] = orc_weight(P, R);
        if (rho_out) rho_out[a] = rho;
        if (P->spm > 1 && rho > P->rho_max) status |= ORC_STRETCH;
    }
    if (P->region == ORC_REGION_SPHERES) {
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < n; ++a)
            w[a] = orc_weight_of_distance(orc_anchor_distance(P, com, a), P->d_at, P->d_hy);
    }
    return status;
}

/* Unordered molecule pairs {a < b} whose minimum-image centre-of-mass distance is
 * below r_list (strict), by brute force over all pairs, in lexicographic order.
 * The test is r2 < rl2 with r2 = (dx^2 + dy^2) + dz^2 of mi(R_b - R_a).
 * pairs: 2 x cap int32 (row-major [k][2]).  Returns the pair count (may exceed cap;
 * only the first cap pairs are written). */
int64_t orc_pairs(const orc_params *P, const double *com, double rl2, int32_t *pairs, int64_t cap)
{
    int64_t n = P->n_mol;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        int64_t c = 0;
        for (int64_t b = a + 1; b < n; ++b) {
            double q[3];
            for (int d = 0; d < 3; ++d) q[d] = orc_mi(com[d * n + b] - com[d * n + a], P->box[d]);
            double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
            if (r2 < rl2) ++c;
        }
        cnt[a + 1] = c;
    }
    for (int64_t a = 0; a < n; ++a) cnt[a + 1] += cnt[a];
    int64_t total = cnt[n];
    if (pairs) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; ++a) {
            int64_t k = cnt[a];
            for (int64_t b = a + 1; b < n; ++b) {
                double q[3];
                for (int d = 0; d < 3; ++d) q[d] = orc_mi(com[d * n + b] - com[d * n + a], P->box[d]);
                double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
                if (r2 < rl2) {
                    if (k < cap) { pairs[2 * k] = (int32_t)a; pairs[2 * k + 1] = (int32_t)b; }
                    ++k;
                }
            }
        }
    }
    free(cnt);
    return total;
}

/* WCA pair term: returns f/r (so the force on the first particle is (f/r) * d with
 * d = x_first - x_second) and the potential 4 eps (s^12 - s^6) + eps, r2 < rc2. */
static void orc_wca(double r2, double eps, double sig, double *f_over_r, double *u)
{
    double s = (sig * sig) / r2;
    double s6 = s * s * s;
    *f_over_r = 24.0 * eps * s6 * (2.0 * s6 - 1.0) / r2;
    *u = 4.0 * eps * s6 * (s6 - 1.0) + eps;
}

/* Magnitude scale of a WCA pair term before cancellation: |48 eps s^12| + |24 eps s^6|,
 * divided by r^2 like f/r (the two terms of the force cancel at the cutoff). */
static double orc_wca_scale(double r2, double eps, double sig)
{
    double s = (sig * sig) / r2;
    double s6 = s * s * s;
    return 24.0 * eps * s6 * (2.0 * s6 + 1.0) / r2;
}

/* Cubic table of the CG force magnitude: interval k = clamp(floor((r - lo)/h), 0, n-2),
 * t = (r - lo)/h - k, f = ((c3 t + c2) t + c1) t + c0 with the FP32 coefficients
 * promoted to FP64.  r < lo raises the table-range flag (reading). */
double orc_table_eval(const float *tab, int n, double lo, double hi, double r, int *status)
{
    double h = (hi - lo) / (double)(n - 1);
    double u = (r - lo) / h;
    if (r < lo && status) *status |= ORC_TABLE_RANGE;
    double kf = floor(u);
    if (kf < 0.0) kf = 0.0;
    if (kf > (double)(n - 2)) kf = (double)(n - 2);
    int k = (int)kf;
    double t = u - kf;
    const float *c = tab + 4 * k;
    return (((double)c[3] * t + (double)c[2]) * t + (double)c[1]) * t + (double)c[0];
}

/* Sum of the magnitudes of the four Horner terms of a table lookup. */
static double orc_table_scale(const float *tab, int n, double lo, double hi, double r)
{
    double h = (hi - lo) / (double)(n - 1);
    double u = (r - lo) / h;
    double kf = floor(u);
    if (kf < 0.0) kf = 0.0;
    if (kf > (double)(n - 2)) kf = (double)(n - 2);
    double t = u - kf;
    const float *c = tab + 4 * (int)kf;
    return fabs((double)c[0]) + fabs((double)c[1] * t) + fabs((double)c[2] * t * t) + fabs((double)c[3] * t * t * t);
}

static double orc_silu(double z) { return z / (1.0 + exp(-z)); }

/* Learned CG force magnitude (reading of the learned-CG extension):
 * f(r) = scale * taper(r) * [W3 . silu(W2 silu(W1 x + b1) + b2) + b3], x = r / rc,
 * taper = 1 below rc - tw, cos^2 ramp to 0 at rc; below r_min the table is used. */
double orc_mlp_eval(const orc_params *P, double r, int *status)
{
    if (r < P->mlp_rmin && P->tab)
        return orc_table_eval(P->tab, P->tab_n, P->tab_lo, P->tab_hi, r, status);
    int H = P->mlp_hidden;
    const double *W1 = P->mlp, *b1 = W1 + H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
    double xin = r / P->mlp_rc;
    double h1[256];
    for (int k = 0; k < H; ++k) h1[k] = orc_silu(W1[k] * xin + b1[k]);
    double y = b3[0];
    for (int o = 0; o < H; ++o) {
        double z = b2[o];
        for (int k = 0; k < H; ++k) z += W2[o * H + k] * h1[k];
        y += W3[o] * orc_silu(z);
    }
    double tp = orc_weight_of_distance(r, P->mlp_rc - P->mlp_taper, P->mlp_taper);
    return P->mlp_scale * tp * y;
}

/* CG force between centres of mass: returns f/r and the potential (0 for table/MLP). */
static void orc_cg(const orc_params *P, double r2, double *f_over_r, double *u, int *status)
{
    if (P->cg_kind == ORC_CG_WCA) {
        orc_wca(r2, P->eps_cg, P->sig_cg, f_over_r, u);
        return;
    }
    double r = sqrt(r2);
    double f = (P->cg_kind == ORC_CG_TABLE)
                   ? orc_table_eval(P->tab, P->tab_n, P->tab_lo, P->tab_hi, r, status)
                   : orc_mlp_eval(P, r, status);
    *f_over_r = f / r;
    *u = 0.0;
}

static double orc_norm3(double a, double b, double c) { return sqrt((a * a + b * b) + c * c); }

/* Term-magnitude scale of the CG force, divided by r like f/r. */
static double orc_cg_scale(const orc_params *P, double r2, double f_over_r)
{
    if (P->cg_kind == ORC_CG_WCA) return orc_wca_scale(r2, P->eps_cg, P->sig_cg);
    double r = sqrt(r2);
    if (P->cg_kind == ORC_CG_TABLE) return orc_table_scale(P->tab, P->tab_n, P->tab_lo, P->tab_hi, r) / r;
    return fabs(f_over_r);
}

/* Forces on the sites of molecule a, summed over every other molecule b (no list):
 *   Eq. (1): ww = w_a w_b;  AT part if ww > 0: ww * sum of atom-atom WCA forces;
 *   (Eq. (2) instead: ww = (w_a + w_b) / 2 for both parts, energies w_a V^AT_a and
 *   (1 - w_a) V^CG_a, and the drift force of a hybrid molecule shared by mass fraction);
 *   CG part if ww < 1: (1 - ww) * F^CG(R_a - R_b), shared among a's sites by mass
 *   fraction m_i / M (reading: the paper leaves the distribution to sites open);
 *   plus the non-interpolated bonded terms.
 * Writes fa[3][spm], the absolute-sum scale amag[spm] and the molecule's half-share
 * of the energies e[0..2] = U_AT, U_CG, U_bond (each pair term counted half from
 * each side).  amag sums, over all contributions to a site, the magnitudes of the
 * terms each contribution is made of before they cancel: 24 eps s^6 (2 s^6 + 1)/r
 * for a WCA pair (the two terms cancel at the cutoff), (1 + ww) for the CG share
 * (1 - ww cancels as ww -> 1), K (r + b0) for a harmonic bond (r - b0 cancels at
 * rest), the four Horner terms of a table lookup, |f| (1 + r^2/R0^2)/(1 - r^2/R0^2)
 * for FENE; it bounds the rounding error of any evaluation order of the same
 * formulas, including sites whose net force is pure rounding noise. */
/* part selects the terms for multiple time stepping (Sec. 2.6): ORC_PART_ALL every term;
 * ORC_PART_FAST the atomistic pair part, the atomistic share -V^AT grad w of the drift and
 * the bonds; ORC_PART_SLOW the CG pair part, the CG share +V^CG grad w of the drift and the
 * correction force.  The energies are those of the included terms. */
static int orc_mol_forces(const orc_params *P, const double *x, const double *com, const double *w,
                          int64_t a, double *fa, double *amag, double e[4], int part)
{
    int status = 0;
    int spm = P->spm;
    int64_t n = P->n_mol;
    double M = orc_mol_mass(P);
    double rcA2 = P->rc_at * P->rc_at, rcC2 = P->rc_cg * P->rc_cg;
    for (int k = 0; k < 3 * spm; ++k) fa[k] = 0.0;
    for (int k = 0; k < spm; ++k) amag[k] = 0.0;
    e[0] = e[1] = e[2] = e[3] = 0.0;
    double Ra[3] = {com[a], com[n + a], com[2 * n + a]};
    const int hamiltonian = P->scheme == ORC_SCHEME_HAMILTONIAN;
    /* Eq. (2): the molecule's single-molecule potentials V^AT_a, V^CG_a (half of each
     * intermolecular pair potential, so that the sum over molecules is the total) and
     * their term scales */
    double vat = 0.0, vcg = 0.0, avat = 0.0, avcg = 0.0;

    for (int64_t b = 0; b < n; ++b) {
        if (b == a) continue;
        /* weight of the AT part of the pair force: Eq. (1) w_a w_b; Eq. (2) gives
         * -grad of (w_a V^AT_a + w_b V^AT_b), i.e. (w_a + w_b) / 2 per pair potential */
        double ww = hamiltonian ? 0.5 * (w[a] + w[b]) : w[a] * w[b];
        if (ww > 0.0 && part != ORC_PART_SLOW) {
            for (int i = 0; i < spm; ++i) {
                for (int j = 0; j < spm; ++j) {
                    double d[3];
                    for (int q = 0; q < 3; ++q)
                        d[q] = orc_mi(orc_sx(P, x, q, a * spm + i) - orc_sx(P, x, q, b * spm + j), P->box[q]);
                    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                    if (r2 < rcA2) {
                        double fr, u;
                        orc_wca(r2, P->eps_at, P->sig_at, &fr, &u);
                        double c[3] = {ww * fr * d[0], ww * fr * d[1], ww * fr * d[2]};
                        for (int q = 0; q < 3; ++q) fa[3 * i + q] += c[q];
                        amag[i] += ww * orc_wca_scale(r2, P->eps_at, P->sig_at) * sqrt(r2);
                        if (hamiltonian) {
                            double s6 = pow(P->sig_at * P->sig_at / r2, 3);
                            vat += 0.5 * u;
                            avat += 0.5 * (4.0 * P->eps_at * s6 * (s6 + 1.0) + P->eps_at);
                        } else {
                            e[0] += 0.5 * ww * u;
                        }
                    }
                }
            }
        }
        if (ww < 1.0 && part != ORC_PART_FAST) {
            double D[3];
            for (int q = 0; q < 3; ++q) D[q] = orc_mi(Ra[q] - com[q * n + b], P->box[q]);
            double r2 = (D[0] * D[0] + D[1] * D[1]) + D[2] * D[2];
            if (r2 < rcC2) {
                double fr, u;
                orc_cg(P, r2, &fr, &u, &status);
                double scale = (1.0 + ww) * orc_cg_scale(P, r2, fr) * sqrt(r2);
                for (int i = 0; i < spm; ++i) {
                    double sc = (1.0 - ww) * (P->mass[i] / M) * fr;
                    double c[3] = {sc * D[0], sc * D[1], sc * D[2]};
                    for (int q = 0; q < 3; ++q) fa[3 * i + q] += c[q];
                    amag[i] += (P->mass[i] / M) * scale;
                }
                if (hamiltonian) {
                    double s6 = pow(P->sig_cg * P->sig_cg / r2, 3);
                    vcg += 0.5 * u;
                    avcg += 0.5 * (4.0 * P->eps_cg * s6 * (s6 + 1.0) + P->eps_cg);
                } else {
                    e[1] += 0.5 * (1.0 - ww) * u;
                }
            }
        }
    }
    if (hamiltonian) {
        e[0] += w[a] * vat;
        e[1] += (1.0 - w[a]) * vcg;
        /* drift force: -(V^AT_a - V^CG_a) grad_x w(R_a); grad_{x_i} R_a = (m_i / M) I */
        double g[3];
        orc_weight_gradient(P, Ra, g);
        double gn = orc_norm3(g[0], g[1], g[2]);
        if (gn > 0.0) {
            for (int i = 0; i < spm; ++i) {
                double mf = P->mass[i] / M;
                for (int q = 0; q < 3; ++q) fa[3 * i + q] += -(vat - vcg) * g[q] * mf;
                amag[i] += (avat + avcg) * gn * mf;
            }
        }
    }

    if (P->td_n > 0 && part != ORC_PART_FAST) {
        double dir[3], ut, sc;
        double ft = orc_td_force(P, com, Ra, dir, &ut, &sc);
        for (int i = 0; i < spm; ++i) {
            double mf = P->mass[i] / M;
            for (int q = 0; q < 3; ++q) fa[3 * i + q] += mf * ft * dir[q];
            amag[i] += mf * sc;
        }
        e[3] += ut;
    }

    if (part == ORC_PART_SLOW) {
        /* no bonds in the slow part */
    } else if (P->bond_kind == ORC_BOND_HARMONIC) {
        /* every pair of sites of the molecule is bonded: U = K/2 (r - b0)^2 */
        for (int i = 0; i < spm; ++i) {
            for (int k = 0; k < spm; ++k) {
                if (k == i) continue;
                double d[3];
                for (int q = 0; q < 3; ++q)
                    d[q] = orc_mi(orc_sx(P, x, q, a * spm + i) - orc_sx(P, x, q, a * spm + k), P->box[q]);
                double r = orc_norm3(d[0], d[1], d[2]);
                double fr = -P->k_bond * (r - P->r0_bond) / r;
                double c[3] = {fr * d[0], fr * d[1], fr * d[2]};
                for (int q = 0; q < 3; ++q) fa[3 * i + q] += c[q];
                amag[i] += P->k_bond * (r + P->r0_bond);
                if (k > i) e[2] += 0.5 * P->k_bond * (r - P->r0_bond) * (r - P->r0_bond);
            }
        }
    } else if (P->bond_kind == ORC_BOND_FENE) {
        /* beads a-1, a, a+1 of one chain (chains are runs of chain_len consecutive
         * molecules): U = -k R0^2 / 2 * ln(1 - (r / R0)^2) */
        int64_t chain = a / P->chain_len;
        for (int side = -1; side <= 1; side += 2) {
            int64_t b = a + side;
            if (b < 0 || b >= n || b / P->chain_len != chain) continue;
            double d[3];
            for (int q = 0; q < 3; ++q)
                d[q] = orc_mi(orc_sx(P, x, q, a) - orc_sx(P, x, q, b), P->box[q]);
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            double R02 = P->r0_bond * P->r0_bond;
            if (r2 >= R02) { status |= ORC_FENE; continue; }
            double fr = -P->k_bond / (1.0 - r2 / R02);
            double c[3] = {fr * d[0], fr * d[1], fr * d[2]};
            for (int q = 0; q < 3; ++q) fa[q] += c[q];
            amag[0] += orc_norm3(c[0], c[1], c[2]) * (1.0 + r2 / R02) / (1.0 - r2 / R02);
            e[2] += 0.5 * (-0.5 * P->k_bond * R02 * log(1.0 - r2 / R02));
        }
    }
    for (int k = 0; k < 3 * spm; ++k)
        if (!isfinite(fa[k])) status |= ORC_NONFINITE;
    return status;
}

/* Forces on every site (f: 3 x N_s SoA), absolute-sum scales (amag: N_s) and the
 * energies e[0..3] = U_AT, U_CG, U_bond, U_corr (the correction force's potential).
 * Returns the status bit mask. */
int orc_forces_part(const orc_params *P, const double *x, double *f, double *amag, double *energy, int part)
{
    int64_t n = P->n_mol, spm = P->spm, ns = n * spm;
    double *com = (double *)malloc(sizeof(double) * 3 * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *em = (double *)malloc(sizeof(double) * 4 * n);
    int status = orc_weights(P, x, com, w, NULL);
#pragma omp parallel for schedule(dynamic, 16) reduction(| : status)
    for (int64_t a = 0; a < n; ++a) {
        double fa[3 * ORC_MAX_SITES], am[ORC_MAX_SITES];
        status |= orc_mol_forces(P, x, com, w, a, fa, am, em + 4 * a, part);
        for (int i = 0; i < spm; ++i) {
            for (int q = 0; q < 3; ++q) f[q * ns + a * spm + i] = fa[3 * i + q];
            if (amag) amag[a * spm + i] = am[i];
        }
    }
    if (energy) {
        energy[0] = energy[1] = energy[2] = energy[3] = 0.0;
        for (int64_t a = 0; a < n; ++a)
            for (int k = 0; k < 4; ++k) energy[k] += em[4 * a + k];
    }
    free(com); free(w); free(em);
    return status;
}

int orc_forces(const orc_params *P, const double *x, double *f, double *amag, double *energy)
{
    return orc_forces_part(P, x, f, amag, energy, ORC_PART_ALL);
}

/* Forces on the sites of the selected molecules only (f: [n_sel][3][spm] ... stored as
 * f[(s * 3 + q) * spm + i]), same definition as orc_forces; O(n_mol) per molecule. */
int orc_forces_sampled(const orc_params *P, const double *x, const int64_t *sel, int64_t n_sel,
                       double *f, double *amag)
{
    int64_t n = P->n_mol, spm = P->spm;
    double *com = (double *)malloc(sizeof(double) * 3 * n);
    double *w = (double *)malloc(sizeof(double) * n);
    int status = orc_weights(P, x, com, w, NULL);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : status)
    for (int64_t s = 0; s < n_sel; ++s) {
        double fa[3 * ORC_MAX_SITES], am[ORC_MAX_SITES], e[4];
        status |= orc_mol_forces(P, x, com, w, sel[s], fa, am, e, ORC_PART_ALL);
        for (int i = 0; i < spm; ++i) {
            for (int q = 0; q < 3; ++q) f[(s * 3 + q) * spm + i] = fa[3 * i + q];
            if (amag) amag[s * spm + i] = am[i];
        }
    }
    free(com); free(w);
    return status;
}

double orc_kinetic(const orc_params *P, const double *v)
{
    int64_t n = P->n_mol, spm = P->spm, ns = n * spm;
    double ke = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        double m = P->mass[s % spm];
        ke += 0.5 * m * ((v[s] * v[s] + v[ns + s] * v[ns + s]) + v[2 * ns + s] * v[2 * ns + s]);
    }
    return ke;
}

/* Velocity Verlet, n_steps of size dt, in place on x, v (f returns F(x_final)):
 *   v += F dt / (2m); x += v dt; fold each site into [0, L); F = F(x); v += F dt / (2m).
 * Force interpolation has no conserved energy (Sec. 2.3); energies are diagnostics.
 * e_out (optional): (n_steps + 1) x 5 rows of U_AT, U_CG, U_bond, U_corr, KE. */
int orc_vv(const orc_params *P, double *x, double *v, double *f, double dt, int32_t n_steps,
           double *e_out)
{
    int64_t n = P->n_mol, spm = P->spm, ns = n * spm;
    double e[4];
    int status = orc_forces(P, x, f, NULL, e);
    if (e_out) { for (int k = 0; k < 4; ++k) e_out[k] = e[k]; e_out[4] = orc_kinetic(P, v); }
    for (int32_t step = 0; step < n_steps; ++step) {
        for (int q = 0; q < 3; ++q) {
            double L = P->box[q];
            for (int64_t s = 0; s < ns; ++s) {
                double m = P->mass[s % spm];
                v[q * ns + s] += f[q * ns + s] * dt / (2.0 * m);
                double y = x[q * ns + s] + v[q * ns + s] * dt;
                if (y >= L) y -= L;
                else if (y < 0.0) y += L;
                x[q * ns + s] = y;
            }
        }
        status |= orc_forces(P, x, f, NULL, e);
        for (int q = 0; q < 3; ++q)
            for (int64_t s = 0; s < ns; ++s)
                v[q * ns + s] += f[q * ns + s] * dt / (2.0 * P->mass[s % spm]);
        if (e_out) {
            double *r = e_out + 5 * (step + 1);
            for (int k = 0; k < 4; ++k) r[k] = e[k];
            r[4] = orc_kinetic(P, v);
        }
    }
    return status;
}

/* Multiple time stepping (Sec. 2.6): reversible RESPA (Tuckerman, Berne & Martyna 1992)
 * with the slow part (CG pair forces, the CG share of the drift, the correction force)
 * on the outer step Dt = n_inner dt and the fast part (atomistic pair forces, the
 * atomistic share of the drift, bonds) on the inner step dt.  One outer step:
 *   v += F_slow Dt / (2m);
 *   n_inner times: v += F_fast dt / (2m); x += v dt (folded); v += F_fast(x) dt / (2m);
 *   v += F_slow(x) Dt / (2m).
 * f returns the total force F_fast + F_slow at the final positions.  e_out (optional):
 * (n_outer + 1) x 5 rows of U_AT, U_CG, U_bond, U_corr, KE after each outer step. */
int orc_respa(const orc_params *P, double *x, double *v, double *f, double dt, int32_t n_inner,
              int32_t n_outer, double *e_out)
{
    int64_t n = P->n_mol, spm = P->spm, ns = n * spm;
    double Dt = dt * n_inner;
    double *ff = (double *)malloc(sizeof(double) * 3 * ns);
    double *fs = (double *)malloc(sizeof(double) * 3 * ns);
    double e[4];
    int status = orc_forces_part(P, x, ff, NULL, NULL, ORC_PART_FAST);
    status |= orc_forces_part(P, x, fs, NULL, NULL, ORC_PART_SLOW);
    if (e_out) {
        status |= orc_forces(P, x, f, NULL, e);
        for (int k = 0; k < 4; ++k) e_out[k] = e[k];
        e_out[4] = orc_kinetic(P, v);
    }
    for (int32_t o = 0; o < n_outer; ++o) {
        for (int q = 0; q < 3; ++q)
            for (int64_t s = 0; s < ns; ++s)
                v[q * ns + s] += fs[q * ns + s] * Dt / (2.0 * P->mass[s % spm]);
        for (int32_t j = 0; j < n_inner; ++j) {
            for (int q = 0; q < 3; ++q) {
                double L = P->box[q];
                for (int64_t s = 0; s < ns; ++s) {
                    v[q * ns + s] += ff[q * ns + s] * dt / (2.0 * P->mass[s % spm]);
                    double y = x[q * ns + s] + v[q * ns + s] * dt;
                    if (y >= L) y -= L;
                    else if (y < 0.0) y += L;
                    x[q * ns + s] = y;
                }
            }
            status |= orc_forces_part(P, x, ff, NULL, NULL, ORC_PART_FAST);
            for (int q = 0; q < 3; ++q)
                for (int64_t s = 0; s < ns; ++s)
                    v[q * ns + s] += ff[q * ns + s] * dt / (2.0 * P->mass[s % spm]);
        }
        status |= orc_forces_part(P, x, fs, NULL, NULL, ORC_PART_SLOW);
        for (int q = 0; q < 3; ++q)
            for (int64_t s = 0; s < ns; ++s)
                v[q * ns + s] += fs[q * ns + s] * Dt / (2.0 * P->mass[s % spm]);
        if (e_out) {
            status |= orc_forces(P, x, f, NULL, e);
            double *r = e_out + 5 * (o + 1);
            for (int k = 0; k < 4; ++k) r[k] = e[k];
            r[4] = orc_kinetic(P, v);
        }
    }
    for (int64_t k = 0; k < 3 * ns; ++k) f[k] = ff[k] + fs[k];
    free(ff); free(fs);
    return status;
}

/* Density profile along the resolution coordinate (Sec. 2.4): adds to counts[k] the
 * number of molecules whose centre-of-mass distance d from the AT centre satisfies
 * lo + k h <= d < lo + (k + 1) h, h = (hi - lo) / n_bins, with the bin index taken as
 * floor((d - lo) / h) (the top bin also takes a d that rounds to n_bins below hi). */
int orc_density_profile(const orc_params *P, const double *x, int32_t n_bins, double lo, double hi,
                        int64_t *counts)
{
    int64_t n = P->n_mol;
    double *com = (double *)malloc(sizeof(double) * 3 * n);
    double *w = (double *)malloc(sizeof(double) * n);
    int status = orc_weights(P, x, com, w, NULL);
    double h = (hi - lo) / n_bins;
    for (int64_t a = 0; a < n; ++a) {
        double R[3] = {com[a], com[n + a], com[2 * n + a]};
        double d = P->region == ORC_REGION_SPHERES ? orc_anchor_distance(P, com, a) : orc_region_distance(P, R);
        if (d < lo || d >= hi) continue;
        int64_t k = (int64_t)floor((d - lo) / h);
        if (k > n_bins - 1) k = n_bins - 1;
        counts[k] += 1;
    }
    free(com); free(w);
    return status;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output for counter value k of a
 * stream with key s is the finaliser applied to s + (k + 1) * 0x9E3779B97F4A7C15. */
static uint64_t orc_splitmix64(uint64_t s, uint64_t k)
{
    uint64_t z = s + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Bin volumes by sampling, for the density profile of a region whose bins have no closed
 * form (a union of moving spheres, Sec. 2.5 with Sec. 2.4).  Reading: n_samples points
 * uniform in the box, coordinate c of point i at L_c * u with u = (top 53 bits of
 * SplitMix64(seed, 3 i + c)) / 2^53; each point is binned by its resolution distance like a
 * centre of mass (for anchor spheres, the nearest anchor centre of the configuration x).
 * Adds to counts; V_k is then counts_k / n_samples times the box volume. */
int orc_region_volumes(const orc_params *P, const double *x, int64_t n_samples, uint64_t seed, int32_t n_bins,
                       double lo, double hi, int64_t *counts)
{
    int64_t n = P->n_mol;
    double *com = (double *)malloc(sizeof(double) * 3 * n);
    double *w = (double *)malloc(sizeof(double) * n);
    int status = orc_weights(P, x, com, w, NULL);
    double h = (hi - lo) / n_bins;
    for (int64_t i = 0; i < n_samples; ++i) {
        double p[3];
        for (int c = 0; c < 3; ++c) {
            uint64_t z = orc_splitmix64(seed, 3 * (uint64_t)i + (uint64_t)c);
            p[c] = P->box[c] * ((double)(z >> 11) * 0x1.0p-53);
        }
        double d;
        if (P->region == ORC_REGION_SPHERES) {
            double best = INFINITY;
            for (int32_t k = 0; k < P->n_anchors; ++k) {
                int64_t b = P->anchors[k];
                double q[3];
                for (int c = 0; c < 3; ++c) q[c] = orc_mi(p[c] - com[c * n + b], P->box[c]);
                double r2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
                if (r2 < best) best = r2;
            }
            d = sqrt(best);
        } else {
            d = orc_region_distance(P, p);
        }
        if (d < lo || d >= hi) continue;
        int64_t k = (int64_t)floor((d - lo) / h);
        if (k > n_bins - 1) k = n_bins - 1;
        counts[k] += 1;
    }
    free(com); free(w);
    return status;
}

/* One refinement of the correction force from a density profile (Sec. 2.4: the force is
 * built from the distorted density profile and refined iteratively).  Readings: the
 * number density of bin k is rho_k = counts_k / (n_frames V_k), V_k the bin's volume (slab:
 * both sides of the mid-plane, 2 h L_y L_z; sphere: the shell 4/3 pi (r_k+1^3 - r_k^3),
 * r_k = lo + k h); its slope at bin centre k is the central difference
 * (rho_k+1 - rho_k-1) / (2 h), one-sided at the two end bins, 0 for a single bin; and
 * the update is F_k <- F_k - prefactor * slope_k (the usual prefactor is
 * M / (rho_0^2 kappa_T)).  With vol_counts the volumes are sampled ones
 * (orc_region_volumes over n_vol_samples points in total), for any region. */
void orc_tdforce_update(const orc_params *P, double *F, int32_t n, double lo, double hi,
                        const int64_t *counts, int64_t n_frames, double prefactor,
                        const int64_t *vol_counts, int64_t n_vol_samples)
{
    double h = (hi - lo) / n;
    double *rho = (double *)malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        double V;
        if (vol_counts) {
            /* sampled volumes (orc_region_volumes); an unsampled bin counts as empty */
            V = ((double)vol_counts[k] / (double)n_vol_samples) * ((P->box[0] * P->box[1]) * P->box[2]);
            if (vol_counts[k] == 0) {
                rho[k] = 0.0;
                continue;
            }
        } else if (P->region == ORC_REGION_SLAB) {
            V = 2.0 * h * P->box[1] * P->box[2];
        } else {
            double r0 = lo + k * h, r1 = lo + (k + 1) * h;
            V = (4.0 / 3.0) * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        }
        rho[k] = (double)counts[k] / ((double)n_frames * V);
    }
    for (int k = 0; k < n; ++k) {
        double slope;
        if (n == 1) slope = 0.0;
        else if (k == 0) slope = (rho[1] - rho[0]) / h;
        else if (k == n - 1) slope = (rho[n - 1] - rho[n - 2]) / h;
        else slope = (rho[k + 1] - rho[k - 1]) / (2.0 * h);
        F[k] = F[k] - prefactor * slope;
    }
    free(rho);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads later oracle calls use (timing runs). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
