// Linked-cell list of molecule centres of mass (Sec. 5, introduction: the
// linked-cell list behind ESPResSo++'s domain decomposition), rebuilt as a
// Morton-ordered counting sort on the GPU:
//   keys (cell -> Morton rank) -> per-cell counts (atomics) -> exclusive scan
//   (one workgroup, wavefront shuffles) -> scatter -> per-cell insertion sort by
//   caller index (makes the order a pure function of the positions) -> permute
//   the state into the new order.
// and the Verlet list of molecule pairs: every molecule scans the 27 cells around
// its own (fewer when a dimension has < 3 cells) and keeps the molecules whose
// minimum-image centre distance is strictly below r_list.  The list is stored
// row-major (ELL): nbr[slot * cap + k]; every row is padded with the row's own
// slot up to a multiple of 4 so that the force kernel can fetch four entries with
// one 16-byte load and issue their gathers unconditionally.
#include "adres_internal.h"

namespace adres {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_cell_keys(DevParams P, Grid G, const int *__restrict__ cell_rank,
                                                      const double4 *__restrict__ Rw, int *__restrict__ key,
                                                      int *__restrict__ count)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    const double4 r = Rw[t];
    int cx = cell_coord(r.x, G.inv_len[0], G.n[0]);
    int cy = cell_coord(r.y, G.inv_len[1], G.n[1]);
    int cz = cell_coord(r.z, G.inv_len[2], G.n[2]);
    int k = cell_rank[cx + G.n[0] * (cy + G.n[1] * cz)];
    key[t] = k;
    atomicAdd(&count[k], 1);
}

// Exclusive scan of count[0..n) into start[0..n] in three launches: each workgroup
// scans a tile of 1024 counts (4 per thread; wavefront shuffles, then the 4 wave
// totals), one workgroup scans the tile totals, a third pass adds the tile offsets
// and resets count and fill for the next build.
constexpr int kScanThreads = 256;
constexpr int kScanTile = 4 * kScanThreads;

__device__ __forceinline__ int block_exclusive_scan(int v, int &total)
{
    __shared__ int wave_tot[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        before += w < wave ? wave_tot[w] : 0;
        total += wave_tot[w];
    }
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int *__restrict__ count, int n,
                                                             int *__restrict__ start, int *__restrict__ tiles)
{
    const int base = blockIdx.x * kScanTile + 4 * threadIdx.x;
    int c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = base + j < n ? count[base + j] : 0;
    const int mine = (c[0] + c[1]) + (c[2] + c[3]);
    int total;
    int run = block_exclusive_scan(mine, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) start[base + j] = run;
        run += c[j];
    }
    if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

// scans up to kScanTile tile totals in one workgroup; start[n] = grand total
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_totals(int *__restrict__ tiles, int n_tiles,
                                                                   int *__restrict__ start, int n)
{
    const int base = 4 * threadIdx.x;
    int c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = base + j < n_tiles ? tiles[base + j] : 0;
    const int mine = (c[0] + c[1]) + (c[2] + c[3]);
    int total;
    int run = block_exclusive_scan(mine, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n_tiles) tiles[base + j] = run;
        run += c[j];
    }
    if (threadIdx.x == 0) start[n] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int *__restrict__ count, int n, int *__restrict__ start,
                                                           const int *__restrict__ tiles, int *__restrict__ fill)
{
    const int i = blockIdx.x * kScanThreads + threadIdx.x;
    if (i >= n) return;
    start[i] += tiles[i / kScanTile];
    count[i] = 0;
    if (fill) fill[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_scatter_slots(int n_mol, const int *__restrict__ key,
                                                          const int *__restrict__ start, int *__restrict__ fill,
                                                          int *__restrict__ new_from)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_mol) return;
    int k = key[i];
    int pos = start[k] + atomicAdd(&fill[k], 1);
    new_from[pos] = i;
}

__global__ __launch_bounds__(kBlock) void k_sort_within_cells(int n_cells, const int *__restrict__ start,
                                                              const int *__restrict__ perm_old,
                                                              int *__restrict__ new_from)
{
    int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= n_cells) return;
    int lo = start[c], hi = start[c + 1];
    for (int i = lo + 1; i < hi; ++i) {
        int v = new_from[i];
        int tag = perm_old[v];
        int j = i - 1;
        while (j >= lo && perm_old[new_from[j]] > tag) {
            new_from[j + 1] = new_from[j];
            --j;
        }
        new_from[j + 1] = v;
    }
}

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_permute(DevParams P, const int *__restrict__ new_from, StateBufs src,
                                                    StateBufs dst, int *__restrict__ inv_perm,
                                                    double4 *__restrict__ R_ref, int with_v)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    const int64_t ns = P.n_sites;
    int i = new_from[t];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < SPM; ++k) {
            dst.x[d * ns + (int64_t)t * SPM + k] = src.x[d * ns + (int64_t)i * SPM + k];
            if (with_v) dst.v[d * ns + (int64_t)t * SPM + k] = src.v[d * ns + (int64_t)i * SPM + k];
        }
    }
    const double4 r = src.Rw[i];
    dst.Rw[t] = r;
    R_ref[t] = r;
    dst.rho[t] = src.rho[i];
#pragma unroll
    for (int j = 0; j < 3 * SPM; ++j) dst.off[(int64_t)t * (3 * SPM) + j] = src.off[(int64_t)i * (3 * SPM) + j];
    dst.key[t] = src.key[i];
    int caller = src.perm[i];
    dst.perm[t] = caller;
    inv_perm[caller] = t;
}

__device__ __forceinline__ int wrap_cell(int c, int n)
{
    c += n;
    return c >= n ? (c >= 2 * n ? c - 2 * n : c - n) : c;
}

__global__ __launch_bounds__(kBlock) void k_list_build(DevParams P, Grid G, const int *__restrict__ rank_cell,
                                                       const int *__restrict__ cell_rank,
                                                       const int *__restrict__ start, const double4 *__restrict__ Rw,
                                                       const int *__restrict__ key, double rl2,
                                                       int *__restrict__ nbr, int *__restrict__ cnt, int cap,
                                                       Ctrl *ctrl)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_mol) return;
    const double4 me = Rw[t];
    const int c = rank_cell[key[t]];
    const int cx = c % G.n[0], cy = (c / G.n[0]) % G.n[1], cz = c / (G.n[0] * G.n[1]);
    int *row = nbr + (int64_t)t * cap;
    int k = 0;
    for (int oz = G.off_lo[2]; oz <= G.off_hi[2]; ++oz) {
        const int z = wrap_cell(cz + oz, G.n[2]);
        for (int oy = G.off_lo[1]; oy <= G.off_hi[1]; ++oy) {
            const int y = wrap_cell(cy + oy, G.n[1]);
            for (int ox = G.off_lo[0]; ox <= G.off_hi[0]; ++ox) {
                const int x = wrap_cell(cx + ox, G.n[0]);
                const int r = cell_rank[x + G.n[0] * (y + G.n[1] * z)];
                const int hi = start[r + 1];
                for (int u = start[r]; u < hi; ++u) {
                    if (u == t) continue;
                    const double4 o = Rw[u];
                    double dx = mi(o.x - me.x, P.box[0], P.half[0]);
                    double dy = mi(o.y - me.y, P.box[1], P.half[1]);
                    double dz = mi(o.z - me.z, P.box[2], P.half[2]);
                    if (dist2_exact(dx, dy, dz) < rl2) {
                        if (k < cap) row[k] = u;
                        ++k;
                    }
                }
            }
        }
    }
    cnt[t] = k;
    if (k > cap) {
        atomicOr(&ctrl->overflow, 1);
        atomicMax(&ctrl->max_count, k);
        atomicMin(&ctrl->halt, -1);   // stops every kernel of a step chunk until regrown
    } else {
        for (int j = k; j < ((k + 3) & ~3); ++j) row[j] = t;   // padding: the row's own slot
    }
}

// LDS-staged build: one workgroup per brick of kBrick^3 cells stages the centres of
// the (kBrick+2)^3 halo cells in LDS, then each home molecule of the brick scans its 27
// neighbour cells from LDS.  Rows come out in the same order as k_list_build (stencil
// order, then slot order inside a cell).  A brick whose halo holds more molecules than
// fit in LDS falls back to global loads.  Needs >= 3 cells per dimension.
constexpr int kBrick = 4;
constexpr int kHalo = kBrick + 2;
constexpr int kHaloCells = kHalo * kHalo * kHalo;
constexpr int kBrickCells = kBrick * kBrick * kBrick;
constexpr int kLdsMol = 1536;

__global__ __launch_bounds__(kBlock) void k_list_build_lds(DevParams P, Grid G, const int *__restrict__ cell_rank,
                                                           const int *__restrict__ start,
                                                           const double4 *__restrict__ Rw, double rl2,
                                                           int *__restrict__ nbr, int *__restrict__ cnt, int cap,
                                                           Ctrl *ctrl, int3 nbricks)
{
    __shared__ double4 sR[kLdsMol];
    __shared__ int sFirst[kHaloCells];   // first slot of each halo cell
    __shared__ int sOff[kHaloCells + 1]; // LDS offset of each halo cell
    __shared__ int sHome[kBrickCells + 1];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int bx = b % nbricks.x, by = (b / nbricks.x) % nbricks.y, bz = b / (nbricks.x * nbricks.y);
    const int ox0 = bx * kBrick - 1, oy0 = by * kBrick - 1, oz0 = bz * kBrick - 1;

    // halo cell sizes, exclusive scan into sOff (one thread per halo cell)
    int my_cnt = 0;
    if (tid < kHaloCells) {
        const int hx = tid % kHalo, hy = (tid / kHalo) % kHalo, hz = tid / (kHalo * kHalo);
        const int cx = wrap_cell(ox0 + hx, G.n[0]), cy = wrap_cell(oy0 + hy, G.n[1]), cz = wrap_cell(oz0 + hz, G.n[2]);
        const int r = cell_rank[cx + G.n[0] * (cy + G.n[1] * cz)];
        sFirst[tid] = start[r];
        my_cnt = start[r + 1] - start[r];
    }
    {
        __shared__ int wave_tot[kBlock / 64];
        const int lane = tid & 63, wave = tid >> 6;
        int incl = my_cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wave_tot[wave] = incl;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            before += w < wave ? wave_tot[w] : 0;
            total += wave_tot[w];
        }
        if (tid < kHaloCells) sOff[tid] = before + incl - my_cnt;
        if (tid == 0) sOff[kHaloCells] = total;
    }
    __syncthreads();
    // home cells of the brick (inside the grid) and their counts
    if (tid == 0) {
        int acc = 0;
        for (int c = 0; c < kBrickCells; ++c) {
            sHome[c] = acc;
            const int lx = c % kBrick, ly = (c / kBrick) % kBrick, lz = c / (kBrick * kBrick);
            const int gx = bx * kBrick + lx, gy = by * kBrick + ly, gz = bz * kBrick + lz;
            if (gx < G.n[0] && gy < G.n[1] && gz < G.n[2]) {
                const int h = (lx + 1) + kHalo * ((ly + 1) + kHalo * (lz + 1));
                acc += sOff[h + 1] - sOff[h];
            }
        }
        sHome[kBrickCells] = acc;
    }
    __syncthreads();
    const bool staged = sOff[kHaloCells] <= kLdsMol;
    if (staged) {
        // stage: LDS entry i belongs to the halo cell h with sOff[h] <= i < sOff[h + 1], whose
        // molecules are the contiguous slots sFirst[h] ..
        const int total = sOff[kHaloCells];
        for (int i = tid; i < total; i += kBlock) {
            int lo = 0, hi = kHaloCells - 1;   // largest h with sOff[h] <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sOff[mid] <= i) lo = mid; else hi = mid - 1;
            }
            const int slot = sFirst[lo] + (i - sOff[lo]);
            sR[i] = Rw[slot];
        }
    }
    __syncthreads();

    const int n_home = sHome[kBrickCells];
    for (int hm = tid; hm < n_home; hm += kBlock) {
        int c = 0;
        while (sHome[c + 1] <= hm) ++c;   // brick cell of this home molecule
        const int lx = c % kBrick, ly = (c / kBrick) % kBrick, lz = c / (kBrick * kBrick);
        const int hh = (lx + 1) + kHalo * ((ly + 1) + kHalo * (lz + 1));
        const int t = sFirst[hh] + (hm - sHome[c]);
        const double4 me = staged ? sR[sOff[hh] + (hm - sHome[c])] : Rw[t];
        int *row = nbr + (int64_t)t * cap;
        int k = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int h = (lx + 1 + dx) + kHalo * ((ly + 1 + dy) + kHalo * (lz + 1 + dz));
                    const int n_h = sOff[h + 1] - sOff[h];
                    for (int i = 0; i < n_h; ++i) {
                        const int u = sFirst[h] + i;
                        if (u == t) continue;
                        const double4 o = staged ? sR[sOff[h] + i] : Rw[u];
                        const double ddx = mi(o.x - me.x, P.box[0], P.half[0]);
                        const double ddy = mi(o.y - me.y, P.box[1], P.half[1]);
                        const double ddz = mi(o.z - me.z, P.box[2], P.half[2]);
                        if (dist2_exact(ddx, ddy, ddz) < rl2) {
                            if (k < cap) row[k] = u;
                            ++k;
                        }
                    }
                }
        cnt[t] = k;
        if (k > cap) {
            atomicOr(&ctrl->overflow, 1);
            atomicMax(&ctrl->max_count, k);
            atomicMin(&ctrl->halt, -1);
        } else {
            for (int j = k; j < ((k + 3) & ~3); ++j) row[j] = t;
        }
    }
}

// Half list for per-pair work (the learned CG force): every unordered pair once,
// as (t, u) with t < u, and for every full-list entry the id of its pair.
__global__ __launch_bounds__(kBlock) void k_up_count(int n, const int *__restrict__ nbr, const int *__restrict__ cnt,
                                                     int cap, int *__restrict__ cnt_up)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const int *row = nbr + (int64_t)t * cap;
    int c = 0;
    for (int k = 0; k < cnt[t]; ++k) c += row[k] > t;
    cnt_up[t] = c;
}

__global__ __launch_bounds__(kBlock) void k_up_fill(int n, const int *__restrict__ nbr, const int *__restrict__ cnt,
                                                    int cap, const int *__restrict__ up_off, int2 *__restrict__ pairs,
                                                    int *__restrict__ pid)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const int *row = nbr + (int64_t)t * cap;
    int p = up_off[t];
    for (int k = 0; k < cnt[t]; ++k) {
        const int u = row[k];
        if (u > t) {
            pairs[p] = make_int2(t, u);
            pid[(int64_t)t * cap + k] = p;
            ++p;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_up_mirror(int n, const int *__restrict__ nbr, const int *__restrict__ cnt,
                                                      int cap, int *__restrict__ pid)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const int *row = nbr + (int64_t)t * cap;
    for (int k = 0; k < cnt[t]; ++k) {
        const int u = row[k];
        if (u >= t) continue;
        const int *ru = nbr + (int64_t)u * cap;
        const int cu = cnt[u];
        int kk = 0;
        while (kk < cu && ru[kk] != t) ++kk;   // the list is symmetric: t is in row u
        pid[(int64_t)t * cap + k] = kk < cu ? pid[(int64_t)u * cap + kk] : 0;
    }
}

}  // namespace

void launch_half_list(hipStream_t s, int n, const int *nbr, const int *cnt, int cap, int *cnt_up, int *up_off,
                      int *scratch, int2 *pairs, int *pid)
{
    k_up_count<<<blocks_for(n), kBlock, 0, s>>>(n, nbr, cnt, cap, cnt_up);
    launch_scan_cells(s, cnt_up, n, up_off, nullptr, scratch);
    k_up_fill<<<blocks_for(n), kBlock, 0, s>>>(n, nbr, cnt, cap, up_off, pairs, pid);
    k_up_mirror<<<blocks_for(n), kBlock, 0, s>>>(n, nbr, cnt, cap, pid);
}

void launch_cell_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank,
                      const double4 *Rw, int *key, int *count)
{
    k_cell_keys<<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, G, cell_rank, Rw, key, count);
}

void launch_scan_cells(hipStream_t s, int *count, int n, int *start, int *fill, int *tiles)
{
    const int n_tiles = (n + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<n_tiles, kScanThreads, 0, s>>>(count, n, start, tiles);
    k_scan_tile_totals<<<1, kScanThreads, 0, s>>>(tiles, n_tiles, start, n);
    k_scan_add<<<(n + kScanThreads - 1) / kScanThreads, kScanThreads, 0, s>>>(count, n, start, tiles, fill);
}

int scan_max_elements() { return kScanTile * kScanTile; }

void launch_scatter_slots(hipStream_t s, int n_mol, const int *key, const int *start, int *fill, int *new_from)
{
    k_scatter_slots<<<blocks_for(n_mol), kBlock, 0, s>>>(n_mol, key, start, fill, new_from);
}

void launch_sort_within_cells(hipStream_t s, int n_cells, const int *start, const int *perm_old, int *new_from)
{
    k_sort_within_cells<<<blocks_for(n_cells), kBlock, 0, s>>>(n_cells, start, perm_old, new_from);
}

void launch_permute(hipStream_t s, const DevParams &P, const int *new_from, const StateBufs &src,
                    const StateBufs &dst, int *inv_perm, double4 *R_ref, bool with_v)
{
    switch (P.spm) {
    case 1: k_permute<1><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, new_from, src, dst, inv_perm, R_ref, with_v); break;
    case 2: k_permute<2><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, new_from, src, dst, inv_perm, R_ref, with_v); break;
    case 3: k_permute<3><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, new_from, src, dst, inv_perm, R_ref, with_v); break;
    default: k_permute<4><<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, new_from, src, dst, inv_perm, R_ref, with_v); break;
    }
}

void launch_list_build(hipStream_t s, const DevParams &P, const Grid &G, const int *rank_cell,
                       const int *cell_rank, const int *start, const double4 *Rw, const int *key, double rl2,
                       int *nbr, int *cnt, int cap, Ctrl *ctrl)
{
    if (G.n[0] >= 3 && G.n[1] >= 3 && G.n[2] >= 3) {
        const int3 nb = make_int3((G.n[0] + kBrick - 1) / kBrick, (G.n[1] + kBrick - 1) / kBrick,
                                  (G.n[2] + kBrick - 1) / kBrick);
        k_list_build_lds<<<nb.x * nb.y * nb.z, kBlock, 0, s>>>(P, G, cell_rank, start, Rw, rl2, nbr, cnt, cap, ctrl,
                                                                 nb);
    } else {
        k_list_build<<<blocks_for(P.n_mol), kBlock, 0, s>>>(P, G, rank_cell, cell_rank, start, Rw, key, rl2, nbr,
                                                           cnt, cap, ctrl);
    }
}

}  // namespace adres
