// Linked-cell list of molecule centres of mass (Sec. 5, introduction: the
// linked-cell list behind ESPResSo++'s domain decomposition), rebuilt as a
// Morton-ordered counting sort on the GPU:
//   keys (cell -> Morton rank) -> per-cell counts (atomics) -> exclusive scan (each
//   tile of 1024 cells in place, the tile totals by every workgroup of the scatter)
//   -> scatter -> per-cell order by caller index (makes the order a pure function of
//   the positions), fused with the move of the state into the new order.
// The Verlet list of molecule pairs is built cell by cell: a wavefront takes a cell's
// molecules as homes and the molecules of the 27 cells around it (fewer when a
// dimension has < 3 cells) as candidates, and keeps those whose minimum-image centre
// distance is strictly below r_list.  The list is stored row-major (ELL):
// nbr[slot * cap + k]; every row is padded with the row's own slot up to a multiple
// of 4.  The tile halos and the dispatch order of the force kernel's tiles are built
// from it at the end of this file.
#include <algorithm>
#include <climits>

#include "adres_internal.h"

namespace adres {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_cell_keys(const int *__restrict__ go, DevParams P, Grid G, const int *__restrict__ cell_rank,
                                                      const double4 *__restrict__ Rw, int *__restrict__ key,
                                                      int *__restrict__ count, const double4 *__restrict__ Rw_alt,
                                                      ChainHead head)
{
    bool sw;   // the chunk's positions sit in the other buffer
    if (!chain_go(head, go, sw)) return;   // a guarded rebuild that was not asked for
    if (sw) Rw = Rw_alt;
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

// Exclusive scan of count[0..n) into start[0..n] in two launches: each workgroup scans a
// tile of 1024 counts (4 per thread; wavefront shuffles, then the 4 wave totals) and
// records the tile's total; a second pass adds to every tile the totals before it.
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

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int *__restrict__ go, const int *__restrict__ count, int n,
                                                             int *__restrict__ start, int *__restrict__ tiles)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
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

// Second pass: workgroup T adds the sum of the tile totals before tile T to its tile
// (each workgroup sums at most kScanTile totals itself), resets count and fill for the
// next build, and the last workgroup writes start[n], the grand total.
__global__ __launch_bounds__(kScanThreads) void k_scan_add(const int *__restrict__ go, int *__restrict__ count, int n, int *__restrict__ start,
                                                           const int *__restrict__ tiles, int n_tiles,
                                                           int *__restrict__ fill)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    const int T = blockIdx.x;
    int part = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * threadIdx.x + j;
        part += k < T ? tiles[k] : 0;
    }
    int before;
    block_exclusive_scan(part, before);   // before = sum of the totals of tiles 0 .. T-1
    if (T == n_tiles - 1 && threadIdx.x == 0) start[n] = before + tiles[T];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = T * kScanTile + j * kScanThreads + threadIdx.x;
        if (i < n) {
            start[i] += before;
            count[i] = 0;
            if (fill) fill[i] = 0;
        }
    }
}

// The cell sort's scan in one pass plus the scatter: k_scan_local leaves each tile of 1024
// cells its in-tile exclusive prefix (in place of the counts) and its total, and clears the
// fill counters; k_scatter_slots then scans the tile totals in every workgroup (at most
// kScanTile of them), writes the cells' global starts and places every molecule at its
// cell's start plus an atomic fill index (the order within a cell is fixed afterwards by
// k_sort_permute, which also clears the counts for the next build).
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int *__restrict__ go, int *__restrict__ count, int n,
                                                             int *__restrict__ tiles, int *__restrict__ fill,
                                                             Ctrl *__restrict__ reset)
{
    if (reset && blockIdx.x == 0 && threadIdx.x == 0) {   // published by the kernel before
        reset->halt = INT_MAX;
        reset->overflow = 0;
        reset->max_count = 0;
        reset->max_halo = 0;
    }
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    const int base = blockIdx.x * kScanTile + 4 * threadIdx.x;
    int c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = base + j < n ? count[base + j] : 0;
    const int mine = (c[0] + c[1]) + (c[2] + c[3]);
    int total;
    int run = block_exclusive_scan(mine, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) {
            count[base + j] = run;
            fill[base + j] = 0;
        }
        run += c[j];
    }
    if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scatter_slots(const int *__restrict__ go, int n_mol, const int *__restrict__ key,
                                                          const int *__restrict__ lstart, const int *__restrict__ tiles,
                                                          int n_tiles, int n_cells, int *__restrict__ start,
                                                          int *__restrict__ fill, int *__restrict__ new_from)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    static_assert(kBlock == kScanThreads, "the tile totals are scanned by the whole workgroup");
    __shared__ int toff[kScanTile];
    int tt[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) tt[j] = 4 * (int)threadIdx.x + j < n_tiles ? tiles[4 * threadIdx.x + j] : 0;
    int total;
    int run = block_exclusive_scan((tt[0] + tt[1]) + (tt[2] + tt[3]), total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        toff[4 * threadIdx.x + j] = run;
        run += tt[j];
    }
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n_cells) start[i] = lstart[i] + toff[i / kScanTile];
    else if (i == n_cells) start[i] = total;
    if (i >= n_mol) return;
    const int k = key[i];
    const int pos = lstart[k] + toff[k / kScanTile] + atomicAdd(&fill[k], 1);
    new_from[pos] = i;
}

// Caller order within each cell (the atomic scatter leaves the molecules of a cell in
// arbitrary order), then the state gathered into the new slot order, in one launch: the
// slots of a cell depend on that cell alone, so a workgroup takes kSortCells consecutive
// cells, its first wavefront orders them (a thread per cell) and the whole workgroup then
// moves the molecules of their slot range.
// Ordering: a cell of at most 16 molecules is loaded into registers at once and every
// molecule is written to the slot given by its rank (the number of cell mates with a
// smaller caller index; indices are distinct); larger cells use an insertion sort.
// Moving: one lane per site (perm_lanes<SPM>() lanes per molecule; lane 0 also moves the
// per-molecule arrays), all of a lane's loads issued before its first store (source and
// destination are distinct buffers, which the compiler cannot know).
constexpr int kSortCell = 16;
constexpr int kSortCells = 32;

__device__ __forceinline__ void sort_cell(int lo, int hi, const int *__restrict__ perm_old, int *__restrict__ new_from)
{
    const int m = hi - lo;
    if (m <= 1) return;
    if (m <= kSortCell) {
        int v[kSortCell], tag[kSortCell];
#pragma unroll
        for (int i = 0; i < kSortCell; ++i) v[i] = i < m ? new_from[lo + i] : 0;
#pragma unroll
        for (int i = 0; i < kSortCell; ++i) tag[i] = i < m ? perm_old[v[i]] : INT_MAX;
#pragma unroll
        for (int i = 0; i < kSortCell; ++i) {
            if (i >= m) break;
            int r = 0;
#pragma unroll
            for (int j = 0; j < kSortCell; ++j) r += tag[j] < tag[i];
            new_from[lo + r] = v[i];
        }
        return;
    }
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
constexpr int perm_lanes() { return SPM == 1 ? 1 : (SPM == 2 ? 2 : 4); }

template <int SPM>
__global__ __launch_bounds__(kBlock) void k_sort_permute(const int *__restrict__ go, DevParams P, int n_cells,
                                                         const int *__restrict__ start, int *__restrict__ new_from,
                                                         int *__restrict__ count, StateBufs src, StateBufs dst,
                                                         int *__restrict__ inv_perm, double4 *__restrict__ R_ref,
                                                         int with_v)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    // (go points at Ctrl::go, followed by Ctrl::fix: the chunk's positions sit in the other buffer)
    if (go && go[1] != 0) {   // the source positions are in the destination's buffer and the other way round
        double *tx = src.x; src.x = dst.x; dst.x = tx;
        double4 *tr = src.Rw; src.Rw = dst.Rw; dst.Rw = tr;
    }
    const int c0 = blockIdx.x * kSortCells;
    const int c1 = min(c0 + kSortCells, n_cells);
    if (threadIdx.x < kSortCells && c0 + (int)threadIdx.x < c1) {
        const int c = c0 + threadIdx.x;
        count[c] = 0;   // (the in-tile prefixes of k_scan_local: cleared for the next build)
        sort_cell(start[c], start[c + 1], src.perm, new_from);
    }
    __syncthreads();   // the workgroup's own global stores are visible to it after the barrier
    constexpr int L = perm_lanes<SPM>();
    static_assert(SPM <= L, "one lane per site");
    const int lo = start[c0], hi = start[c1];
    const int64_t ns = P.n_sites;
    for (int64_t g = (int64_t)lo * L + threadIdx.x; g < (int64_t)hi * L; g += kBlock) {
        const int t = (int)(g / L), k = (int)(g % L);
        const int i = new_from[t];
        const bool site = k < SPM;
        const int64_t from = (int64_t)i * SPM + k, to = (int64_t)t * SPM + k;
        double xs[3] = {0.0, 0.0, 0.0}, vs[3] = {0.0, 0.0, 0.0};
        if (site) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xs[d] = src.x[d * ns + from];
                if (with_v) vs[d] = src.v[d * ns + from];
            }
        }
        double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
        int caller = 0;
        if (k == 0) {
            r = src.Rw[i];
            caller = src.perm[i];
        }
        if (site) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                dst.x[d * ns + to] = xs[d];
                if (with_v) dst.v[d * ns + to] = vs[d];
            }
        }
        if (k == 0) {
            dst.Rw[t] = r;
            R_ref[t] = r;
            dst.perm[t] = caller;
            inv_perm[caller] = t;
        }
    }
}

// Cell-major build: one wavefront per cell of Morton rank r, four cells per workgroup.  The
// cell's 27 stencil neighbours come from a table fixed at set-up (rank, or -1 for offsets
// skipped on grids with fewer than 3 cells along a dimension, so that no cell is visited
// twice; stencil order z, then y, then x offset); lanes 0..26 fetch their slot ranges and
// a scan gives every candidate of the stencil an index k (stencil order, then slot order).  Home
// molecules are taken 64 at a time (lane h holds home h's running row length, its centre
// comes from scalar loads, one home ahead); candidates 128 at a time (two per lane, the
// stencil cell found by a branch-free search of the scanned starts in LDS), each tested
// against every home of the batch: a ballot gives the hits' positions in the home's row,
// so rows come out in stencil order, then slot order.  Each candidate centre is loaded once
// per batch of homes, not once per home molecule.  The kernel is bound by VALU issue: the
// home's centre and row address are wave-uniform (scalar registers), so that the vector
// work per (home, candidate) test is the FP64 minimum-image distance and the ballot.
constexpr int kCmWaves = 4;

__global__ __launch_bounds__(kBlock) void k_list_build_cm(const int *__restrict__ go, DevParams P, int n_cells, const int *__restrict__ stencil,
                                                          const int *__restrict__ start,
                                                          const double4 *__restrict__ Rw, double rl2,
                                                          int *__restrict__ nbr, int *__restrict__ cnt, int cap,
                                                          unsigned *__restrict__ mcost, Ctrl *ctrl,
                                                          const double4 *__restrict__ Rw_alt)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    // (go points at Ctrl::go, followed by Ctrl::fix: the chunk's positions sit in the other buffer)
    const bool sw = go && go[1] != 0;
    if (sw) Rw = Rw_alt;
    __shared__ int s_lo[kCmWaves][32], s_ex[kCmWaves][32];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int r = blockIdx.x * kCmWaves + wv;
    if (r >= n_cells) return;   // whole wavefront
    const int h0 = start[r], h1 = start[r + 1];
    int lo = 0, c = 0;
    if (lane < 27) {
        const int nr = stencil[(int64_t)r * 27 + lane];
        if (nr >= 0) {
            lo = start[nr];
            c = start[nr + 1] - lo;
        }
    }
    if (h0 == h1) return;
    int incl = c;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const int total_c = __shfl(incl, 31, 64);   // lanes 27..31 carry the full sum
    if (lane < 32) {
        s_lo[wv][lane] = lo;
        s_ex[wv][lane] = incl - c;   // entries 27..31 hold total_c: above every candidate index
    }
    // lanes of one wavefront read what the others wrote above: LDS operations of a
    // wavefront complete in order, and this keeps the compiler from moving the reads up
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const unsigned heavy = (unsigned)(P.spm * P.spm);
    for (int hb = h0; hb < h1; hb += 64) {
        const int nb = min(64, h1 - hb);
        int base = 0;   // lane h: entries found so far for home hb + h
        // candidates 128 at a time, two per lane, both centres requested before the tests
        for (int c0 = 0; c0 < total_c; c0 += 128) {
            int slot[2] = {0, 0};
            bool vk[2];
            double4 o[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = c0 + 64 * u + lane;
                vk[u] = k < total_c;
                // the stencil cell holding candidate k: the largest j with ex_j <= k (ex_0 = 0)
                int j = 0;
#pragma unroll
                for (int step = 16; step >= 1; step >>= 1) j += s_ex[wv][j + step] <= k ? step : 0;
                slot[u] = s_lo[wv][j] + (k - s_ex[wv][j]);
                o[u] = make_double4(0.0, 0.0, 0.0, 0.0);
                if (vk[u]) o[u] = Rw[slot[u]];
            }
            double4 nx = Rw[hb];   // the next home's centre (uniform: scalar loads)
            for (int h = 0; h < nb; ++h) {
                const double mx = nx.x, my = nx.y, mz = nx.z;
                if (h + 1 < nb) nx = Rw[hb + h + 1];
                const int t = hb + h;
                int *row = nbr + (int64_t)t * cap;
                int bh = __builtin_amdgcn_readlane(base, h);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    bool hit = false;
                    if (vk[u] && slot[u] != t) {
                        const double dx = mi(o[u].x - mx, P.box[0], P.inv_box[0]);
                        const double dy = mi(o[u].y - my, P.box[1], P.inv_box[1]);
                        const double dz = mi(o[u].z - mz, P.box[2], P.inv_box[2]);
                        hit = dist2_exact(dx, dy, dz) < rl2;
                    }
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    if (hit) {
                        const unsigned pos = (unsigned)bh + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                        if (pos < (unsigned)cap) row[pos] = slot[u];
                    }
                    bh += __popcll(m);
                }
                if (lane == h) base = bh;
            }
        }
        if (lane < nb) {
            const int t = hb + lane;
            const int total = base;
            cnt[t] = total;
            mcost[t] = (unsigned)min(total, cap) * (Rw[t].w > 0.0 ? heavy : 1u) + 4u;
            if (total > cap) {
                atomicOr(&ctrl->overflow, 1);
                atomicMax(&ctrl->max_count, total);
                atomicMin(&ctrl->halt, -1);
            } else {
                int *row = nbr + (int64_t)t * cap;
                for (int j = total; j < ((total + 3) & ~3); ++j) row[j] = t;   // padding: own slot
            }
        }
    }
}

// Half list for per-pair work (the learned CG force): every unordered listed pair once,
// as (t, u) with t < u, ordered by t then u, plus for every full-list entry the index of
// its pair.  Rows are first sorted by neighbour slot (32 lanes per row, rank sort in
// LDS); then a row's upper neighbours (u > t) are a suffix starting at lb[t] = number of
// neighbours below t, and the pair of an entry (t, k) is found without search for u > t
// and by binary search for t in the sorted row u for u < t (the list is symmetric).
constexpr int kSortRows = kBlock / 32;

__global__ __launch_bounds__(kBlock) void k_sort_rows(const int *__restrict__ go, int n, int *__restrict__ nbr, const int *__restrict__ cnt,
                                                     int cap, int *__restrict__ cnt_up)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    extern __shared__ int srow[];   // kSortRows rows of cap entries
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    const int t = blockIdx.x * kSortRows + g;
    // a row that overflowed its capacity (count > cap) holds only cap entries; the list is
    // rebuilt with a larger capacity before anything reads it, so clamping keeps this safe
    const int c = t < n ? min(cnt[t], cap) : 0;
    int *row = nbr + (int64_t)(t < n ? t : 0) * cap;
    int *sr = srow + g * cap;
    for (int k = lane; k < c; k += 32) sr[k] = row[k];
    __syncthreads();
    int below = 0;
    for (int k = lane; k < c; k += 32) {
        const int e = sr[k];
        int rank = 0;
        for (int j = 0; j < c; ++j) rank += sr[j] < e;   // entries of a row are distinct
        row[rank] = e;
        below += e < t;
    }
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) below += __shfl_xor(below, off, 32);
    if (t < n && lane == 0) cnt_up[t] = c - below;
}

__global__ __launch_bounds__(kBlock) void k_up_entries(const int *__restrict__ go, int n, const int *__restrict__ nbr, const int *__restrict__ cnt,
                                                      int cap, const int *__restrict__ up_off, int2 *__restrict__ pairs,
                                                      int64_t pairs_cap, int *__restrict__ pid)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)n * cap) return;
    const int t = (int)(e / cap), k = (int)(e - (int64_t)t * cap);
    const int ct = min(cnt[t], cap);   // see k_sort_rows
    if (k >= ct) return;
    const int u = nbr[e];
    if (u > t) {
        const int lb = ct - (up_off[t + 1] - up_off[t]);
        const int p = up_off[t] + k - lb;
        if (p < pairs_cap) pairs[p] = make_int2(t, u);   // only an overflowed list can exceed it
        pid[e] = p;
    } else {
        const int *ru = nbr + (int64_t)u * cap;
        const int cu = min(cnt[u], cap);
        int lo = 0, hi = cu;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ru[mid] < t) lo = mid + 1;
            else hi = mid;
        }
        const int lbu = cu - (up_off[u + 1] - up_off[u]);
        pid[e] = up_off[u] + lo - lbu;
    }
}

}  // namespace

void launch_half_list(hipStream_t s, int n, int *nbr, const int *cnt, int cap, int *cnt_up, int *up_off,
                      int *scratch, int2 *pairs, int64_t pairs_cap, int *pid, const int *go)
{
    k_sort_rows<<<(n + kSortRows - 1) / kSortRows, kBlock, (size_t)kSortRows * cap * sizeof(int), s>>>(go, n, nbr, cnt, cap,
                                                                                                     cnt_up);
    launch_scan_cells(s, cnt_up, n, up_off, nullptr, scratch, go);
    const int64_t entries = (int64_t)n * cap;
    k_up_entries<<<(unsigned)((entries + kBlock - 1) / kBlock), kBlock, 0, s>>>(go, n, nbr, cnt, cap, up_off, pairs, pairs_cap, pid);
}

void launch_cell_keys(hipStream_t s, const DevParams &P, const Grid &G, const int *cell_rank,
                      const double4 *Rw, int *key, int *count, const int *go, const double4 *Rw_alt,
                      const ChainHead &head)
{
    k_cell_keys<<<blocks_for(P.n_mol), kBlock, 0, s>>>(go, P, G, cell_rank, Rw, key, count, Rw_alt, head);
}

void launch_scan_cells(hipStream_t s, int *count, int n, int *start, int *fill, int *tiles, const int *go)
{
    const int n_tiles = (n + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<n_tiles, kScanThreads, 0, s>>>(go, count, n, start, tiles);
    k_scan_add<<<n_tiles, kScanThreads, 0, s>>>(go, count, n, start, tiles, n_tiles, fill);
}

int scan_max_elements() { return kScanTile * kScanTile; }

void launch_scatter_slots(hipStream_t s, int n_mol, int n_cells, const int *key, int *count, int *start, int *fill,
                          int *tiles, int *new_from, const int *go, Ctrl *reset)
{
    const int n_tiles = (n_cells + kScanTile - 1) / kScanTile;
    k_scan_local<<<n_tiles, kScanThreads, 0, s>>>(go, count, n_cells, tiles, fill, reset);
    k_scatter_slots<<<blocks_for(std::max(n_mol, n_cells + 1)), kBlock, 0, s>>>(go, n_mol, key, count, tiles, n_tiles,
                                                                               n_cells, start, fill, new_from);
}

void launch_sort_permute(hipStream_t s, const DevParams &P, int n_cells, const int *start, int *new_from,
                         int *count, const StateBufs &src, const StateBufs &dst, int *inv_perm, double4 *R_ref,
                         bool with_v, const int *go)
{
    const int nb = (n_cells + kSortCells - 1) / kSortCells;
    const int v = with_v ? 1 : 0;
    switch (P.spm) {
    case 1: k_sort_permute<1><<<nb, kBlock, 0, s>>>(go, P, n_cells, start, new_from, count, src, dst, inv_perm, R_ref, v); break;
    case 2: k_sort_permute<2><<<nb, kBlock, 0, s>>>(go, P, n_cells, start, new_from, count, src, dst, inv_perm, R_ref, v); break;
    case 3: k_sort_permute<3><<<nb, kBlock, 0, s>>>(go, P, n_cells, start, new_from, count, src, dst, inv_perm, R_ref, v); break;
    default: k_sort_permute<4><<<nb, kBlock, 0, s>>>(go, P, n_cells, start, new_from, count, src, dst, inv_perm, R_ref, v); break;
    }
}

void launch_list_build(hipStream_t s, const DevParams &P, const Grid &G, const int *stencil, const int *start,
                       const double4 *Rw, double rl2, int *nbr, int *cnt, int cap, unsigned *mcost, Ctrl *ctrl, const int *go,
                       const double4 *Rw_alt)
{
    const int blocks = (G.n_cells + kCmWaves - 1) / kCmWaves;
    k_list_build_cm<<<blocks, kBlock, 0, s>>>(go, P, G.n_cells, stencil, start, Rw, rl2, nbr, cnt, cap, mcost, ctrl, Rw_alt);
}

namespace {

// Neighbour halo of one force-kernel tile (kHaloTile consecutive slots, one workgroup): every
// slot its molecules' rows reference is entered once into an LDS hash table (open
// addressing, linear probing); the distinct slots are then ranked by value and numbered in
// slot order after the tile's own slots, which take halo positions 0..kHaloTile-1 (slot
// order keeps the runs of a cell's molecules together, so that neighbouring lanes of the
// force kernel's staging read neighbouring addresses).  The rows are rewritten as local
// halo indices, lane q of a quad owning entries q, q + 4, ...  The kernel is bound by the
// latency of its dependent chains (row loads, hash probes): a lane takes its entries in
// groups of kHaloGroup, each group's loads, first probes and lookups issued together, and
// keeps its first group in registers for the second pass.  The table takes 6 bytes a
// position (4-byte key, 2-byte halo position) and the compacted list 8 bytes a distinct
// slot (at most hcap - kHaloTile).  Its size is a power of two in [kBlock, kHaloHashMax]:
// a grid that one round of workgroups covers (four per compute unit) is bound by one
// workgroup's latency and takes the largest table (fewest collisions, hence the shortest
// probe chains); a larger grid is bound by how many workgroups a compute unit holds and
// takes the smallest table with at most half of its positions filled.
constexpr int kHaloHashMin = kBlock;   // table positions: a power of two in [kBlock, kHaloHashMax]
constexpr int kHaloHashMax = 2048;
constexpr int kHaloGroup = 4;          // row entries per lane in flight together

__device__ __forceinline__ int halo_hash(int u, int shift) { return (int)(((unsigned)u * 2654435761u) >> shift); }

// Inserts u, whose first probe returned prev, by linear probing from there.
__device__ __forceinline__ void halo_insert_rest(int *keys, int mask, int shift, int u, int prev, int *lost)
{
    if (prev == -1 || prev == u) return;
    int h = halo_hash(u, shift), probe = 1;
#pragma unroll 1
    for (; probe <= mask; ++probe) {
        h = (h + 1) & mask;
        const int p = atomicCAS(&keys[h], -1, u);
        if (p == -1 || p == u) break;
    }
    if (probe > mask) atomicOr(lost, 1);
}

// Table position of u (present), given the key found at its first probe position.
__device__ __forceinline__ int halo_find(const int *keys, int mask, int shift, int u, int first)
{
    int h = halo_hash(u, shift);
    if (first == u) return h;
#pragma unroll 1
    for (int probe = 1; probe <= mask; ++probe) {
        h = (h + 1) & mask;
        if (keys[h] == u) break;
    }
    return h;
}

// log2 of the table size for a halo capacity hcap and a grid of `tiles` workgroups on
// n_cu compute units
int halo_table_log2(int hcap, int tiles, int n_cu)
{
    int lg = 0;
    if (n_cu > 0 && tiles <= 4 * n_cu) {
        while ((1 << lg) < kHaloHashMax) ++lg;
        return lg;
    }
    while ((1 << lg) < kHaloHashMin || ((1 << lg) < 2 * (hcap - kHaloTile) && (1 << lg) < kHaloHashMax)) ++lg;
    return lg;
}

__global__ __launch_bounds__(kBlock) void k_halo_build(const int *__restrict__ go, int n_mol, const int *__restrict__ nbr,
                                                       const int *__restrict__ cnt, int cap, int hcap, int lcap,
                                                       int lg, const unsigned *__restrict__ mcost,
                                                       const int *__restrict__ tile_pos, int *__restrict__ hid,
                                                       int *__restrict__ hn, int *__restrict__ hcnt,
                                                       uint16_t *__restrict__ lnbr, uint8_t *__restrict__ tperm,
                                                       Ctrl *ctrl)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    // keys and vals by table position, then the distinct slots compacted (key, position):
    // room for the hcap - kHaloTile a halo may hold (more overflow the capacity)
    extern __shared__ int tab[];
    const int T = 1 << lg, mask = T - 1, shift = 32 - lg, D = hcap - kHaloTile;
    int *keys = tab, *dkey = tab + T, *dpos = tab + T + D;
    uint16_t *vals = reinterpret_cast<uint16_t *>(tab + T + 2 * D);   // halo positions (< hcap)
    __shared__ int wave_tot[kBlock / 64];
    __shared__ int lost;
    __shared__ unsigned tcost[kHaloTile];
    __shared__ int trank[kHaloTile];   // each molecule's place in the cost order
    const int b = blockIdx.x;
    const int pb = tile_pos[b];   // the dispatch position, where the outputs go
    const int base = b * kHaloTile;
    const int n_home = min(kHaloTile, n_mol - base);
    // (the tail of a short last tile costs 0: it sorts last; valid costs are at least 4)
    const unsigned my_cost = (int)threadIdx.x < n_home ? mcost[base + threadIdx.x] : 0u;
    const int m = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int t = base + m;
    // a row that overflowed holds only cap entries; the list is rebuilt before any use
    const int c = m < n_home ? min(cnt[t], cap) : 0;
    const int per = c > q ? (c - q + 3) >> 2 : 0;   // lane q's entries k = q + 4 i, i < per
    const int *row = nbr + (int64_t)t * cap + q;
    auto own = [base, n_home](int v) { return (unsigned)(v - base) < (unsigned)n_home; };
    int u0[kHaloGroup];   // the first group, kept for the second pass
#pragma unroll
    for (int i = 0; i < kHaloGroup; ++i) u0[i] = i < per ? row[4 * i] : base;

    for (int i = threadIdx.x; i < T; i += kBlock) keys[i] = -1;
    if (threadIdx.x == 0) lost = 0;
    if (threadIdx.x < kHaloTile) tcost[threadIdx.x] = my_cost;
    __syncthreads();
    // the tile's molecules by falling cost, ties in slot order
    if (threadIdx.x < kHaloTile) {
        const unsigned cme = tcost[threadIdx.x];
        int rank = 0;
#pragma unroll 8
        for (int j = 0; j < kHaloTile; ++j) {
            const unsigned o = tcost[j];
            rank += (o > cme || (o == cme && j < (int)threadIdx.x)) ? 1 : 0;
        }
        tperm[(int64_t)pb * kHaloTile + rank] = (uint8_t)threadIdx.x;
        trank[threadIdx.x] = rank;
    }
    // insertion, a group at a time: its first probes back to back, then the rare collisions
    // (entries past the row's length are the tile's own first slot: skipped as own)
    for (int i0 = 0; i0 < per; i0 += kHaloGroup) {
        int v[kHaloGroup], prev[kHaloGroup];
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i) v[i] = i0 == 0 ? u0[i] : (i0 + i < per ? row[4 * (i0 + i)] : base);
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i)
            prev[i] = own(v[i]) ? -1 : atomicCAS(&keys[halo_hash(v[i], shift)], -1, v[i]);
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i)
            if (!own(v[i])) halo_insert_rest(keys, mask, shift, v[i], prev[i], &lost);
    }
    __syncthreads();
    // number the occupied positions: each thread owns T / kBlock consecutive ones
    const int kPer = T / kBlock;
    int occ = 0;
    for (int j = 0; j < kPer; ++j) occ += keys[threadIdx.x * kPer + j] >= 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = occ;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        before += w < wv ? wave_tot[w] : 0;
        total += wave_tot[w];
    }
    int r = before + incl - occ;
    for (int j = 0; j < kPer; ++j) {
        const int pos = threadIdx.x * kPer + j;
        const int key = keys[pos];
        if (key >= 0) {
            if (r < D) {
                dkey[r] = key;
                dpos[r] = pos;
            }
            ++r;
        }
    }
    __syncthreads();
    // rank of each distinct slot among them (the slots are distinct: ranks are a permutation);
    // a halo over the capacity is only reported (the capacity grows, the halos are rebuilt)
    int *h_out = hid + (int64_t)pb * hcap;
    for (int j = threadIdx.x; j < (total > D ? 0 : total); j += kBlock) {
        const int key = dkey[j];
        int rank = 0;
#pragma unroll 8
        for (int i = 0; i < total; ++i) rank += dkey[i] < key;
        const int lpos = kHaloTile + rank;
        vals[dpos[j]] = (uint16_t)lpos;
        if (lpos < hcap) h_out[lpos] = key;
    }
    // the tile's own slots first (a short last tile repeats its last slot: never referenced)
    if (threadIdx.x < kHaloTile) h_out[threadIdx.x] = base + min((int)threadIdx.x, n_home - 1);
    // a full table held more than T distinct slots: report T + 1 of them, so that the
    // capacity (and with it the table) grows
    const int n_halo = kHaloTile + (lost ? T + 1 : total);
    if (threadIdx.x == 0) {
        hn[pb] = min(n_halo, hcap);
        if (n_halo > hcap) {
            atomicOr(&ctrl->overflow, 2);
            atomicMax(&ctrl->max_halo, n_halo);
            atomicMin(&ctrl->halt, -1);
        }
    }
    __syncthreads();
    if (n_halo > hcap) return;
    // rows as local halo indices, lane q's entries contiguous in its quarter of the row, a
    // group's lookups issued together and its entries stored as one 8-byte word (the
    // quarter is a multiple of 8 entries long and 16-byte aligned; entries past the row's
    // length are never read)
    const int64_t rrow = (int64_t)pb * kHaloTile + trank[m];   // the row's dispatch-ordered place
    if (q == 0) hcnt[rrow] = c;
    uint16_t *lrow = lnbr + rrow * lcap + q * (lcap / 4);
    static_assert(kHaloGroup == 4, "a group is stored as one 8-byte word");
    for (int i0 = 0; i0 < per; i0 += kHaloGroup) {
        int v[kHaloGroup], first[kHaloGroup];
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i) v[i] = i0 == 0 ? u0[i] : (i0 + i < per ? row[4 * (i0 + i)] : base);
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i) first[i] = own(v[i]) ? 0 : keys[halo_hash(v[i], shift)];
        unsigned loc[kHaloGroup];
#pragma unroll
        for (int i = 0; i < kHaloGroup; ++i)
            loc[i] = own(v[i]) ? (unsigned)(v[i] - base) : (unsigned)vals[halo_find(keys, mask, shift, v[i], first[i])];
        uint2 pk;
        pk.x = (loc[0] & 0xFFFFu) | (loc[1] << 16);
        pk.y = (loc[2] & 0xFFFFu) | (loc[3] << 16);
        *reinterpret_cast<uint2 *>(lrow + i0) = pk;
    }
}

}  // namespace

void launch_halo_build(hipStream_t s, int n_mol, const int *nbr, const int *cnt, int cap, int hcap, int lcap,
                       const unsigned *mcost, const int *tile_pos, int *hid, int *hn, int *hcnt, uint16_t *lnbr,
                       uint8_t *tperm, Ctrl *ctrl, const int *go)
{
    const int tiles = (n_mol + kHaloTile - 1) / kHaloTile;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 0;
    const int lg = halo_table_log2(hcap, tiles, n_cu);
    const size_t lds = ((size_t)6 << lg) + (size_t)8 * (hcap - kHaloTile);
    k_halo_build<<<tiles, kBlock, lds, s>>>(go, n_mol, nbr, cnt, cap, hcap, lcap, lg, mcost, tile_pos, hid, hn, hcnt, lnbr,
                                            tperm, ctrl);
}


namespace {

// Dispatch order of the force kernel's workgroups (longest processing time first): one
// workgroup per XCD range of tiles (64 molecules each, the force kernel's workgroup).  A
// tile's cost estimate is the sum over its four wavefronts of the largest per-molecule
// cost in each (lanes of a wavefront run in lockstep); the list build stores the
// per-molecule costs (row length, times SPM^2 when the molecule can be atomistic).  Tiles are
// ranked by falling cost (ties by index) within chunks of kTileRound consecutive tiles, so
// that the heaviest tiles of an XCD round are dispatched first, one per compute unit,
// instead of piling up on the compute units that receive neighbouring parts of the slab.  Any order
// is a valid permutation; ranges longer than kTileSortMax keep the identity.
constexpr int kTileSortMax = 4096;
constexpr int kTileThreads = 1024;
constexpr int kTileRankMax = 512;    // longer ranges are sorted (bitonic) instead of ranked

// About as many force workgroups as one XCD holds at once (32 compute units x 4): tiles are
// ranked by cost within consecutive chunks of this many, so that when a range takes several
// rounds (large systems) each round stays a compact piece of space whose halos share the
// XCD's L2, while the heaviest tiles of a round still start first.
constexpr int kTileRound = 128;

// Sort key of tile i of a range (falling order): its chunk (earlier first), its cost (as
// summed below, at most 4 x (2048 x 16 + 4) < 2^20), then the lower index; distinct, nonzero.
__device__ __forceinline__ unsigned long long tile_key(unsigned cost, int i)
{
    const unsigned long long chunk = 4095u - (unsigned)(i / kTileRound);   // (i < kTileSortMax)
    return (chunk << 52) | ((unsigned long long)(cost & 0xFFFFFu) << 32) | (unsigned)(~(unsigned)i);
}

__global__ __launch_bounds__(kTileThreads) void k_tile_order(const int *__restrict__ go, int n_mol, const unsigned *__restrict__ mcost, int n_tiles,
                                                            int *__restrict__ order, int *__restrict__ pos)
{
    if (go && *go == 0) return;   // a guarded rebuild that was not asked for
    __shared__ unsigned tcost[kTileSortMax];
    __shared__ unsigned long long key[kTileSortMax];
    const int x = blockIdx.x;
    const int q = n_tiles / 8, r = n_tiles % 8;
    const int start = x * q + (x < r ? x : r), len = q + (x < r ? 1 : 0);
    if (len == 0) return;   // fewer tiles than XCDs: this range is empty
    if (len > kTileSortMax) {
        for (int i = threadIdx.x; i < len; i += kTileThreads) order[start + i] = pos[start + i] = start + i;
        return;
    }
    for (int i = threadIdx.x; i < len; i += kTileThreads) tcost[i] = 0u;
    __syncthreads();
    // per-molecule costs in runs of 16 consecutive molecules (one force-kernel wavefront):
    // each thread reads whole runs as four 16-byte vectors, two runs in flight, and adds the
    // run's largest cost to its tile's total with an LDS integer atomic (order-independent).
    // The cost array is padded to a multiple of 16 entries; the address of a run past the
    // end is moved to the first run, and entries at or beyond n_mol are masked.
    const int64_t m0 = (int64_t)start * 64;
    const int n_runs = len * 4;
    for (int r0 = 0; r0 < n_runs; r0 += 2 * kTileThreads) {
        uint4 a[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int run = r0 + u * kTileThreads + threadIdx.x;
            const int64_t t0 = m0 + (int64_t)run * 16;
            const uint4 *p = reinterpret_cast<const uint4 *>(mcost + (run < n_runs && t0 < n_mol ? t0 : 0));
#pragma unroll
            for (int w = 0; w < 4; ++w) a[u][w] = p[w];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int run = r0 + u * kTileThreads + threadIdx.x;
            const int64_t t0 = m0 + (int64_t)run * 16;
            const unsigned e[16] = {a[u][0].x, a[u][0].y, a[u][0].z, a[u][0].w, a[u][1].x, a[u][1].y,
                                    a[u][1].z, a[u][1].w, a[u][2].x, a[u][2].y, a[u][2].z, a[u][2].w,
                                    a[u][3].x, a[u][3].y, a[u][3].z, a[u][3].w};
            unsigned v = 0u;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const unsigned c = t0 + k < n_mol ? e[k] : 0u;
                v = c > v ? c : v;
            }
            if (run < n_runs) atomicAdd(&tcost[run / 4], v);
        }
    }
    __syncthreads();
    // keys (chunk, cost, then the lower index first) are distinct and nonzero
    if (len <= kTileRankMax) {
        // short ranges: rank of tile i = number of larger keys, counted by all threads in
        // C chunks of the j range per tile, partial counts added with LDS atomics
        for (int i = threadIdx.x; i < len; i += kTileThreads) key[i] = tile_key(tcost[i], i);
        for (int i = threadIdx.x; i < len; i += kTileThreads) tcost[i] = 0u;   // now the ranks
        __syncthreads();
        const int C = len < kTileThreads ? kTileThreads / len : 1;
        const int per = (len + C - 1) / C;
        for (int wk = threadIdx.x; wk < len * C; wk += kTileThreads) {
            const int i = wk % len, c = wk / len;
            const unsigned long long k = key[i];
            const int j0 = c * per, j1 = min(len, j0 + per);
            unsigned n_gt = 0u;
#pragma unroll 4
            for (int j = j0; j < j1; ++j) n_gt += key[j] > k ? 1u : 0u;
            atomicAdd(&tcost[i], n_gt);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += kTileThreads) {
            order[start + (int)tcost[i]] = start + i;
            pos[start + i] = start + (int)tcost[i];
        }
        return;
    }
    // long ranges: bitonic sort into falling order over a power-of-two padding of zeros
    // (which sort last), log2(P2) (log2(P2) + 1) / 2 compare-exchange stages
    int P2 = 1;
    while (P2 < len) P2 <<= 1;
    for (int i = threadIdx.x; i < P2; i += kTileThreads)
        key[i] = i < len ? tile_key(tcost[i], i) : 0ull;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P2; i += kTileThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], b = key[l];
                    if ((i & k) == 0 ? a < b : a > b) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // position p holds the p-th largest key, whose low word is the complement of its tile
    for (int p = threadIdx.x; p < len; p += kTileThreads) {
        const int i = (int)(~(unsigned)(key[p] & 0xffffffffull));
        order[start + p] = start + i;
        pos[start + i] = start + p;
    }
}

}  // namespace

void launch_tile_order(hipStream_t s, const DevParams &P, const unsigned *mcost, int n_tiles, int *order, int *pos, const int *go)
{
    k_tile_order<<<8, kTileThreads, 0, s>>>(go, P.n_mol, mcost, n_tiles, order, pos);
}

}  // namespace adres
