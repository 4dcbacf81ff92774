// Host side of libadres: context, parameter checks, list-rebuild orchestration
// and the velocity-Verlet step loop.  Every numerical step runs in the HIP
// kernels of this directory; the host only allocates, launches and reads the
// device control word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "adres_internal.h"
#include "adres_mlp.h"

using namespace adres;

struct adres_ctx {
    adres_params prm{};
    DevParams P{};
    Grid G{};
    hipStream_t stream = nullptr;
    int device = 0;
    double r_list = 0.0, rl2 = 0.0;

    // two buffer sets; positions (x, Rw, rho) and order (v, perm, key) flip independently:
    // a fused step flips the positions, a reorder flips both.
    StateBufs S[2]{};
    int pos = 0, ord = 0;
    double *f = nullptr;     // forces, Morton order
    double4 *R_ref = nullptr;
    int *inv_perm = nullptr;
    int *cell_rank = nullptr;      // Morton rank of every cell (row-major cell index -> rank)
    int *count = nullptr, *start = nullptr, *fill = nullptr, *new_from = nullptr, *scan_tiles = nullptr;
    int *nbr = nullptr, *cnt = nullptr;
    int cap = 0;
    // tile halos of the force kernel and the rows as local halo indices
    int *hid = nullptr, *hn = nullptr;
    uint16_t *lnbr = nullptr;
    uint8_t *tperm = nullptr;                // each tile's molecules by falling cost
    int hcap = 0, lcap = 0;
    bool rw_stale = false;   // the step kernels moved the positions without storing centres
    Ctrl *ctrl = nullptr;
    Ctrl *ctrl_host = nullptr;     // last values read by the host
    CtrlPub *pub = nullptr;        // host-mapped pinned copy (k_publish, or a rebuild's first kernel)
    CtrlPub *pub_dev = nullptr;    // its device address
    unsigned pub_seq = 0;
    double *epart = nullptr;
    int epart_blocks = 0;
    float4 *tab = nullptr;
    double *td = nullptr, *td_u = nullptr;   // correction force table and its integrals
    int *anchors = nullptr;                  // anchor molecules of a self-adjusting region
    int *aslot = nullptr;                    // their slots in the current order
    double4 *near = nullptr;                 // offset from the nearest anchor per slot
    double *anchor_cen = nullptr;            // anchor centres of a caller configuration [K][3]
    int *tile_order = nullptr;               // force kernel dispatch order (per list build)
    int *tile_pos = nullptr;                 // its inverse: each tile's dispatch position
    int *hcnt = nullptr;                     // row lengths in dispatch order (halo build)
    unsigned *mcost = nullptr;               // per-molecule cost estimates (list build)
    int *stencil = nullptr;                  // [n_cells][27] neighbour cell ranks (static grid)

    // learned CG force
    float *mlp = nullptr;          // FP32 master parameters (kMlpParams)
    __bf16 *mlp_w2 = nullptr;      // BF16 copy of W2 (kHidden^2) followed by its transpose
    int *mlp_w2q = nullptr;        // FP8 copy of W2 (kHidden^2 bytes)
    float *mlp_fp8s = nullptr;     // its scales (3 floats)
    float *adam_m = nullptr, *adam_v = nullptr;
    int64_t adam_t = 0;
    double *grad = nullptr, *loss = nullptr, *res_part = nullptr, *resid = nullptr;
    float *gpart = nullptr;
    double *gred = nullptr;        // chunk sums of the gradient reduction
    double mlp_rc = 0.0, mlp_scale = 1.0, mlp_tw = 0.0, mlp_rmin = 0.0;
    bool have_mlp = false;
    // half list (every unordered pair once) for per-pair network outputs
    int *cnt_up = nullptr, *up_off = nullptr, *up_scratch = nullptr, *pid = nullptr;
    int2 *up_pairs = nullptr;
    float *f_pair = nullptr;
    int64_t half_rows_cap = 0, half_pairs_cap = 0;

    bool have_state = false;
    bool list_valid = false;
    uint64_t step_counter = 0;
    int last_interval = 8;

    bool no_alloc = false;   // inside adres_forces_noalloc: capacities may not grow
    double *scratch_epart = nullptr;   // this device's static energy-partials scratch

    int timing = 0;   // 0 off, 1 force kernel, 2 network pre-pass
    int timing_every = 1;
    int64_t timing_count = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
    // per recorded launch: its kernel's index within the step chunk (-1 outside the step
    // loop), and whether it returned at once (an earlier kernel of its chunk asked for a
    // rebuild, or a list overflow stopped the chunk): such launches are not counted
    std::vector<int> event_k;
    std::vector<char> event_skip;

    std::string err = "no error";
};

namespace {

// Energy partials of adres_forces_noalloc (one slot of 4 per force workgroup), in a static
// device array instead of a context allocation: at most 8192 workgroups, i.e. 524,288
// molecules (256 KiB).  Each device holds its own copy; its address is taken once per device.
constexpr int kNoallocBlocks = 8192;
__device__ __align__(256) double scratch[kNoallocBlocks * 4];
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mutex;

// The device address of this device's scratch (the current device must be `device`).
hipError_t scratch_address(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

adres_status fail(adres_ctx *c, adres_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

StateBufs view(const adres_ctx *c, int pos, int ord)
{
    StateBufs b;
    b.x = c->S[pos].x;
    b.Rw = c->S[pos].Rw;
    b.v = c->S[ord].v;
    b.perm = c->S[ord].perm;
    b.key = c->S[ord].key;
    return b;
}
StateBufs cur(const adres_ctx *c) { return view(c, c->pos, c->ord); }

#define HIPCHK(ctx, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(ctx, ADRES_E_HIP, std::string(#call " failed: ") + hipGetErrorString(e_));      \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

uint32_t spread3(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

// Reads the device control block once all work enqueued so far has finished: a
// one-thread kernel publishes it into host-mapped memory with a sequence number the
// host polls (cheaper than a copy plus a stream synchronisation).  Converts latched
// error bits into a status and clears them.
// The step loop has the first launch of the rebuild behind each chunk publish instead
// (ChainHead) and waits for it after enqueueing the rest of the rebuild.
unsigned publish_ctrl(adres_ctx *c)
{
    const unsigned seq = ++c->pub_seq;
    launch_publish(c->stream, c->ctrl, c->pub_dev, seq);
    return seq;
}

adres_status wait_ctrl(adres_ctx *c, unsigned seq)
{
    HIPCHK(c, hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    int v[kPubFields];
    auto published = [c, seq, &v]() {
        for (int i = 0; i < kPubFields; ++i) {
            const unsigned long long w = __atomic_load_n(&c->pub->w[i], __ATOMIC_ACQUIRE);
            if ((unsigned)(w >> 32) != seq) return false;
            v[i] = (int)(unsigned)w;
        }
        return true;
    };
    for (long spin = 0; !published(); ++spin) {
        if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5)) {
            // something is wrong with the stream: let the runtime report it
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (!published()) return fail(c, ADRES_E_HIP, "control word was not published");
        }
    }
    c->ctrl_host->halt = v[kPubHalt];
    c->ctrl_host->err = v[kPubErr];
    c->ctrl_host->overflow = v[kPubOverflow];
    c->ctrl_host->max_count = v[kPubMaxCount];
    c->ctrl_host->max_halo = v[kPubMaxHalo];
    int e = c->ctrl_host->err;
    if (e) {
        HIPCHK(c, hipMemsetAsync(&c->ctrl->err, 0, sizeof(int), c->stream));
        if (e & kErrNonFinite) return fail(c, ADRES_E_NONFINITE, "non-finite position or force");
        if (e & kErrStretch) return fail(c, ADRES_E_STRETCH, "a site is farther than rho_max + r_skin/2 from its centre of mass");
        if (e & kErrFene) return fail(c, ADRES_E_FENE, "a FENE bond reached its maximum extension R0");
        if (e & kErrTableRange) return fail(c, ADRES_E_TABLE_RANGE, "CG table lookup below the first knot");
    }
    return ADRES_OK;
}

adres_status read_ctrl(adres_ctx *c)
{
    return wait_ctrl(c, publish_ctrl(c));
}

adres_status gather(adres_ctx *c, const double *x, const double *v, bool check_disp)
{
    launch_gather(c->stream, c->P, x, v, cur(c), check_disp ? c->R_ref : nullptr, c->ctrl);
    c->rw_stale = false;
    if (c->P.region == ADRES_REGION_SPHERES)
        launch_anchor_weights(c->stream, c->P, cur(c).Rw, c->inv_perm, c->aslot, 1, c->ctrl, 0, 0, c->near);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

// Morton reorder: the launches (guarded by go when non-null: a rebuild enqueued before the
// host knows whether it is needed; head: the publication of the step chunk before it, taken
// by the first launch, which then also stores go) and the host's bookkeeping once it has run
void enqueue_resort(adres_ctx *c, bool with_v, const int *go, const ChainHead &head = ChainHead{})
{
    const StateBufs src = cur(c);
    const StateBufs dst = view(c, 1 - c->pos, 1 - c->ord);
    // (each position-reading kernel also gets the other position buffer, which a guarded
    // rebuild reads instead when the chunk's positions sit there: Ctrl::fix)
    if (c->rw_stale)   // the step kernels moved the positions without storing centres
        launch_centres_keys(c->stream, c->P, c->G, c->cell_rank, src.x, src.Rw, src.key, c->count, go, dst.x,
                            dst.Rw, head);
    else
        launch_cell_keys(c->stream, c->P, c->G, c->cell_rank, src.Rw, src.key, c->count, go, dst.Rw, head);
    // (after a head, the scan's launch clears the halt index and the list reports it published)
    launch_scatter_slots(c->stream, c->P.n_mol, c->G.n_cells, src.key, c->count, c->start, c->fill, c->scan_tiles,
                         c->new_from, go, head.ctrl);
    launch_sort_permute(c->stream, c->P, c->G.n_cells, c->start, c->new_from, c->count, src, dst, c->inv_perm,
                        c->R_ref, with_v, go);
    // the nearest-anchor offsets are per slot: recompute them in the new order
    if (c->P.region == ADRES_REGION_SPHERES)
        launch_anchor_weights(c->stream, c->P, dst.Rw, c->inv_perm, c->aslot, 1, c->ctrl, 0, 0, c->near, go, src.Rw);
}

void commit_resort(adres_ctx *c)
{
    c->rw_stale = false;
    c->pos = 1 - c->pos;
    c->ord = 1 - c->ord;
    c->list_valid = false;
}

adres_status resort(adres_ctx *c, bool with_v)
{
    enqueue_resort(c, with_v, nullptr);
    HIPCHK(c, hipGetLastError());
    commit_resort(c);
    return ADRES_OK;
}

bool is_mlp(const adres_ctx *c) { return c->P.cg_kind >= ADRES_CG_MLP; }

// The step kernels store the new centres only when something reads them before the next
// list build: the network's pair pre-pass and the anchor pass of a self-adjusting region.
bool keep_centres(const adres_ctx *c) { return is_mlp(c) || c->P.region == ADRES_REGION_SPHERES; }

// Row length of the local-index rows: each lane's quarter holds ceil(cap / 4) entries,
// rounded up to whole 16-byte loads (8 entries).
int local_cap(int cap) { return 4 * ((((cap + 3) / 4) + 7) / 8 * 8); }

// (Re)allocates the tile halos for capacity hcap and the local rows for the list capacity.
adres_status alloc_halo(adres_ctx *c, int hcap)
{
    const int tiles = (c->P.n_mol + kHaloTile - 1) / kHaloTile;
    const int lcap = local_cap(c->cap);
    if (hcap != c->hcap || !c->hid) {
        hipFree(c->hid);
        c->hid = nullptr;
        if (dalloc(&c->hid, (size_t)tiles * hcap) != hipSuccess)
            return fail(c, ADRES_E_NOMEM, "could not allocate the tile halos");
        c->hcap = hcap;
    }
    if (lcap != c->lcap || !c->lnbr) {
        hipFree(c->lnbr);
        c->lnbr = nullptr;
        if (dalloc(&c->lnbr, (size_t)lcap * c->P.n_mol) != hipSuccess)
            return fail(c, ADRES_E_NOMEM, "could not allocate the local rows");
        c->lcap = lcap;
    }
    return ADRES_OK;
}

void launch_halo(adres_ctx *c, const int *go = nullptr)
{
    launch_halo_build(c->stream, c->P.n_mol, c->nbr, c->cnt, c->cap, c->hcap, c->lcap, c->mcost, c->tile_pos,
                      c->hid, c->hn, c->hcnt, c->lnbr, c->tperm, c->ctrl, go);
}

// Every unordered pair of the Verlet list once (t < u) and, for every list entry, the
// id of its pair; the network is evaluated per pair, so both directions of a pair
// read the same value (exact Newton's third law).  The pair count stays on the
// device (up_off[n]).
adres_status build_half_list(adres_ctx *c)
{
    const int n = c->P.n_mol;
    if (c->cap > 2048) return fail(c, ADRES_E_CAPACITY, "neighbour rows longer than 2048 entries");
    if (c->half_rows_cap < c->cap) {
        if (c->no_alloc)
            return fail(c, ADRES_E_CAPACITY, "the half list must grow, which adres_forces_noalloc does not do");
        hipFree(c->pid); hipFree(c->up_pairs); hipFree(c->f_pair);
        c->pid = nullptr; c->up_pairs = nullptr; c->f_pair = nullptr;
        const size_t cap_pairs = (size_t)n * c->cap / 2 + 16;
        if (dalloc(&c->pid, (size_t)n * c->cap) != hipSuccess || dalloc(&c->up_pairs, cap_pairs) != hipSuccess ||
            dalloc(&c->f_pair, cap_pairs) != hipSuccess)
            return fail(c, ADRES_E_NOMEM, "could not allocate the half list");
        c->half_rows_cap = c->cap;
        c->half_pairs_cap = (int64_t)cap_pairs;
    }
    launch_half_list(c->stream, n, c->nbr, c->cnt, c->cap, c->cnt_up, c->up_off, c->up_scratch, c->up_pairs,
                     c->half_pairs_cap, c->pid);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

MlpDev mlp_dev(const adres_ctx *c)
{
    MlpDev M;
    M.w1 = c->mlp;
    M.b1 = c->mlp + kHidden;
    M.w2 = c->mlp + 2 * kHidden;
    M.b2 = c->mlp + 2 * kHidden + kHidden * kHidden;
    M.w3 = M.b2 + kHidden;
    M.w2_bf16 = c->mlp_w2;
    M.w2t_bf16 = c->mlp_w2 + kHidden * kHidden;
    M.w2_fp8 = c->mlp_w2q;
    M.fp8_scale = c->mlp_fp8s;
    M.fp8 = c->P.cg_kind == ADRES_CG_MLP_FP8;
    M.rc = c->mlp_rc;
    M.scale = c->mlp_scale;
    M.tw = c->mlp_tw;
    M.r_min = c->mlp_rmin;
    return M;
}

// Verlet list from the current (sorted) centres and the tile halos from it; grows the list
// and halo capacities on overflow.  The halos are built last: the learned CG force's half
// list reorders every row, and the local rows must follow the final row order.
adres_status build_list(adres_ctx *c)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        HIPCHK(c, hipMemsetAsync(&c->ctrl->overflow, 0, 3 * sizeof(int), c->stream));
        const StateBufs b = cur(c);
        launch_list_build(c->stream, c->P, c->G, c->stencil, c->start, b.Rw, c->rl2, c->nbr, c->cnt, c->cap,
                          c->mcost, c->ctrl);
        HIPCHK(c, hipGetLastError());
        adres_status st = read_ctrl(c);
        if (st != ADRES_OK) return st;
        if (!c->ctrl_host->overflow) break;
        if (attempt == 3) return fail(c, ADRES_E_CAPACITY, "neighbour list capacity did not converge");
        if (c->no_alloc)
            return fail(c, ADRES_E_CAPACITY, "the neighbour list must grow, which adres_forces_noalloc does not do");
        int need = c->ctrl_host->max_count;
        int new_cap = ((need + need / 4 + 8) + 15) & ~15;
        HIPCHK(c, hipFree(c->nbr));
        c->nbr = nullptr;
        if (dalloc(&c->nbr, (size_t)new_cap * c->P.n_mol) != hipSuccess)
            return fail(c, ADRES_E_CAPACITY, "could not grow the neighbour list");
        c->cap = new_cap;
        st = alloc_halo(c, c->hcap);
        if (st != ADRES_OK) return st;
    }
    launch_tile_order(c->stream, c->P, c->mcost, c->epart_blocks, c->tile_order, c->tile_pos);
    if (is_mlp(c)) {
        adres_status st = build_half_list(c);
        if (st != ADRES_OK) return st;
    }
    for (int attempt = 0; attempt < 4; ++attempt) {
        launch_halo(c);
        HIPCHK(c, hipGetLastError());
        adres_status st = read_ctrl(c);
        if (st != ADRES_OK) return st;
        if (!(c->ctrl_host->overflow & 2)) {
            c->list_valid = true;
            launch_reset_halt(c->stream, c->ctrl);   // an earlier overflow may have left halt = -1
            return ADRES_OK;
        }
        // a tile's halo outgrew its capacity
        if (c->no_alloc)
            return fail(c, ADRES_E_CAPACITY, "a tile halo must grow, which adres_forces_noalloc does not do");
        const int need = c->ctrl_host->max_halo;
        const int limit = halo_capacity_limit(c->P.spm, c->prm.pair_precision);
        if (need > limit)
            return fail(c, ADRES_E_CAPACITY, "a tile's neighbour halo (" + std::to_string(need) +
                                                 " molecules) exceeds the force kernel's LDS (" +
                                                 std::to_string(limit) + ")");
        HIPCHK(c, hipMemsetAsync(&c->ctrl->overflow, 0, 3 * sizeof(int), c->stream));
        st = alloc_halo(c, std::min(limit, ((need + need / 8 + 16) + 31) & ~31));
        if (st != ADRES_OK) return st;
    }
    return fail(c, ADRES_E_CAPACITY, "tile halo capacity did not converge");
}

// Verlet list without waiting: an overflowing row sets ctrl->halt = -1, which stops
// every kernel of the next step chunk; the host then regrows (regrow_list).  With go, the
// launches are guarded (see enqueue_resort) and the half list reuses its allocation, which
// only a synchronous regrow enlarges.
adres_status enqueue_list(adres_ctx *c, const int *go)
{
    // overflow / max_count were cleared by the halt reset launched before the reorder
    const StateBufs b = cur(c);
    launch_list_build(c->stream, c->P, c->G, c->stencil, c->start, b.Rw, c->rl2, c->nbr, c->cnt, c->cap,
                      c->mcost, c->ctrl, go, view(c, 1 - c->pos, c->ord).Rw);
    launch_tile_order(c->stream, c->P, c->mcost, c->epart_blocks, c->tile_order, c->tile_pos, go);
    HIPCHK(c, hipGetLastError());
    if (is_mlp(c)) {
        if (go) {
            if (c->half_rows_cap < c->cap) return fail(c, ADRES_E_STATE, "half list smaller than the list");
            launch_half_list(c->stream, c->P.n_mol, c->nbr, c->cnt, c->cap, c->cnt_up, c->up_off, c->up_scratch,
                             c->up_pairs, c->half_pairs_cap, c->pid, go);
        } else {
            adres_status st = build_half_list(c);
            if (st != ADRES_OK) return st;
        }
    }
    launch_halo(c, go);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status build_list_async(adres_ctx *c)
{
    adres_status st = enqueue_list(c, nullptr);
    if (st != ADRES_OK) return st;
    c->list_valid = true;
    return ADRES_OK;
}

ForceArgs force_args(adres_ctx *c)
{
    const StateBufs S = cur(c);
    ForceArgs a{};
    a.P = c->P;
    a.x = S.x;
    a.Rw = S.Rw;
    a.cap = c->cap;
    a.hid = c->hid;
    a.hn = c->hn;
    a.hcap = c->hcap;
    a.lnbr = c->lnbr;
    a.lcap = c->lcap;
    a.tperm = c->tperm;
    a.hcnt = c->hcnt;
    a.perm = S.perm;
    a.inv_perm = c->inv_perm;
    a.ctrl = c->ctrl;
    a.mode = kModeForce;
    a.slow_scale = 1.0;
    a.tile_order = c->tile_order;
    a.near = c->near;
    return a;
}

adres_status run_forces(adres_ctx *c, ForceArgs a)
{
    // timing mode 1 brackets the force kernel, mode 2 the network's pair-force pre-pass;
    // one launch in timing_every is recorded, picked by a hash of the launch count so that
    // the sample does not lock onto the rebuild cycle
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool sample = false;
    if (c->timing != 0 && !c->no_alloc && (c->timing == 1 || is_mlp(c))) {
        const uint32_t h = (uint32_t)(c->timing_count++) * 2654435761u;
        sample = (h >> 16) % (uint32_t)c->timing_every == 0;
    }
    if (sample) {
        if (c->events_used == c->events.size()) {
            hipEvent_t p, q;
            HIPCHK(c, hipEventCreate(&p));
            HIPCHK(c, hipEventCreate(&q));
            c->events.emplace_back(p, q);
        }
        if (c->event_k.size() < c->events.size()) {
            c->event_k.resize(c->events.size());
            c->event_skip.resize(c->events.size());
        }
        e0 = c->events[c->events_used].first;
        e1 = c->events[c->events_used].second;
        c->event_k[c->events_used] = a.check_halt ? a.step : -1;
        c->event_skip[c->events_used] = 0;
        ++c->events_used;
    }
    if (is_mlp(c) && a.slow_scale != 0.0) {
        if (sample && c->timing == 2) HIPCHK(c, hipEventRecord(e0, c->stream));
        launch_mlp_forward_pairs(c->stream, mlp_dev(c), c->P, c->up_pairs, a.Rw, c->f_pair, c->up_off + c->P.n_mol,
                                 c->half_pairs_cap, c->ctrl, a.check_halt, a.step);
        HIPCHK(c, hipGetLastError());
        if (sample && c->timing == 2) HIPCHK(c, hipEventRecord(e1, c->stream));
    }
    if (is_mlp(c)) {
        a.pid = c->pid;
        a.f_pair = c->f_pair;
    }
    const bool ev = sample && c->timing == 1;
    launch_forces(c->stream, a, c->prm.pair_precision, ev ? e0 : nullptr, ev ? e1 : nullptr);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status check_cg_ready(adres_ctx *c)
{
    if (c->P.region == ADRES_REGION_SPHERES && c->P.n_anchors == 0)
        return fail(c, ADRES_E_STATE, "self-adjusting region without anchors (adres_set_anchors)");
    if (c->P.cg_kind == ADRES_CG_TABLE && !c->tab)
        return fail(c, ADRES_E_STATE, "cg_kind is TABLE but no table was installed");
    if (is_mlp(c) && !c->have_mlp)
        return fail(c, ADRES_E_STATE, "MLP CG force requested but no network is installed");
    return ADRES_OK;
}

adres_status full_build(adres_ctx *c, const double *x, const double *v)
{
    adres_status st = gather(c, x, v, false);
    if (st != ADRES_OK) return st;
    st = resort(c, v != nullptr);
    if (st != ADRES_OK) return st;
    c->have_state = true;
    return build_list(c);
}

}  // namespace

extern "C" {

adres_status adres_create(const adres_params *p, void *hip_stream, adres_ctx **out)
{
    if (!p || !out) return ADRES_E_ARG;
    const adres_params &q = *p;
    if (q.n_mol < 1 || q.sites_per_mol < 1 || q.sites_per_mol > ADRES_MAX_SITES) return ADRES_E_ARG;
    for (int d = 0; d < 3; ++d)
        if (!(q.box[d] > 0.0) || !std::isfinite(q.box[d])) return ADRES_E_ARG;
    for (int k = 0; k < q.sites_per_mol; ++k)
        if (!(q.site_mass[k] > 0.0)) return ADRES_E_ARG;
    if (q.region < ADRES_REGION_ALL_AT || q.region > ADRES_REGION_SPHERES) return ADRES_E_ARG;
    if ((q.region == ADRES_REGION_SLAB_X || q.region == ADRES_REGION_SPHERE || q.region == ADRES_REGION_SPHERES) &&
        (q.d_at < 0.0 || q.d_hy < 0.0))
        return ADRES_E_ARG;
    if (q.cg_kind < ADRES_CG_WCA || q.cg_kind > ADRES_CG_MLP_FP8) return ADRES_E_ARG;
    if (q.bond_kind < ADRES_BOND_NONE || q.bond_kind > ADRES_BOND_FENE) return ADRES_E_ARG;
    if (q.bond_kind == ADRES_BOND_FENE && (q.sites_per_mol != 1 || q.chain_len < 1 || !(q.r0_bond > 0.0)))
        return ADRES_E_ARG;
    if (q.region != ADRES_REGION_ALL_CG && !(q.rc_at > 0.0 && q.sig_at > 0.0)) return ADRES_E_ARG;
    if (q.region != ADRES_REGION_ALL_AT && !(q.rc_cg > 0.0 && q.sig_cg > 0.0)) return ADRES_E_ARG;
    if (q.r_skin < 0.0 || q.rho_max < 0.0) return ADRES_E_ARG;
    if (q.sites_per_mol > 1 && !(q.rho_max > 0.0)) return ADRES_E_ARG;
    if (q.pair_precision != 32 && q.pair_precision != 64) return ADRES_E_ARG;
    if (q.scheme != ADRES_SCHEME_FORCE && q.scheme != ADRES_SCHEME_HAMILTONIAN) return ADRES_E_ARG;
    if (q.scheme == ADRES_SCHEME_HAMILTONIAN && q.cg_kind != ADRES_CG_WCA) return ADRES_E_ARG;
    // moving anchors would add drift forces on the anchors themselves: force interpolation only
    if (q.scheme == ADRES_SCHEME_HAMILTONIAN && q.region == ADRES_REGION_SPHERES) return ADRES_E_ARG;
    if (q.n_mol > scan_max_elements()) return ADRES_E_ARG;

    adres_ctx *c = new adres_ctx();
    c->prm = q;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return ADRES_E_HIP;
    }
    // the static scratch of adres_forces_noalloc: its address on this device, taken once
    if (scratch_address(c->device, &c->scratch_epart) != hipSuccess) {
        delete c;
        return ADRES_E_HIP;
    }

    // list radius: largest centre distance at which two molecules can interact, plus skin
    double r_mol = 0.0;
    if (q.region != ADRES_REGION_ALL_AT) r_mol = std::max(r_mol, q.rc_cg);
    if (q.region != ADRES_REGION_ALL_CG) r_mol = std::max(r_mol, q.rc_at + 2.0 * q.rho_max);
    c->r_list = r_mol + q.r_skin;
    c->rl2 = c->r_list * c->r_list;

    DevParams &P = c->P;
    P.n_mol = q.n_mol;
    P.spm = q.sites_per_mol;
    P.n_sites = (int64_t)q.n_mol * q.sites_per_mol;
    P.M = 0.0;
    for (int k = 0; k < P.spm; ++k) P.M = P.M + q.site_mass[k];
    {
        int ex = 0;
        P.M_pow2 = std::frexp(P.M, &ex) == 0.5 ? 1 : 0;
        P.inv_M = 1.0 / P.M;
    }
    for (int k = 0; k < kMaxSites; ++k) {
        P.mass[k] = k < P.spm ? q.site_mass[k] : 1.0;
        P.mfrac[k] = k < P.spm ? q.site_mass[k] / P.M : 0.0;
        P.inv_2m[k] = 1.0 / (2.0 * P.mass[k]);
    }
    Grid &G = c->G;
    G.n_cells = 1;
    for (int d = 0; d < 3; ++d) {
        P.box[d] = q.box[d];
        P.half[d] = 0.5 * q.box[d];
        P.inv_box[d] = 1.0 / q.box[d];
        P.center[d] = q.center[d];
        if (q.box[d] < 2.0 * c->r_list) {
            delete c;
            return ADRES_E_BOX;
        }
        int nd = (int)std::floor(q.box[d] / (c->r_list * (1.0 + 1e-12)));
        nd = std::max(1, std::min(nd, 1023));
        G.n[d] = nd;
        G.inv_len[d] = (double)nd / q.box[d];
        G.off_lo[d] = nd >= 3 ? -1 : 0;
        G.off_hi[d] = nd >= 2 ? 1 : 0;
        G.n_cells *= nd;
    }
    if (G.n_cells > scan_max_elements()) {   // the cell scan covers at most 2^20 cells
        delete c;
        return ADRES_E_BOX;
    }
    P.region = q.region;
    P.d_at = q.d_at;
    P.d_hy = q.d_hy;
    P.d_end = q.d_at + q.d_hy;
    P.eps_at = q.eps_at;
    P.sig2_at = q.sig_at * q.sig_at;
    P.rc_at = q.rc_at;
    P.rcA2 = q.rc_at * q.rc_at;
    P.eps_cg = q.eps_cg;
    P.sig2_cg = q.sig_cg * q.sig_cg;
    P.rcC2 = q.rc_cg * q.rc_cg;
    P.cg_kind = q.cg_kind;
    P.scheme = q.scheme;
    P.bond_kind = q.bond_kind;
    P.k_bond = q.k_bond;
    P.r0_bond = q.r0_bond;
    P.R02 = q.r0_bond * q.r0_bond;
    P.chain_len = std::max(1, q.chain_len);
    P.rho_max = q.rho_max;
    P.rho_lim = q.sites_per_mol > 1 ? q.rho_max + 0.5 * q.r_skin : 0.0;   // (a single site is its centre)
    P.half_skin = 0.5 * q.r_skin;
    P.cg_half = q.region != ADRES_REGION_ALL_AT ? 0.5 * (c->r_list - q.rc_cg) : 1e300;
    P.at_half = q.region != ADRES_REGION_ALL_CG ? q.rho_max + P.half_skin : 1e300;
    P.w0_cg = q.scheme == ADRES_SCHEME_FORCE && (q.region == ADRES_REGION_SLAB_X || q.region == ADRES_REGION_SPHERE);

    // Morton order of the cells
    std::vector<std::pair<uint32_t, int>> codes(G.n_cells);
    for (int z = 0; z < G.n[2]; ++z)
        for (int y = 0; y < G.n[1]; ++y)
            for (int x = 0; x < G.n[0]; ++x) {
                int cidx = x + G.n[0] * (y + G.n[1] * z);
                codes[cidx] = {spread3(x) | (spread3(y) << 1) | (spread3(z) << 2), cidx};
            }
    std::sort(codes.begin(), codes.end());
    std::vector<int> rank(G.n_cells);
    for (int r = 0; r < G.n_cells; ++r) rank[codes[r].second] = r;

    // neighbour-list capacity: twice the mean count at this density, plus slack
    double vol = q.box[0] * q.box[1] * q.box[2];
    double mean = (double)q.n_mol / vol * (4.0 / 3.0) * M_PI * c->rl2 * c->r_list;
    c->cap = (((int)std::ceil(2.0 * mean) + 16) + 15) & ~15;

    // the 27 stencil neighbours of every cell, by Morton rank (stencil order z, y, x offset;
    // offsets outside [off_lo, off_hi] skipped so that small grids visit no cell twice)
    std::vector<int> stencil((size_t)G.n_cells * 27);
    for (int r = 0; r < G.n_cells; ++r) {
        const int cidx = codes[r].second;
        const int cx = cidx % G.n[0], cy = (cidx / G.n[0]) % G.n[1], cz = cidx / (G.n[0] * G.n[1]);
        for (int l = 0; l < 27; ++l) {
            const int oz = l / 9 - 1, oy = (l / 3) % 3 - 1, ox = l % 3 - 1;
            const bool used = ox >= G.off_lo[0] && ox <= G.off_hi[0] && oy >= G.off_lo[1] && oy <= G.off_hi[1] &&
                              oz >= G.off_lo[2] && oz <= G.off_hi[2];
            const int wx = (cx + ox + G.n[0]) % G.n[0], wy = (cy + oy + G.n[1]) % G.n[1],
                      wz = (cz + oz + G.n[2]) % G.n[2];
            stencil[(size_t)r * 27 + l] = used ? rank[wx + G.n[0] * (wy + G.n[1] * wz)] : -1;
        }
    }

    const int n = q.n_mol;
    const int64_t ns = P.n_sites;
    bool ok = true;
    for (int b = 0; b < 2; ++b) {
        ok = ok && dalloc(&c->S[b].x, 3 * ns) == hipSuccess && dalloc(&c->S[b].v, 3 * ns) == hipSuccess &&
             dalloc(&c->S[b].Rw, n) == hipSuccess &&
             dalloc(&c->S[b].perm, n) == hipSuccess && dalloc(&c->S[b].key, n) == hipSuccess;
    }
    ok = ok && dalloc(&c->f, 3 * ns) == hipSuccess;
    ok = ok && dalloc(&c->R_ref, (size_t)n) == hipSuccess && dalloc(&c->inv_perm, n) == hipSuccess &&
         dalloc(&c->cell_rank, G.n_cells) == hipSuccess &&
         dalloc(&c->count, G.n_cells) == hipSuccess && dalloc(&c->start, G.n_cells + 1) == hipSuccess &&
         dalloc(&c->fill, G.n_cells) == hipSuccess && dalloc(&c->new_from, n) == hipSuccess &&
         dalloc(&c->nbr, (size_t)c->cap * n) == hipSuccess && dalloc(&c->cnt, n) == hipSuccess &&
         dalloc(&c->ctrl, 1) == hipSuccess &&
         dalloc(&c->scan_tiles, (size_t)std::max(G.n_cells, n) / 1024 + 2) == hipSuccess;
    ok = ok && dalloc(&c->cnt_up, n) == hipSuccess && dalloc(&c->up_off, (size_t)n + 1) == hipSuccess &&
         dalloc(&c->up_scratch, n) == hipSuccess;
    c->epart_blocks = force_blocks(n);
    ok = ok && dalloc(&c->epart, 4 * (size_t)c->epart_blocks) == hipSuccess;
    ok = ok && dalloc(&c->hn, (size_t)c->epart_blocks) == hipSuccess;
    ok = ok && dalloc(&c->tperm, (size_t)c->epart_blocks * kHaloTile) == hipSuccess;
    ok = ok && alloc_halo(c, std::min(320, halo_capacity_limit(q.sites_per_mol, q.pair_precision))) == ADRES_OK;
    ok = ok && dalloc(&c->tile_pos, (size_t)c->epart_blocks) == hipSuccess &&
         dalloc(&c->hcnt, (size_t)c->epart_blocks * kHaloTile) == hipSuccess;
    ok = ok && dalloc(&c->tile_order, (size_t)c->epart_blocks) == hipSuccess &&
         dalloc(&c->mcost, ((size_t)n + 15) / 16 * 16) == hipSuccess &&   // whole 16-entry runs
         dalloc(&c->stencil, (size_t)G.n_cells * 27) == hipSuccess;
    if (q.region == ADRES_REGION_SPHERES) ok = ok && dalloc(&c->near, (size_t)n) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&c->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&c->pub, sizeof(CtrlPub), hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
    if (ok) {
        std::memset(c->pub, 0, sizeof(CtrlPub));
        ok = hipHostGetDevicePointer((void **)&c->pub_dev, c->pub, 0) == hipSuccess;
    }
    if (!ok) {
        adres_destroy(c);
        return ADRES_E_NOMEM;
    }
    std::vector<int> ident(n);
    for (int i = 0; i < n; ++i) ident[i] = i;
    Ctrl c0{INT_MAX, 0, 0, 0, 0, 0, 0};
    bool cp = hipMemcpy(c->cell_rank, rank.data(), sizeof(int) * G.n_cells, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->S[0].perm, ident.data(), sizeof(int) * n, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->S[1].perm, ident.data(), sizeof(int) * n, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->inv_perm, ident.data(), sizeof(int) * n, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->stencil, stencil.data(), sizeof(int) * stencil.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(c->count, 0, sizeof(int) * G.n_cells) == hipSuccess &&
              hipMemset(c->cnt_up, 0, sizeof(int) * n) == hipSuccess &&
              hipMemcpy(c->ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice) == hipSuccess;
    if (!cp) {
        adres_destroy(c);
        return ADRES_E_HIP;
    }
    *out = c;
    return ADRES_OK;
}

void adres_destroy(adres_ctx *c)
{
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    for (int b = 0; b < 2; ++b) {
        hipFree(c->S[b].x); hipFree(c->S[b].v); hipFree(c->S[b].Rw);
        hipFree(c->S[b].perm); hipFree(c->S[b].key);
    }
    hipFree(c->f);
    hipFree(c->R_ref); hipFree(c->inv_perm); hipFree(c->cell_rank);
    hipFree(c->count); hipFree(c->start); hipFree(c->fill); hipFree(c->new_from); hipFree(c->scan_tiles);
    hipFree(c->nbr); hipFree(c->cnt); hipFree(c->hid); hipFree(c->hn); hipFree(c->lnbr); hipFree(c->tperm); hipFree(c->ctrl); hipFree(c->epart); hipFree(c->tab);
    hipFree(c->td); hipFree(c->td_u); hipFree(c->anchors); hipFree(c->aslot); hipFree(c->near); hipFree(c->anchor_cen); hipFree(c->tile_order); hipFree(c->tile_pos); hipFree(c->hcnt); hipFree(c->mcost); hipFree(c->stencil);
    hipFree(c->mlp); hipFree(c->mlp_w2); hipFree(c->mlp_w2q); hipFree(c->mlp_fp8s); hipFree(c->cnt_up); hipFree(c->up_off); hipFree(c->up_scratch);
    hipFree(c->pid); hipFree(c->up_pairs); hipFree(c->f_pair);
    hipFree(c->adam_m); hipFree(c->adam_v); hipFree(c->grad); hipFree(c->loss); hipFree(c->res_part);
    hipFree(c->resid); hipFree(c->gpart); hipFree(c->gred);
    if (c->ctrl_host) hipHostFree(c->ctrl_host);
    if (c->pub) hipHostFree(c->pub);
    for (auto &e : c->events) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    delete c;
}

adres_status adres_weights(adres_ctx *c, const double *x, double *com, double *w)
{
    if (!c || !x || !com || !w) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.region == ADRES_REGION_SPHERES && c->P.n_anchors == 0)
        return fail(c, ADRES_E_STATE, "self-adjusting region without anchors (adres_set_anchors)");
    launch_weights_caller(c->stream, c->P, x, com, w, c->ctrl);
    if (c->P.region == ADRES_REGION_SPHERES) launch_anchor_weights_caller(c->stream, c->P, com, w);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_build_cells(adres_ctx *c, const double *x)
{
    if (!c || !x) return fail(c, ADRES_E_ARG, "null argument");
    adres_status st = gather(c, x, nullptr, false);
    if (st != ADRES_OK) return st;
    st = resort(c, false);
    if (st == ADRES_OK) c->have_state = true;
    return st;
}

adres_status adres_build_verlet(adres_ctx *c, const double *x, int64_t *n_pairs)
{
    if (!c || !x) return fail(c, ADRES_E_ARG, "null argument");
    adres_status st = full_build(c, x, nullptr);
    if (st != ADRES_OK) return st;
    if (n_pairs) {
        std::vector<int> h(c->P.n_mol);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->cnt, sizeof(int) * h.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int64_t s = 0;
        for (int v : h) s += v;
        *n_pairs = s / 2;
    }
    return ADRES_OK;
}

namespace {

adres_status forces_impl(adres_ctx *c, const double *x, double *f, double *energy, double *epart);

}  // namespace

adres_status adres_forces(adres_ctx *c, const double *x, double *f, double *energy)
{
    if (!c || !x || !f) return fail(c, ADRES_E_ARG, "null argument");
    return forces_impl(c, x, f, energy, c->epart);
}

adres_status adres_forces_noalloc(adres_ctx *c, const double *x, double *f, double *energy)
{
    if (!c || !x || !f) return fail(c, ADRES_E_ARG, "null argument");
    if (c->epart_blocks > kNoallocBlocks)
        return fail(c, ADRES_E_CAPACITY, "adres_forces_noalloc takes at most 524288 molecules (" +
                                             std::to_string(kNoallocBlocks) + " workgroup partials)");
    if (!c->scratch_epart) return fail(c, ADRES_E_STATE, "no static scratch address for this device");
    c->no_alloc = true;
    const adres_status st = forces_impl(c, x, f, energy, c->scratch_epart);
    c->no_alloc = false;
    return st;
}

namespace {

adres_status forces_impl(adres_ctx *c, const double *x, double *f, double *energy, double *epart)
{
    adres_status st = check_cg_ready(c);
    if (st != ADRES_OK) return st;
    if (!c->list_valid) {
        st = full_build(c, x, nullptr);
        if (st != ADRES_OK) return st;
    } else {
        launch_reset_halt(c->stream, c->ctrl);
        st = gather(c, x, nullptr, true);
        if (st != ADRES_OK) return st;
        st = read_ctrl(c);
        if (st != ADRES_OK) return st;
        if (c->ctrl_host->halt != INT_MAX) {
            st = resort(c, false);
            if (st != ADRES_OK) return st;
            st = build_list(c);
            if (st != ADRES_OK) return st;
        }
    }
    ForceArgs a = force_args(c);
    a.f = f;
    a.out_perm = cur(c).perm;
    a.epart = energy ? epart : nullptr;
    st = run_forces(c, a);
    if (st != ADRES_OK) return st;
    if (energy) {
        launch_energy_reduce(c->stream, epart, c->epart_blocks, energy);
        HIPCHK(c, hipGetLastError());
    }
    return ADRES_OK;
}

}  // namespace

namespace {

// Velocity Verlet (n_inner = 1) or RESPA with n_inner inner steps of dt per outer step
// (n_steps a multiple of n_inner).  In RESPA the half kicks of the slow part at the end
// of one outer step and the start of the next meet at the same positions, as do the fast
// part's half kicks at every inner boundary, so every kernel g kicks with
// F_fast + s_g F_slow: s_g = n_inner at outer boundaries (g a multiple of n_inner), else 0
// (the slow part is then not computed).  n_inner = 1 gives s_g = 1: plain VV.
adres_status integrate_impl(adres_ctx *c, double *x, double *v, double *f, double dt, int32_t n_steps,
                            int32_t n_inner, double gamma, double kT, uint64_t seed, int32_t *n_rebuilds)
{
    adres_status st = check_cg_ready(c);
    if (st != ADRES_OK) return st;
    st = full_build(c, x, v);
    if (st != ADRES_OK) return st;
    auto slow_scale = [n_inner](int g) { return g % n_inner == 0 ? (double)n_inner : 0.0; };

    // F(x_0) into the Morton-ordered force buffer
    ForceArgs a0 = force_args(c);
    a0.f = c->f;
    a0.slow_scale = slow_scale(0);
    st = run_forces(c, a0);
    if (st != ADRES_OK) return st;

    // Kernel g (0 <= g <= n_steps) finishes/starts steps around time g:
    //   g = 0:            opening kick + drift of step 1 (needs F(x_0))
    //   0 < g < n_steps:  fused: F(x_g), closing kick of step g, opening kick + drift of step g+1
    //   g = n_steps:      F(x_N) and the closing kick of the last step
    // Kernels with g < n_steps drift (positions flip buffers).  They are launched in
    // chunks; a drift whose centres moved more than skin/2 sets ctrl->halt to its
    // chunk index and every later kernel of the chunk returns at once.
    int rebuilds = 0;
    int g = 0;
    int since = 0;   // kernels since the last rebuild
    const int *go = &c->ctrl->go;
    launch_reset_halt(c->stream, c->ctrl);
    while (g <= n_steps && n_steps > 0) {
        // one kernel past the expected rebuild: a chunk without one costs a rebuild's worth of
        // guarded launches that return at once, one past it only a kernel that does
        const int len = std::min(std::max(2, c->last_interval - since) + 1, n_steps + 1 - g);
        int p = c->pos;
        int len_drift = 0;
        const size_t ev0 = c->events_used;   // this chunk's timed launches start here
        for (int k = 0; k < len; ++k) {
            const int gk = g + k;
            StepArgs sa{dt, gamma, kT, seed, c->step_counter + (uint64_t)gk};
            const StateBufs in = view(c, p, c->ord), out = view(c, 1 - p, c->ord);
            if (gk == 0) {
                launch_kick_drift(c->stream, c->P, in.x, in.v, c->f, out.x, out.Rw, c->R_ref, in.perm, c->ctrl, k,
                                  sa);
                if (c->P.region == ADRES_REGION_SPHERES)
                    launch_anchor_weights(c->stream, c->P, out.Rw, c->inv_perm, c->aslot, 0, c->ctrl, k, 1, c->near);
                HIPCHK(c, hipGetLastError());
            } else {
                ForceArgs a = force_args(c);
                a.x = in.x;
                a.Rw = in.Rw;
                a.v = in.v;
                a.st = sa;
                a.step = k;
                a.check_halt = 1;
                a.slow_scale = slow_scale(gk);
                if (gk < n_steps) {
                    a.mode = kModeStep;
                    a.x_out = out.x;
                    a.Rw_out = keep_centres(c) ? out.Rw : nullptr;
                    a.R_ref = c->R_ref;
                    if (!keep_centres(c)) c->rw_stale = true;
                } else {
                    a.mode = kModeClose;
                    a.f = c->f;
                }
                st = run_forces(c, a);
                if (st != ADRES_OK) return st;
                if (gk < n_steps && c->P.region == ADRES_REGION_SPHERES) {
                    launch_anchor_weights(c->stream, c->P, out.Rw, c->inv_perm, c->aslot, 0, c->ctrl, k, 1, c->near);
                    HIPCHK(c, hipGetLastError());
                }
            }
            if (gk < n_steps) {
                p = 1 - p;
                ++len_drift;
            }
        }
        // A reorder + list rebuild that runs only if a drift asked for one (Ctrl::go), whose
        // first launch publishes the chunk's control word (its second clears halt): the GPU
        // goes on while the host reads the publication.  The rebuild is enqueued as if every
        // drift ran (positions in buffer p); if an odd number did not, its kernels read the
        // other buffer (Ctrl::fix).  The host keeps the rebuild's bookkeeping only if it ran.
        const unsigned seq = ++c->pub_seq;
        c->pos = p;
        const int pos0 = c->pos, ord0 = c->ord;
        const bool stale0 = c->rw_stale, valid0 = c->list_valid;
        enqueue_resort(c, true, go, ChainHead{c->ctrl, c->pub_dev, seq, len_drift});
        commit_resort(c);
        st = enqueue_list(c, go);
        if (st != ADRES_OK) return st;
        c->list_valid = true;
        // the one synchronisation per chunk; on an error latched by the chunk the fields are
        // still read, so that the context's buffers stay where the device left them
        st = wait_ctrl(c, seq);
        if (st != ADRES_OK && __atomic_load_n(&c->pub->w[kPubHalt], __ATOMIC_ACQUIRE) >> 32 != seq) return st;
        const adres_status chunk_st = st;
        const int h = c->ctrl_host->halt;
        for (size_t i = ev0; i < c->events_used; ++i)
            if (c->event_k[i] >= 0 && (h < 0 || (h != INT_MAX && c->event_k[i] > h))) c->event_skip[i] = 1;
        // the drifts that ran, and whether the positions sit in the other buffer (as on the device)
        const int ran_drift = h == INT_MAX ? len_drift : (h < 0 ? 0 : std::min(h + 1, len_drift));
        const int fix = (len_drift - ran_drift) & 1;
        if (h < 0 || h == INT_MAX) {   // the rebuild did not run
            c->pos = pos0 ^ fix;
            c->ord = ord0;
            c->rw_stale = stale0;
            c->list_valid = valid0;
        } else {
            c->pos = pos0 ^ fix ^ 1;   // the reorder wrote the buffer its source was not in
        }
        if (chunk_st != ADRES_OK) return chunk_st;
        if (h < 0) {
            // the last list build overflowed: nothing of this chunk ran; regrow, rebuild
            st = build_list(c);
            if (st != ADRES_OK) return st;
            continue;
        }
        const int ran = h == INT_MAX ? len : h + 1;   // kernels that completed
        g += ran;
        since += ran;
        if (h == INT_MAX) continue;
        // kernel g-1 drifted, asked for a rebuild, and the rebuild ran
        ++rebuilds;
        c->last_interval = std::max(2, since);
        since = 0;
    }
    c->step_counter += (uint64_t)n_steps;
    if (n_inner > 1) {
        // the closing kernel kicked with F_fast + n_inner F_slow; report the total force
        ForceArgs af = force_args(c);
        af.f = c->f;
        st = run_forces(c, af);
        if (st != ADRES_OK) return st;
    }
    const StateBufs fin = cur(c);
    launch_scatter_out(c->stream, c->P, fin.perm, fin.x, fin.v, c->f, x, v, f);
    HIPCHK(c, hipGetLastError());
    st = read_ctrl(c);
    if (n_rebuilds) *n_rebuilds = rebuilds;
    return st;
}

}  // namespace

adres_status adres_integrate(adres_ctx *c, double *x, double *v, double *f, double dt, int32_t n_steps,
                             double gamma, double kT, uint64_t seed, int32_t *n_rebuilds)
{
    if (!c || !x || !v || !f) return fail(c, ADRES_E_ARG, "null argument");
    if (n_steps < 0 || !(dt > 0.0) || gamma < 0.0 || (gamma > 0.0 && !(kT >= 0.0)))
        return fail(c, ADRES_E_ARG, "invalid dt, n_steps, gamma or kT");
    return integrate_impl(c, x, v, f, dt, n_steps, 1, gamma, kT, seed, n_rebuilds);
}

adres_status adres_integrate_respa(adres_ctx *c, double *x, double *v, double *f, double dt, int32_t n_inner,
                                   int32_t n_outer, double gamma, double kT, uint64_t seed, int32_t *n_rebuilds)
{
    if (!c || !x || !v || !f) return fail(c, ADRES_E_ARG, "null argument");
    if (n_inner < 1 || n_outer < 0 || (int64_t)n_inner * n_outer > INT32_MAX || !(dt > 0.0) || gamma < 0.0 ||
        (gamma > 0.0 && !(kT >= 0.0)))
        return fail(c, ADRES_E_ARG, "invalid dt, n_inner, n_outer, gamma or kT");
    return integrate_impl(c, x, v, f, dt, n_inner * n_outer, n_inner, gamma, kT, seed, n_rebuilds);
}

adres_status adres_get_pairs(adres_ctx *c, int32_t *pairs_host, int64_t cap, int64_t *n)
{
    if (!c || !n || (cap > 0 && !pairs_host)) return fail(c, ADRES_E_ARG, "null argument");
    if (!c->list_valid) return fail(c, ADRES_E_STATE, "no neighbour list has been built");
    const int nm = c->P.n_mol;
    std::vector<int> cnt(nm), perm(nm), nbr((size_t)c->cap * nm);
    HIPCHK(c, hipMemcpyAsync(cnt.data(), c->cnt, sizeof(int) * nm, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(perm.data(), cur(c).perm, sizeof(int) * nm, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(nbr.data(), c->nbr, sizeof(int) * nbr.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<std::pair<int, int>> pr;
    for (int t = 0; t < nm; ++t)
        for (int k = 0; k < std::min(cnt[t], c->cap); ++k) {
            int a = perm[t], b = perm[nbr[(size_t)t * c->cap + k]];
            if (a < b) pr.emplace_back(a, b);
        }
    std::sort(pr.begin(), pr.end());
    *n = (int64_t)pr.size();
    for (int64_t i = 0; i < std::min<int64_t>(cap, *n); ++i) {
        pairs_host[2 * i] = pr[i].first;
        pairs_host[2 * i + 1] = pr[i].second;
    }
    return ADRES_OK;
}

adres_status adres_get_cells(adres_ctx *c, int32_t *cell_start_host, int32_t *perm_host, int32_t *n_cells)
{
    if (!c) return ADRES_E_ARG;
    if (!c->have_state) return fail(c, ADRES_E_STATE, "no cell list has been built");
    if (n_cells) *n_cells = c->G.n_cells;
    if (cell_start_host)
        HIPCHK(c, hipMemcpyAsync(cell_start_host, c->start, sizeof(int) * (c->G.n_cells + 1), hipMemcpyDeviceToHost,
                                 c->stream));
    if (perm_host)
        HIPCHK(c, hipMemcpyAsync(perm_host, cur(c).perm, sizeof(int) * c->P.n_mol, hipMemcpyDeviceToHost,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ADRES_OK;
}

adres_status adres_set_cg_table(adres_ctx *c, const float *coef4, int32_t n_knots, double r_lo, double r_hi)
{
    if (!c || !coef4) return fail(c, ADRES_E_ARG, "null argument");
    if (n_knots < 2 || n_knots > 4096 || !(r_hi > r_lo) || !(r_lo > 0.0))
        return fail(c, ADRES_E_ARG, "table needs 2..4096 knots on 0 < r_lo < r_hi");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->tab) HIPCHK(c, hipFree(c->tab));
    c->tab = nullptr;
    HIPCHK(c, dalloc(&c->tab, (size_t)(n_knots - 1)));
    HIPCHK(c, hipMemcpy(c->tab, coef4, sizeof(float4) * (n_knots - 1), hipMemcpyHostToDevice));
    c->P.tab = c->tab;
    c->P.tab_n = n_knots;
    c->P.tab_lo = r_lo;
    c->P.tab_h = (r_hi - r_lo) / (double)(n_knots - 1);
    c->P.tab_inv_h = (double)(n_knots - 1) / (r_hi - r_lo);
    return ADRES_OK;
}

adres_status adres_set_tdforce(adres_ctx *c, const double *table, int32_t n, double d_lo, double d_hi)
{
    if (!c) return fail(c, ADRES_E_ARG, "null argument");
    if (n == 0) {
        c->P.td_n = 0;
        return ADRES_OK;
    }
    if (!table) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.region != ADRES_REGION_SLAB_X && c->P.region != ADRES_REGION_SPHERE &&
        c->P.region != ADRES_REGION_SPHERES)
        return fail(c, ADRES_E_ARG, "a correction force needs a slab, sphere or anchor-sphere region");
    if (n < 0 || n > kTdMaxBins || !std::isfinite(d_lo) || !std::isfinite(d_hi) || !(d_lo >= 0.0) ||
        !(d_hi > d_lo))
        return fail(c, ADRES_E_ARG, "correction table needs 1..4096 values on 0 <= d_lo < d_hi");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(table[k])) return fail(c, ADRES_E_ARG, "correction table value is not finite");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->td) {
        HIPCHK(c, dalloc(&c->td, (size_t)kTdMaxBins));
        HIPCHK(c, dalloc(&c->td_u, (size_t)kTdMaxBins));
    }
    HIPCHK(c, hipMemcpy(c->td, table, sizeof(double) * n, hipMemcpyHostToDevice));
    c->P.td = c->td;
    c->P.td_u = c->td_u;
    c->P.td_n = n;
    c->P.td_lo = d_lo;
    c->P.td_hi = d_hi;
    c->P.td_h = (d_hi - d_lo) / (double)n;
    launch_td_update(c->stream, c->P, c->td, c->td_u, nullptr, 1, 0.0, nullptr, 0);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_set_anchors(adres_ctx *c, const int32_t *mols, int32_t k)
{
    if (!c || !mols) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.region != ADRES_REGION_SPHERES) return fail(c, ADRES_E_ARG, "anchors need region ADRES_REGION_SPHERES");
    if (k < 1 || k > kMaxAnchors) return fail(c, ADRES_E_ARG, "1..1024 anchors");
    for (int i = 0; i < k; ++i)
        if (mols[i] < 0 || mols[i] >= c->P.n_mol) return fail(c, ADRES_E_ARG, "anchor index out of range");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->anchors) {
        HIPCHK(c, dalloc(&c->anchors, (size_t)kMaxAnchors));
        HIPCHK(c, dalloc(&c->aslot, (size_t)kMaxAnchors));
        HIPCHK(c, dalloc(&c->anchor_cen, (size_t)kMaxAnchors * 3));
    }
    HIPCHK(c, hipMemcpy(c->anchors, mols, sizeof(int) * k, hipMemcpyHostToDevice));
    c->P.anchors = c->anchors;
    c->P.n_anchors = k;
    c->list_valid = false;   // the weights of the stored state are stale
    return ADRES_OK;
}

adres_status adres_get_tdforce(adres_ctx *c, double *table_host, int32_t n)
{
    if (!c || !table_host) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.td_n == 0) return fail(c, ADRES_E_STATE, "no correction force installed");
    if (n != c->P.td_n) return fail(c, ADRES_E_ARG, "n differs from the installed table's length");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(table_host, c->td, sizeof(double) * n, hipMemcpyDeviceToHost));
    return ADRES_OK;
}

adres_status adres_density_profile(adres_ctx *c, const double *x, int64_t *counts)
{
    if (!c || !x || !counts) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.td_n == 0) return fail(c, ADRES_E_STATE, "no correction table (its bins define the profile)");
    const double *cen = nullptr;
    if (c->P.region == ADRES_REGION_SPHERES) {
        if (c->P.n_anchors == 0) return fail(c, ADRES_E_STATE, "self-adjusting region without anchors");
        launch_anchor_centres(c->stream, c->P, x, c->anchor_cen);
        cen = c->anchor_cen;
    }
    launch_density_profile(c->stream, c->P, x, cen, reinterpret_cast<unsigned long long *>(counts));
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_region_volumes(adres_ctx *c, const double *x, int64_t n_samples, uint64_t seed,
                                  int64_t *vol_counts)
{
    if (!c || !vol_counts) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.td_n == 0) return fail(c, ADRES_E_STATE, "no correction table (its bins define the volumes)");
    if (n_samples < 1) return fail(c, ADRES_E_ARG, "need n_samples >= 1");
    const double *cen = nullptr;
    if (c->P.region == ADRES_REGION_SPHERES) {
        if (!x) return fail(c, ADRES_E_ARG, "anchor spheres need the configuration x");
        if (c->P.n_anchors == 0) return fail(c, ADRES_E_STATE, "self-adjusting region without anchors");
        launch_anchor_centres(c->stream, c->P, x, c->anchor_cen);
        cen = c->anchor_cen;
    }
    launch_region_volumes(c->stream, c->P, cen, (long long)n_samples, (unsigned long long)seed,
                          reinterpret_cast<unsigned long long *>(vol_counts));
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_tdforce_update(adres_ctx *c, const int64_t *counts, int64_t n_frames, double prefactor)
{
    if (!c || !counts) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.td_n == 0) return fail(c, ADRES_E_STATE, "no correction force installed");
    if (n_frames < 1 || !std::isfinite(prefactor)) return fail(c, ADRES_E_ARG, "need n_frames >= 1, finite prefactor");
    if (c->P.region == ADRES_REGION_SPHERES)
        return fail(c, ADRES_E_ARG, "anchor spheres have no closed-form bin volumes: use adres_tdforce_update_sampled");
    launch_td_update(c->stream, c->P, c->td, c->td_u, reinterpret_cast<const long long *>(counts),
                     (long long)n_frames, prefactor, nullptr, 0);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_tdforce_update_sampled(adres_ctx *c, const int64_t *counts, int64_t n_frames,
                                          const int64_t *vol_counts, int64_t n_vol_samples, double prefactor)
{
    if (!c || !counts || !vol_counts) return fail(c, ADRES_E_ARG, "null argument");
    if (c->P.td_n == 0) return fail(c, ADRES_E_STATE, "no correction force installed");
    if (n_frames < 1 || n_vol_samples < 1 || !std::isfinite(prefactor))
        return fail(c, ADRES_E_ARG, "need n_frames >= 1, n_vol_samples >= 1, finite prefactor");
    launch_td_update(c->stream, c->P, c->td, c->td_u, reinterpret_cast<const long long *>(counts),
                     (long long)n_frames, prefactor, reinterpret_cast<const long long *>(vol_counts),
                     (long long)n_vol_samples);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_mlp_set(adres_ctx *c, const float *params, int32_t n_params, double rc, double scale,
                           double taper_width, double r_min)
{
    if (!c || !params) return fail(c, ADRES_E_ARG, "null argument");
    if (n_params != kMlpParams) return fail(c, ADRES_E_ARG, "the network has 4353 parameters (hidden width 64)");
    if (!(rc > 0.0) || !(taper_width > 0.0) || taper_width > rc || !(r_min >= 0.0) || !std::isfinite(scale))
        return fail(c, ADRES_E_ARG, "need rc > 0, 0 < taper_width <= rc, r_min >= 0, finite scale");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->mlp) {
        HIPCHK(c, dalloc(&c->mlp, kMlpParams));
        HIPCHK(c, dalloc(&c->mlp_w2, (size_t)2 * kHidden * kHidden));
        HIPCHK(c, dalloc(&c->mlp_w2q, (size_t)kHidden * kHidden / 4));
        HIPCHK(c, dalloc(&c->mlp_fp8s, 4));
        HIPCHK(c, dalloc(&c->adam_m, kMlpParams));
        HIPCHK(c, dalloc(&c->adam_v, kMlpParams));
    }
    HIPCHK(c, hipMemcpy(c->mlp, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(c->adam_m, 0, sizeof(float) * kMlpParams));
    HIPCHK(c, hipMemset(c->adam_v, 0, sizeof(float) * kMlpParams));
    c->adam_t = 0;
    launch_mlp_convert(c->stream, c->mlp, c->mlp_w2, c->mlp_w2 + kHidden * kHidden);
    launch_mlp_fp8_prepare(c->stream, c->mlp, c->mlp_w2q, c->mlp_fp8s);
    HIPCHK(c, hipGetLastError());
    c->mlp_rc = rc;
    c->mlp_scale = scale;
    c->mlp_tw = taper_width;
    c->mlp_rmin = r_min;
    c->have_mlp = true;
    return ADRES_OK;
}

adres_status adres_mlp_get(adres_ctx *c, float *params, int32_t n_params)
{
    if (!c || !params) return fail(c, ADRES_E_ARG, "null argument");
    if (!c->have_mlp) return fail(c, ADRES_E_STATE, "no network installed");
    if (n_params != kMlpParams) return fail(c, ADRES_E_ARG, "the network has 4353 parameters");
    HIPCHK(c, hipMemcpyAsync(params, c->mlp, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ADRES_OK;
}

adres_status adres_mlp_eval(adres_ctx *c, const double *r, float *f, int64_t n)
{
    if (!c || (n > 0 && (!r || !f)) || n < 0) return fail(c, ADRES_E_ARG, "null argument or negative count");
    if (!c->have_mlp) return fail(c, ADRES_E_STATE, "no network installed");
    if (n == 0) return ADRES_OK;
    launch_mlp_forward_r(c->stream, mlp_dev(c), c->P, r, f, n, c->ctrl);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

}  // extern "C"

namespace {

// Loss and gradient of force matching over n_frames frames of CG sites (accumulated
// on the device in c->loss and c->grad).
adres_status fm_accumulate(adres_ctx *c, const double *com, const double *fmap, int32_t n_frames)
{
    if (!com || !fmap || n_frames < 1) return fail(c, ADRES_E_ARG, "need frames of centres and mapped forces");
    if (c->P.spm != 1 || c->P.region != ADRES_REGION_ALL_CG || c->P.cg_kind != ADRES_CG_MLP)
        return fail(c, ADRES_E_STATE, "force matching needs a context of CG sites (1 site, all CG, MLP kind)");
    if (!c->have_mlp) return fail(c, ADRES_E_STATE, "no network installed");
    const int n = c->P.n_mol;
    if (!c->grad) {
        const bool ok = dalloc(&c->grad, kMlpParams) == hipSuccess && dalloc(&c->loss, 1) == hipSuccess &&
                        dalloc(&c->res_part, (size_t)(n + 255) / 256) == hipSuccess &&
                        dalloc(&c->resid, 3 * (size_t)n) == hipSuccess &&
                        dalloc(&c->gpart, (size_t)mlp_backward_waves() * kMlpParams) == hipSuccess &&
                        dalloc(&c->gred, (size_t)mlp_reduce_chunks() * kMlpParams) == hipSuccess;
        if (!ok) return fail(c, ADRES_E_NOMEM, "could not allocate training buffers");
    }
    launch_zero(c->stream, c->grad, kMlpParams);
    launch_zero(c->stream, c->loss, 1);
    const double cc = 1.0 / (3.0 * (double)n_frames * (double)n);
    for (int fr = 0; fr < n_frames; ++fr) {
        const double *x = com + (size_t)fr * 3 * n;
        const double *fm = fmap + (size_t)fr * 3 * n;
        adres_status st = full_build(c, x, nullptr);
        if (st != ADRES_OK) return st;
        ForceArgs a = force_args(c);
        a.f = c->f;
        st = run_forces(c, a);
        if (st != ADRES_OK) return st;
        const StateBufs b = cur(c);
        int n_part = 0;
        launch_fm_residual(c->stream, n, b.perm, c->f, fm, c->resid, c->res_part, &n_part);
        launch_loss_accumulate(c->stream, c->res_part, n_part, cc, c->loss);
        launch_mlp_backward(c->stream, mlp_dev(c), c->P, c->up_pairs, c->up_off + n, b.Rw, c->resid, 2.0 * cc,
                            c->gpart, c->gred, c->grad);
        HIPCHK(c, hipGetLastError());
    }
    return ADRES_OK;
}

}  // namespace

extern "C" {

adres_status adres_mlp_fm_grad(adres_ctx *c, const double *com, const double *f_map, int32_t n_frames,
                               double *grad_host, double *loss_host)
{
    if (!c) return ADRES_E_ARG;
    adres_status st = fm_accumulate(c, com, f_map, n_frames);
    if (st != ADRES_OK) return st;
    if (grad_host)
        HIPCHK(c, hipMemcpyAsync(grad_host, c->grad, sizeof(double) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
    if (loss_host) HIPCHK(c, hipMemcpyAsync(loss_host, c->loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return read_ctrl(c);
}

adres_status adres_mlp_train_step(adres_ctx *c, const double *com, const double *f_map, int32_t n_frames, double lr,
                                  double *loss_host)
{
    if (!c) return ADRES_E_ARG;
    if (!(lr > 0.0)) return fail(c, ADRES_E_ARG, "learning rate must be positive");
    adres_status st = fm_accumulate(c, com, f_map, n_frames);
    if (st != ADRES_OK) return st;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    ++c->adam_t;
    const double bc1 = 1.0 - std::pow(b1, (double)c->adam_t), bc2 = 1.0 - std::pow(b2, (double)c->adam_t);
    launch_adam(c->stream, c->mlp, c->adam_m, c->adam_v, c->grad, lr, b1, b2, bc1, bc2, eps);
    launch_mlp_convert(c->stream, c->mlp, c->mlp_w2, c->mlp_w2 + kHidden * kHidden);
    HIPCHK(c, hipGetLastError());
    if (loss_host) HIPCHK(c, hipMemcpyAsync(loss_host, c->loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return read_ctrl(c);
}

adres_status adres_map_cg(adres_ctx *c, const double *x, double *f, double *com, double *f_map)
{
    if (!c || !x || !f || !com || !f_map) return fail(c, ADRES_E_ARG, "null argument");
    adres_status st = adres_forces(c, x, f, nullptr);
    if (st != ADRES_OK) return st;
    launch_map_cg(c->stream, c->P, x, f, com, f_map);
    HIPCHK(c, hipGetLastError());
    return ADRES_OK;
}

adres_status adres_kernel_timing(adres_ctx *c, int32_t enable, int32_t every, double *ms, int64_t *launches)
{
    if (!c) return ADRES_E_ARG;
    if (enable < 0 || enable > 2 || every < 1) return fail(c, ADRES_E_ARG, "timing mode must be 0, 1 or 2 and every >= 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    int64_t counted = 0;
    for (size_t i = 0; i < c->events_used; ++i) {
        if (c->event_skip[i]) continue;
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->events[i].first, c->events[i].second));
        sum += t;
        ++counted;
    }
    if (ms) *ms = sum;
    if (launches) *launches = counted;
    c->events_used = 0;
    c->timing = enable;
    c->timing_every = every;
    c->timing_count = 0;
    return ADRES_OK;
}

const char *adres_last_error(const adres_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

}  // extern "C"
