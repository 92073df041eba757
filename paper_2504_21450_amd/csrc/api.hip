// C ABI of libvlasov.so (declared in include/vlasov.h): argument checks,
// workspace carving, initial upload, and the stream-ordered launch sequence of
// the ghost update, the three shears and the end-of-step pruning.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "vl_internal.h"
#include "vl_storage.h"

using namespace vl;

namespace {

constexpr size_t ALIGN = 256;
constexpr int RED_DOUBLES = 1024;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t pool, ring, lstart, lcount, lcapa, lsorted, lid, lslot, litem, rows, items, masks, resid, penfirst,
        pencnt, pensum, ctl, cover, cellred, red, cellcnt, mom, lg_ids[4], lg_res[4], lg_kfirst[4],
        lg_kcnt[4], lg_src, accel, total;
    int64_t N, nlocal, nghost, LA, LG, row_cap, item_cap, pen_cap, mom_parts, lg_cap;
    int wlmax, cover_stride;
};

bool desc_ok(const vl_desc *d)
{
    if (!d) return false;
    int64_t nb = 1;
    for (int k = 0; k < 3; k++) {
        if (d->n[k] < 1 || d->n[k] + 2 * H > MAXL) return false;
        if (d->nblk[k] < 1 || d->nblk[k] > 1024) return false;
        nb *= d->nblk[k];
        if (!(d->dx[k] > 0.0) || !(d->dv[k] > 0.0) || !isfinite(d->vmin[k])) return false;
        if (!isfinite(d->dx[k]) || !isfinite(d->dv[k])) return false;
    }
    if (nb > NB_MAX) return false;
    int seen = 0;
    for (int k = 0; k < 3; k++) {
        if (d->order[k] < 0 || d->order[k] > 2) return false;
        seen |= 1 << d->order[k];
    }
    if (seen != 7) return false;
    if (d->storage != VL_F64 && d->storage != VL_F32 && d->storage != VL_BF16) return false;
    if (d->stencil != 2 || d->gt_level < 1 || d->gt_level > H) return false;
    if (d->vbuffer != 0 && d->vbuffer != 6 && d->vbuffer != 26) return false;
    if (d->edges < 0 || d->edges > 63) return false;
    if (!isfinite(d->sparse_min)) return false;
    if (d->block_capacity < 1 || d->ghost_block_capacity < 1) return false;
    // slots (and the scratch slot) must stay below the row flag bit
    if (d->block_capacity + d->ghost_block_capacity + 1 + NSINK >= (int64_t)NEWFLAG - 1) return false;
    return true;
}

Layout make_layout(const vl_desc *d)
{
    Layout L{};
    int64_t P[3];
    for (int k = 0; k < 3; k++) P[k] = d->n[k] + 2 * H;
    L.N = P[0] * P[1] * P[2];
    L.nlocal = (int64_t)d->n[0] * d->n[1] * d->n[2];
    L.nghost = L.N - L.nlocal;
    const int64_t lcap = d->block_capacity, gcap = d->ghost_block_capacity;
    // list regions: the lists as written (25 % + 32 slack per cell) and room
    // for the lists that outgrow them within a step and move to the region's
    // end (at most once per cell and shear, again with 25 % + 32 slack)
    L.LA = lcap + 3 * (lcap / 4) + 64 * L.nlocal;
    L.LG = gcap + 3 * (gcap / 4) + 64 * L.nghost;
    L.row_cap = lcap + gcap + 64;
    const int64_t tot = lcap + gcap;
    // one item per block of a pencil's union: at most one per (cell, block)
    // of the shear's box; large partitions hold many cells per item
    L.item_cap = tot <= (1 << 24) ? tot + 64 : std::max<int64_t>(1 << 24, tot / 8);
    L.pen_cap = std::max(P[0] * P[1], std::max(P[0] * P[2], P[1] * P[2]));
    int maxP = std::max(P[0], std::max(P[1], P[2]));
    L.wlmax = (maxP + 31) / 32;
    int maxnv = 4 * std::max(d->nblk[0], std::max(d->nblk[1], d->nblk[2]));
    L.cover_stride = maxnv;
    const int bs = storage_bytes(d->storage);
    size_t o = 0;
    L.pool = o;    o = align_up(o + (size_t)(tot + 1 + NSINK) * BLK * bs);  // + zero block + sinks
    L.ring = o;    o = align_up(o + (size_t)lcap * 4);
    L.lstart = o;  o = align_up(o + (size_t)L.N * 8);
    L.lcount = o;  o = align_up(o + (size_t)L.N * 4);
    L.lcapa = o;   o = align_up(o + (size_t)L.N * 4);
    L.lsorted = o; o = align_up(o + (size_t)L.N * 4);
    const size_t nl = (size_t)(2 * L.LA + L.LG);
    L.lid = o;     o = align_up(o + nl * 4);
    L.lslot = o;   o = align_up(o + nl * 4);
    L.litem = o;   o = align_up(o + nl * 4);
    L.rows = o;    o = align_up(o + (size_t)L.row_cap * 4);
    L.items = o;   o = align_up(o + (size_t)L.item_cap * sizeof(Item));
    L.masks = o;   o = align_up(o + (size_t)L.item_cap * L.wlmax * 4);
    L.resid = o;   o = align_up(o + (d->storage == VL_F64 ? 0 : (size_t)L.item_cap * 8));
    L.penfirst = o; o = align_up(o + (size_t)L.pen_cap * 8);
    L.pencnt = o;  o = align_up(o + (size_t)L.pen_cap * 4);
    L.pensum = o;  o = align_up(o + (size_t)L.pen_cap * 8);
    L.ctl = o;     o = align_up(o + sizeof(Ctl));
    L.cover = o;   o = align_up(o + (size_t)3 * maxnv * 8);
    L.cellred = o; o = align_up(o + (size_t)L.nlocal * 8);
    L.red = o;     o = align_up(o + (size_t)RED_DOUBLES * 8);
    L.cellcnt = o; o = align_up(o + (size_t)L.nlocal * 4);
    // moments: a split cell has fewer than 2 cnt / MOM_CHUNK chunks
    L.mom_parts = 2 * lcap / MOM_CHUNK + 64;
    L.mom = o;     o = align_up(o + (size_t)moments_scratch_bytes(L.nlocal, L.mom_parts, L.mom_parts));
    // per-line mass ledger (reduced storage): three stores, one per shear
    // axis, and a fourth that the next shear writes; each holds a shear's
    // items (block id and FP64 residual) and per pencil key its item range
    L.lg_cap = d->storage == VL_F64 ? 0 : L.item_cap;
    for (int k = 0; k < 4; k++) {
        L.lg_ids[k] = o;    o = align_up(o + (size_t)L.lg_cap * 4);
        L.lg_res[k] = o;    o = align_up(o + (size_t)L.lg_cap * 8);
        L.lg_kfirst[k] = o; o = align_up(o + (size_t)(L.lg_cap ? L.pen_cap : 0) * 4);
        L.lg_kcnt[k] = o;   o = align_up(o + (size_t)(L.lg_cap ? L.pen_cap : 0) * 4);
    }
    L.lg_src = o;  o = align_up(o + (size_t)L.lg_cap * 4);
    // acceleration: the velocity maps of the local cells
    L.accel = o;   o = align_up(o + (size_t)L.nlocal * ACC_MAP_DOUBLES * 8);
    L.total = o;
    return L;
}

}  // namespace

struct Prof {
    bool on = false;
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> cls;
};

// Executable graphs of one whole step (coalesced fill when the mode has one,
// then the translation kernels), one per starting list region and ledger
// store rotation (the stores a step reads and writes).  They hold
// dt, the mode, the shear variant and the Courant table pointer as launch
// arguments, so any change of these drops them.
struct GraphCache {
    hipStream_t cap = nullptr;  // private stream, used only to record captures
    hipGraphExec_t exec[8] = {};  // by starting list region + 2 x ledger rotation phase
    double dt = 0.0;
    int mode = -1;
    int variant[3] = {-1, -1, -1};
};

// Ledger store rotation: store axis[a] holds the residuals of the last shear
// along axis a; a shear along a writes store `spare` and then the two swap.
// A step makes three swaps, so the assignment repeats every four steps.
struct LedgerRot {
    int axis[3] = {0, 1, 2};
    int spare = 3;
    int phase = 0;  // steps mod 4 (0 without a ledger)
};

struct vl_partition {
    Prof prof;
    GraphCache graph;
    SrcTable src;       // ghost sources of the last vl_fill_ghosts_from (per-sweep face fills use them)
    bool has_src;
    vl_desc desc;
    Layout lay;
    Dev D;
    hipStream_t stream;
    char *ws;
    int cur;            // local list region in use (0 or 1)
    int64_t init_blocks; // blocks given at init; their slots are 0 .. init_blocks - 1
    bool loadable;      // no step yet: vl_load_values may still overwrite values
    bool ghosts_valid;
    bool bad;
    bool has_cover;
    std::vector<double> cover_host;
    MomScratch mom;       // moments scratch in the workspace
    void *mom_static;     // device address of the fixed scratch array (vl_moments_static)
    LedgerStore lgs[4];   // per-line ledger stores (reduced storage)
    LedgerRot rot;        // which store holds each axis's residuals
};

namespace {

int hip_ok(hipError_t e) { return e == hipSuccess ? VL_OK : VL_ERR_HIP; }

#define VL_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) {                             \
            fprintf(stderr, "libvlasov: %s failed: %s\n", #call, hipGetErrorString(e_)); \
            return VL_ERR_HIP;                              \
        }                                                   \
    } while (0)

// kernel classes timed by the profiler
enum { K_FILL = 0, K_PLAN = 1, K_SWEEP = 2, K_PRUNE = 3, K_OTHER = 4, K_SHEAR0 = 5, K_ACCEL = 8, K_NCLS = 9 };

struct ProfScope {
    vl_partition *p;
    int slot = -1;
    ProfScope(vl_partition *pp, int c) : p(pp)
    {
        Prof &f = p->prof;
        if (f.on && f.used < f.cap) {
            slot = f.used++;
            f.cls[slot] = c;
            (void)hipEventRecord(f.ev[2 * slot], p->stream);
        }
    }
    ~ProfScope()
    {
        if (slot >= 0) (void)hipEventRecord(p->prof.ev[2 * slot + 1], p->stream);
    }
};

double host_courant(const vl_partition *p, int d, int j, double dt)
{
    if (p->has_cover) return p->cover_host[(size_t)d * p->lay.cover_stride + j];
    const vl_desc &s = p->desc;
    volatile double v = s.vmin[d] + ((double)j + 0.5) * s.dv[d];
    volatile double num = v * dt;
    return num / s.dx[d];
}

int check_cfl(const vl_partition *p, double dt)
{
    for (int d = 0; d < 3; d++)
        for (int j = 0; j < 4 * p->desc.nblk[d]; j++) {
            double c = host_courant(p, d, j, dt);
            if (!(fabs(c) <= 1.0)) return VL_ERR_CFL;
        }
    return VL_OK;
}

int device_status(vl_partition *p)
{
    unsigned long long err = 0;
    VL_HIP(hipMemcpyAsync(&err, &p->D.ctl->err, sizeof(err), hipMemcpyDeviceToHost, p->stream));
    VL_HIP(hipStreamSynchronize(p->stream));
    if (err) {
        p->bad = true;
        return VL_ERR_CAPACITY;
    }
    return VL_OK;
}

void update_box(const vl_partition *p, int mode, int s, int lo[3], int hi[3])
{
    for (int e = 0; e < 3; e++) {
        lo[e] = H;
        hi[e] = H + p->desc.n[e];
    }
    if (mode == VL_COALESCED)  // the later axes' ghost layers within the GT level,
        for (int t = s + 1; t < 3; t++) {  // none beyond a simulation edge
            const int e = p->desc.order[t], ed = p->desc.edges;
            lo[e] = (ed >> (2 * e) & 1) ? H : H - p->desc.gt_level;
            hi[e] = (ed >> (2 * e + 1) & 1) ? H + p->desc.n[e] : H + p->desc.n[e] + p->desc.gt_level;
        }
}

// the ledger stores after one step from `r`
void rotate(LedgerRot &r, const int order[3], bool on)
{
    if (!on) return;
    for (int s = 0; s < 3; s++) std::swap(r.axis[order[s]], r.spare);
    r.phase = (r.phase + 1) & 3;
}

// The kernels of one translation step (growth, work list and shear per axis,
// then pruning into the other local list region), enqueued on st with no
// host read-back, so that the sequence can also be captured into a graph.
// The ledger stores are those of p->rot, which the caller advances (rotate)
// once the step is enqueued or launched.
// ledger3 (device, optional): the change of the FP64 rounding residuals that
// each shear leaves outside f on the local pencils, one sum per shear.
void enqueue_translate(vl_partition *p, double dt, int mode, double *ledger3, hipStream_t st)
{
    const Dev &D = p->D;
    const int nxt = 1 - p->cur;
    const bool ledger = p->lay.lg_cap > 0;
    LedgerRot rot = p->rot;
    p->loadable = false;
    launch_book(D, BOOK_STEP_RESET, st);
    for (int s = 0; s < 3; s++) {
        const int d = p->desc.order[s];
        int lo[3], hi[3];
        update_box(p, mode, s, lo, hi);
        if (mode == VL_PER_SWEEP) {
            int flo[3], fhi[3];
            for (int e = 0; e < 3; e++) {
                flo[e] = H;
                fhi[e] = H + D.n[e];
            }
            flo[d] = 0;
            fhi[d] = D.P[d];
            launch_book(D, BOOK_GHOST_RESET, st);
            ProfScope ps(p, K_FILL);
            if (p->has_src)
                launch_fill_box(D, p->src, flo, fhi, st);
            else
                launch_fill(D, flo, fhi, st);
        }
        launch_book(D, BOOK_SWEEP_RESET, st);
        LedgerIO lg{};
        if (ledger) {
            lg.old = p->lgs[rot.axis[d]];
            lg.nw = p->lgs[rot.spare];
            lg.src = (int32_t *)(p->ws + p->lay.lg_src);
            lg.cap = p->lay.lg_cap;
            std::swap(rot.axis[d], rot.spare);
        }
        {
            ProfScope ps(p, K_PLAN);
            if (ledger) launch_zero_i32(lg.nw.kcnt, p->lay.pen_cap, st);
            launch_plan(D, d, s, lo, hi, dt, p->cur, lg, st);
        }
        {
            ProfScope ps(p, K_SHEAR0 + s);
            launch_sweep(D, d, s, lo, hi, dt, s == 2, lg, st);
        }
        if (ledger3) launch_ledger_sum(D, d, lo, hi, ledger3 + s, st);
    }
    launch_book(D, nxt == 0 ? BOOK_PRUNE_RESET_A : BOOK_PRUNE_RESET_B, st);
    {
        ProfScope ps(p, K_PRUNE);
        launch_prune(D, nxt, p->desc.order[2], st);
    }
}


void enqueue_fill(vl_partition *p, hipStream_t st)
{
    const Dev &D = p->D;
    int lo[3] = {0, 0, 0}, hi[3] = {D.P[0], D.P[1], D.P[2]};
    launch_book(D, BOOK_GHOST_RESET, st);
    ProfScope ps(p, K_FILL);
    if (p->has_src)  // the sources of the last vl_fill_ghosts_from
        launch_fill_from(D, p->src, st);
    else
        launch_fill(D, lo, hi, st);
}

void drop_graphs(vl_partition *p)
{
    GraphCache &g = p->graph;
    for (auto &e : g.exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    g.mode = -1;
    for (int &v : g.variant) v = -1;
}

// Record the step that starts from list region p->cur and ledger rotation
// p->rot into its slot of g.exec.
int capture_step(vl_partition *p, double dt, int mode)
{
    GraphCache &g = p->graph;
    if (!g.cap) VL_HIP(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
    const bool prof = p->prof.on;
    p->prof.on = false;  // no event records inside the graph
    VL_HIP(hipStreamBeginCapture(g.cap, hipStreamCaptureModeRelaxed));
    if (mode == VL_COALESCED) enqueue_fill(p, g.cap);
    enqueue_translate(p, dt, mode, nullptr, g.cap);
    hipGraph_t graph = nullptr;
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(g.cap, &graph);
    p->prof.on = prof;
    if (le != hipSuccess || ee != hipSuccess || !graph) {
        fprintf(stderr, "libvlasov: step capture failed: %s / %s\n", hipGetErrorString(le), hipGetErrorString(ee));
        if (graph) (void)hipGraphDestroy(graph);
        return VL_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        fprintf(stderr, "libvlasov: graph instantiation failed: %s\n", hipGetErrorString(ie));
        return VL_ERR_HIP;
    }
    g.exec[p->cur + 2 * p->rot.phase] = exec;
    return VL_OK;
}

}  // namespace

extern "C" {

size_t vl_workspace_bytes(const vl_desc *d)
{
    if (!desc_ok(d)) return 0;
    return make_layout(d).total;
}

const char *vl_status_string(int s)
{
    switch (s) {
    case VL_OK: return "ok";
    case VL_ERR_ARG: return "invalid argument";
    case VL_ERR_CFL: return "Courant number above 1 (|v dt / dx| > 1)";
    case VL_ERR_CAPACITY: return "capacity exceeded (blocks, lists or work items); re-initialise larger";
    case VL_ERR_STALE_GHOSTS: return "coalesced step without a ghost update since the last step";
    case VL_ERR_HIP: return "HIP runtime error";
    case VL_ERR_STATE: return "partition invalid after an earlier error";
    case VL_ERR_SCRATCH: return "the partition needs more scratch than the fixed device array of vl_moments_static holds";
    case VL_ERR_SPLIT: return "a cell's velocity map cannot be split into three one-coordinate remaps (rotation too large for the step)";
    default: return "unknown status";
    }
}

int vl_init_partition(const vl_desc *d, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                      const int64_t *cell_offsets, const int32_t *block_ids, const double *f,
                      vl_partition **out)
{
    if (!out) return VL_ERR_ARG;
    *out = nullptr;
    if (!desc_ok(d) || !dev_workspace || !cell_offsets) return VL_ERR_ARG;
    if (((uintptr_t)dev_workspace) % ALIGN) return VL_ERR_ARG;
    Layout L = make_layout(d);
    if (ws_bytes < L.total) return VL_ERR_ARG;
    const int64_t NB = (int64_t)d->nblk[0] * d->nblk[1] * d->nblk[2];
    if (cell_offsets[0] != 0) return VL_ERR_ARG;
    for (int64_t q = 0; q < L.nlocal; q++)
        if (cell_offsets[q + 1] < cell_offsets[q]) return VL_ERR_ARG;
    const int64_t total = cell_offsets[L.nlocal];
    if (total > 0 && !block_ids) return VL_ERR_ARG;
    for (int64_t q = 0; q < L.nlocal; q++)
        for (int64_t k = cell_offsets[q]; k < cell_offsets[q + 1]; k++) {
            if (block_ids[k] < 0 || block_ids[k] >= NB) return VL_ERR_ARG;
            if (k > cell_offsets[q] && block_ids[k] <= block_ids[k - 1]) return VL_ERR_ARG;
        }
    if (total > d->block_capacity) return VL_ERR_CAPACITY;

    vl_partition *p = new vl_partition();
    p->desc = *d;
    p->lay = L;
    p->stream = (hipStream_t)hip_stream;
    p->ws = (char *)dev_workspace;
    p->cur = 0;
    p->init_blocks = total;
    p->loadable = true;
    p->has_src = false;
    p->ghosts_valid = false;
    p->bad = false;
    p->has_cover = false;

    Dev &D = p->D;
    memset(&D, 0, sizeof(D));
    for (int k = 0; k < 3; k++) {
        D.n[k] = d->n[k];
        D.P[k] = d->n[k] + 2 * H;
        D.nblk[k] = d->nblk[k];
        D.vmin[k] = d->vmin[k];
        D.dv[k] = d->dv[k];
        D.dx[k] = d->dx[k];
    }
    D.NB = (int)NB;
    D.W = (int)((NB + 31) / 32);
    D.storage = d->storage;
    D.vbuffer = d->vbuffer;
    D.N = L.N;
    D.nlocal = L.nlocal;
    D.s[0] = 1;
    D.s[1] = D.P[0];
    D.s[2] = (int64_t)D.P[0] * D.P[1];
    D.sparse_min = d->sparse_min;
    char *w = p->ws;
    D.pool = w + L.pool;
    D.lcap = d->block_capacity;
    D.gcap = d->ghost_block_capacity;
    D.trash = D.lcap + D.gcap;
    D.ring = (int32_t *)(w + L.ring);
    D.lstart = (int64_t *)(w + L.lstart);
    D.lcount = (int32_t *)(w + L.lcount);
    D.lcapa = (int32_t *)(w + L.lcapa);
    D.lsorted = (int32_t *)(w + L.lsorted);
    D.lid = (int32_t *)(w + L.lid);
    D.lslot = (int32_t *)(w + L.lslot);
    D.litem = (int32_t *)(w + L.litem);
    D.reg_off[0] = 0;
    D.reg_cap[0] = L.LA;
    D.reg_off[1] = L.LA;
    D.reg_cap[1] = L.LA;
    D.reg_off[2] = 2 * L.LA;
    D.reg_cap[2] = L.LG;
    D.rows = (int32_t *)(w + L.rows);
    D.row_cap = L.row_cap;
    D.items = (Item *)(w + L.items);
    D.masks = (uint32_t *)(w + L.masks);
    D.item_cap = L.item_cap;
    D.resid = (double *)(w + L.resid);
    D.pen_first = (int64_t *)(w + L.penfirst);
    D.pen_cnt = (int32_t *)(w + L.pencnt);
    D.pen_sum = (double *)(w + L.pensum);
    D.pen_cap = L.pen_cap;
    D.wlmax = L.wlmax;
    D.ctl = (Ctl *)(w + L.ctl);
    D.cover = nullptr;
    D.cover_stride = L.cover_stride;
    D.cell_red = (double *)(w + L.cellred);
    D.red = (double *)(w + L.red);
    D.cell_cnt = (int32_t *)(w + L.cellcnt);
    for (int k = 0; k < 4; k++) {
        LedgerStore &g = p->lgs[k];
        const bool on = L.lg_cap > 0;
        g.ids = on ? (int32_t *)(w + L.lg_ids[k]) : nullptr;
        g.res = on ? (double *)(w + L.lg_res[k]) : nullptr;
        g.kfirst = on ? (int32_t *)(w + L.lg_kfirst[k]) : nullptr;
        g.kcnt = on ? (int32_t *)(w + L.lg_kcnt[k]) : nullptr;
    }
    p->mom = carve_moments_scratch(w + L.mom, L.nlocal, L.mom_parts, L.mom_parts, MOM_CHUNK);
    // the fixed scratch array of vl_moments_static on this device (its
    // address, taken once per device)
    p->mom_static = nullptr;
    if (static_moments_scratch(&p->mom_static) != 0) p->mom_static = nullptr;  // vl_moments_static reports it

    // host-side construction of cell metadata and local lists (region 0)
    std::vector<int64_t> lstart(L.N, D.reg_off[2]);
    std::vector<int32_t> lcount(L.N, 0), lcapa(L.N, 0);
    std::vector<int32_t> lid, lslot;
    lid.reserve(total + total / 4 + 32 * L.nlocal);
    lslot.reserve(lid.capacity());
    int64_t run = 0;
    for (int64_t q = 0; q < L.nlocal; q++) {
        const int x = (int)(q % d->n[0]), y = (int)((q / d->n[0]) % d->n[1]),
                  z = (int)(q / ((int64_t)d->n[0] * d->n[1]));
        const int64_t c = cell_index(D, x + H, y + H, z + H);
        const int64_t b0 = cell_offsets[q], b1 = cell_offsets[q + 1];
        const int cnt = (int)(b1 - b0);
        const int cap = cnt + cnt / 4 + 32;
        lstart[c] = run;
        lcount[c] = cnt;
        lcapa[c] = cap;
        for (int64_t k = b0; k < b1; k++) {
            lid.push_back(block_ids[k]);
            lslot.push_back((int32_t)k);
        }
        for (int k = cnt; k < cap; k++) {
            lid.push_back(0);
            lslot.push_back(0);
        }
        run += cap;
    }
    int rc = VL_OK;
    do {
        Ctl ctl;
        memset(&ctl, 0, sizeof(ctl));
        ctl.ring_head = 0;
        ctl.ring_tail = (unsigned long long)(D.lcap - total);
        ctl.ring_limit = ctl.ring_tail;
        ctl.list_top[0] = (unsigned long long)run;
        if (hipMemcpy(D.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (hipMemcpy(D.lstart, lstart.data(), L.N * 8, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (hipMemcpy(D.lcount, lcount.data(), L.N * 4, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (hipMemcpy(D.lsorted, lcount.data(), L.N * 4, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (hipMemcpy(D.lcapa, lcapa.data(), L.N * 4, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (!lid.empty()) {
            if (hipMemcpy(D.lid, lid.data(), lid.size() * 4, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
            if (hipMemcpy(D.lslot, lslot.data(), lslot.size() * 4, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        }
        // empty ledger stores: no line has a residual yet
        if (L.lg_cap > 0) {
            bool ok = true;
            for (int k = 0; k < 4 && ok; k++) ok = hipMemset(p->lgs[k].kcnt, 0, (size_t)L.pen_cap * 4) == hipSuccess;
            if (!ok) { rc = VL_ERR_HIP; break; }
        }
        // the scratch block reads as zero in the shears
        if (hipMemset((char *)D.pool + (size_t)D.trash * BLK * storage_bytes(d->storage), 0,
                      (size_t)BLK * storage_bytes(d->storage)) != hipSuccess) { rc = VL_ERR_HIP; break; }
        // payload, converted to the storage type in chunks
        const int bs = storage_bytes(d->storage);
        const int64_t nval = total * BLK;
        if (!f) {  // values follow through vl_load_values
            if (nval > 0 && hipMemset(D.pool, 0, (size_t)nval * bs) != hipSuccess) { rc = VL_ERR_HIP; break; }
        } else if (d->storage == VL_F64) {
            if (nval > 0 && hipMemcpy(D.pool, f, (size_t)nval * 8, hipMemcpyHostToDevice) != hipSuccess) { rc = VL_ERR_HIP; break; }
        } else {
            const int64_t chunk = 1 << 24;
            std::vector<unsigned char> buf((size_t)std::min<int64_t>(chunk, std::max<int64_t>(nval, 1)) * bs);
            for (int64_t o = 0; o < nval && rc == VL_OK; o += chunk) {
                const int64_t m = std::min(chunk, nval - o);
                if (d->storage == VL_F32) {
                    float *bf = (float *)buf.data();
                    for (int64_t i = 0; i < m; i++) bf[i] = (float)f[o + i];
                } else {
                    uint16_t *bh = (uint16_t *)buf.data();
                    for (int64_t i = 0; i < m; i++) {
                        // FP64 -> FP32 rounded to odd -> BF16 nearest even
                        const double v = f[o + i];
                        float t = (float)v;
                        if ((double)t != v) {
                            // round toward zero, then set the sticky bit
                            if (fabs((double)t) > fabs(v)) t = nextafterf(t, 0.0f);
                            uint32_t u;
                            memcpy(&u, &t, 4);
                            u |= 1u;
                            memcpy(&t, &u, 4);
                        }
                        bh[i] = f32_to_bf16_rne(t);
                    }
                }
                if (hipMemcpy((char *)D.pool + (size_t)o * bs, buf.data(), (size_t)m * bs, hipMemcpyHostToDevice) !=
                    hipSuccess)
                    rc = VL_ERR_HIP;
            }
            if (rc) break;
        }
        launch_iota_ring(D, total, D.lcap - total, p->stream);
        if (hipGetLastError() != hipSuccess) { rc = VL_ERR_HIP; break; }
        if (hipStreamSynchronize(p->stream) != hipSuccess) { rc = VL_ERR_HIP; break; }
    } while (0);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return VL_OK;
}

int vl_load_values(vl_partition *p, int64_t first_block, int64_t nblocks, const double *dev_f)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad || !p->loadable) return VL_ERR_STATE;
    if (first_block < 0 || nblocks < 0 || first_block > p->init_blocks - nblocks) return VL_ERR_ARG;
    if (nblocks == 0) return VL_OK;
    if (!dev_f) return VL_ERR_ARG;
    launch_load(p->D, first_block, nblocks, dev_f, p->stream);
    VL_HIP(hipGetLastError());
    p->ghosts_valid = false;
    return VL_OK;
}

int vl_fill_ghosts(vl_partition *p)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    if (p->desc.edges) return VL_ERR_ARG;  // boundary cells need their sources
    if (p->has_src) drop_graphs(p);
    p->has_src = false;
    enqueue_fill(p, p->stream);
    VL_HIP(hipGetLastError());
    p->ghosts_valid = true;
    return VL_OK;
}

int vl_fill_ghosts_from(vl_partition *p, vl_partition *const *nbr)
{
    if (!p || !nbr || nbr[13] != p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const vl_desc &a = p->desc;
    SrcTable src;
    memset(&src, 0, sizeof(src));
    src.remote = 1;
    for (int q = 0; q < 27; q++) {
        const vl_partition *o = nbr[q];
        if (!o) return VL_ERR_ARG;
        if (o->bad) return VL_ERR_STATE;
        const vl_desc &b = o->desc;
        for (int d = 0; d < 3; d++)
            if (b.n[d] != a.n[d] || a.n[d] < H || b.nblk[d] != a.nblk[d] || b.vmin[d] != a.vmin[d] ||
                b.dv[d] != a.dv[d])
                return VL_ERR_ARG;
        if (b.storage != a.storage) return VL_ERR_ARG;
        src.part[q] = self_source(o->D);
    }
    launch_book(p->D, BOOK_GHOST_RESET, p->stream);
    {
        ProfScope ps(p, K_FILL);
        launch_fill_from(p->D, src, p->stream);
    }
    VL_HIP(hipGetLastError());
    p->src = src;
    p->has_src = true;
    drop_graphs(p);
    p->ghosts_valid = true;
    return VL_OK;
}

int vl_translate_step(vl_partition *p, double dt, int32_t mode, vl_step_stats *stats)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    if (mode != VL_COALESCED && mode != VL_PER_SWEEP) return VL_ERR_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return VL_ERR_ARG;
    if (check_cfl(p, dt)) return VL_ERR_CFL;
    if (mode == VL_COALESCED && !p->ghosts_valid) return VL_ERR_STALE_GHOSTS;
    if (mode == VL_PER_SWEEP && p->desc.edges && !p->has_src) return VL_ERR_STALE_GHOSTS;
    const Dev &D = p->D;
    hipStream_t st = p->stream;
    if (stats) {
        launch_cell_mass(D, st);
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 0, st);
    }
    enqueue_translate(p, dt, mode, stats ? D.red + 8 : nullptr, st);
    const int nxt = 1 - p->cur;
    VL_HIP(hipGetLastError());
    p->cur = nxt;
    rotate(p->rot, p->desc.order, p->lay.lg_cap > 0);
    p->ghosts_valid = false;
    if (stats) {
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 2, st);  // pruned mass
        launch_cell_mass(D, st);
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 1, st);
        launch_cell_counts(D, st);
        VL_HIP(hipGetLastError());
        double red[11];
        Ctl ctl;
        std::vector<int32_t> cc((size_t)D.nlocal);
        VL_HIP(hipMemcpyAsync(red, D.red, sizeof(red), hipMemcpyDeviceToHost, st));
        VL_HIP(hipMemcpyAsync(&ctl, D.ctl, sizeof(ctl), hipMemcpyDeviceToHost, st));
        VL_HIP(hipMemcpyAsync(cc.data(), D.cell_cnt, cc.size() * 4, hipMemcpyDeviceToHost, st));
        VL_HIP(hipStreamSynchronize(st));
        const double vol = D.dx[0] * D.dx[1] * D.dx[2] * D.dv[0] * D.dv[1] * D.dv[2];
        memset(stats, 0, sizeof(*stats));
        stats->mass_before = red[0] * vol;
        stats->mass_after = red[1] * vol;
        stats->pruned_mass = red[2];
        stats->ledger_mass = ((red[8] + red[9]) + red[10]) * vol;
        int64_t nb = 0;
        for (int32_t v : cc) nb += v;
        stats->local_blocks = nb;
        for (int s = 0; s < 3; s++) {
            stats->updated_ps[s] = (int64_t)ctl.upd_ps[s];
            stats->read_ps[s] = (int64_t)ctl.read_ps[s];
            stats->items[s] = (int64_t)ctl.items[s];
        }
        stats->device_errors = (uint64_t)ctl.err;
        if (ctl.err) {
            p->bad = true;
            return VL_ERR_CAPACITY;
        }
    }
    return VL_OK;
}

int vl_graph_step(vl_partition *p, double dt, int32_t mode, int32_t nsteps)
{
    if (!p || nsteps < 0) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    if (mode != VL_COALESCED && mode != VL_PER_SWEEP) return VL_ERR_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return VL_ERR_ARG;
    if (check_cfl(p, dt)) return VL_ERR_CFL;
    if (p->desc.edges && !p->has_src) return VL_ERR_STALE_GHOSTS;
    GraphCache &g = p->graph;
    const int *sv = p->D.sweep_variant;
    if (g.dt != dt || g.mode != mode || g.variant[0] != sv[0] || g.variant[1] != sv[1] || g.variant[2] != sv[2]) {
        drop_graphs(p);
        g.dt = dt;
        g.mode = mode;
        for (int s = 0; s < 3; s++) g.variant[s] = sv[s];
    }
    for (int k = 0; k < nsteps; k++) {
        const int gi = p->cur + 2 * p->rot.phase;
        if (!g.exec[gi]) {
            int rc = capture_step(p, dt, mode);
            if (rc) {
                drop_graphs(p);
                return rc;
            }
        }
        VL_HIP(hipGraphLaunch(g.exec[gi], p->stream));
        p->cur = 1 - p->cur;
        rotate(p->rot, p->desc.order, p->lay.lg_cap > 0);
        p->ghosts_valid = false;
    }
    return VL_OK;
}

int vl_accelerate(vl_partition *p, double dt, double qm, const double *dev_fields, const int32_t *slice_order,
                  vl_step_stats *stats)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    if (!(dt > 0.0) || !isfinite(dt) || !isfinite(qm) || !dev_fields) return VL_ERR_ARG;
    int order[3] = {0, 1, 2};
    if (slice_order) {
        int seen = 0;
        for (int k = 0; k < 3; k++) {
            if (slice_order[k] < 0 || slice_order[k] > 2) return VL_ERR_ARG;
            order[k] = slice_order[k];
            seen |= 1 << order[k];
        }
        if (seen != 7) return VL_ERR_ARG;
    }
    const Dev &D = p->D;
    hipStream_t st = p->stream;
    {
        int ncols = 0, hc = 0, dev = 0, maxlds = 0;
        const size_t lds = accel_lds_bytes(D, &ncols, &hc);
        VL_HIP(hipGetDevice(&dev));
        VL_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (lds == 0 || lds + 2048 > (size_t)maxlds) return VL_ERR_ARG;  // + the kernel's static LDS
    }
    double *maps = (double *)(p->ws + p->lay.accel);
    int *bad = (int *)(D.red + 64);
    // the maps first: a cell whose map cannot be split leaves f untouched
    launch_zero_i32(bad, 1, st);
    launch_accel_maps(D, dev_fields, maps, bad, qm, dt, order, st);
    VL_HIP(hipGetLastError());
    int hbad = 0;
    VL_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    VL_HIP(hipStreamSynchronize(st));
    if (hbad) return VL_ERR_SPLIT;
    if (stats) {
        launch_cell_mass(D, st);
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 0, st);
    }
    const int nxt = 1 - p->cur;
    p->loadable = false;
    launch_book(D, BOOK_STEP_RESET, st);
    launch_book(D, BOOK_SWEEP_RESET, st);  // ring limit <- tail
    {
        ProfScope ps(p, K_ACCEL);
        if (launch_accel(D, maps, order, p->cur, st)) return VL_ERR_ARG;
    }
    launch_book(D, nxt == 0 ? BOOK_PRUNE_RESET_A : BOOK_PRUNE_RESET_B, st);
    {
        ProfScope ps(p, K_PRUNE);
        launch_prune(D, nxt, -1, st);
    }
    VL_HIP(hipGetLastError());
    p->cur = nxt;
    p->ghosts_valid = false;
    if (stats) {
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 2, st);  // pruned mass
        launch_cell_mass(D, st);
        launch_reduce(D, D.cell_red, D.nlocal, D.red + 1, st);
        launch_cell_counts(D, st);
        VL_HIP(hipGetLastError());
        double red[3];
        Ctl ctl;
        std::vector<int32_t> cc((size_t)D.nlocal);
        VL_HIP(hipMemcpyAsync(red, D.red, sizeof(red), hipMemcpyDeviceToHost, st));
        VL_HIP(hipMemcpyAsync(&ctl, D.ctl, sizeof(ctl), hipMemcpyDeviceToHost, st));
        VL_HIP(hipMemcpyAsync(cc.data(), D.cell_cnt, cc.size() * 4, hipMemcpyDeviceToHost, st));
        VL_HIP(hipStreamSynchronize(st));
        const double vol = D.dx[0] * D.dx[1] * D.dx[2] * D.dv[0] * D.dv[1] * D.dv[2];
        memset(stats, 0, sizeof(*stats));
        stats->mass_before = red[0] * vol;
        stats->mass_after = red[1] * vol;
        stats->pruned_mass = red[2];
        int64_t nb = 0;
        for (int32_t v : cc) nb += v;
        stats->local_blocks = nb;
        stats->device_errors = (uint64_t)ctl.err;
        if (ctl.err) {
            p->bad = true;
            return VL_ERR_CAPACITY;
        }
    }
    return VL_OK;
}

int vl_moments(vl_partition *p, double *dev_n, double *dev_V3, double *dev_P6, double *host_total_mass)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const Dev &D = p->D;
    {
        ProfScope ps(p, K_OTHER);
        launch_moments(D, p->mom, dev_n, dev_V3, dev_P6, p->stream);
    }
    VL_HIP(hipGetLastError());
    if (host_total_mass) {
        launch_reduce(D, p->mom.cell_mass, D.nlocal, D.red + 5, p->stream);
        VL_HIP(hipMemcpyAsync(host_total_mass, D.red + 5, sizeof(double), hipMemcpyDeviceToHost, p->stream));
        return device_status(p);
    }
    return VL_OK;
}

int vl_moments_static(vl_partition *p, double *dev_n, double *dev_V3, double *dev_P6, double *dev_total_mass)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const Dev &D = p->D;
    const Layout &L = p->lay;
    if (!p->mom_static) return VL_ERR_HIP;
    // the chunk size that keeps every possible split within the array: the
    // workspace's when it fits, else larger
    const int64_t fixed = moments_scratch_bytes(L.nlocal, 0, 0);
    const int64_t per_part = 80 + 8;
    if (fixed + 64 * per_part + 1024 > STATIC_MOMENTS_SCRATCH_BYTES) return VL_ERR_SCRATCH;
    const int64_t parts = (STATIC_MOMENTS_SCRATCH_BYTES - fixed - 1024) / per_part;
    int64_t chunk = MOM_CHUNK;
    if (2 * D.lcap / chunk + 64 > parts) chunk = (2 * D.lcap + parts - 65) / (parts - 64);
    if (chunk > (int64_t)1 << 30) return VL_ERR_SCRATCH;
    const MomScratch M = carve_moments_scratch(p->mom_static, L.nlocal, parts, parts, (int)chunk);
    {
        ProfScope ps(p, K_OTHER);
        launch_moments(D, M, dev_n, dev_V3, dev_P6, p->stream);
        if (dev_total_mass) launch_reduce(D, M.cell_mass, D.nlocal, dev_total_mass, p->stream);
    }
    VL_HIP(hipGetLastError());
    return VL_OK;
}

int vl_counters(vl_partition *p, uint64_t *out, int32_t n)
{
    if (!p || !out || n < 0 || n > 32) return VL_ERR_ARG;
    Ctl ctl;
    VL_HIP(hipMemcpyAsync(&ctl, p->D.ctl, sizeof(ctl), hipMemcpyDeviceToHost, p->stream));
    VL_HIP(hipStreamSynchronize(p->stream));
    uint64_t v[32] = {ctl.ring_head, ctl.ring_tail, ctl.ring_limit, ctl.ghost_top, ctl.ghost_list_top,
                      ctl.list_top[0], ctl.list_top[1], ctl.n_items, ctl.row_top, ctl.work, ctl.err,
                      ctl.upd_ps[0], ctl.upd_ps[1], ctl.upd_ps[2], ctl.read_ps[0], ctl.read_ps[1],
                      ctl.read_ps[2], ctl.items[0], ctl.items[1], ctl.items[2], (uint64_t)p->cur,
                      ctl.cum_upd, ctl.cum_read};
    for (int i = 0; i < n; i++) out[i] = v[i];
    return VL_OK;
}

int vl_profile_start(vl_partition *p, int32_t max_launches)
{
    if (!p || max_launches < 1 || max_launches > (1 << 20)) return VL_ERR_ARG;
    Prof &f = p->prof;
    for (hipEvent_t e : f.ev) (void)hipEventDestroy(e);
    f.ev.assign(2 * (size_t)max_launches, nullptr);
    f.cls.assign(max_launches, 0);
    for (auto &e : f.ev) VL_HIP(hipEventCreate(&e));
    f.cap = max_launches;
    f.used = 0;
    f.on = true;
    return VL_OK;
}

int vl_profile_stop(vl_partition *p, double *ms, int64_t *launches)
{
    if (!p || !ms || !launches) return VL_ERR_ARG;
    Prof &f = p->prof;
    for (int c = 0; c < K_NCLS; c++) {
        ms[c] = 0.0;
        launches[c] = 0;
    }
    VL_HIP(hipStreamSynchronize(p->stream));
    for (int i = 0; i < f.used; i++) {
        float t = 0.0f;
        VL_HIP(hipEventElapsedTime(&t, f.ev[2 * i], f.ev[2 * i + 1]));
        ms[f.cls[i]] += t;
        launches[f.cls[i]] += 1;
        if (f.cls[i] >= K_SHEAR0) {  // all shears together as well
            ms[K_SWEEP] += t;
            launches[K_SWEEP] += 1;
        }
    }
    for (hipEvent_t e : f.ev) (void)hipEventDestroy(e);
    f.ev.clear();
    f.cls.clear();
    f.on = false;
    f.cap = f.used = 0;
    return VL_OK;
}

int vl_set_variant(vl_partition *p, int32_t variant)
{
    if (!p || variant < 0 || variant >= sweep_variants()) return VL_ERR_ARG;
    for (int s = 0; s < 3; s++) p->D.sweep_variant[s] = variant;
    drop_graphs(p);
    return VL_OK;
}

int vl_set_shear_variants(vl_partition *p, const int32_t variants[3])
{
    if (!p || !variants) return VL_ERR_ARG;
    for (int s = 0; s < 3; s++)
        if (variants[s] < 0 || variants[s] >= sweep_variants()) return VL_ERR_ARG;
    for (int s = 0; s < 3; s++) p->D.sweep_variant[s] = variants[s];
    drop_graphs(p);
    return VL_OK;
}

int vl_get_shear_variants(const vl_partition *p, int32_t variants[3], int32_t *count)
{
    if (!p || !variants) return VL_ERR_ARG;
    for (int s = 0; s < 3; s++) variants[s] = p->D.sweep_variant[s];
    if (count) *count = sweep_variants();
    return VL_OK;
}

int vl_autotune(vl_partition *p, double dt, int32_t mode, int32_t steps_per_variant, int32_t best[3],
                double *ms_out, int32_t ms_cap)
{
    if (!p || steps_per_variant < 1 || !best) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    if (mode != VL_COALESCED && mode != VL_PER_SWEEP) return VL_ERR_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return VL_ERR_ARG;
    if (check_cfl(p, dt)) return VL_ERR_CFL;
    if (p->desc.edges && !p->has_src) return VL_ERR_STALE_GHOSTS;  // boundary cells need their sources
    const int nv = sweep_variants();
    const int budget = steps_per_variant * nv;      // real steps in all
    std::vector<double> t((size_t)nv * 4, 0.0);     // per variant: summed ms of shears 1..3, all
    // per variant and shear: summed ms per 1e9 phase-space cells the shear
    // read and updated, so steps taken as the lists grow compare alike
    std::vector<double> r((size_t)nv * 3, 0.0);
    std::vector<int> k((size_t)nv, 0);              // steps run with each variant
    auto run = [&](int v) -> int {
        for (int s = 0; s < 3; s++) p->D.sweep_variant[s] = v;
        int rc = vl_profile_start(p, 64);
        if (rc) return rc;
        if (mode == VL_COALESCED) {
            // the ghost update a real step would take: from the sources of the
            // last vl_fill_ghosts_from if there was one, else periodic images
            enqueue_fill(p, p->stream);
            VL_HIP(hipGetLastError());
            p->ghosts_valid = true;
        }
        if ((rc = vl_translate_step(p, dt, mode, nullptr))) return rc;
        double ms[K_NCLS];
        int64_t n[K_NCLS];
        if ((rc = vl_profile_stop(p, ms, n))) return rc;
        Ctl ctl;
        VL_HIP(hipMemcpyAsync(&ctl, p->D.ctl, sizeof(ctl), hipMemcpyDeviceToHost, p->stream));
        VL_HIP(hipStreamSynchronize(p->stream));
        for (int s = 0; s < 3; s++) {
            t[(size_t)v * 4 + s] += ms[K_SHEAR0 + s];
            const double cells = (double)(ctl.upd_ps[s] + ctl.read_ps[s]);
            r[(size_t)v * 3 + s] += ms[K_SHEAR0 + s] * 1e9 / std::max(cells, 1.0);
        }
        t[(size_t)v * 4 + 3] += ms[K_SWEEP];
        k[v]++;
        return VL_OK;
    };
    auto mean = [&](int v, int s) { return r[(size_t)v * 3 + s] / k[v]; };
    // One step with every variant, then rounds over the variants within 25 %
    // of the best mean on some shear until the steps are spent; each shear's
    // time is taken per cell it read and updated, so the growth of the lists
    // from step to step does not favour the variants tried first.
    int done = 0, rc;
    for (int v = 0; v < nv; v++, done++)
        if ((rc = run(v))) return rc;
    while (done < budget) {
        double bm[3];
        for (int s = 0; s < 3; s++) {
            bm[s] = mean(0, s);
            for (int v = 1; v < nv; v++) bm[s] = std::min(bm[s], mean(v, s));
        }
        for (int v = 0; v < nv && done < budget; v++) {
            bool live = false;
            for (int s = 0; s < 3; s++) live = live || mean(v, s) <= 1.25 * bm[s];
            if (!live) continue;
            if ((rc = run(v))) return rc;
            done++;
        }
    }
    for (int s = 0; s < 3; s++) {
        int bv = 0;
        for (int v = 1; v < nv; v++)
            if (mean(v, s) < mean(bv, s)) bv = v;
        p->D.sweep_variant[s] = bv;
        best[s] = bv;
    }
    if (ms_out)
        for (int v = 0; v < nv && v < ms_cap; v++) ms_out[v] = t[(size_t)v * 4 + 3] / k[v];
    return device_status(p);
}

int vl_sync(vl_partition *p)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    return device_status(p);
}

int vl_local_block_count(vl_partition *p, int64_t *out)
{
    if (!p || !out) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const Dev &D = p->D;
    launch_cell_counts(D, p->stream);
    std::vector<int32_t> cc((size_t)D.nlocal);
    VL_HIP(hipMemcpyAsync(cc.data(), D.cell_cnt, cc.size() * 4, hipMemcpyDeviceToHost, p->stream));
    int rc = device_status(p);
    if (rc) return rc;
    int64_t nb = 0;
    for (int32_t v : cc) nb += v;
    *out = nb;
    return VL_OK;
}

int vl_export_cells(vl_partition *p, const int64_t *cells, int64_t ncells, int64_t *cell_offsets,
                    int32_t *block_ids, double *f, int64_t cap_blocks)
{
    if (!p || !cells || ncells < 0 || !cell_offsets) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const Dev &D = p->D;
    for (int64_t i = 0; i < ncells; i++)
        if (cells[i] < 0 || cells[i] >= D.nlocal) return VL_ERR_ARG;
    int rc = device_status(p);
    if (rc) return rc;
    // cell metadata and the current local list region
    std::vector<int64_t> ls(ncells);
    std::vector<int32_t> lc(ncells);
    for (int64_t i = 0; i < ncells; i++) {
        const int64_t q = cells[i];
        const int x = (int)(q % D.n[0]), y = (int)((q / D.n[0]) % D.n[1]), z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
        const int64_t c = cell_index(D, x + H, y + H, z + H);
        VL_HIP(hipMemcpy(&ls[i], D.lstart + c, 8, hipMemcpyDeviceToHost));
        VL_HIP(hipMemcpy(&lc[i], D.lcount + c, 4, hipMemcpyDeviceToHost));
    }
    int64_t total = 0;
    cell_offsets[0] = 0;
    for (int64_t i = 0; i < ncells; i++) {
        total += lc[i];
        cell_offsets[i + 1] = total;
    }
    if (total > cap_blocks) return VL_ERR_ARG;
    if (total > 0 && !block_ids) return VL_ERR_ARG;
    std::vector<int32_t> slots((size_t)total);
    std::vector<std::pair<int32_t, int32_t>> ent;
    for (int64_t i = 0; i < ncells; i++) {
        ent.resize(lc[i]);
        std::vector<int32_t> a(lc[i]), b(lc[i]);
        if (lc[i] > 0) {
            VL_HIP(hipMemcpy(a.data(), D.lid + ls[i], (size_t)lc[i] * 4, hipMemcpyDeviceToHost));
            VL_HIP(hipMemcpy(b.data(), D.lslot + ls[i], (size_t)lc[i] * 4, hipMemcpyDeviceToHost));
        }
        for (int k = 0; k < lc[i]; k++) ent[k] = {a[k], b[k]};
        std::sort(ent.begin(), ent.end());
        for (int k = 0; k < lc[i]; k++) {
            block_ids[cell_offsets[i] + k] = ent[k].first;
            slots[cell_offsets[i] + k] = ent[k].second;
        }
    }
    // gather payloads through dead work-list buffers: slot list in the item
    // area, FP64 values in the row area
    const int64_t chunk = std::min<int64_t>((int64_t)(p->lay.row_cap * 4) / (BLK * 8),
                                            (int64_t)(p->lay.item_cap * sizeof(Item)) / 4);
    if (chunk < 1) return VL_ERR_STATE;
    int32_t *dslots = (int32_t *)D.items;
    double *dvals = (double *)D.rows;
    for (int64_t o = 0; o < total; o += chunk) {
        const int64_t m = std::min(chunk, total - o);
        VL_HIP(hipMemcpyAsync(dslots, slots.data() + o, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
        launch_gather(D, dslots, m, dvals, p->stream);
        VL_HIP(hipGetLastError());
        VL_HIP(hipMemcpyAsync(f + o * BLK, dvals, (size_t)m * BLK * 8, hipMemcpyDeviceToHost, p->stream));
        VL_HIP(hipStreamSynchronize(p->stream));
    }
    return VL_OK;
}

int vl_export_state(vl_partition *p, int64_t *cell_offsets, int32_t *block_ids, double *f, int64_t cap_blocks)
{
    if (!p || !cell_offsets) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    const Dev &D = p->D;
    int rc = device_status(p);
    if (rc) return rc;
    // bulk metadata copy, then per-cell assembly on the host
    std::vector<int64_t> lstart((size_t)D.N);
    std::vector<int32_t> lcount((size_t)D.N);
    VL_HIP(hipMemcpy(lstart.data(), D.lstart, (size_t)D.N * 8, hipMemcpyDeviceToHost));
    VL_HIP(hipMemcpy(lcount.data(), D.lcount, (size_t)D.N * 4, hipMemcpyDeviceToHost));
    const int64_t roff = D.reg_off[p->cur], rcap = D.reg_cap[p->cur];
    std::vector<int32_t> lid((size_t)rcap), lslot((size_t)rcap);
    VL_HIP(hipMemcpy(lid.data(), D.lid + roff, (size_t)rcap * 4, hipMemcpyDeviceToHost));
    VL_HIP(hipMemcpy(lslot.data(), D.lslot + roff, (size_t)rcap * 4, hipMemcpyDeviceToHost));
    int64_t total = 0;
    cell_offsets[0] = 0;
    for (int64_t q = 0; q < D.nlocal; q++) {
        const int x = (int)(q % D.n[0]), y = (int)((q / D.n[0]) % D.n[1]), z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
        total += lcount[cell_index(D, x + H, y + H, z + H)];
        cell_offsets[q + 1] = total;
    }
    if (total > cap_blocks) return VL_ERR_ARG;
    if (total > 0 && !block_ids) return VL_ERR_ARG;
    std::vector<int32_t> slots((size_t)total);
    std::vector<std::pair<int32_t, int32_t>> ent;
    for (int64_t q = 0; q < D.nlocal; q++) {
        const int x = (int)(q % D.n[0]), y = (int)((q / D.n[0]) % D.n[1]), z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
        const int64_t c = cell_index(D, x + H, y + H, z + H);
        const int64_t s0 = lstart[c] - roff;
        const int cnt = lcount[c];
        if (cnt > 0 && (s0 < 0 || s0 + cnt > rcap)) return VL_ERR_STATE;
        ent.resize(cnt);
        for (int k = 0; k < cnt; k++) ent[k] = {lid[s0 + k], lslot[s0 + k]};
        std::sort(ent.begin(), ent.end());
        for (int k = 0; k < cnt; k++) {
            block_ids[cell_offsets[q] + k] = ent[k].first;
            slots[cell_offsets[q] + k] = ent[k].second;
        }
    }
    const int64_t chunk = std::min<int64_t>((int64_t)(p->lay.row_cap * 4) / (BLK * 8),
                                            (int64_t)(p->lay.item_cap * sizeof(Item)) / 4);
    if (chunk < 1) return VL_ERR_STATE;
    int32_t *dslots = (int32_t *)D.items;
    double *dvals = (double *)D.rows;
    for (int64_t o = 0; o < total; o += chunk) {
        const int64_t m = std::min(chunk, total - o);
        VL_HIP(hipMemcpyAsync(dslots, slots.data() + o, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
        launch_gather(D, dslots, m, dvals, p->stream);
        VL_HIP(hipGetLastError());
        VL_HIP(hipMemcpyAsync(f + o * BLK, dvals, (size_t)m * BLK * 8, hipMemcpyDeviceToHost, p->stream));
        VL_HIP(hipStreamSynchronize(p->stream));
    }
    return VL_OK;
}

int vl_set_courant_override(vl_partition *p, const double *table, int32_t stride)
{
    if (!p) return VL_ERR_ARG;
    if (p->bad) return VL_ERR_STATE;
    drop_graphs(p);
    if (!table) {
        p->has_cover = false;
        p->D.cover = nullptr;
        return VL_OK;
    }
    const int cs = p->lay.cover_stride;
    for (int d = 0; d < 3; d++)
        if (stride < 4 * p->desc.nblk[d]) return VL_ERR_ARG;
    std::vector<double> t((size_t)3 * cs, 0.0);
    for (int d = 0; d < 3; d++)
        for (int j = 0; j < 4 * p->desc.nblk[d]; j++) {
            double v = table[(size_t)d * stride + j];
            if (!(fabs(v) <= 1.0)) return VL_ERR_CFL;
            t[(size_t)d * cs + j] = v;
        }
    double *dst = (double *)(p->ws + p->lay.cover);
    VL_HIP(hipStreamSynchronize(p->stream));
    VL_HIP(hipMemcpy(dst, t.data(), t.size() * 8, hipMemcpyHostToDevice));
    p->cover_host = t;
    p->has_cover = true;
    p->D.cover = dst;
    return VL_OK;
}

void vl_destroy(vl_partition *p)
{
    if (!p) return;
    for (hipEvent_t e : p->prof.ev) (void)hipEventDestroy(e);
    drop_graphs(p);
    if (p->graph.cap) (void)hipStreamDestroy(p->graph.cap);
    delete p;
}

}  // extern "C"
