// Internal layout of a partition in device memory, shared by the kernels and
// the C-ABI host code of libvlasov.so.  Not part of the public ABI.
//
// Device layout (all inside the caller's workspace):
//   pool    : (lcap + gcap + 1 + NSINK) blocks x 64 values of the storage type.
//             Slots [0, lcap) belong to local cells, [lcap, lcap+gcap) to ghost
//             cells; slot lcap+gcap is an all-zero block (what the shears read
//             for a cell without the block; also handed out, with the error flag
//             set, when an allocation fails) and the NSINK slots after it are
//             write-only sinks for the shears' discarded stores, one per
//             resident wavefront so the stores spread over the memory channels.
//   ring    : lcap int32 free local slots, a FIFO addressed by 64-bit counters
//             (head = next to hand out, tail = next free position).
//   cells   : per padded cell (x fastest) list start / count / capacity.
//   lists   : block ids and slots of every cell; three regions: two for the
//             local cells (rebuilt alternately by the end-of-step pruning) and
//             one for the ghost cells (rebuilt by every ghost update).  Lists
//             grow in place during a shear (new entries appended) and are
//             sorted again by the pruning.
//   rows    : per shear, for each (pencil, block) work item the slots of the
//             cells of the pencil that hold the block (compacted, pencil order).
//   items   : per shear, block id, row offset and presence mask of every item;
//             the items of one pencil are contiguous, one per block of the
//             union of the pencil's lists in ascending id order (blocks with no
//             updated cell get an empty item), so pencil p's items are
//             [pen_first[p], pen_first[p] + pen_cnt[p]).
//   resid   : per item, the FP32/BF16 rounding residual left at the end of the
//             item's pencil line, summed over the block's 64 velocity cells
//             (FP64), reduced per pencil in a fixed order for the mass ledger.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vlasov.h"

namespace vl {

constexpr int H = 3;                   // ghost depth: stencil 2 + 1 face neighbour
constexpr int BLK = 64;                // values per velocity block (4 x 4 x 4)
constexpr uint32_t NEWFLAG = 0x80000000u;  // row entry of a block created by growth
constexpr int MAXL = 256;              // longest pencil (padded extent)
constexpr int MAXWL = MAXL / 32;       // presence-mask words per item
constexpr int NB_MAX = 131072;         // block ids per velocity mesh
constexpr int WAVE = 64;
constexpr int NSINK = 8192;            // sink blocks (>= resident wavefronts)

// device error bits (Ctl::err)
enum : unsigned long long {
    E_RING = 1, E_GHOST_SLOTS = 2, E_LIST = 4, E_ITEMS = 8, E_ROWS = 16,
    E_GHOST_LIST = 32, E_LOCAL_LIST = 64, E_MOMENTS = 128
};

struct Ctl {
    unsigned long long ring_head, ring_tail, ring_limit;
    unsigned long long ghost_top, ghost_list_top;
    unsigned long long list_top[2];
    unsigned long long n_items, row_top, work;
    unsigned long long upd_ps[3], read_ps[3], items[3];
    unsigned long long cum_upd, cum_read;  // never reset: totals since init
    // error bits on a cache line of their own: every kernel reads them at its
    // start (fail-stop) while the counters above take atomics
    alignas(128) unsigned long long err;
    unsigned long long pad[15];
};

struct Item {
    int32_t id;       // velocity block id
    int32_t pencil;   // pencil index within the shear
    int64_t rowoff;   // first row entry
};

struct Dev {
    int n[3], P[3], nblk[3];
    int NB, W;               // block ids, 32-bit words of a block bitmap
    int storage;
    int vbuffer;
    int64_t N, nlocal;       // padded cells, local cells
    int64_t s[3];            // cell strides in the padded box
    double vmin[3], dv[3], dx[3];
    double sparse_min;
    void *pool;
    int64_t lcap, gcap, trash;
    int32_t *ring;
    int64_t *lstart;
    int32_t *lcount, *lcapa;
    int32_t *lsorted;        // length of the ascending prefix of each list (growth appends after it)
    int32_t *lid, *lslot;
    int32_t *litem;          // per list entry: the last shear's work item of the block
    int64_t reg_off[3], reg_cap[3];
    int32_t *rows;
    int64_t row_cap;
    Item *items;
    uint32_t *masks;         // per item: presence along the pencil; after the last
                             // shear, the content flags of the updated cells
    int64_t item_cap;
    double *resid;           // per item: terminal rounding residual of its line (item_cap)
    int64_t *pen_first;      // per pencil of the current shear: first item
    int32_t *pen_cnt;        //   and number of items (pen_cap entries)
    double *pen_sum;         //   and the sum of its items' residuals (ledger scratch)
    int64_t pen_cap;
    int wlmax;
    Ctl *ctl;
    const double *cover;     // Courant override (3 x cover_stride) or null
    int cover_stride;
    double *cell_red;        // nlocal doubles of per-cell partial sums
    double *red;             // small reduction scratch (>= 1024 doubles)
    int32_t *cell_cnt;       // nlocal ints (export helper)
    int sweep_variant[3];    // shear kernel variant of each shear of the order (autotuner)
};

// Fail-stop: once a capacity error is recorded, every later kernel of the
// partition returns at once, so a partition whose lists or slots may be
// inconsistent is never read (the host reports VL_ERR_CAPACITY at its next
// synchronising call and refuses further work).
__device__ inline bool failed(const Dev &D)
{
    // errors of earlier kernels are visible at launch; one raised by another
    // workgroup of the same kernel may be missed, which every kernel tolerates
    return D.ctl->err != 0ull;
}

__host__ __device__ inline int64_t cell_index(const Dev &D, int x, int y, int z)
{
    return (int64_t)x + D.s[1] * y + D.s[2] * z;
}

__host__ __device__ inline bool is_local(const Dev &D, int x, int y, int z)
{
    return x >= H && x < H + D.n[0] && y >= H && y < H + D.n[1] && z >= H && z < H + D.n[2];
}

// Courant number of velocity index j along axis d: v_j dt / dx_d with the
// cell-centre velocity v_j = vmin + (j + 1/2) dv (no fused operations, so host
// and device agree bit for bit).
__device__ inline double courant(const Dev &D, int d, int j, double dt)
{
    if (D.cover) return D.cover[d * D.cover_stride + j];
    double v = __dadd_rn(D.vmin[d], __dmul_rn((double)j + 0.5, D.dv[d]));
    return __ddiv_rn(__dmul_rn(v, dt), D.dx[d]);
}

__device__ inline int block_coord(const Dev &D, int d, int32_t b)
{
    if (d == 0) return b % D.nblk[0];
    if (d == 1) return (b / D.nblk[0]) % D.nblk[1];
    return b / (D.nblk[0] * D.nblk[1]);
}

// bit 0: some velocity cell of the block moves towards +d; bit 1: towards -d
__device__ inline int block_dirs(const Dev &D, int d, int32_t b, double dt)
{
    int bd = block_coord(D, d, b);
    int r = 0;
    for (int q = 0; q < 4; q++) {
        double c = courant(D, d, 4 * bd + q, dt);
        r |= (c > 0.0) ? 1 : 0;
        r |= (c < 0.0) ? 2 : 0;
    }
    return r;
}

// Per-line mass ledger of the reduced storage types.  A store holds, for one
// shear axis, the work items of its last shear: per item the block id and
// the FP64 carry left at the end of the pencil line, summed over the block's
// 64 velocity cells; per pencil (keyed by its padded transverse coordinates
// t1 + P[e1] t2) the first item and the item count.  The next shear along
// the same axis starts the carry of each velocity cell of the same (line,
// block) from 1/64 of that sum (exact in FP64), so rounding residuals go back
// into f instead of piling up.
struct LedgerStore {
    int32_t *ids;     // block id per item
    double *res;      // residual per item
    int32_t *kfirst;  // per pencil key: first item
    int32_t *kcnt;    //   and item count (0: none)
};
// the stores one shear reads (old) and writes (nw), and its item -> old item
// map; all null (cap 0) in FP64 storage, which has no rounding carry
struct LedgerIO {
    LedgerStore old, nw;
    int32_t *src;     // per item of the shear: item of the old store with the same line and block, or -1
    int64_t cap;      // items a store holds
};

// ---- launches (defined in the kernel sources, called by the host API) ----
void launch_book(const Dev &D, int op, hipStream_t st);
void launch_iota_ring(const Dev &D, int64_t first_free, int64_t count, hipStream_t st);
void launch_load(const Dev &D, int64_t first, int64_t n, const double *f, hipStream_t st);
// source of a ghost update: the partition itself (periodic images) or the 27
// partitions around it (index (dx+1) + 3(dy+1) + 9(dz+1), same local box)
struct SrcPart {
    const int64_t *lstart;
    const int32_t *lcount, *lsorted, *lid, *lslot;
    const void *pool;
};
struct SrcTable {
    SrcPart part[27];
    int remote;  // 0: periodic images of the partition's own cells
};
void launch_fill(const Dev &D, const int lo[3], const int hi[3], hipStream_t st);
void launch_fill_from(const Dev &D, const SrcTable &src, hipStream_t st);
void launch_fill_box(const Dev &D, const SrcTable &src, const int lo[3], const int hi[3], hipStream_t st);
SrcPart self_source(const Dev &D);
void launch_plan(const Dev &D, int d, int sidx, const int lo[3], const int hi[3], double dt, int cur,
                 const LedgerIO &lg, hipStream_t st);
int sweep_variants();
void launch_sweep(const Dev &D, int d, int sidx, const int lo[3], const int hi[3], double dt, bool last,
                  const LedgerIO &lg, hipStream_t st);
// n int32 zeros at p (a kernel, so that graph captures hold no memset node)
void launch_zero_i32(int32_t *p, int64_t n, hipStream_t st);
// FP64 sum of the terminal residuals of the shear's local pencils into *out:
// per pencil over its items in id order, then over the pencils in order
void launch_ledger_sum(const Dev &D, int d, const int lo[3], const int hi[3], double *out, hipStream_t st);
// last_axis < 0: the acceleration step's flags per list entry (bit 0 content,
// bit 1 nonzero, bit 2 created in the step) instead of a shear's content flags
void launch_prune(const Dev &D, int nxt_region, int last_axis, hipStream_t st);
// acceleration step: per local cell the three one-coordinate maps of the
// velocity map in the given order (ACC_MAP doubles each; *bad set to nonzero
// if a cell's map cannot be split), then the three remaps of every cell's
// velocity space; launch_accel returns -1 if the velocity mesh is beyond the
// kernel's limits (more than ACC_MAX_NBLK blocks along an axis)
constexpr int ACC_MAX_NBLK = 64;
constexpr int ACC_MAP_DOUBLES = 12;
void launch_accel_maps(const Dev &D, const double *fields, double *maps, int *bad, double qm, double dt,
                       const int order[3], hipStream_t st);
size_t accel_lds_bytes(const Dev &D, int *ncols, int *hc);
int launch_accel(const Dev &D, double *maps, const int order[3], int cur, hipStream_t st);
void launch_cell_mass(const Dev &D, hipStream_t st);
void launch_reduce(const Dev &D, const double *in, int64_t n, double *out, hipStream_t st);
// scratch of the moments: per local cell the first partial slot of a split
// cell (-1: one chunk) and the cell's mass; per chunk of a split cell ten
// partial sums; the further chunks (cell, chunk) as work units; two counters
struct MomScratch {
    unsigned long long *ctr;
    int32_t *cell_base;
    double *cell_mass;
    double *part;
    int2 *extra;
    int64_t cap_part, cap_extra;
    int chunk;
};
constexpr int MOM_CHUNK = 1024;  // blocks per moments work unit (cells with more are split)
int64_t moments_scratch_bytes(int64_t nlocal, int64_t parts, int64_t extras);
MomScratch carve_moments_scratch(void *base, int64_t nlocal, int64_t parts, int64_t extras, int chunk);
void launch_moments(const Dev &D, const MomScratch &M, double *dn, double *dV, double *dP, hipStream_t st);
// the fixed device array of the allocation-free moments entry point: its
// address on the current device (taken once per device), and its size
int static_moments_scratch(void **ptr);
constexpr int64_t STATIC_MOMENTS_SCRATCH_BYTES = 64ll << 20;
void launch_cell_counts(const Dev &D, hipStream_t st);
void launch_gather(const Dev &D, const int32_t *slots, int64_t n, double *out, hipStream_t st);

// book-keeping operations (launch_book)
enum {
    BOOK_GHOST_RESET = 1,     // ghost slot and ghost list allocators to zero
    BOOK_SWEEP_RESET = 2,     // work list counters to zero, ring limit <- tail
    BOOK_PRUNE_RESET_A = 3,   // ring limit <- tail, local list region A allocator to zero
    BOOK_PRUNE_RESET_B = 4,   // same for region B
    BOOK_STEP_RESET = 5,      // per-step statistics counters to zero
};

}  // namespace vl
