// Shear planner: one workgroup per pencil (a line of padded cells along the
// shear axis d).  It
//   1. builds the union of the block ids held by the pencil's cells (an LDS
//      bitmap over the block-id space) and ranks it,
//   2. records, per block of the union, which cells of the pencil hold it (a
//      presence mask over the pencil),
//   3. grows the block lists of the updated cells: a cell gains every block of
//      its upwind face neighbour that moves into it (bit shifts of the
//      presence masks), allocating slots for the new blocks,
//   4. emits one work item per block of the union, in ascending id order and
//      contiguous per pencil (taken with one counter update per pencil): for
//      a block held by an updated cell its presence mask and a compacted row
//      of the slots of the cells holding it, for any other block an empty
//      item; in the last shear of a step it also records, per list entry of
//      the pencil's cells, the item of the entry's block (where the shear
//      leaves the content flags that the pruning reads).
//   5. in the reduced storage types, records the pencil's items in the
//      axis's new ledger store and maps each of them to the item of the same
//      block in the store of the previous shear along the axis (a bitmap
//      look-up per old item), so the shear can take that line's residual.
// Each cell belongs to exactly one pencil of a shear, so the workgroup owns the
// lists it grows.  Block ids of a chunk of the union are processed at a time
// so the LDS footprint is bounded.
#include <algorithm>

#include "vl_internal.h"

namespace vl {

struct PlanParams {
    int d, sidx;
    int e1, e2;          // transverse axes
    int lo1, n1, lo2, n2;  // pencil ranges (padded coordinates)
    int L, WL;           // pencil length (padded extent along d), mask words
    int ulo, uhi;        // updated cells along d
    int R;               // chunk capacity (block ids per chunk)
    int cur;             // local list region in use
    int kstride;         // pencil key of (t1, t2): t1 + kstride t2
    double dt;
    LedgerIO lg;
};

__device__ inline int popc(uint32_t v) { return __popc(v); }

// threads and wavefronts of a planner workgroup, and its LDS budget: four
// workgroups fit a compute unit's 160 KiB (and its registers), and a
// pencil's union is taken in chunks of as many block ids as the budget holds
// (larger chunks in fewer, larger workgroups were slower on the mixture)
constexpr int PNT = 256;
constexpr int PNW = PNT / 64;
constexpr size_t PLAN_LDS_BUDGET = 34 * 1024;

// cells of a pencil rounded up to a multiple of 8 (LDS array length)
__host__ __device__ inline int plan_cells(int L) { return (L + 7) & ~7; }

// exclusive scan of a[0..n) in place (LDS) by the workgroup: each thread
// sums a run of consecutive entries, the runs' sums are scanned within each
// wavefront by shuffles and across the wavefronts through s_w[PNW]; returns
// the total
__device__ int block_scan_excl(int *a, int n, int *s_w)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + PNT - 1) / PNT;
    const int b = min(tid * per, n), e = min(b + per, n);
    int sum = 0;
    for (int i = b; i < e; i++) sum += a[i];
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    int run = incl - sum, total = 0;
    for (int w = 0; w < PNW; w++) {
        const int t = s_w[w];
        run += (w < wave) ? t : 0;
        total += t;
    }
    for (int i = b; i < e; i++) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

__device__ inline long long block_sum_ll(long long v, long long *s_w)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    long long r = 0;
    for (int w = 0; w < PNW; w++) r += s_w[w];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(PNT) void k_plan(Dev D, PlanParams pp)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_tmp[PNW];
    __shared__ long long s_ll[PNW];
    __shared__ unsigned long long s_base[4];  // (unused), row, new-slot bases, status
    __shared__ long long s_ibp;               // the pencil's first item
    const int tid = threadIdx.x;
    const int L = pp.L, WL = pp.WL, W = D.W, R = pp.R;

    // dynamic LDS carve (per-cell arrays sized by the pencil, a multiple of 8)
    const int LP = plan_cells(L);
    unsigned char *q = smem;
    int64_t *s_cs = (int64_t *)q; q += sizeof(int64_t) * LP;
    int64_t *s_mvsrc = (int64_t *)q; q += sizeof(int64_t) * LP;  // list moved: its old place
    int *s_cnt = (int *)q; q += sizeof(int) * LP;
    int *s_cap = (int *)q; q += sizeof(int) * LP;
    int *s_new = (int *)q; q += sizeof(int) * LP;
    int *s_req = (int *)q; q += sizeof(int) * LP;   // new blocks of this chunk per cell
    int *s_pos = (int *)q; q += sizeof(int) * LP;   // first list entry of the current chunk
    int *s_cc = (int *)q; q += sizeof(int) * LP;    // list entries in the current chunk
    int *s_srt = (int *)q; q += sizeof(int) * LP;   // ascending prefix length of each list
    int *s_mvn = (int *)q; q += sizeof(int) * LP;   // list moved: entries to copy
    uint32_t *s_bm = (uint32_t *)q; q += sizeof(uint32_t) * W;
    int *s_rank = (int *)q; q += sizeof(int) * (W + 1);
    uint32_t *s_pres = (uint32_t *)q; q += sizeof(uint32_t) * R * WL;
    uint32_t *s_newb = (uint32_t *)q; q += sizeof(uint32_t) * R * WL;
    int *s_id = (int *)q; q += sizeof(int) * R;
    int *s_ro = (int *)q; q += sizeof(int) * (R + 1);  // row prefix
    int *s_np = (int *)q; q += sizeof(int) * (R + 1);  // new-block prefix
    // per block of the chunk and mask word w: the cells of its row in words
    // before w (at most 224), or 255 for a block no updated cell holds
    uint8_t *s_cum = (uint8_t *)q; q += (size_t)R * WL;

    const int p = blockIdx.x;
    const int t1 = pp.lo1 + p % pp.n1;
    const int t2 = pp.lo2 + p / pp.n1;
    int co[3];
    co[pp.e1] = t1;
    co[pp.e2] = t2;
    co[pp.d] = 0;
    const int64_t base = cell_index(D, co[0], co[1], co[2]);
    const int64_t sd = D.s[pp.d];
    const bool local_pencil = t1 >= H && t1 < H + D.n[pp.e1] && t2 >= H && t2 < H + D.n[pp.e2];
    const bool last = pp.sidx == 2;  // last shear of the step: record list entry -> item

    // 0. cell metadata
    for (int i = tid; i < L; i += PNT) {
        const int64_t c = base + sd * i;
        s_cs[i] = D.lstart[c];
        s_cnt[i] = D.lcount[c];
        s_cap[i] = D.lcapa[c];
        s_new[i] = 0;
        s_req[i] = 0;
        s_pos[i] = 0;
        s_srt[i] = D.lsorted[c];
    }
    for (int w = tid; w < W; w += PNT) s_bm[w] = 0u;
    if (tid == 0) s_base[3] = failed(D) ? 1ull : 0ull;
    __syncthreads();
    if (s_base[3]) return;  // fail-stop, one decision per workgroup (nothing written yet)
    const int lane = tid & 63, wave = tid >> 6;

    // 1. union bitmap: a wavefront reads one cell's sorted list at a time,
    //    four coalesced loads per lane, and the first 256 entries of its next
    //    cell are in flight while it files the current one
    auto load_ids = [&](int i, int e0, int32_t (&ids)[4]) {
        const int cnt = s_cnt[i];
        const int32_t *lst = D.lid + s_cs[i];
#pragma unroll
        for (int k = 0; k < 4; k++) ids[k] = (e0 + 64 * k < cnt) ? lst[e0 + 64 * k] : -1;
    };
    auto file_ids = [&](const int32_t (&ids)[4]) {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (ids[k] >= 0) atomicOr(&s_bm[ids[k] >> 5], 1u << (ids[k] & 31));
    };
    {
        int32_t nxt[4] = {-1, -1, -1, -1};
        if (wave < L) load_ids(wave, lane, nxt);
        for (int i = wave; i < L; i += PNW) {
            int32_t ids[4];
#pragma unroll
            for (int k = 0; k < 4; k++) ids[k] = nxt[k];
            if (i + PNW < L) load_ids(i + PNW, lane, nxt);
            file_ids(ids);
            for (int e0 = lane + 256; e0 < s_cnt[i]; e0 += 256) {  // lists longer than 256
                load_ids(i, e0, ids);
                file_ids(ids);
            }
        }
    }
    __syncthreads();
    // 2. ranks
    for (int w = tid; w < W; w += PNT) s_rank[w] = popc(s_bm[w]);
    __syncthreads();
    const int U = block_scan_excl(s_rank, W, s_tmp);
    // the pencil's items: item first + r for the block of union rank r
    if (tid == 0) {
        const unsigned long long ib = U > 0 ? atomicAdd(&D.ctl->n_items, (unsigned long long)U) : 0ull;
        if ((int64_t)(ib + U) > D.item_cap) atomicOr(&D.ctl->err, (unsigned long long)E_ITEMS);
        s_ibp = (long long)ib;
        if (p < D.pen_cap) {
            D.pen_first[p] = (int64_t)ib;
            D.pen_cnt[p] = U;
        }
        if (pp.lg.src) {  // the pencil in the new ledger store (its count was cleared)
            if ((int64_t)(ib + U) > pp.lg.cap) {
                atomicOr(&D.ctl->err, (unsigned long long)E_ITEMS);
            } else {
                const int key = t1 + pp.kstride * t2;
                pp.lg.nw.kfirst[key] = (int32_t)ib;
                pp.lg.nw.kcnt[key] = U;
            }
        }
    }
    __syncthreads();
    const int64_t ibp = (int64_t)s_ibp;

    // update-range mask
    uint32_t um[MAXWL];
#pragma unroll
    for (int w = 0; w < MAXWL; w++) {
        uint32_t m = 0;
        for (int b = 0; b < 32; b++) {
            int i = 32 * w + b;
            if (i >= pp.ulo && i < pp.uhi) m |= 1u << b;
        }
        um[w] = m;
    }

    long long st_upd = 0, st_read = 0, st_items = 0;

    for (int r0 = 0; r0 < U; r0 += R) {
        const int rn = min(R, U - r0);
        for (int k = tid; k < rn * WL; k += PNT) s_pres[k] = 0u;
        __syncthreads();
        // presence masks of this chunk.  Ranks grow along the ascending
        // prefix of a list, so a cell's prefix entries in the chunk are the
        // run that starts at s_pos[i] and ends at the first rank beyond the
        // chunk; the entries appended by earlier shears of the step (the
        // tail) are all looked at in every chunk.
        // The first 256 run entries and the first tail entries of a wavefront's
        // next cell are loaded while it files the current one.
        auto load_run = [&](int i, int32_t (&ids)[4], int32_t &tail0) {
            const int cnt = s_cnt[i], srt = s_srt[i], pos = s_pos[i];
            const int32_t *lst = D.lid + s_cs[i];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int e = pos + 64 * u + lane;
                ids[u] = (e < srt) ? lst[e] : -1;
            }
            tail0 = (srt + lane < cnt) ? lst[srt + lane] : -1;
        };
        int32_t nid[4] = {-1, -1, -1, -1}, ntail = -1;
        if (wave < L) load_run(wave, nid, ntail);
        for (int i = wave; i < L; i += PNW) {
            const int cnt = s_cnt[i], srt = s_srt[i];
            const int32_t *lst = D.lid + s_cs[i];
            const uint32_t cbit = 1u << (i & 31);
            const int cw = i >> 5;
            int32_t ids[4];
#pragma unroll
            for (int u = 0; u < 4; u++) ids[u] = nid[u];
            const int32_t tail0 = ntail;
            if (i + PNW < L) load_run(i + PNW, nid, ntail);
            // 256 entries are loaded at once (the run usually continues) and
            // taken 64 at a time until the first one beyond the chunk
            int pos = s_pos[i];
            bool more = pos < srt;
            bool first = true;
            while (more) {
                if (!first) {
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int e = pos + 64 * u + lane;
                        ids[u] = (e < srt) ? lst[e] : -1;
                    }
                }
                first = false;
                // the ranks of all four groups are read before any is filed,
                // so their LDS reads overlap
                int kq[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t id = ids[u];
                    const int w = id >= 0 ? id >> 5 : 0;
                    const int k = s_rank[w] + popc(s_bm[w] & ((1u << (id & 31)) - 1u)) - r0;
                    kq[u] = id >= 0 ? k : rn;
                }
                int taken = 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (more) {
                        const int32_t id = ids[u];
                        const int k = kq[u];
                        const bool in = k < rn;
                        if (in) {
                            atomicOr(&s_pres[k * WL + cw], cbit);
                            s_id[k] = id;
                        }
                        const int n_in = (int)__popcll(__ballot(in));
                        taken += n_in;
                        if (n_in < 64) more = false;
                    }
                }
                pos += taken;
                more = more && pos < srt;
            }
            if (lane == 0) s_cc[i] = pos - s_pos[i];
            for (int e = srt + lane; e < cnt; e += 64) {
                const int32_t id = (e == srt + lane) ? tail0 : lst[e];
                const int w = id >> 5;
                const int k = s_rank[w] + popc(s_bm[w] & ((1u << (id & 31)) - 1u)) - r0;
                if (k >= 0 && k < rn) {
                    atomicOr(&s_pres[k * WL + cw], cbit);
                    s_id[k] = id;
                }
            }
        }
        __syncthreads();
        // growth and per-block counts
        for (int k = tid; k < rn; k += PNT) {
            uint32_t P[MAXWL], G[MAXWL];
#pragma unroll
            for (int w = 0; w < MAXWL; w++) P[w] = (w < WL) ? s_pres[k * WL + w] : 0u;
            const int dirs = block_dirs(D, pp.d, s_id[k], pp.dt);
#pragma unroll
            for (int w = 0; w < MAXWL; w++) {
                uint32_t g = 0;
                if (dirs & 1) g |= (P[w] << 1) | (w > 0 ? (P[w - 1] >> 31) : 0u);
                if (dirs & 2) g |= (P[w] >> 1) | (w + 1 < MAXWL ? (P[w + 1] << 31) : 0u);
                G[w] = g & ~P[w] & um[w];
            }
            int rowlen = 0, nnew = 0, upd = 0, rd = 0;
            bool active = false;
#pragma unroll
            for (int w = 0; w < MAXWL; w++) {
                if (w < WL) {
                    const uint32_t pn = P[w] | G[w];
                    s_pres[k * WL + w] = pn;
                    s_newb[k * WL + w] = G[w];
                    active |= (pn & um[w]) != 0u;
                    rowlen += popc(pn);
                    nnew += popc(G[w]);
                    upd += popc(pn & um[w]);
                    rd += popc(P[w]);
                }
            }
            if (nnew > 0) {
#pragma unroll
                for (int w = 0; w < MAXWL; w++) {
                    uint32_t g = G[w];
                    while (g) {
                        const int bit = __ffs(g) - 1;
                        g &= g - 1;
                        atomicAdd(&s_req[32 * w + bit], 1);
                    }
                }
            }
            s_ro[k] = active ? rowlen : 0;
            s_np[k] = active ? nnew : 0;
            {
                int run = 0;
#pragma unroll
                for (int w = 0; w < MAXWL; w++) {
                    if (w < WL) {
                        s_cum[k * WL + w] = active ? (uint8_t)run : (uint8_t)255;
                        run += popc(P[w] | G[w]);
                    }
                }
            }
            if (active) {
                st_upd += upd;
                st_read += rd;
                st_items += 1;
            }
        }
        __syncthreads();
        // a cell whose list cannot take this chunk's new blocks moves its
        // list to a larger place at the end of its list region: the places
        // are taken per cell, then each wavefront copies the lists of its
        // cells (coalesced; the old places are not reused within the step)
        for (int i = tid; i < L; i += PNT) {
            s_mvn[i] = 0;
            const int req = s_req[i];  // cleared when the cell's new entries are written
            if (req == 0) continue;
            const int have = s_cnt[i] + s_new[i];
            if (have + req <= s_cap[i]) continue;
            const int ncap = (have + req) + (have + req) / 4 + 32;  // the slack of a fresh list
            const int reg = local_pencil ? pp.cur : 2;
            unsigned long long *top = local_pencil ? &D.ctl->list_top[pp.cur] : &D.ctl->ghost_list_top;
            const unsigned long long nb0 = atomicAdd(top, (unsigned long long)ncap);
            if ((int64_t)(nb0 + ncap) > D.reg_cap[reg]) {
                atomicOr(&D.ctl->err, (unsigned long long)E_LIST);
                continue;
            }
            const int64_t ns = D.reg_off[reg] + (int64_t)nb0;
            s_mvsrc[i] = s_cs[i];
            s_mvn[i] = have;
            s_cs[i] = ns;
            s_cap[i] = ncap;
            const int64_t c = base + sd * i;
            D.lstart[c] = ns;
            D.lcapa[c] = ncap;
        }
        __syncthreads();
        for (int i = wave; i < L; i += PNW) {
            const int n = s_mvn[i];
            if (n == 0) continue;
            const int64_t from = s_mvsrc[i], to = s_cs[i];
            for (int e = lane; e < n; e += 64) {
                D.lid[to + e] = D.lid[from + e];
                D.lslot[to + e] = D.lslot[from + e];
                if (last) D.litem[to + e] = D.litem[from + e];  // entries of earlier chunks
            }
        }
        __syncthreads();
        const int nrow = block_scan_excl(s_ro, rn, s_tmp);
        const int nnew = block_scan_excl(s_np, rn, s_tmp);
        if (tid == 0) {
            s_ro[rn] = nrow;
            s_np[rn] = nnew;
            unsigned long long err = 0;
            unsigned long long rb = atomicAdd(&D.ctl->row_top, (unsigned long long)nrow);
            unsigned long long nb = 0;
            unsigned long long ok = 1;
            if ((int64_t)(rb + nrow) > D.row_cap) {
                err |= E_ROWS;
                ok = 0;
            }
            if (nnew > 0) {
                if (local_pencil) {
                    nb = atomicAdd(&D.ctl->ring_head, (unsigned long long)nnew);
                    if (nb + nnew > D.ctl->ring_limit) {
                        err |= E_RING;
                        ok |= 2;  // allocation failed: new blocks go to the scratch slot
                    }
                } else {
                    nb = atomicAdd(&D.ctl->ghost_top, (unsigned long long)nnew);
                    if ((int64_t)(nb + nnew) > D.gcap) {
                        err |= E_GHOST_SLOTS;
                        ok |= 2;
                    }
                }
            }
            if (err) atomicOr(&D.ctl->err, err);
            s_base[1] = rb;
            s_base[2] = nb;
            s_base[3] = ok;
        }
        __syncthreads();
        const unsigned long long rb = s_base[1], nb = s_base[2];
        const bool rows_ok = (s_base[3] & 1) != 0;
        const bool alloc_failed = (s_base[3] & 2) != 0;

        // items and new blocks
        for (int k = tid; k < rn; k += PNT) {
            const int64_t it = ibp + r0 + k;
            if (pp.lg.src && it < pp.lg.cap) {  // no old residual unless matched below
                pp.lg.nw.ids[it] = s_id[k];
                pp.lg.src[it] = -1;
            }
            if (s_ro[k + 1] == s_ro[k]) {  // no updated cell holds the block: empty item
                if (it < D.item_cap) {
                    Item item;
                    item.id = s_id[k];
                    item.pencil = p;
                    item.rowoff = 0;
                    D.items[it] = item;
                    for (int w = 0; w < D.wlmax; w++) D.masks[it * D.wlmax + w] = 0u;
                }
                continue;
            }
            const int64_t rowoff = (int64_t)rb + s_ro[k];
            if (it < D.item_cap) {
                Item item;
                item.id = s_id[k];
                item.pencil = p;
                item.rowoff = rows_ok ? rowoff : 0;
                D.items[it] = item;
                for (int w = 0; w < D.wlmax; w++)
                    D.masks[it * D.wlmax + w] = (rows_ok && w < WL) ? s_pres[k * WL + w] : 0u;
            }
            int qn = s_np[k];
            for (int w = 0; w < WL; w++) {
                uint32_t nbits = s_newb[k * WL + w];
                while (nbits) {
                    const int bit = __ffs(nbits) - 1;
                    nbits &= nbits - 1;
                    const int i = 32 * w + bit;
                    int64_t slot;
                    if (alloc_failed) {
                        slot = D.trash;
                    } else if (local_pencil) {
                        slot = D.ring[(int64_t)((nb + qn) % (unsigned long long)D.lcap)];
                    } else {
                        slot = D.lcap + (int64_t)nb + qn;
                    }
                    qn++;
                    if (rows_ok) {
                        const int pos = s_cum[k * WL + w] + popc(s_pres[k * WL + w] & ((1u << bit) - 1u));
                        D.rows[rowoff + pos] = (int32_t)((uint32_t)slot | NEWFLAG);
                    }
                }
            }
        }
        // the new list entries, per cell in ascending block id (the same order
        // in every run): a wavefront per cell tests 64 chunk ranks at a time
        // and places the cell's new blocks in rank order; the slot of the
        // block of chunk rank k new in cell i is the one the row above took,
        // number s_np[k] + (rank of i among k's new cells) of this chunk's
        // allocation
        for (int i = wave; i < L; i += PNW) {
            const int want = s_req[i];
            if (want == 0) continue;
            const int have = s_new[i];
            const int iw = i >> 5;
            const uint32_t ibit = 1u << (i & 31);
            int done = 0;
            for (int k0 = 0; k0 < rn && done < want && !alloc_failed; k0 += 64) {
                const int k = k0 + lane;
                const uint32_t nw = (k < rn) ? s_newb[k * WL + iw] : 0u;
                const bool is_new = (nw & ibit) != 0u;
                const unsigned long long bal = __ballot(is_new);
                if (is_new) {
                    int qn = s_np[k];
                    for (int w2 = 0; w2 < iw; w2++) qn += popc(s_newb[k * WL + w2]);
                    qn += popc(nw & (ibit - 1u));
                    const int64_t slot = local_pencil
                                             ? (int64_t)D.ring[(int64_t)((nb + qn) % (unsigned long long)D.lcap)]
                                             : D.lcap + (int64_t)nb + qn;
                    const int lp = have + done + (int)__popcll(bal & ((1ull << lane) - 1ull));
                    if (s_cnt[i] + lp < s_cap[i]) {
                        const int64_t at = s_cs[i] + s_cnt[i] + lp;
                        D.lid[at] = s_id[k];
                        D.lslot[at] = (int32_t)slot;
                        if (last) __builtin_nontemporal_store((int32_t)(ibp + r0 + k), &D.litem[at]);
                    } else {
                        atomicOr(&D.ctl->err, (unsigned long long)E_LIST);
                    }
                }
                done += (int)__popcll(bal);
            }
            if (lane == 0) {
                s_req[i] = 0;
                if (!alloc_failed) s_new[i] = have + done;
            }
        }
        // rows of the blocks already held: the chunk's run of each list
        // (its place may have moved, its entries have not)
        if (rows_ok) {
            // the first 256 run entries and the first tail entries of the
            // wavefront's next cell are loaded while it writes the current one
            auto load_rows = [&](int i, int32_t (&ids)[4], int32_t (&sls)[4], int32_t &tid0, int32_t &tsl0) {
                const int64_t at0 = s_cs[i] + s_pos[i];
                const int n = s_cc[i];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int e = lane + 64 * k;
                    ids[k] = (e < n) ? D.lid[at0 + e] : -1;
                    sls[k] = (e < n) ? D.lslot[at0 + e] : 0;
                }
                const int64_t te = s_cs[i] + s_srt[i] + lane;
                const bool has = s_srt[i] + lane < s_cnt[i];
                tid0 = has ? D.lid[te] : -1;
                tsl0 = has ? D.lslot[te] : 0;
            };
            int32_t nids[4] = {-1, -1, -1, -1}, nsls[4] = {0, 0, 0, 0}, ntid = -1, ntsl = 0;
            if (wave < L) load_rows(wave, nids, nsls, ntid, ntsl);
            for (int i = wave; i < L; i += PNW) {
                const int64_t at0 = s_cs[i] + s_pos[i];
                const int n = s_cc[i];
                const int iw = i >> 5;
                const uint32_t below = (1u << (i & 31)) - 1u;
                int32_t ids[4], sls[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    ids[k] = nids[k];
                    sls[k] = nsls[k];
                }
                const int32_t tid0 = ntid, tsl0 = ntsl;
                if (i + PNW < L) load_rows(i + PNW, nids, nsls, ntid, ntsl);
                for (int e0 = lane; e0 < n; e0 += 256) {
                    if (e0 != lane) {  // lists with more than 256 entries in the chunk
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const int e = e0 + 64 * k;
                            ids[k] = (e < n) ? D.lid[at0 + e] : -1;
                            sls[k] = (e < n) ? D.lslot[at0 + e] : 0;
                        }
                    }
                    // the four groups' ranks, then their row bases, prefix
                    // counts and presence words, so the LDS reads overlap (the
                    // run's blocks lie in the chunk)
                    int kq[4], ro[4], cm[4];
                    uint32_t pw[4];
#pragma unroll
                    for (int kk = 0; kk < 4; kk++) {
                        const int32_t id = ids[kk];
                        const int w = id >= 0 ? id >> 5 : 0;
                        const int k = s_rank[w] + popc(s_bm[w] & ((1u << (id & 31)) - 1u)) - r0;
                        kq[kk] = id >= 0 ? k : 0;
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; kk++) {
                        ro[kk] = s_ro[kq[kk]];
                        cm[kk] = s_cum[kq[kk] * WL + iw];
                        pw[kk] = s_pres[kq[kk] * WL + iw];
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; kk++) {
                        if (ids[kk] < 0 || cm[kk] == 255) continue;  // no updated cell holds it: no row
                        D.rows[(int64_t)rb + ro[kk] + cm[kk] + popc(pw[kk] & below)] = sls[kk];
                        if (last)
                            __builtin_nontemporal_store((int32_t)(ibp + r0 + kq[kk]), &D.litem[at0 + e0 + 64 * kk]);
                    }
                }
                // the tail
                const int64_t cs = s_cs[i];
                for (int e = s_srt[i] + lane; e < s_cnt[i]; e += 64) {
                    const bool pre = e == s_srt[i] + lane;
                    const int32_t id = pre ? tid0 : D.lid[cs + e];
                    const int w = id >> 5;
                    const int k = s_rank[w] + popc(s_bm[w] & ((1u << (id & 31)) - 1u)) - r0;
                    if (k < 0 || k >= rn) continue;
                    const int cm = s_cum[k * WL + iw];
                    if (cm == 255) continue;
                    D.rows[(int64_t)rb + s_ro[k] + cm + popc(s_pres[k * WL + iw] & below)] = pre ? tsl0 : D.lslot[cs + e];
                    if (last) __builtin_nontemporal_store((int32_t)(ibp + r0 + k), &D.litem[cs + e]);
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < L; i += PNT) s_pos[i] += s_cc[i];
        __syncthreads();
    }

    // the line's residuals of the last shear along d: an old item whose block
    // is in the union gives its index to the item of that block (the union
    // bitmap and ranks still hold; the -1 entries above were written before
    // the last barrier of the chunk loop)
    if (pp.lg.src) {
        const int key = t1 + pp.kstride * t2;
        const int ocnt = pp.lg.old.kcnt[key];
        const int64_t ofirst = pp.lg.old.kfirst[key];
        for (int j = tid; j < ocnt; j += PNT) {
            const int32_t b = pp.lg.old.ids[ofirst + j];
            const uint32_t w = s_bm[b >> 5];
            if ((w >> (b & 31)) & 1u) {
                const int64_t it = ibp + s_rank[b >> 5] + popc(w & ((1u << (b & 31)) - 1u));
                if (it < pp.lg.cap) pp.lg.src[it] = (int32_t)(ofirst + j);
            }
        }
    }

    // commit list growth
    for (int i = tid; i < L; i += PNT) {
        const int a = s_new[i];
        if (a > 0) D.lcount[base + sd * i] = min(s_cnt[i] + a, s_cap[i]);
    }
    const long long u = block_sum_ll(st_upd, s_ll);
    const long long r = block_sum_ll(st_read, s_ll);
    const long long n = block_sum_ll(st_items, s_ll);
    if (tid == 0 && n > 0) {
        atomicAdd(&D.ctl->upd_ps[pp.sidx], (unsigned long long)(u * BLK));
        atomicAdd(&D.ctl->read_ps[pp.sidx], (unsigned long long)(r * BLK));
        atomicAdd(&D.ctl->items[pp.sidx], (unsigned long long)n);
        atomicAdd(&D.ctl->cum_upd, (unsigned long long)(u * BLK));
        atomicAdd(&D.ctl->cum_read, (unsigned long long)(r * BLK));
    }
}

size_t plan_lds_bytes(int W, int R, int WL, int L)
{
    const size_t lp = (size_t)plan_cells(L);
    size_t b = sizeof(int64_t) * lp * 2 + sizeof(int) * lp * 8;
    b += sizeof(uint32_t) * W + sizeof(int) * (W + 1);
    b += (size_t)R * WL * 4 * 2 + (size_t)R * 4 + (size_t)(R + 1) * 4 * 2 + (size_t)R * WL;
    return b + 64;
}

__global__ __launch_bounds__(256) void k_zero_i32(int32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

void launch_zero_i32(int32_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)g), dim3(256), 0, st, p, n);
}

void launch_plan(const Dev &D, int d, int sidx, const int lo[3], const int hi[3], double dt, int cur,
                 const LedgerIO &lg, hipStream_t st)
{
    PlanParams pp;
    pp.cur = cur;
    pp.lg = lg;
    pp.d = d;
    pp.sidx = sidx;
    pp.e1 = (d == 0) ? 1 : 0;
    pp.e2 = (d == 2) ? 1 : 2;
    pp.lo1 = lo[pp.e1];
    pp.n1 = hi[pp.e1] - lo[pp.e1];
    pp.lo2 = lo[pp.e2];
    pp.n2 = hi[pp.e2] - lo[pp.e2];
    pp.L = D.P[d];
    pp.WL = (pp.L + 31) / 32;
    pp.kstride = D.P[pp.e1];
    pp.ulo = lo[d];
    pp.uhi = hi[d];
    pp.dt = dt;
    // chunk size: as many block ids as the LDS budget holds
    const size_t budget = PLAN_LDS_BUDGET;
    size_t fixed = plan_lds_bytes(D.W, 0, pp.WL, pp.L);
    size_t per = (size_t)pp.WL * 9 + 12;
    int R = (fixed < budget) ? (int)((budget - fixed) / per) : 64;
    if (R < 64) R = 64;
    pp.R = R;
    size_t lds = plan_lds_bytes(D.W, R, pp.WL, pp.L);
    int64_t np = (int64_t)pp.n1 * pp.n2;
    if (np <= 0) return;
    hipLaunchKernelGGL(k_plan, dim3((unsigned)np), dim3(PNT), lds, st, D, pp);
}

}  // namespace vl
