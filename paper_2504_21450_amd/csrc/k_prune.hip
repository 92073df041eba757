// End-of-step block pruning of the local cells (sparse velocity space,
// Section 2: the velocity space gains and loses blocks as needed).  One workgroup per
// local cell:
//   content = blocks with a value >= sparse_min: bit t (the cell's place along
//             the last shear's pencil) of the content-flag words that the last
//             shear left in its work item of the block (list entry -> item);
//             after an acceleration step, bit 0 of the flags it left per list
//             entry,
//   keep    = content dilated by the velocity-space buffer (0, 6 or 26
//             neighbours, clipped to the mesh); if pruning is off, all blocks
//             (after an acceleration step: all but the blocks it created that
//             hold only zeros),
//   removed blocks: their mass goes to the pruned-mass ledger and their slots
//             back to the free ring; created blocks get zeroed slots,
//   the list is rewritten sorted by block id into the other local list
//             region, with fresh slack for the next step's growth.
// The cell's list is staged through LDS in chunks so every global access is
// coalesced and independent.
#include "vl_internal.h"
#include "vl_storage.h"

namespace vl {

constexpr int PR_CHUNK = 1024;   // list entries staged in LDS at a time
constexpr int PR_QUEUE = 512;    // removed / created blocks queued for the wavefronts

__device__ inline int popc32(uint32_t v) { return __popc(v); }

template <int ST>
__device__ inline double lane_value(const Dev &D, int32_t slot, int lane)
{
    return Storage<ST>::load(D.pool, (int64_t)slot * BLK + lane);
}

template <int ST>
__global__ __launch_bounds__(256) void k_prune(Dev D, int nxt, int last_axis, double vol)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_tmp[256];
    __shared__ int32_t s_eid[PR_CHUNK], s_eslot[PR_CHUNK];
    __shared__ int32_t s_q[PR_QUEUE];
    __shared__ double s_wmass[4];
    __shared__ unsigned long long s_base[3];
    __shared__ unsigned long long s_rbase;
    __shared__ int s_cnt[4];
    __shared__ int s_wrem[4];
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = D.W;
    uint32_t *s_old = (uint32_t *)smem;
    uint32_t *s_keep = s_old + W;
    int *s_rank = (int *)(s_keep + W);

    const int64_t q = blockIdx.x;
    const int x = (int)(q % D.n[0]), y = (int)((q / D.n[0]) % D.n[1]), z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
    const int64_t c = cell_index(D, x + H, y + H, z + H);
    const int cnt = D.lcount[c];
    const int64_t cs = D.lstart[c];
    const bool prune = D.sparse_min > 0.0;
    const int nbx = D.nblk[0], nby = D.nblk[1], nbz = D.nblk[2];
    // the cell's word and bit in the last shear's content flags
    const bool accel = last_axis < 0;
    const int tc = H + (last_axis == 0 ? x : last_axis == 1 ? y : z);
    const uint32_t *fw = D.masks + (tc >> 5);
    const uint32_t fbit = 1u << (tc & 31);
    const uint64_t nitems = (uint64_t)min((int64_t)D.ctl->n_items, D.item_cap);

    for (int w = tid; w < W; w += 256) {
        s_old[w] = 0u;
        s_keep[w] = 0u;
    }
    if (tid < 4) s_cnt[tid] = 0;
    if (tid == 0) s_fail = failed(D) ? 1 : 0;
    __syncthreads();
    if (s_fail) return;  // fail-stop, one decision per workgroup (nothing written yet)
    // old set and dilated content
    for (int e = tid; e < cnt; e += 256) {
        const int32_t id = D.lid[cs + e];
        const int32_t slot = D.lslot[cs + e];
        atomicOr(&s_old[id >> 5], 1u << (id & 31));
        if (accel) {
            const int fl = D.litem[cs + e];
            if (!prune) {
                if (!(fl & 4) || (fl & 2)) atomicOr(&s_keep[id >> 5], 1u << (id & 31));
                continue;
            }
            if (!(fl & 1)) continue;
        } else {
            if (!prune) {
                atomicOr(&s_keep[id >> 5], 1u << (id & 31));
                continue;
            }
            if ((int64_t)slot >= D.lcap) continue;  // scratch slot of a failed allocation
            const uint32_t it = (uint32_t)D.litem[cs + e];
            if ((uint64_t)it >= nitems || !(fw[(int64_t)it * D.wlmax] & fbit)) continue;
        }
        const int bx = id % nbx, by = (id / nbx) % nby, bz = id / (nbx * nby);
        for (int oz = -1; oz <= 1; oz++)
            for (int oy = -1; oy <= 1; oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    const int nz = (ox != 0) + (oy != 0) + (oz != 0);
                    if (nz > 1 && D.vbuffer != 26) continue;
                    if (nz == 1 && D.vbuffer == 0) continue;
                    const int xx = bx + ox, yy = by + oy, zz = bz + oz;
                    if (xx < 0 || yy < 0 || zz < 0 || xx >= nbx || yy >= nby || zz >= nbz) continue;
                    const int32_t nid = xx + nbx * (yy + nby * zz);
                    atomicOr(&s_keep[nid >> 5], 1u << (nid & 31));
                }
    }
    __syncthreads();
    // ranks of the kept blocks (exclusive scan over W words) and counts
    int ncreate = 0;
    {
        const int per = (W + 255) / 256;
        const int b = min(tid * per, W), e = min(b + per, W);
        int sum = 0;
        for (int i = b; i < e; i++) {
            sum += popc32(s_keep[i]);
            ncreate += popc32(s_keep[i] & ~s_old[i]);
        }
        s_tmp[tid] = sum;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            int v = (tid >= o) ? s_tmp[tid - o] : 0;
            __syncthreads();
            s_tmp[tid] += v;
            __syncthreads();
        }
        int run = s_tmp[tid] - sum;
        for (int i = b; i < e; i++) {
            s_rank[i] = run;
            run += popc32(s_keep[i]);
        }
        if (tid == 255) s_cnt[0] = s_tmp[255];
    }
    atomicAdd(&s_cnt[1], ncreate);
    __syncthreads();
    const int nkeep = s_cnt[0];
    const int ncr = s_cnt[1];
    const int cap = nkeep + nkeep / 4 + 32;
    if (tid == 0) {
        unsigned long long err = 0;
        unsigned long long lb = atomicAdd(&D.ctl->list_top[nxt], (unsigned long long)cap);
        unsigned long long ok = 1;
        if ((int64_t)(lb + cap) > D.reg_cap[nxt]) {
            err |= E_LOCAL_LIST;
            ok = 0;
        }
        unsigned long long rb = 0;
        if (ok && ncr > 0) {
            rb = atomicAdd(&D.ctl->ring_head, (unsigned long long)ncr);
            if (rb + ncr > D.ctl->ring_limit) {
                err |= E_RING;
                ok |= 2;
            }
        }
        if (err) atomicOr(&D.ctl->err, err);
        s_base[0] = lb;
        s_rbase = rb;
        s_base[2] = ok;
    }
    __syncthreads();
    if (!(s_base[2] & 1)) {
        if (tid == 0) D.cell_red[q] = 0.0;
        return;  // list region full: the cell keeps its old list (error flagged)
    }
    const int64_t ns = D.reg_off[nxt] + (int64_t)s_base[0];
    const bool ring_failed = (s_base[2] & 2) != 0;
    double lmass = 0.0;  // this lane's share of the removed blocks of this wavefront

    // old entries: kept ones move to their sorted position, removed ones are
    // queued (slot) for the mass sum and returned to the ring
    for (int e0 = 0; e0 < cnt; e0 += PR_CHUNK) {
        const int m = min(PR_CHUNK, cnt - e0);
        for (int e = tid; e < m; e += 256) {
            s_eid[e] = D.lid[cs + e0 + e];
            s_eslot[e] = D.lslot[cs + e0 + e];
        }
        __syncthreads();
        // removed entries are queued in entry order (a prefix count over the
        // workgroup per 256 entries), so their mass is summed in the same order
        // in every run
        int nrem_run = 0;
        for (int r = 0; r < m; r += 256) {
            const int e = r + tid;
            bool removed = false;
            int32_t slot = 0;
            if (e < m) {
                const int32_t id = s_eid[e];
                slot = s_eslot[e];
                const int w = id >> 5;
                const uint32_t bit = 1u << (id & 31);
                if (s_keep[w] & bit) {
                    const int pos = s_rank[w] + popc32(s_keep[w] & (bit - 1u));
                    D.lid[ns + pos] = id;
                    D.lslot[ns + pos] = slot;
                } else {
                    removed = true;
                }
            }
            const unsigned long long bal = __ballot(removed);
            if (lane == 0) s_wrem[wv] = (int)__popcll(bal);
            __syncthreads();
            int before = nrem_run;
            for (int j = 0; j < wv; j++) before += s_wrem[j];
            const int k = before + (int)__popcll(bal & ((1ull << lane) - 1ull));
            if (removed) {
                if (k < PR_QUEUE) s_q[k] = slot;
                else s_eslot[e] = -1 - slot;  // summed below from the staged entries
            }
            nrem_run += ((s_wrem[0] + s_wrem[1]) + s_wrem[2]) + s_wrem[3];
            __syncthreads();
        }
        if (tid == 0) s_cnt[2] = nrem_run;
        __syncthreads();
        // return the removed slots to the free ring: one counter update per chunk
        {
            const int nrem = s_cnt[2];
            if (tid == 0 && nrem > 0) s_base[1] = atomicAdd(&D.ctl->ring_tail, (unsigned long long)nrem);
            __syncthreads();
            const unsigned long long t0 = s_base[1];
            for (int k = tid; k < min(nrem, PR_QUEUE); k += 256) {
                const int32_t slot = s_q[k];
                D.ring[(int64_t)((t0 + k) % (unsigned long long)D.lcap)] = (int64_t)slot < D.lcap ? slot : (int32_t)D.trash;
            }
            if (nrem > PR_QUEUE) {
                // queue overflow: the remaining removed slots in entry order
                if (tid == 0) {
                    int k = PR_QUEUE;
                    for (int e = 0; e < m; e++) {
                        const int32_t sl = s_eslot[e];
                        if (sl < 0) {
                            const int32_t slot = -1 - sl;
                            D.ring[(int64_t)((t0 + k) % (unsigned long long)D.lcap)] =
                                (int64_t)slot < D.lcap ? slot : (int32_t)D.trash;
                            k++;
                        }
                    }
                }
            }
            __syncthreads();
        }
        const int nq = min(s_cnt[2], PR_QUEUE);
        // removed mass: per lane over the wavefront's blocks, four loads in
        // flight, reduced across the lanes once at the end
        int k = wv;
        for (; k + 12 < nq; k += 16) {
            const double a0 = lane_value<ST>(D, s_q[k], lane), a1 = lane_value<ST>(D, s_q[k + 4], lane);
            const double a2 = lane_value<ST>(D, s_q[k + 8], lane), a3 = lane_value<ST>(D, s_q[k + 12], lane);
            lmass += (a0 + a1) + (a2 + a3);
        }
        for (; k < nq; k += 4) lmass += lane_value<ST>(D, s_q[k], lane);
        if (s_cnt[2] > PR_QUEUE) {
            // overflow of the queue: sum the rest entry by entry
            for (int e = wv; e < m; e += 4) {
                const int32_t sl = s_eslot[e];
                if (sl < 0) lmass += lane_value<ST>(D, -1 - sl, lane);
            }
        }
        __syncthreads();
    }
    // created blocks: take slots, record them, zero them
    if (ncr > 0) {
        if (tid == 0) s_cnt[3] = 0;
        __syncthreads();
        const int per = (W + 255) / 256;
        const int b = min(tid * per, W), e = min(b + per, W);
        for (int w = b; w < e; w++) {
            uint32_t cr = s_keep[w] & ~s_old[w];
            while (cr) {
                const int bit = __ffs(cr) - 1;
                cr &= cr - 1;
                const int32_t id = 32 * w + bit;
                const int pos = s_rank[w] + popc32(s_keep[w] & ((1u << bit) - 1u));
                const int ci = atomicAdd(&s_cnt[3], 1);
                const int64_t slot = ring_failed ? D.trash
                                                 : (int64_t)D.ring[(int64_t)((s_rbase + ci) % (unsigned long long)D.lcap)];
                D.lid[ns + pos] = id;
                D.lslot[ns + pos] = (int32_t)slot;
                if (ci < PR_QUEUE) {
                    s_q[ci] = (int32_t)slot;
                } else {
                    for (int l = 0; l < BLK; l++) Storage<ST>::store(D.pool, slot * BLK + l, 0.0);
                }
            }
        }
        __syncthreads();
        const int nq = min(s_cnt[3], PR_QUEUE);
        for (int k = wv; k < nq; k += 4) Storage<ST>::store(D.pool, (int64_t)s_q[k] * BLK + lane, 0.0);
    }
    double wmass = lmass;
    for (int o = 32; o > 0; o >>= 1) wmass += __shfl_xor(wmass, o);
    if (lane == 0) s_wmass[wv] = wmass;
    __syncthreads();
    if (tid == 0) {
        D.cell_red[q] = (((s_wmass[0] + s_wmass[1]) + s_wmass[2]) + s_wmass[3]) * vol;
        D.lstart[c] = ns;
        D.lcount[c] = nkeep;
        D.lcapa[c] = cap;
        D.lsorted[c] = nkeep;
    }
}

void launch_prune(const Dev &D, int nxt, int last_axis, hipStream_t st)
{
    size_t lds = sizeof(uint32_t) * D.W * 2 + sizeof(int) * (D.W + 1) + 64;
    const double vol = D.dx[0] * D.dx[1] * D.dx[2] * D.dv[0] * D.dv[1] * D.dv[2];
    dim3 g((unsigned)D.nlocal), b(256);
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_prune<VL_F64>, g, b, lds, st, D, nxt, last_axis, vol); break;
    case VL_F32: hipLaunchKernelGGL(k_prune<VL_F32>, g, b, lds, st, D, nxt, last_axis, vol); break;
    default: hipLaunchKernelGGL(k_prune<VL_BF16>, g, b, lds, st, D, nxt, last_axis, vol); break;
    }
}

}  // namespace vl
