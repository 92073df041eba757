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
// Every pass over the cell's list takes four entries per thread at a time
// with their loads issued together; removed blocks are ordered by block id
// (a prefix count over the bitmap of removed blocks), so each entry finds its
// place in the new list or in the free ring by itself, and their mass is
// summed from the slots the workgroup wrote to its part of the ring.
#include "vl_internal.h"
#include "vl_storage.h"

namespace vl {

constexpr int PR_QUEUE = 512;  // created blocks queued for the wavefronts
constexpr int PR_UNROLL = 4;   // list entries per thread per pass iteration

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
    __shared__ int s_tmp[3][4];
    __shared__ int32_t s_q[PR_QUEUE];
    __shared__ double s_wmass[4];
    __shared__ unsigned long long s_base[4];
    __shared__ int s_cnt[4];
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = D.W;
    uint32_t *s_old = (uint32_t *)smem;
    uint32_t *s_keep = s_old + W;
    int *s_rank = (int *)(s_keep + W);   // kept blocks before each word
    int *s_rrank = s_rank + (W + 1);     // removed blocks before each word

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
    if (tid == 0) s_fail = failed(D) ? 1 : 0;
    __syncthreads();
    if (s_fail) return;  // fail-stop, one decision per workgroup (nothing written yet)
    // old set and dilated content
    for (int e0 = tid; e0 < cnt; e0 += 256 * PR_UNROLL) {
        int32_t id[PR_UNROLL], slot[PR_UNROLL], fl[PR_UNROLL];
        uint32_t word[PR_UNROLL];
#pragma unroll
        for (int u = 0; u < PR_UNROLL; u++) {
            const int e = e0 + 256 * u;
            const bool v = e < cnt;
            id[u] = v ? D.lid[cs + e] : -1;
            slot[u] = v ? D.lslot[cs + e] : 0;
            fl[u] = (v && (accel || prune)) ? D.litem[cs + e] : 0;
        }
        // the content flag word of each entry's item (last shear)
#pragma unroll
        for (int u = 0; u < PR_UNROLL; u++) {
            const bool need = id[u] >= 0 && !accel && prune && (int64_t)slot[u] < D.lcap && (uint64_t)(uint32_t)fl[u] < nitems;
            word[u] = need ? fw[(int64_t)(uint32_t)fl[u] * D.wlmax] : 0u;
        }
#pragma unroll
        for (int u = 0; u < PR_UNROLL; u++) {
            const int32_t bid = id[u];
            if (bid < 0) continue;
            atomicOr(&s_old[bid >> 5], 1u << (bid & 31));
            bool content;
            if (accel) {
                if (!prune) {
                    if (!(fl[u] & 4) || (fl[u] & 2)) atomicOr(&s_keep[bid >> 5], 1u << (bid & 31));
                    continue;
                }
                content = (fl[u] & 1) != 0;
            } else {
                if (!prune) {
                    atomicOr(&s_keep[bid >> 5], 1u << (bid & 31));
                    continue;
                }
                content = (word[u] & fbit) != 0;  // zero for the scratch slot of a failed allocation
            }
            if (!content) continue;
            const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
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
    }
    __syncthreads();
    // kept and removed blocks before each word (exclusive scans: per thread a
    // run of words, within the wavefront by shuffles, across the wavefronts
    // through LDS), and the created blocks
    {
        const int per = (W + 255) / 256;
        const int b = min(tid * per, W), e = min(b + per, W);
        int sk = 0, sr = 0, sc = 0;
        for (int i = b; i < e; i++) {
            sk += popc32(s_keep[i]);
            sr += popc32(s_old[i] & ~s_keep[i]);
            sc += popc32(s_keep[i] & ~s_old[i]);
        }
        int ik = sk, ir = sr, ic = sc;
        for (int o = 1; o < 64; o <<= 1) {
            const int vk = __shfl_up(ik, o), vr = __shfl_up(ir, o), vc = __shfl_up(ic, o);
            if (lane >= o) {
                ik += vk;
                ir += vr;
                ic += vc;
            }
        }
        if (lane == 63) {
            s_tmp[0][wv] = ik;
            s_tmp[1][wv] = ir;
            s_tmp[2][wv] = ic;
        }
        __syncthreads();
        int rk = ik - sk, rr = ir - sr;
        for (int w = 0; w < wv; w++) {
            rk += s_tmp[0][w];
            rr += s_tmp[1][w];
        }
        for (int i = b; i < e; i++) {
            s_rank[i] = rk;
            s_rrank[i] = rr;
            rk += popc32(s_keep[i]);
            rr += popc32(s_old[i] & ~s_keep[i]);
        }
        if (tid == 0) {
            s_cnt[0] = ((s_tmp[0][0] + s_tmp[0][1]) + s_tmp[0][2]) + s_tmp[0][3];
            s_cnt[1] = ((s_tmp[2][0] + s_tmp[2][1]) + s_tmp[2][2]) + s_tmp[2][3];
            s_cnt[2] = ((s_tmp[1][0] + s_tmp[1][1]) + s_tmp[1][2]) + s_tmp[1][3];
        }
    }
    __syncthreads();
    const int nkeep = s_cnt[0];
    const int ncr = s_cnt[1];
    const int nrem = s_cnt[2];
    const int cap = nkeep + nkeep / 4 + 32;
    // the new list's place, the created blocks' slots and the removed blocks'
    // places in the free ring, one counter update each
    if (tid == 0) {
        unsigned long long err = 0;
        unsigned long long lb = atomicAdd(&D.ctl->list_top[nxt], (unsigned long long)cap);
        unsigned long long ok = 1;
        if ((int64_t)(lb + cap) > D.reg_cap[nxt]) {
            err |= E_LOCAL_LIST;
            ok = 0;
        }
        unsigned long long rb = 0, tb = 0;
        if (ok && ncr > 0) {
            rb = atomicAdd(&D.ctl->ring_head, (unsigned long long)ncr);
            if (rb + ncr > D.ctl->ring_limit) {
                err |= E_RING;
                ok |= 2;
            }
        }
        if (ok && nrem > 0) tb = atomicAdd(&D.ctl->ring_tail, (unsigned long long)nrem);
        if (err) atomicOr(&D.ctl->err, err);
        s_base[0] = lb;
        s_base[1] = tb;
        s_base[2] = ok;
        s_base[3] = rb;
    }
    __syncthreads();
    if (!(s_base[2] & 1)) {
        if (tid == 0) D.cell_red[q] = 0.0;
        return;  // list region full: the cell keeps its old list (error flagged)
    }
    const int64_t ns = D.reg_off[nxt] + (int64_t)s_base[0];
    const int64_t r0 = (int64_t)(s_base[1] % (unsigned long long)D.lcap);  // the removed blocks' first ring place
    const unsigned long long rbase = s_base[3];
    const bool ring_failed = (s_base[2] & 2) != 0;

    // old entries: kept ones to their sorted place in the new list, removed
    // ones to their place in the free ring (in block-id order)
    for (int e0 = tid; e0 < cnt; e0 += 256 * PR_UNROLL) {
        int32_t id[PR_UNROLL], slot[PR_UNROLL];
#pragma unroll
        for (int u = 0; u < PR_UNROLL; u++) {
            const int e = e0 + 256 * u;
            const bool v = e < cnt;
            id[u] = v ? D.lid[cs + e] : -1;
            slot[u] = v ? D.lslot[cs + e] : 0;
        }
#pragma unroll
        for (int u = 0; u < PR_UNROLL; u++) {
            const int32_t bid = id[u];
            if (bid < 0) continue;
            const int w = bid >> 5;
            const uint32_t bit = 1u << (bid & 31), below = bit - 1u;
            const uint32_t kw = s_keep[w];
            if (kw & bit) {
                const int pos = s_rank[w] + popc32(kw & below);
                D.lid[ns + pos] = bid;
                D.lslot[ns + pos] = slot[u];
            } else {
                const int k = s_rrank[w] + popc32(s_old[w] & ~kw & below);
                int64_t r = r0 + k;  // k < nrem <= lcap
                if (r >= D.lcap) r -= D.lcap;
                D.ring[r] = (int64_t)slot[u] < D.lcap ? slot[u] : (int32_t)D.trash;
            }
        }
    }
    __syncthreads();
    // removed mass: each wavefront takes 64 removed blocks at a time, their
    // slots read back from the workgroup's places in the ring (one coalesced
    // vector load; written above by this workgroup), the blocks summed per
    // lane with eight loads in flight; reduced across the lanes at the end
    double lmass = 0.0;
    for (int k0 = 64 * wv; k0 < nrem; k0 += 256) {
        const int n = min(64, nrem - k0);
        int32_t myslot = (int32_t)D.trash;
        if (lane < n) {
            int64_t r = r0 + k0 + lane;
            if (r >= D.lcap) r -= D.lcap;
            myslot = D.ring[r];
        }
        int j = 0;
        for (; j + 8 <= n; j += 8) {
            double a[8];
#pragma unroll
            for (int i = 0; i < 8; i++) a[i] = lane_value<ST>(D, __builtin_amdgcn_readlane(myslot, j + i), lane);
            lmass += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
        for (; j < n; j++) lmass += lane_value<ST>(D, __builtin_amdgcn_readlane(myslot, j), lane);
    }
    __syncthreads();
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
                                                 : (int64_t)D.ring[(int64_t)((rbase + ci) % (unsigned long long)D.lcap)];
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
    size_t lds = sizeof(uint32_t) * D.W * 2 + sizeof(int) * (D.W + 1) * 2 + 64;
    const double vol = D.dx[0] * D.dx[1] * D.dx[2] * D.dv[0] * D.dv[1] * D.dv[2];
    dim3 g((unsigned)D.nlocal), b(256);
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_prune<VL_F64>, g, b, lds, st, D, nxt, last_axis, vol); break;
    case VL_F32: hipLaunchKernelGGL(k_prune<VL_F32>, g, b, lds, st, D, nxt, last_axis, vol); break;
    default: hipLaunchKernelGGL(k_prune<VL_BF16>, g, b, lds, st, D, nxt, last_axis, vol); break;
    }
}

}  // namespace vl
