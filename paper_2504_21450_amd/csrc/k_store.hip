// Block-store kernels: allocator book-keeping, the ghost update (periodic
// image copy of block lists and payloads), per-cell mass, deterministic
// reductions and the FP64 velocity moments.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "vl_internal.h"
#include "vl_storage.h"

namespace vl {

// ---------------------------------------------------------------------------
// single-thread book-keeping between phases (stream ordered)
// ---------------------------------------------------------------------------
__global__ void k_book(Dev D, int op)
{
    Ctl *c = D.ctl;
    switch (op) {
    case BOOK_GHOST_RESET:
        c->ghost_top = 0;
        c->ghost_list_top = 0;
        break;
    case BOOK_SWEEP_RESET:
        c->n_items = 0;
        c->row_top = 0;
        c->work = 0;
        c->ring_limit = c->ring_tail;
        break;
    case BOOK_PRUNE_RESET_A:
    case BOOK_PRUNE_RESET_B:
        c->ring_limit = c->ring_tail;
        c->list_top[op == BOOK_PRUNE_RESET_A ? 0 : 1] = 0;
        break;
    case BOOK_STEP_RESET:
        for (int s = 0; s < 3; s++) {
            c->upd_ps[s] = 0;
            c->read_ps[s] = 0;
            c->items[s] = 0;
        }
        break;
    default:
        break;
    }
}

void launch_book(const Dev &D, int op, hipStream_t st)
{
    hipLaunchKernelGGL(k_book, dim3(1), dim3(1), 0, st, D, op);
}

__global__ __launch_bounds__(256) void k_iota_ring(Dev D, int64_t first, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) D.ring[i] = (int32_t)(first + i);
}

void launch_iota_ring(const Dev &D, int64_t first, int64_t count, hipStream_t st)
{
    if (count <= 0) return;
    int64_t g = (count + 255) / 256;
    hipLaunchKernelGGL(k_iota_ring, dim3((unsigned)g), dim3(256), 0, st, D, first, count);
}

// values of blocks [first, first + n) given in FP64, converted to the storage
// type (slot k holds block k of the initial CSR order)
template <int ST>
__global__ __launch_bounds__(256) void k_load(Dev D, int64_t first, int64_t nval, const double *f)
{
    using S = Storage<ST>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nval; i += stride)
        S::store(D.pool, first * BLK + i, f[i]);
}

void launch_load(const Dev &D, int64_t first, int64_t n, const double *f, hipStream_t st)
{
    const int64_t nval = n * BLK;
    const unsigned g = (unsigned)std::min<int64_t>((nval + 255) / 256, 1 << 20);
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_load<VL_F64>, dim3(g), dim3(256), 0, st, D, first, nval, f); break;
    case VL_F32: hipLaunchKernelGGL(k_load<VL_F32>, dim3(g), dim3(256), 0, st, D, first, nval, f); break;
    default: hipLaunchKernelGGL(k_load<VL_BF16>, dim3(g), dim3(256), 0, st, D, first, nval, f); break;
    }
}

// ---------------------------------------------------------------------------
// ghost update: every non-local cell of the box [lo, lo + ext) receives the
// list and payload of its periodic image.  One wavefront per cell.
// ---------------------------------------------------------------------------
__device__ inline int wrap_coord(int g, int n)
{
    int l = (g - H) % n;
    if (l < 0) l += n;
    return l + H;
}

template <int ST>
__global__ __launch_bounds__(256) void k_fill(Dev D, SrcTable src, int lo0, int lo1, int lo2, int e0, int e1, int e2)
{
    using SW = typename Storage<ST>::Word;
    constexpr int WPB = Storage<ST>::WORDS_PER_BLOCK;  // words per block (<= 64)
    __shared__ unsigned long long s_need[4][2], s_wgbase[2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    const int64_t total = (int64_t)e0 * e1 * e2;
    // one wave per cell; every wave reaches the workgroup's two barriers
    const int x = lo0 + (int)(w % e0);
    const int y = lo1 + (int)((w / e0) % e1);
    const int z = lo2 + (int)(w / ((int64_t)e0 * e1));
    const bool active = w < total && !failed(D) && !is_local(D, x, y, z);
    const int64_t c = cell_index(D, x, y, z);
    // source cell: the periodic image in this partition, or the cell of the
    // neighbouring partition that holds this position (all local boxes equal,
    // each at least 3 cells wide, so the neighbour is one box away)
    int64_t s = 0;
    SrcPart sp = src.part[13];
    if (!active) {
    } else if (!src.remote) {
        s = cell_index(D, wrap_coord(x, D.n[0]), wrap_coord(y, D.n[1]), wrap_coord(z, D.n[2]));
        sp = src.part[13];
    } else {
        const int g[3] = {x - H, y - H, z - H};
        int l[3], q = 0, m = 1;
        for (int d = 0; d < 3; d++) {
            const int dir = g[d] < 0 ? -1 : (g[d] >= D.n[d] ? 1 : 0);
            l[d] = g[d] - dir * D.n[d] + H;
            q += (dir + 1) * m;
            m *= 3;
        }
        s = cell_index(D, l[0], l[1], l[2]);
        sp = src.part[q];
    }
    const int cnt = active ? sp.lcount[s] : 0;
    const int64_t ss = active ? sp.lstart[s] : 0;
    const int cap = cnt + cnt / 4 + 32;
    // list and slot space: one pair of counter updates per workgroup
    if (lane == 0) {
        s_need[wv][0] = active ? (unsigned long long)cap : 0ull;
        s_need[wv][1] = active ? (unsigned long long)cnt : 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long nl = s_need[0][0] + s_need[1][0] + s_need[2][0] + s_need[3][0];
        const unsigned long long ns = s_need[0][1] + s_need[1][1] + s_need[2][1] + s_need[3][1];
        s_wgbase[0] = nl ? atomicAdd(&D.ctl->ghost_list_top, nl) : 0ull;
        s_wgbase[1] = ns ? atomicAdd(&D.ctl->ghost_top, ns) : 0ull;
    }
    __syncthreads();
    if (!active) return;
    unsigned long long lb = s_wgbase[0], sb = s_wgbase[1];
    for (int j = 0; j < wv; j++) {
        lb += s_need[j][0];
        sb += s_need[j][1];
    }
    const bool lok = (int64_t)(lb + cap) <= D.reg_cap[2];
    const bool sok = (int64_t)(sb + cnt) <= D.gcap;
    if (!lok || !sok) {
        if (lane == 0) {
            atomicOr(&D.ctl->err, (unsigned long long)((lok ? 0 : E_GHOST_LIST) | (sok ? 0 : E_GHOST_SLOTS)));
            D.lstart[c] = D.reg_off[2];
            D.lcount[c] = 0;
            D.lcapa[c] = 0;
            D.lsorted[c] = 0;
        }
        return;
    }
    const int64_t ls = D.reg_off[2] + (int64_t)lb;
    const int64_t gslot0 = D.lcap + (int64_t)sb;
    if (lane == 0) {
        D.lstart[c] = ls;
        D.lcount[c] = cnt;
        D.lcapa[c] = cap;
        D.lsorted[c] = sp.lsorted[s];
    }
    for (int e = lane; e < cnt; e += 64) {
        D.lid[ls + e] = sp.lid[ss + e];
        D.lslot[ls + e] = (int32_t)(gslot0 + e);
    }
    // source slots are read 64 at a time (one per lane) and broadcast from
    // the lanes; 8 block copies in flight
    SW *pool = (SW *)D.pool;
    const SW *spool = (const SW *)sp.pool;
    for (int g = 0; g < cnt; g += 64) {
        const int ng = min(64, cnt - g);
        const int32_t mys = lane < ng ? sp.lslot[ss + g + lane] : 0;
        if (lane < WPB) {
            int k = 0;
            for (; k + 8 <= ng; k += 8) {
                SW v[8];
#pragma unroll
                for (int j = 0; j < 8; j++)
                    v[j] = spool[(int64_t)__builtin_amdgcn_readlane(mys, k + j) * WPB + lane];
#pragma unroll
                for (int j = 0; j < 8; j++) pool[(gslot0 + g + k + j) * WPB + lane] = v[j];
            }
            for (; k < ng; k++)
                pool[(gslot0 + g + k) * WPB + lane] = spool[(int64_t)__builtin_amdgcn_readlane(mys, k) * WPB + lane];
        }
    }
}

SrcPart self_source(const Dev &D)
{
    SrcPart p;
    p.lstart = D.lstart;
    p.lcount = D.lcount;
    p.lsorted = D.lsorted;
    p.lid = D.lid;
    p.lslot = D.lslot;
    p.pool = D.pool;
    return p;
}

template <int ST>
static void launch_fill_st(const Dev &D, const SrcTable &src, const int lo[3], const int hi[3], hipStream_t st)
{
    const int e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    const int64_t waves = (int64_t)e0 * e1 * e2;
    if (waves <= 0) return;
    hipLaunchKernelGGL(k_fill<ST>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, D, src, lo[0], lo[1], lo[2],
                       e0, e1, e2);
}

static void launch_fill_any(const Dev &D, const SrcTable &src, const int lo[3], const int hi[3], hipStream_t st)
{
    switch (D.storage) {
    case VL_F64: launch_fill_st<VL_F64>(D, src, lo, hi, st); break;
    case VL_F32: launch_fill_st<VL_F32>(D, src, lo, hi, st); break;
    default: launch_fill_st<VL_BF16>(D, src, lo, hi, st); break;
    }
}

void launch_fill_box(const Dev &D, const SrcTable &src, const int lo[3], const int hi[3], hipStream_t st)
{
    launch_fill_any(D, src, lo, hi, st);
}

void launch_fill_from(const Dev &D, const SrcTable &src, hipStream_t st)
{
    const int lo[3] = {0, 0, 0}, hi[3] = {D.P[0], D.P[1], D.P[2]};
    launch_fill_any(D, src, lo, hi, st);
}

void launch_fill(const Dev &D, const int lo[3], const int hi[3], hipStream_t st)
{
    SrcTable src;
    memset(&src, 0, sizeof(src));
    src.part[13] = self_source(D);
    src.remote = 0;
    launch_fill_any(D, src, lo, hi, st);
}

// ---------------------------------------------------------------------------
// wave reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline void local_coords(const Dev &D, int64_t q, int &x, int &y, int &z)
{
    x = (int)(q % D.n[0]);
    y = (int)((q / D.n[0]) % D.n[1]);
    z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
}

// per local cell: sum of f (FP64), one wavefront per cell
template <int ST>
__global__ __launch_bounds__(256) void k_cell_mass(Dev D)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= D.nlocal || failed(D)) return;
    int x, y, z;
    local_coords(D, q, x, y, z);
    const int64_t c = cell_index(D, x + H, y + H, z + H);
    const int cnt = D.lcount[c];
    const int64_t ls = D.lstart[c];
    double acc = 0.0;
    for (int e = 0; e < cnt; e++) {
        int64_t slot = D.lslot[ls + e];
        acc += Storage<ST>::load(D.pool, slot * BLK + lane);
    }
    acc = wave_sum(acc);
    if (lane == 0) D.cell_red[q] = acc;
}

void launch_cell_mass(const Dev &D, hipStream_t st)
{
    dim3 g((unsigned)((D.nlocal + 3) / 4));
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_cell_mass<VL_F64>, g, dim3(256), 0, st, D); break;
    case VL_F32: hipLaunchKernelGGL(k_cell_mass<VL_F32>, g, dim3(256), 0, st, D); break;
    default: hipLaunchKernelGGL(k_cell_mass<VL_BF16>, g, dim3(256), 0, st, D); break;
    }
}

// deterministic sum of n doubles into *out (one workgroup, fixed order)
__global__ __launch_bounds__(1024) void k_reduce(const double *in, int64_t n, double *out)
{
    __shared__ double s[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += in[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

void launch_reduce(const Dev &D, const double *in, int64_t n, double *out, hipStream_t st)
{
    (void)D;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, in, n, out);
}

__global__ __launch_bounds__(256) void k_cell_counts(Dev D)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D.nlocal) return;
    int x, y, z;
    local_coords(D, q, x, y, z);
    D.cell_cnt[q] = D.lcount[cell_index(D, x + H, y + H, z + H)];
}

void launch_cell_counts(const Dev &D, hipStream_t st)
{
    hipLaunchKernelGGL(k_cell_counts, dim3((unsigned)((D.nlocal + 255) / 256)), dim3(256), 0, st, D);
}

// ---------------------------------------------------------------------------
// velocity moments, FP64 (textbook definitions).  Sums are taken about a
// reference velocity R of the cell, the centre of the block in the middle of
// its id-sorted list (within a few thermal speeds of the bulk velocity for
// the distributions here), so the pressure tensor
// P = m dv^3 (S2 - S1 S1^T / S0) does not subtract two large raw moments:
//   S0 = sum f, S1 = sum f (v - R), S2 = sum f (v - R)(v - R)^T.
// Work units: the first `chunk` blocks of every local cell, and every further
// chunk of a cell with more blocks (its own unit), so the hot cells of a
// mixture are spread over many wavefronts.  A unit of a cell with one chunk
// writes the cell's moments; the units of a split cell leave ten partial sums
// each, which the cell's combine pass adds in chunk order (the same result in
// every run).  Per block the lanes add f, f k, f k k^T with k the block
// centre's offset from R in units of 4 dv per axis (uniform over the block,
// computed from the two blocks' packed coordinates; the units are applied to
// the sums at the end);
// each lane's offset o within the block enters once at the end:
//   sum f (c + o) = S1c + o S0,  sum f (c+o)(c+o)^T = S2c + S1c o^T + o S1c^T + S0 o o^T.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// packed block coordinates bx | by << 10 | bz << 20
__device__ inline int32_t pack_coords(const Dev &D, int32_t id)
{
    return (id % D.nblk[0]) | (((id / D.nblk[0]) % D.nblk[1]) << 10) | ((id / (D.nblk[0] * D.nblk[1])) << 20);
}

// moments of one cell from its sums about R (lane 0 writes)
__device__ inline void moments_finish(const Dev &D, int64_t q, const double (&S)[10], const double R[3],
                                      double *dn, double *dV, double *dP, double *cell_mass)
{
    const double dv3 = D.dv[0] * D.dv[1] * D.dv[2];
    const double mp = 1.67262192e-27;
    const double s0 = S[0];
    const double nd = dv3 * s0;
    double u[3] = {0.0, 0.0, 0.0};
    if (s0 != 0.0)
        for (int a = 0; a < 3; a++) u[a] = S[1 + a] / s0;
    if (dn) dn[q] = nd;
    if (dV)
        for (int a = 0; a < 3; a++) dV[3 * q + a] = R[a] + u[a];
    if (dP) {
        const double k = mp * dv3;
        dP[6 * q + 0] = k * (S[4] - S[1] * u[0]);
        dP[6 * q + 1] = k * (S[5] - S[2] * u[1]);
        dP[6 * q + 2] = k * (S[6] - S[3] * u[2]);
        dP[6 * q + 3] = k * (S[7] - S[1] * u[1]);
        dP[6 * q + 4] = k * (S[8] - S[1] * u[2]);
        dP[6 * q + 5] = k * (S[9] - S[2] * u[2]);
    }
    cell_mass[q] = nd * D.dx[0] * D.dx[1] * D.dx[2];
}

__device__ inline void reference_velocity(const Dev &D, int32_t idR, int cnt, double R[3], int32_t &pkR)
{
    pkR = cnt > 0 ? pack_coords(D, idR) : 0;
    const int b[3] = {pkR & 1023, (pkR >> 10) & 1023, pkR >> 20};
    for (int a = 0; a < 3; a++) R[a] = cnt > 0 ? D.vmin[a] + (4 * b[a] + 2) * D.dv[a] : 0.0;
}

// counters to zero (a kernel, not a memset, so graph captures replay it
// faithfully)
__global__ __launch_bounds__(256) void k_mom_reset(MomScratch M)
{
    if (threadIdx.x == 0) {
        M.ctr[0] = 0ull;
        M.ctr[1] = 0ull;
    }
}

// per local cell: the partial slots of a split cell and its further chunks
__global__ __launch_bounds__(256) void k_mom_plan(Dev D, MomScratch M)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D.nlocal || failed(D)) return;
    int x, y, z;
    local_coords(D, q, x, y, z);
    const int cnt = D.lcount[cell_index(D, x + H, y + H, z + H)];
    const int nch = (cnt + M.chunk - 1) / M.chunk;
    if (nch <= 1) {
        M.cell_base[q] = -1;
        return;
    }
    const unsigned long long base = atomicAdd(&M.ctr[0], (unsigned long long)nch);
    const unsigned long long eb = atomicAdd(&M.ctr[1], (unsigned long long)(nch - 1));
    if ((int64_t)(base + nch) > M.cap_part || (int64_t)(eb + nch - 1) > M.cap_extra) {
        atomicOr(&D.ctl->err, (unsigned long long)E_MOMENTS);  // not reached: capacities cover any list
        M.cell_base[q] = -1;
        return;
    }
    M.cell_base[q] = (int32_t)base;
    for (int j = 1; j < nch; j++) M.extra[eb + j - 1] = make_int2((int)q, j);
}

// five waves per SIMD for the narrow storage types (95 VGPRs, 37.6 instead of
// 39.5 ms per step on the 128x128x64 BF16 mixture); FP64 keeps the default,
// where five would spill
template <int ST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == VL_F64 ? 4 : 5))) void k_mom_units(
    Dev D, MomScratch M, double *dn, double *dV, double *dP)
{
    if (failed(D)) return;
    const int lane = threadIdx.x & 63;
    // the wavefront's index, made visibly uniform so the unit's cell and its
    // metadata are read with scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nunits = D.nlocal + (int64_t)min(M.ctr[1], (unsigned long long)M.cap_extra);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    // raw storage words, widened when summed (BF16 bits held in 32-bit
    // registers, which the compiler does not pack in pairs)
    using T = typename Storage<ST>::T;
    using RW = typename std::conditional<ST == VL_BF16, uint32_t, T>::type;
    constexpr int NF = 8;  // blocks per group; two groups are in flight
    const uint32_t lane_off = (uint32_t)lane * Storage<ST>::BYTES;
    const uint32_t zslot = (uint32_t)D.trash;  // the all-zero block
    // the lane's velocity offset from its block's centre
    const double o[3] = {((lane & 3) - 1.5) * D.dv[0], (((lane >> 2) & 3) - 1.5) * D.dv[1],
                         ((lane >> 4) - 1.5) * D.dv[2]};
    for (int64_t u = (int64_t)blockIdx.x * 4 + wv; u < nunits; u += nwaves) {
        int64_t q;
        int j;
        if (u < D.nlocal) {
            q = u;
            j = 0;
        } else {
            const int2 e = M.extra[u - D.nlocal];
            q = __builtin_amdgcn_readfirstlane(e.x);
            j = __builtin_amdgcn_readfirstlane(e.y);
        }
        int x, y, z;
        local_coords(D, q, x, y, z);
        const int64_t c = cell_index(D, x + H, y + H, z + H);
        const int cnt = __builtin_amdgcn_readfirstlane(D.lcount[c]);
        const int64_t ls = D.lstart[c];
        double R[3];
        int32_t pkR;
        reference_velocity(D, cnt > 0 ? __builtin_amdgcn_readfirstlane(D.lid[ls + cnt / 2]) : 0, cnt, R, pkR);
        pkR = __builtin_amdgcn_readfirstlane(pkR);
        const int b0 = j * M.chunk, b1 = min(cnt, b0 + M.chunk);
        // sums with the block centre's offset from R in units of 4 dv per
        // axis (k, uniform over the block, from the packed coordinates in
        // scalar registers); the units are applied once per unit below
        double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0}, s2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        auto acc = [&](double f, int32_t pk) {
            const double kx = (double)((pk & 1023) - (pkR & 1023));
            const double ky = (double)(((pk >> 10) & 1023) - ((pkR >> 10) & 1023));
            const double kz = (double)((pk >> 20) - (pkR >> 20));
            const double fx = f * kx, fy = f * ky, fz = f * kz;
            s0 += f;
            s1[0] += fx;
            s1[1] += fy;
            s1[2] += fz;
            s2[0] = fma(fx, kx, s2[0]);
            s2[1] = fma(fy, ky, s2[1]);
            s2[2] = fma(fz, kz, s2[2]);
            s2[3] = fma(fx, ky, s2[3]);
            s2[4] = fma(fx, kz, s2[4]);
            s2[5] = fma(fy, kz, s2[5]);
        };
        for (int g = b0; g < b1; g += 64) {
            // slots and packed coordinates of up to 64 blocks, one per lane;
            // past the list the all-zero block (f = 0 adds nothing)
            const int ng = min(64, b1 - g);
            const uint32_t myslot = lane < ng ? (uint32_t)D.lslot[ls + g + lane] : zslot;
            const int32_t mypk = lane < ng ? pack_coords(D, D.lid[ls + g + lane]) : pkR;
            // groups of NF blocks, the next group's loads issued before the
            // current group is summed (every load is issued: blocks past the
            // 64 read the all-zero block)
            RW ra[NF], rb[NF];
            auto issue = [&](RW (&r)[NF], int k0) {
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    // (read unconditionally, then chosen: a select, not a branch)
                    const int k = k0 + i;
                    const uint32_t rl = (uint32_t)__builtin_amdgcn_readlane((int)myslot, k & 63);
                    const uint32_t sl = k < 64 ? rl : zslot;
                    r[i] = block_load_raw<ST>(block_rsrc<ST>(D.pool, sl), lane_off);
                }
            };
            auto take = [&](const RW (&r)[NF], int k0) {
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    const int k = k0 + i;
                    const int32_t rl = __builtin_amdgcn_readlane(mypk, k & 63);
                    acc(Storage<ST>::widen((T)r[i]), k < 64 ? rl : pkR);
                }
            };
            // (scheduling barriers keep each group's loads where they are
            // issued, ahead of the other group's sums)
            issue(ra, 0);
            for (int k0 = 0; k0 < ng; k0 += 2 * NF) {
                issue(rb, k0 + NF);
                __builtin_amdgcn_sched_barrier(0);
                take(ra, k0);
                __builtin_amdgcn_sched_barrier(0);
                issue(ra, k0 + 2 * NF);
                __builtin_amdgcn_sched_barrier(0);
                take(rb, k0 + NF);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // the block offsets' units (4 dv per axis)
        const double ux = 4.0 * D.dv[0], uy = 4.0 * D.dv[1], uz = 4.0 * D.dv[2];
        s1[0] *= ux;
        s1[1] *= uy;
        s1[2] *= uz;
        s2[0] *= ux * ux;
        s2[1] *= uy * uy;
        s2[2] *= uz * uz;
        s2[3] *= ux * uy;
        s2[4] *= ux * uz;
        s2[5] *= uy * uz;
        // the lane's offset within its block, then the sums over the lanes
        double S[10];
        S[0] = s0;
        for (int a = 0; a < 3; a++) S[1 + a] = s1[a] + o[a] * s0;
        S[4] = s2[0] + 2.0 * o[0] * s1[0] + o[0] * o[0] * s0;
        S[5] = s2[1] + 2.0 * o[1] * s1[1] + o[1] * o[1] * s0;
        S[6] = s2[2] + 2.0 * o[2] * s1[2] + o[2] * o[2] * s0;
        S[7] = s2[3] + o[0] * s1[1] + o[1] * s1[0] + o[0] * o[1] * s0;
        S[8] = s2[4] + o[0] * s1[2] + o[2] * s1[0] + o[0] * o[2] * s0;
        S[9] = s2[5] + o[1] * s1[2] + o[2] * s1[1] + o[1] * o[2] * s0;
        for (int i = 0; i < 10; i++) S[i] = wave_sum_d(S[i]);
        const int32_t base = M.cell_base[q];
        if (base < 0) {
            if (lane == 0) moments_finish(D, q, S, R, dn, dV, dP, M.cell_mass);
        } else if (lane < 10) {
            double v = S[0];
            for (int i = 1; i < 10; i++) v = (lane == i) ? S[i] : v;
            M.part[((int64_t)base + j) * 10 + lane] = v;
        }
    }
}

// per split cell: its chunks' partial sums added in chunk order
__global__ __launch_bounds__(256) void k_mom_combine(Dev D, MomScratch M, double *dn, double *dV, double *dP)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D.nlocal || failed(D)) return;
    const int32_t base = M.cell_base[q];
    if (base < 0) return;
    int x, y, z;
    local_coords(D, q, x, y, z);
    const int64_t c = cell_index(D, x + H, y + H, z + H);
    const int cnt = D.lcount[c];
    const int nch = (cnt + M.chunk - 1) / M.chunk;
    double S[10];
    for (int i = 0; i < 10; i++) S[i] = 0.0;
    for (int j = 0; j < nch; j++)
        for (int i = 0; i < 10; i++) S[i] += M.part[((int64_t)base + j) * 10 + i];
    double R[3];
    int32_t pkR;
    reference_velocity(D, D.lid[D.lstart[c] + cnt / 2], cnt, R, pkR);
    moments_finish(D, q, S, R, dn, dV, dP, M.cell_mass);
}

template <typename K>
static unsigned resident_groups(K kernel)
{
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || per < 1) per = 1;
    return (unsigned)(per * ncu);
}

template <int ST>
static void launch_mom_units(const Dev &D, const MomScratch &M, double *dn, double *dV, double *dP, hipStream_t st)
{
    static const unsigned g = resident_groups(k_mom_units<ST>);
    hipLaunchKernelGGL(k_mom_units<ST>, dim3(g), dim3(256), 0, st, D, M, dn, dV, dP);
}

void launch_moments(const Dev &D, const MomScratch &M, double *dn, double *dV, double *dP, hipStream_t st)
{
    if (D.nlocal <= 0) return;
    const dim3 gc((unsigned)((D.nlocal + 255) / 256));
    hipLaunchKernelGGL(k_mom_reset, dim3(1), dim3(256), 0, st, M);
    hipLaunchKernelGGL(k_mom_plan, gc, dim3(256), 0, st, D, M);
    switch (D.storage) {
    case VL_F64: launch_mom_units<VL_F64>(D, M, dn, dV, dP, st); break;
    case VL_F32: launch_mom_units<VL_F32>(D, M, dn, dV, dP, st); break;
    default: launch_mom_units<VL_BF16>(D, M, dn, dV, dP, st); break;
    }
    hipLaunchKernelGGL(k_mom_combine, gc, dim3(256), 0, st, D, M, dn, dV, dP);
}

// ---------------------------------------------------------------------------
// the allocation-free moments entry point's scratch: a fixed array in device
// memory (one per device the library runs on, held until the process ends).
// Host code never passes the array's name to a kernel: it takes the array's
// device address once per device with hipGetSymbolAddress and passes that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_MOMENTS_SCRATCH_BYTES];

int static_moments_scratch(void **ptr)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *addr[MAXDEV] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return -1;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return -1;
        addr[dev] = a;
    }
    *ptr = addr[dev];
    return 0;
}

int64_t moments_scratch_bytes(int64_t nlocal, int64_t parts, int64_t extras)
{
    auto al = [](int64_t v) { return (v + 255) / 256 * 256; };
    return al(16) + al(nlocal * 4) + al(nlocal * 8) + al(parts * 80) + al(extras * 8);
}

MomScratch carve_moments_scratch(void *base, int64_t nlocal, int64_t parts, int64_t extras, int chunk)
{
    auto al = [](int64_t v) { return (v + 255) / 256 * 256; };
    char *w = (char *)base;
    MomScratch M;
    M.ctr = (unsigned long long *)w;          w += al(16);
    M.cell_base = (int32_t *)w;               w += al(nlocal * 4);
    M.cell_mass = (double *)w;                w += al(nlocal * 8);
    M.part = (double *)w;                     w += al(parts * 80);
    M.extra = (int2 *)w;
    M.cap_part = parts;
    M.cap_extra = extras;
    M.chunk = chunk;
    return M;
}

// gather blocks (by slot) into a dense FP64 array, one wavefront per block
template <int ST>
__global__ __launch_bounds__(256) void k_gather(Dev D, const int32_t *slots, int64_t n, double *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n) return;
    const int64_t slot = slots[b];
    out[b * BLK + lane] = Storage<ST>::load(D.pool, slot * BLK + lane);
}

void launch_gather(const Dev &D, const int32_t *slots, int64_t n, double *out, hipStream_t st)
{
    if (n <= 0) return;
    dim3 g((unsigned)((n + 3) / 4));
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_gather<VL_F64>, g, dim3(256), 0, st, D, slots, n, out); break;
    case VL_F32: hipLaunchKernelGGL(k_gather<VL_F32>, g, dim3(256), 0, st, D, slots, n, out); break;
    default: hipLaunchKernelGGL(k_gather<VL_BF16>, g, dim3(256), 0, st, D, slots, n, out); break;
    }
}

}  // namespace vl
