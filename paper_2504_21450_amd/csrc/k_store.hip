// Block-store kernels: allocator book-keeping, the ghost update (periodic
// image copy of block lists and payloads), per-cell mass, deterministic
// reductions and the FP64 velocity moments.
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
__global__ __launch_bounds__(256) void k_fill(Dev D, int lo0, int lo1, int lo2, int e0, int e1, int e2)
{
    using SW = typename Storage<ST>::Word;
    constexpr int WPB = Storage<ST>::WORDS_PER_BLOCK;  // words per block (<= 64)
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t total = (int64_t)e0 * e1 * e2;
    if (w >= total) return;
    const int x = lo0 + (int)(w % e0);
    const int y = lo1 + (int)((w / e0) % e1);
    const int z = lo2 + (int)(w / ((int64_t)e0 * e1));
    if (is_local(D, x, y, z)) return;
    const int64_t c = cell_index(D, x, y, z);
    const int64_t s = cell_index(D, wrap_coord(x, D.n[0]), wrap_coord(y, D.n[1]), wrap_coord(z, D.n[2]));
    const int cnt = D.lcount[s];
    const int64_t ss = D.lstart[s];
    const int cap = cnt + cnt / 4 + 32;
    unsigned long long lb = 0, sb = 0;
    if (lane == 0) {
        lb = atomicAdd(&D.ctl->ghost_list_top, (unsigned long long)cap);
        sb = atomicAdd(&D.ctl->ghost_top, (unsigned long long)cnt);
    }
    lb = __shfl(lb, 0);
    sb = __shfl(sb, 0);
    const bool lok = (int64_t)(lb + cap) <= D.reg_cap[2];
    const bool sok = (int64_t)(sb + cnt) <= D.gcap;
    if (!lok || !sok) {
        if (lane == 0) {
            atomicOr(&D.ctl->err, (unsigned long long)((lok ? 0 : E_GHOST_LIST) | (sok ? 0 : E_GHOST_SLOTS)));
            D.lstart[c] = D.reg_off[2];
            D.lcount[c] = 0;
            D.lcapa[c] = 0;
        }
        return;
    }
    const int64_t ls = D.reg_off[2] + (int64_t)lb;
    const int64_t gslot0 = D.lcap + (int64_t)sb;
    if (lane == 0) {
        D.lstart[c] = ls;
        D.lcount[c] = cnt;
        D.lcapa[c] = cap;
    }
    for (int e = lane; e < cnt; e += 64) {
        D.lid[ls + e] = D.lid[ss + e];
        D.lslot[ls + e] = (int32_t)(gslot0 + e);
    }
    SW *pool = (SW *)D.pool;
    int e = 0;
    if (lane < WPB) {
        for (; e + 4 <= cnt; e += 4) {
            int64_t s0 = D.lslot[ss + e], s1 = D.lslot[ss + e + 1];
            int64_t s2 = D.lslot[ss + e + 2], s3 = D.lslot[ss + e + 3];
            SW v0 = pool[s0 * WPB + lane], v1 = pool[s1 * WPB + lane];
            SW v2 = pool[s2 * WPB + lane], v3 = pool[s3 * WPB + lane];
            pool[(gslot0 + e) * WPB + lane] = v0;
            pool[(gslot0 + e + 1) * WPB + lane] = v1;
            pool[(gslot0 + e + 2) * WPB + lane] = v2;
            pool[(gslot0 + e + 3) * WPB + lane] = v3;
        }
        for (; e < cnt; e++) {
            int64_t s0 = D.lslot[ss + e];
            pool[(gslot0 + e) * WPB + lane] = pool[s0 * WPB + lane];
        }
    }
}

void launch_fill(const Dev &D, const int lo[3], const int hi[3], hipStream_t st)
{
    int e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    int64_t waves = (int64_t)e0 * e1 * e2;
    if (waves <= 0) return;
    dim3 g((unsigned)((waves + 3) / 4));
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_fill<VL_F64>, g, dim3(256), 0, st, D, lo[0], lo[1], lo[2], e0, e1, e2); break;
    case VL_F32: hipLaunchKernelGGL(k_fill<VL_F32>, g, dim3(256), 0, st, D, lo[0], lo[1], lo[2], e0, e1, e2); break;
    default: hipLaunchKernelGGL(k_fill<VL_BF16>, g, dim3(256), 0, st, D, lo[0], lo[1], lo[2], e0, e1, e2); break;
    }
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
    if (q >= D.nlocal) return;
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
// velocity moments, FP64.  One wavefront per local cell.  Per block the wave
// reduces sum f, sum f o and sum f o o^T with o the velocity relative to the
// block centre (|o| <= 1.5 dv, no cancellation); blocks are then merged into
// the cell's count / mean / scatter with the pairwise update of Chan, Golub &
// LeVeque (1979), so the pressure tensor never subtracts large raw moments.
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void k_moments(Dev D, double *dn, double *dV, double *dP)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= D.nlocal) return;
    int x, y, z;
    local_coords(D, q, x, y, z);
    const int64_t c = cell_index(D, x + H, y + H, z + H);
    const int cnt = D.lcount[c];
    const int64_t ls = D.lstart[c];
    const double o0 = ((lane & 3) - 1.5) * D.dv[0];
    const double o1 = (((lane >> 2) & 3) - 1.5) * D.dv[1];
    const double o2 = ((lane >> 4) - 1.5) * D.dv[2];
    double n = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    double M[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < cnt; e++) {
        const int32_t b = D.lid[ls + e];
        const int64_t slot = D.lslot[ls + e];
        const double f = Storage<ST>::load(D.pool, slot * BLK + lane);
        double s0 = wave_sum(f);
        if (s0 == 0.0) continue;
        double s1x = wave_sum(f * o0), s1y = wave_sum(f * o1), s1z = wave_sum(f * o2);
        double sxx = wave_sum(f * o0 * o0), syy = wave_sum(f * o1 * o1), szz = wave_sum(f * o2 * o2);
        double sxy = wave_sum(f * o0 * o1), sxz = wave_sum(f * o0 * o2), syz = wave_sum(f * o1 * o2);
        const int bx = b % D.nblk[0], by = (b / D.nblk[0]) % D.nblk[1], bz = b / (D.nblk[0] * D.nblk[1]);
        const double cbx = D.vmin[0] + (4 * bx + 2) * D.dv[0];
        const double cby = D.vmin[1] + (4 * by + 2) * D.dv[1];
        const double cbz = D.vmin[2] + (4 * bz + 2) * D.dv[2];
        const double ux = s1x / s0, uy = s1y / s0, uz = s1z / s0;  // block mean - block centre
        const double Bxx = sxx - s1x * ux, Byy = syy - s1y * uy, Bzz = szz - s1z * uz;
        const double Bxy = sxy - s1x * uy, Bxz = sxz - s1x * uz, Byz = syz - s1y * uz;
        const double nn = n + s0;
        const double dx_ = (cbx + ux) - m0, dy_ = (cby + uy) - m1, dz_ = (cbz + uz) - m2;
        const double wgt = s0 / nn;
        const double cw = n * wgt;  // n s0 / (n + s0)
        m0 += dx_ * wgt;
        m1 += dy_ * wgt;
        m2 += dz_ * wgt;
        M[0] += Bxx + dx_ * dx_ * cw;
        M[1] += Byy + dy_ * dy_ * cw;
        M[2] += Bzz + dz_ * dz_ * cw;
        M[3] += Bxy + dx_ * dy_ * cw;
        M[4] += Bxz + dx_ * dz_ * cw;
        M[5] += Byz + dy_ * dz_ * cw;
        n = nn;
    }
    if (lane == 0) {
        const double dv3 = D.dv[0] * D.dv[1] * D.dv[2];
        const double mp = 1.67262192e-27;
        const double nd = dv3 * n;
        if (dn) dn[q] = nd;
        if (dV) {
            dV[3 * q + 0] = m0;
            dV[3 * q + 1] = m1;
            dV[3 * q + 2] = m2;
        }
        if (dP)
            for (int k = 0; k < 6; k++) dP[6 * q + k] = mp * dv3 * M[k];
        D.cell_red[q] = nd * D.dx[0] * D.dx[1] * D.dx[2];
    }
}

void launch_moments(const Dev &D, double *dn, double *dV, double *dP, hipStream_t st)
{
    dim3 g((unsigned)((D.nlocal + 3) / 4));
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_moments<VL_F64>, g, dim3(256), 0, st, D, dn, dV, dP); break;
    case VL_F32: hipLaunchKernelGGL(k_moments<VL_F32>, g, dim3(256), 0, st, D, dn, dV, dP); break;
    default: hipLaunchKernelGGL(k_moments<VL_BF16>, g, dim3(256), 0, st, D, dn, dV, dP); break;
    }
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
