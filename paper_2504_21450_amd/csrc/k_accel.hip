// Acceleration step: the Lorentz-force term of the Vlasov equation over one
// time step (Section 2, eq. 1; the velocity-space half of the split step),
// as the three one-coordinate remaps of SLICE-3D (Zerroukat & Allen 2012).
//
// In fields E, B that are constant over the step every velocity moves along
// the exact characteristic of dv/dt = (q/m)(E + v x B): the affine map
// v' = A v + c with A the rotation by -(q/m)|B| dt about B/|B| (Rodrigues)
// and c = (I - A) vE + (q/m)(E.b) dt b (vE = E x B / |B|^2; with B = 0,
// v' = v + (q/m) E dt).  SLICE-3D writes the map as three maps that each set
// one coordinate to its final value as an affine function of the current
// coordinates (rows of the homogeneous form times the inverses of the maps
// before), so the three compose to the map exactly.  Each is a remap of every
// velocity column along its axis: a column moves by u -> alpha u + sigma in
// cell units, and cell i receives the mass of its pre-image under the CW84
// parabolas of the column (the slopes, faces and limiter of the spatial
// remap), cells outside the velocity mesh reading as zero.
//
// k_accel_factors: per local cell, the three maps (12 doubles) and a flag if a
//   map cannot be split (its own coefficient not positive).
// k_accel: one workgroup per local cell runs the three remaps in turn.  Per
//   remap, along axis d:
//   * the cell's block set is an LDS bitmap; a block column (fixed block
//     coordinates across d) spans from its lowest to its highest block,
//     widened to where its image can reach (the map of the column's extent
//     with the extreme shifts of its 16 velocity columns, one cell of margin);
//   * blocks of that span missing from the cell are created: slots from the
//     free ring, entries merged into the sorted list (in place from the end,
//     or into a larger place when the list outgrows it);
//   * the workgroup remaps one block column at a time: it stages the column
//     in LDS (16 velocity columns x its span, missing blocks as zero; eight
//     blocks' loads in flight per wavefront), the limited parabola edges of
//     every cell once (runs of consecutive cells per thread, each slope
//     computed once), then the new averages, writing every block of the
//     span, 64 lanes = the block's 64 cells, so loads and stores are
//     coalesced;
//   * the last remap leaves per list entry the flags the pruning reads:
//     bit 0 a value >= the content threshold, bit 1 a nonzero value, bit 2
//     created by this step.
//   Blocks created but left all zero are dropped by the pruning (as the new
//   block set is the old one plus every block holding a nonzero value).
#include <algorithm>

#include "vl_internal.h"
#include "vl_storage.h"

namespace vl {

struct AccelParams {
    const double *fields;  // per local cell Ex, Ey, Ez, Bx, By, Bz
    double *maps;          // per local cell 3 x 4 map rows (ACC_MAP doubles)
    int *bad;              // set if some cell's map cannot be split
    double qm, dt;
    int order[3];
    int cur;               // local list region in use
    int ncols;             // block columns of the widest cross-section
    int hc;                // staging cells per velocity column (4 max nblk)
};

constexpr int ACC_MAP = ACC_MAP_DOUBLES;

// ---------------------------------------------------------------------------
// per-cell maps
// ---------------------------------------------------------------------------
// identity with row d replaced by `row`, inverted (4x4 homogeneous)
__device__ inline void inv_row_step(const double *row, int d, double (&Mi)[4][4])
{
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) Mi[i][j] = (i == j) ? 1.0 : 0.0;
    for (int j = 0; j < 4; j++) Mi[d][j] = (j == d) ? 1.0 / row[d] : -row[j] / row[d];
}

__device__ inline void row_mul(const double *row, const double (&M)[4][4], double *out)
{
    for (int j = 0; j < 4; j++) {
        double s = 0.0;
        for (int i = 0; i < 4; i++) s += row[i] * M[i][j];
        out[j] = s;
    }
}

__global__ __launch_bounds__(256) void k_accel_factors(Dev D, AccelParams ap)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= D.nlocal) return;
    const double *EB = ap.fields + 6 * q;
    const double E[3] = {EB[0], EB[1], EB[2]}, B[3] = {EB[3], EB[4], EB[5]};
    double T[3][4];
    const double Bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    if (Bm == 0.0) {
        for (int i = 0; i < 3; i++) {
            for (int j = 0; j < 3; j++) T[i][j] = (i == j) ? 1.0 : 0.0;
            T[i][3] = ap.qm * E[i] * ap.dt;
        }
    } else {
        const double b[3] = {B[0] / Bm, B[1] / Bm, B[2] / Bm};
        const double th = -ap.qm * Bm * ap.dt;
        double si, co;
        sincos(th, &si, &co);
        // [b]x: the matrix of v -> b x v
        const double K[3][3] = {{0.0, -b[2], b[1]}, {b[2], 0.0, -b[0]}, {-b[1], b[0], 0.0}};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) T[i][j] = ((i == j) ? co : 0.0) + si * K[i][j] + (1.0 - co) * b[i] * b[j];
        const double B2 = Bm * Bm;
        const double vE[3] = {(E[1] * B[2] - E[2] * B[1]) / B2, (E[2] * B[0] - E[0] * B[2]) / B2,
                              (E[0] * B[1] - E[1] * B[0]) / B2};
        const double Epar = E[0] * b[0] + E[1] * b[1] + E[2] * b[2];
        for (int i = 0; i < 3; i++) {
            const double Av = T[i][0] * vE[0] + T[i][1] * vE[1] + T[i][2] * vE[2];
            T[i][3] = vE[i] - Av + ap.qm * Epar * ap.dt * b[i];
        }
    }
    // the three one-coordinate maps in the slice order
    const int o0 = ap.order[0], o1 = ap.order[1], o2 = ap.order[2];
    double r0[4], r1[4], r2[4], t[4];
    double I0[4][4], I1[4][4];
    for (int j = 0; j < 4; j++) r0[j] = T[o0][j];
    bool ok = r0[o0] > 0.0;
    inv_row_step(r0, o0, I0);
    row_mul(T[o1], I0, r1);
    ok = ok && r1[o1] > 0.0;
    inv_row_step(r1, o1, I1);
    row_mul(T[o2], I0, t);
    row_mul(t, I1, r2);
    ok = ok && r2[o2] > 0.0;
    double *m = ap.maps + ACC_MAP * q;
    for (int j = 0; j < 4; j++) {
        m[j] = r0[j];
        m[4 + j] = r1[j];
        m[8 + j] = r2[j];
    }
    if (!ok) *ap.bad = 1;
}

// ---------------------------------------------------------------------------
// column remap
// ---------------------------------------------------------------------------
// limited slope of cell j of a column (CW84 eq. 1.7-1.8) from its average
// a0 and its neighbours' am, ap: the central difference, limited to twice
// either one-sided difference, zero at an extremum
__device__ __forceinline__ double col_slope(double am, double a0, double ap)
{
    const double dl = a0 - am, dr = ap - a0;
    const double central = 0.5 * (ap - am);
    const double m = fmin(fabs(central), fmin(2.0 * fabs(dl), 2.0 * fabs(dr)));
    return (dr * dl > 0.0) ? copysign(m, central) : 0.0;
}

// limited parabola edges (l, r) of a cell from its average a0, its
// neighbours' am, ap and the limited slopes dm, d0, dp of cells j-1, j, j+1
// (CW84 eq. 1.6 faces, then the eq. 1.10 limiter)
__device__ __forceinline__ void col_edges(double am, double a0, double ap, double dm, double d0, double dp,
                                          double &l, double &r)
{
    constexpr double SIXTH = 1.0 / 6.0;
    l = am + 0.5 * (a0 - am) - (d0 - dm) * SIXTH;
    r = a0 + 0.5 * (ap - a0) - (dp - d0) * SIXTH;
    if ((r - a0) * (a0 - l) <= 0.0) {
        l = a0;
        r = a0;
    } else {
        const double dd = r - l;
        const double mm = a0 - 0.5 * (l + r);
        if (dd * mm > dd * dd * SIXTH)
            l = 3.0 * a0 - 2.0 * r;
        else if (-(dd * dd) * SIXTH > dd * mm)
            r = 3.0 * a0 - 2.0 * l;
    }
}

// mass of source cell j's limited parabola (average a0, edges l, r: CW84
// eq. 1.10's profile) over [0, x] of the cell (0 <= x <= 1, cell units)
__device__ __forceinline__ double col_head(double a0, double l, double r, double x)
{
    constexpr double THIRD = 1.0 / 3.0;
    const double a6 = 6.0 * (a0 - 0.5 * (l + r));
    const double q = 0.5 * ((r - l) + a6);
    return x * (l + x * (q - x * a6 * THIRD));
}

// new average of cell i of a column moved by u -> alpha u + sigma (inv_alpha =
// 1 / alpha): the mass of its pre-image [(i - sigma)/alpha, (i + 1 - sigma)/alpha]
// under the source parabolas, as the tail of the first source cell it meets
// (the cell's average minus its head), the averages of the cells it covers
// whole, and the head of the last; cells outside [base, base + ncell) (the
// staged span) hold zero, and so does all of the mesh beyond it
template <typename A, typename E>
__device__ __forceinline__ double col_remap_cell(const A &a, const E &edges, int base, int ncell, int i,
                                                 double inv_alpha, double sigma)
{
    double lo = ((double)i - sigma) * inv_alpha, hi = ((double)i + 1.0 - sigma) * inv_alpha;
    if (!(hi > (double)base) || !(lo < (double)(base + ncell))) return 0.0;
    lo = fmax(lo, (double)(base - 1));
    hi = fmin(hi, (double)(base + ncell + 1));
    const double fl = floor(lo), fh = floor(hi);
    const int j0 = (int)fl, j1 = (int)fh;
    const double xa = lo - fl, xb = hi - fh;
    double l, r;
    edges(j0, l, r);
    const double a0 = a(j0);
    if (j0 == j1) return col_head(a0, l, r, xb) - col_head(a0, l, r, xa);
    double m = a0 - col_head(a0, l, r, xa);
    for (int j = j0 + 1; j < j1; j++) m += a(j);
    if (xb > 0.0) {
        edges(j1, l, r);
        m += col_head(a(j1), l, r, xb);
    }
    return m;
}

// shift sigma (cell units) of the velocity column at transverse velocity
// indices (i1, i2) under map row `row` along d
__device__ inline double col_sigma(const Dev &D, const double *row, int d, int e1, int e2, int i1, int i2)
{
#pragma clang fp contract(off)
    const double w1 = D.vmin[e1] + ((double)i1 + 0.5) * D.dv[e1];
    const double w2 = D.vmin[e2] + ((double)i2 + 0.5) * D.dv[e2];
    const double s = row[e1] * w1 + row[e2] * w2 + row[3];
    return ((row[d] - 1.0) * D.vmin[d] + s) / D.dv[d];
}

__device__ inline int32_t compose_id(const Dev &D, int d, int e1, int e2, int bd, int b1, int b2)
{
    int c[3];
    c[d] = bd;
    c[e1] = b1;
    c[e2] = b2;
    return c[0] + D.nblk[0] * (c[1] + D.nblk[1] * c[2]);
}

__device__ inline bool has_bit(const uint32_t *bm, int32_t id) { return (bm[id >> 5] >> (id & 31)) & 1u; }

__device__ inline int rank_of(const uint32_t *bm, const int *rk, int32_t id)
{
    return rk[id >> 5] + __popc(bm[id >> 5] & ((1u << (id & 31)) - 1u));
}

// exclusive scan of a[0..n) in place by the workgroup; returns the total
__device__ int acc_scan(int *a, int n, int *s_tmp)
{
    const int tid = threadIdx.x;
    const int per = (n + 255) / 256;
    const int b = min(tid * per, n), e = min(b + per, n);
    int sum = 0;
    for (int i = b; i < e; i++) sum += a[i];
    s_tmp[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = (tid >= o) ? s_tmp[tid - o] : 0;
        __syncthreads();
        s_tmp[tid] += v;
        __syncthreads();
    }
    int run = s_tmp[tid] - sum;
    const int total = s_tmp[255];
    for (int i = b; i < e; i++) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

template <int ST>
__global__ __launch_bounds__(256) void k_accel(Dev D, AccelParams ap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_tmp[256];
    __shared__ double s_map[ACC_MAP];
    __shared__ int s_cnt[4];
    __shared__ long long s_at[2];
    __shared__ unsigned long long s_ring;
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = D.W;
    uint32_t *s_bm = (uint32_t *)smem;     // current block set
    uint32_t *s_old = s_bm + W;            // the set before this remap
    uint32_t *s_start = s_old + W;         // the set before this step
    int *s_rank = (int *)(s_start + W);    // W + 1
    int *s_span = s_rank + (W + 1);        // per block column: lo | hi << 16, or -1
    int *s_new = s_span + ap.ncols;        // per block column: blocks created (then their prefix)
    // per wavefront: the block column it remaps, 16 velocity columns of
    // hc + 1 cells (odd stride: fewer bank conflicts), and the slots of the
    // column's blocks
    // (byte offsets from the LDS array itself, so the compiler keeps these
    // pointers in the LDS address space): the block column being remapped,
    // averages and limited edges of 16 velocity columns of hc + 1 cells (odd
    // stride: fewer bank conflicts)
    const int hcs = ap.hc + 1;
    const int stage_off = (4 * (3 * W + (W + 1) + 2 * ap.ncols) + 15) & ~15;
    double *s_a = (double *)(smem + stage_off);
    double *s_l = s_a + 16 * hcs;
    double *s_r = s_l + 16 * hcs;

    const int64_t q = blockIdx.x;
    const int x = (int)(q % D.n[0]), y = (int)((q / D.n[0]) % D.n[1]), z = (int)(q / ((int64_t)D.n[0] * D.n[1]));
    const int64_t c = cell_index(D, x + H, y + H, z + H);
    if (tid < ACC_MAP) s_map[tid] = ap.maps[ACC_MAP * q + tid];
    if (tid == 0) {
        s_fail = failed(D) ? 1 : 0;
        s_at[0] = D.lstart[c];
        s_cnt[0] = D.lcount[c];
        s_cnt[1] = D.lcapa[c];
    }
    for (int w = tid; w < W; w += 256) s_bm[w] = 0u;
    __syncthreads();
    if (s_fail) return;
    {
        const int cnt = s_cnt[0];
        const int64_t cs = s_at[0];
        for (int e = tid; e < cnt; e += 256) {
            const int32_t id = D.lid[cs + e];
            atomicOr(&s_bm[id >> 5], 1u << (id & 31));
        }
    }
    __syncthreads();
    for (int w = tid; w < W; w += 256) s_start[w] = s_bm[w];

    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    for (int k = 0; k < 3; k++) {
        const int d = ap.order[k];
        const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
        const int nbd = D.nblk[d], nb1 = D.nblk[e1], nb2 = D.nblk[e2];
        const int N = 4 * nbd;
        const int ncol = nb1 * nb2;
        const double *row = s_map + 4 * k;
        const double alpha = row[d];
        for (int w = tid; w < W; w += 256) s_old[w] = s_bm[w];
        __syncthreads();
        // 1. span of every block column and the blocks it lacks
        for (int col = tid; col < ncol; col += 256) {
            const int b1 = col % nb1, b2 = col / nb1;
            int bmin = -1, bmax = -1;
            for (int bd = 0; bd < nbd; bd++)
                if (has_bit(s_bm, compose_id(D, d, e1, e2, bd, b1, b2))) {
                    if (bmin < 0) bmin = bd;
                    bmax = bd;
                }
            if (bmin < 0) {
                s_span[col] = -1;
                s_new[col] = 0;
                continue;
            }
            // extreme shifts: sigma is affine in the velocity column, so at
            // the corners of the block column's 4 x 4
            double smin = 1e300, smax = -1e300;
            for (int u = 0; u < 4; u++) {
                const double s = col_sigma(D, row, d, e1, e2, 4 * b1 + 3 * (u & 1), 4 * b2 + 3 * (u >> 1));
                smin = fmin(smin, s);
                smax = fmax(smax, s);
            }
            // cells that can receive mass from [4 bmin, 4 bmax + 4): those
            // with alpha u0 + sigma - 1 < i < alpha u1 + sigma (a cell of margin)
            const double ilo = floor(alpha * (4.0 * bmin) + smin) - 1.0;
            const double ihi = ceil(alpha * (4.0 * bmax + 4.0) + smax);
            int lo = bmin, hi = bmax;
            if (ihi >= 0.0 && ilo <= (double)(N - 1)) {
                const int i0 = (int)fmax(ilo, 0.0), i1 = (int)fmin(ihi, (double)(N - 1));
                lo = min(lo, i0 >> 2);
                hi = max(hi, i1 >> 2);
            }
            int nn = 0;
            for (int bd = lo; bd <= hi; bd++) nn += has_bit(s_bm, compose_id(D, d, e1, e2, bd, b1, b2)) ? 0 : 1;
            s_span[col] = lo | (hi << 16);
            s_new[col] = nn;
        }
        __syncthreads();
        const int T = acc_scan(s_new, ncol, s_tmp);
        // 2. places: slots for the created blocks, a larger list place if needed
        if (tid == 0) {
            const int cnt = s_cnt[0], cap = s_cnt[1];
            unsigned long long err = 0;
            s_at[1] = s_at[0];
            if (T > 0) {
                const unsigned long long nb = atomicAdd(&D.ctl->ring_head, (unsigned long long)T);
                if (nb + T > D.ctl->ring_limit) err |= E_RING;
                s_ring = nb;
                if (cnt + T > cap) {
                    const int ncap = (cnt + T) + (cnt + T) / 2 + 32;
                    const unsigned long long nb0 = atomicAdd(&D.ctl->list_top[ap.cur], (unsigned long long)ncap);
                    if ((int64_t)(nb0 + ncap) > D.reg_cap[ap.cur]) err |= E_LOCAL_LIST;
                    s_at[1] = D.reg_off[ap.cur] + (int64_t)nb0;
                    s_cnt[1] = ncap;
                }
            }
            if (err) atomicOr(&D.ctl->err, err);
            s_fail = err ? 1 : 0;
        }
        __syncthreads();
        if (s_fail) return;  // the partition is reported as failed; nothing is read again
        const int64_t cs = s_at[0], ns = s_at[1];
        const int cnt = s_cnt[0];
        if (T > 0) {
            // 3. the created blocks join the set; the list is merged in id
            //    order (old entries move up to their new rank, from the end
            //    so that no entry is overwritten before it is read)
            for (int col = tid; col < ncol; col += 256) {
                const int sp = s_span[col];
                if (sp < 0) continue;
                const int b1 = col % nb1, b2 = col / nb1;
                for (int bd = sp & 0xffff; bd <= (sp >> 16); bd++) {
                    const int32_t id = compose_id(D, d, e1, e2, bd, b1, b2);
                    if (!has_bit(s_old, id)) atomicOr(&s_bm[id >> 5], 1u << (id & 31));
                }
            }
            __syncthreads();
            for (int w = tid; w < W; w += 256) s_rank[w] = __popc(s_bm[w]);
            __syncthreads();
            acc_scan(s_rank, W, s_tmp);
            for (int e_hi = cnt; e_hi > 0; e_hi -= 256) {
                const int e = e_hi - 1 - tid;
                int32_t id = 0, slot = 0;
                if (e >= 0) {
                    id = D.lid[cs + e];
                    slot = D.lslot[cs + e];
                }
                __syncthreads();
                if (e >= 0) {
                    const int pos = rank_of(s_bm, s_rank, id);
                    if (ns != cs || pos != e) {
                        D.lid[ns + pos] = id;
                        D.lslot[ns + pos] = slot;
                    }
                }
                __syncthreads();
            }
            for (int col = tid; col < ncol; col += 256) {
                const int sp = s_span[col];
                if (sp < 0) continue;
                const int b1 = col % nb1, b2 = col / nb1;
                int kk = s_new[col];
                for (int bd = sp & 0xffff; bd <= (sp >> 16); bd++) {
                    const int32_t id = compose_id(D, d, e1, e2, bd, b1, b2);
                    if (has_bit(s_old, id)) continue;
                    const int32_t slot = D.ring[(int64_t)((s_ring + kk) % (unsigned long long)D.lcap)];
                    kk++;
                    const int pos = rank_of(s_bm, s_rank, id);
                    D.lid[ns + pos] = id;
                    D.lslot[ns + pos] = slot;
                }
            }
            __syncthreads();
            if (tid == 0) {
                s_cnt[0] = cnt + T;
                s_at[0] = ns;
                D.lstart[c] = ns;
                D.lcount[c] = cnt + T;
                D.lcapa[c] = s_cnt[1];
                D.lsorted[c] = cnt + T;
            }
        } else {
            for (int w = tid; w < W; w += 256) s_rank[w] = __popc(s_bm[w]);
            __syncthreads();
            acc_scan(s_rank, W, s_tmp);
        }
        // 4. remap the block columns one at a time, the workgroup together:
        //    wavefront w stages the blocks lo + w, lo + w + 4, .. (slots and
        //    values of up to eight in flight together), the workgroup computes
        //    the limited edges of every cell once, then wavefront w writes the
        //    new averages of its blocks (64 lanes = a block's 64 cells)
        const bool last = k == 2;
        const double inv_alpha = 1.0 / alpha;
        const int ld = (d == 0) ? lx : (d == 1) ? ly : lz;
        const int l1 = (e1 == 0) ? lx : ly, l2 = (e2 == 1) ? ly : lz;
        const int cc = l1 + 4 * l2;
        for (int col = 0; col < ncol; col++) {
            const int sp = s_span[col];
            if (sp < 0) continue;
            const int lo = sp & 0xffff, hi = sp >> 16;
            const int b1 = col % nb1, b2 = col / nb1;
            const int ncell = 4 * (hi - lo + 1);
            const int nmine = (hi - lo >= wv) ? (hi - lo - wv) / 4 + 1 : 0;  // blocks of this wavefront
            // lane u finds the slot of the wavefront's block u (at most
            // hc / 16 + 1 < 64 of them): negative if the block was created in
            // this remap (it reads as zero)
            int32_t code = -1;
            if (lane < nmine) {
                const int32_t id = compose_id(D, d, e1, e2, lo + wv + 4 * lane, b1, b2);
                const int32_t slot = D.lslot[ns + rank_of(s_bm, s_rank, id)];
                code = has_bit(s_old, id) ? slot : -1 - slot;
            }
            for (int u0 = 0; u0 < nmine; u0 += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    v[u] = 0.0;
                    if (u0 + u < nmine) {
                        const int32_t sl = __builtin_amdgcn_readlane(code, u0 + u);
                        if (sl >= 0) v[u] = Storage<ST>::load(D.pool, (int64_t)sl * BLK + lane);
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (u0 + u < nmine) s_a[cc * hcs + 4 * (wv + 4 * (u0 + u)) + ld] = v[u];
            }
            __syncthreads();
            const int base = 4 * lo;
            {
                // thread (velocity column tc, run q) takes the run of
                // consecutive cells [j0, j1) of its column with a sliding
                // window, so each cell's limited slope is computed once
                const int tc = tid & 15, q = tid >> 4;
                const int per = (ncell + 15) >> 4;
                const int j0 = q * per, j1 = min(j0 + per, ncell);
                const double *ac = s_a + tc * hcs;
                auto A = [&](int j) -> double { return (j >= 0 && j < ncell) ? ac[j] : 0.0; };
                if (j0 < j1) {
                    double am = A(j0 - 1), a0 = A(j0), ap = A(j0 + 1);
                    double dm = col_slope(A(j0 - 2), am, a0), d0 = col_slope(am, a0, ap);
                    for (int j = j0; j < j1; j++) {
                        const double app = A(j + 2);
                        const double dp = col_slope(a0, ap, app);
                        double l, r;
                        col_edges(am, a0, ap, dm, d0, dp, l, r);
                        s_l[tc * hcs + j] = l;
                        s_r[tc * hcs + j] = r;
                        am = a0;
                        a0 = ap;
                        ap = app;
                        dm = d0;
                        d0 = dp;
                    }
                }
            }
            __syncthreads();
            {
                const double *ac = s_a + cc * hcs, *lc = s_l + cc * hcs, *rc = s_r + cc * hcs;
                // cells outside the span hold zero: flat zero parabolas
                auto a = [&](int jj) -> double {
                    const int q = jj - base;
                    return (q >= 0 && q < ncell) ? ac[q] : 0.0;
                };
                auto edges = [&](int jj, double &l, double &r) {
                    const int q = jj - base;
                    const bool in = q >= 0 && q < ncell;
                    l = in ? lc[q] : 0.0;
                    r = in ? rc[q] : 0.0;
                };
                const double sigma = col_sigma(D, row, d, e1, e2, 4 * b1 + l1, 4 * b2 + l2);
                for (int u = 0; u < nmine; u++) {
                    const int bd = lo + wv + 4 * u;
                    const int32_t sl = __builtin_amdgcn_readlane(code, u);
                    const int32_t slot = sl >= 0 ? sl : -1 - sl;
                    const double v = col_remap_cell(a, edges, base, ncell, 4 * bd + ld, inv_alpha, sigma);
                    Storage<ST>::store(D.pool, (int64_t)slot * BLK + lane, v);
                    if (last) {
                        const int32_t id = compose_id(D, d, e1, e2, bd, b1, b2);
                        const double sv = Storage<ST>::round(v);
                        const bool content = sv >= D.sparse_min, nz = sv != 0.0;
                        const unsigned long long bc = __ballot(content), bz = __ballot(nz);
                        if (lane == 0)
                            D.litem[ns + rank_of(s_bm, s_rank, id)] =
                                (bc ? 1 : 0) | (bz ? 2 : 0) | (has_bit(s_start, id) ? 0 : 4);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// LDS of k_accel for a velocity mesh, or 0 if the mesh is beyond its limits
size_t accel_lds_bytes(const Dev &D, int *ncols, int *hc)
{
    int nc = 0, mx = 0;
    for (int d = 0; d < 3; d++) {
        const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
        nc = std::max(nc, D.nblk[e1] * D.nblk[e2]);
        mx = std::max(mx, D.nblk[d]);
    }
    if (mx > ACC_MAX_NBLK) return 0;
    *ncols = nc;
    *hc = 4 * mx;
    size_t b = sizeof(uint32_t) * (size_t)D.W * 3 + sizeof(int) * (size_t)(D.W + 1) + sizeof(int) * (size_t)nc * 2;
    b = (b + 15) & ~(size_t)15;
    return b + sizeof(double) * 3 * 16 * (size_t)(*hc + 1);
}

static AccelParams accel_params(const Dev &D, const double *fields, double *maps, int *bad, double qm, double dt,
                                const int order[3], int cur)
{
    AccelParams ap;
    ap.fields = fields;
    ap.maps = maps;
    ap.bad = bad;
    ap.qm = qm;
    ap.dt = dt;
    for (int k = 0; k < 3; k++) ap.order[k] = order[k];
    ap.cur = cur;
    ap.ncols = 0;
    ap.hc = 0;
    return ap;
}

void launch_accel_maps(const Dev &D, const double *fields, double *maps, int *bad, double qm, double dt,
                       const int order[3], hipStream_t st)
{
    const AccelParams ap = accel_params(D, fields, maps, bad, qm, dt, order, 0);
    hipLaunchKernelGGL(k_accel_factors, dim3((unsigned)((D.nlocal + 255) / 256)), dim3(256), 0, st, D, ap);
}

int launch_accel(const Dev &D, double *maps, const int order[3], int cur, hipStream_t st)
{
    AccelParams ap = accel_params(D, nullptr, maps, nullptr, 0.0, 0.0, order, cur);
    const size_t lds = accel_lds_bytes(D, &ap.ncols, &ap.hc);
    if (lds == 0) return -1;
    const dim3 g((unsigned)D.nlocal), b(256);
    switch (D.storage) {
    case VL_F64: hipLaunchKernelGGL(k_accel<VL_F64>, g, b, lds, st, D, ap); break;
    case VL_F32: hipLaunchKernelGGL(k_accel<VL_F32>, g, b, lds, st, D, ap); break;
    default: hipLaunchKernelGGL(k_accel<VL_BF16>, g, b, lds, st, D, ap); break;
    }
    return 0;
}

}  // namespace vl
