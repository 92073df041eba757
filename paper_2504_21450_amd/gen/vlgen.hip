// Device-side sampling of the seeded synthetic plasma states, for partitions
// too large to sample on the host.  It evaluates the same definition as the
// host sampler in workloads.py: per spatial cell up to NCOMP (bi-)Maxwellian
// components given as a parameter table, point-sampled at velocity-cell
// centres, times (1 + 0.01 u) with u from a SplitMix64 counter stream keyed
// by (seed, cell, block, lane); a block is kept where one of its values
// reaches the threshold, plus its face (6) or full (26) velocity neighbours.
//
// This is input generation only: it holds no part of the translation method
// and shares no code with the solver library.  Compiled without contraction
// of multiplies and adds, so every value is the host sampler's arithmetic up
// to the last-place differences of exp and log.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int NPAR = 10;  // n, Vx, Vy, Vz, Tpar, Tperp, bx, by, bz, unused
constexpr int WG = 256;
constexpr int NWAVE = WG / 64;

struct Geom {
    int nblk[3];
    int NB, W, vbuffer, ncomp;
    double vmin[3], dv[3];
    double thresh;       // content threshold (<= 0: keep every block)
    double kb_over_mp;   // Boltzmann constant over proton mass, as the host rounds it
    double two_pi_15;    // (2 pi)^1.5, as the host rounds it
    unsigned long long seed;
};

__device__ inline double comp_value(const double *q, double vx, double vy, double vz, const Geom &g)
{
    const double ux = vx - q[1], uy = vy - q[2], uz = vz - q[3];
    const double upar = ux * q[6] + uy * q[7] + uz * q[8];
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double uperp2 = fmax(u2 - upar * upar, 0.0);
    const double spa = g.kb_over_mp * q[4];
    const double spe = g.kb_over_mp * q[5];
    const double norm = q[0] / (g.two_pi_15 * spe * sqrt(spa));
    return norm * exp(-0.5 * upar * upar / spa - 0.5 * uperp2 / spe);
}

// f at lane `lane` of block b of a cell with parameter rows q (noise excluded)
__device__ inline double block_value(const double *q, int b, int lane, const Geom &g)
{
    const int bx = b % g.nblk[0], by = (b / g.nblk[0]) % g.nblk[1], bz = b / (g.nblk[0] * g.nblk[1]);
    const double vx = g.vmin[0] + ((double)(4 * bx + (lane & 3)) + 0.5) * g.dv[0];
    const double vy = g.vmin[1] + ((double)(4 * by + ((lane >> 2) & 3)) + 0.5) * g.dv[1];
    const double vz = g.vmin[2] + ((double)(4 * bz + (lane >> 4)) + 0.5) * g.dv[2];
    double f = 0.0;
    for (int k = 0; k < g.ncomp; k++) {
        const double *c = q + k * NPAR;
        if (c[0] > 0.0) f += comp_value(c, vx, vy, vz, g);
    }
    return f;
}

__device__ inline double noise(long long cell, int b, int lane, const Geom &g)
{
    const unsigned long long counter = ((unsigned long long)cell * (unsigned long long)g.NB + (unsigned)b) * 64ull +
                                       (unsigned)lane;
    unsigned long long z = g.seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// squared distance bound beyond which 1.01 times a component stays below half
// the threshold; -1 where its peak is too low (or it is absent)
__device__ inline double comp_radius2(const double *c, const Geom &g)
{
    if (!(c[0] > 0.0)) return -1.0;
    const double spa = g.kb_over_mp * c[4], spe = g.kb_over_mp * c[5];
    const double peak = c[0] / (g.two_pi_15 * spe * sqrt(spa));
    const double r = 1.01 * peak / (0.5 * g.thresh);
    return r > 1.0 ? 2.0 * fmax(spa, spe) * log(r) : -1.0;
}

__device__ inline bool candidate(const double *q, const double *r2, int b, const Geom &g)
{
    const int bc[3] = {b % g.nblk[0], (b / g.nblk[0]) % g.nblk[1], b / (g.nblk[0] * g.nblk[1])};
    for (int k = 0; k < g.ncomp; k++) {
        if (r2[k] < 0.0) continue;
        const double *c = q + k * NPAR;
        double d2 = 0.0;
        for (int d = 0; d < 3; d++) {
            const double lo = g.vmin[d] + (4 * bc[d] + 0.5) * g.dv[d];
            const double hi = g.vmin[d] + (4 * bc[d] + 3.5) * g.dv[d];
            const double V = c[1 + d];
            const double nr = fmin(fmax(V, lo), hi);
            d2 += (nr - V) * (nr - V);
        }
        if (d2 <= r2[k]) return true;
    }
    return false;
}

__device__ inline bool test_bit(const uint32_t *m, int b) { return (m[b >> 5] >> (b & 31)) & 1u; }

__device__ inline bool dilated(const uint32_t *cont, int b, const Geom &g)
{
    if (test_bit(cont, b)) return true;
    if (g.vbuffer == 0) return false;
    const int bx = b % g.nblk[0], by = (b / g.nblk[0]) % g.nblk[1], bz = b / (g.nblk[0] * g.nblk[1]);
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int m = (dx != 0) + (dy != 0) + (dz != 0);
                if (m == 0 || (g.vbuffer == 6 && m != 1)) continue;
                const int x = bx + dx, y = by + dy, z = bz + dz;
                if (x < 0 || y < 0 || z < 0 || x >= g.nblk[0] || y >= g.nblk[1] || z >= g.nblk[2]) continue;
                if (test_bit(cont, x + g.nblk[0] * (y + g.nblk[1] * z))) return true;
            }
    return false;
}

// One workgroup per cell: candidate blocks, content test on the sampled
// values, dilation; writes the kept-block bitmap and the count.
__global__ __launch_bounds__(WG) void k_masks(Geom g, const double *params, long long c0, uint32_t *masks,
                                                int *counts)
{
    extern __shared__ uint32_t lds[];
    uint32_t *cand = lds, *cont = lds + g.W;
    __shared__ int s_cnt;
    const long long cell = c0 + blockIdx.x;
    const double *q = params + cell * (long long)(g.ncomp * NPAR);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_cnt = 0;
    double r2[2];
    for (int k = 0; k < g.ncomp; k++) r2[k] = g.thresh > 0.0 ? comp_radius2(q + k * NPAR, g) : -1.0;
    const int nchunk = (g.NB + 63) / 64;
    for (int ch = wave; ch < nchunk; ch += NWAVE) {
        const int b = ch * 64 + lane;
        const bool bit = b < g.NB && (g.thresh <= 0.0 || candidate(q, r2, b, g));
        const unsigned long long m = __ballot(bit);
        if (lane == 0) {
            cand[2 * ch] = (uint32_t)m;
            if (2 * ch + 1 < g.W) cand[2 * ch + 1] = (uint32_t)(m >> 32);
        }
    }
    __syncthreads();
    for (int j = wave; j < g.W; j += NWAVE) {
        uint32_t bits = cand[j], out = 0;
        if (g.thresh <= 0.0) {
            out = bits;
        } else {
            while (bits) {
                const int t = __builtin_ctz(bits);
                bits &= bits - 1u;
                const int b = 32 * j + t;
                const double f = block_value(q, b, lane, g) * (1.0 + 0.01 * noise(cell, b, lane, g));
                if (__ballot(f >= g.thresh) != 0ull) out |= 1u << t;
            }
        }
        if (lane == 0) cont[j] = out;
    }
    __syncthreads();
    int cnt = 0;
    for (int ch = wave; ch < nchunk; ch += NWAVE) {
        const int b = ch * 64 + lane;
        const bool bit = b < g.NB && (g.thresh <= 0.0 || dilated(cont, b, g));
        const unsigned long long m = __ballot(bit);
        cnt += __popcll(m);
        if (lane == 0) {
            masks[cell * g.W + 2 * ch] = (uint32_t)m;
            if (2 * ch + 1 < g.W) masks[cell * g.W + 2 * ch + 1] = (uint32_t)(m >> 32);
        }
    }
    if (lane == 0) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    if (threadIdx.x == 0) counts[cell] = s_cnt;
}

// One workgroup per cell: ascending block ids from the bitmap.
__global__ __launch_bounds__(WG) void k_ids(const uint32_t *masks, int W, long long c0, const long long *offsets,
                                              int *ids)
{
    __shared__ int s_sum[WG];
    const long long cell = c0 + blockIdx.x;
    const uint32_t *m = masks + cell * W;
    const int per = (W + WG - 1) / WG;
    const int j0 = threadIdx.x * per, j1 = min(W, j0 + per);
    int mine = 0;
    for (int j = j0; j < j1; j++) mine += __popc(m[j]);
    s_sum[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < WG; o <<= 1) {  // inclusive scan
        const int v = threadIdx.x >= o ? s_sum[threadIdx.x - o] : 0;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        __syncthreads();
    }
    long long pos = offsets[cell] + s_sum[threadIdx.x] - mine;
    for (int j = j0; j < j1; j++) {
        uint32_t bits = m[j];
        while (bits) {
            const int t = __builtin_ctz(bits);
            bits &= bits - 1u;
            ids[pos++] = 32 * j + t;
        }
    }
}

// One workgroup per cell of [c0, c0 + gridDim.x): the 64 values of each of
// its blocks, written at (offsets[cell] + k - base) * 64 in FP64.
__global__ __launch_bounds__(WG) void k_values(Geom g, const double *params, long long c0, const long long *offsets,
                                                 const int *ids, long long base, double *out)
{
    const long long cell = c0 + blockIdx.x;
    const double *q = params + cell * (long long)(g.ncomp * NPAR);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long o0 = offsets[cell], o1 = offsets[cell + 1];
    for (long long k = o0 + wave; k < o1; k += NWAVE) {
        const int b = ids[k];
        out[(k - base) * 64 + lane] = block_value(q, b, lane, g) * (1.0 + 0.01 * noise(cell, b, lane, g));
    }
}

int geom(Geom *g, const int32_t nblk[3], const double vmin[3], const double dv[3], double thresh,
         int32_t vbuffer, int32_t ncomp, double kb_over_mp, double two_pi_15, unsigned long long seed)
{
    if (!nblk || !vmin || !dv || ncomp < 1 || ncomp > 2) return -1;  // the radius bound covers two
    if (vbuffer != 0 && vbuffer != 6 && vbuffer != 26) return -1;
    long long NB = 1;
    for (int d = 0; d < 3; d++) {
        if (nblk[d] < 1) return -1;
        g->nblk[d] = nblk[d];
        g->vmin[d] = vmin[d];
        g->dv[d] = dv[d];
        NB *= nblk[d];
    }
    if (NB > 131072) return -1;
    g->NB = (int)NB;
    g->W = (int)((NB + 31) / 32);
    g->vbuffer = vbuffer;
    g->ncomp = ncomp;
    g->thresh = thresh;
    g->kb_over_mp = kb_over_mp;
    g->two_pi_15 = two_pi_15;
    g->seed = seed;
    return 0;
}

}  // namespace

extern "C" {

// Kept-block bitmaps (masks[cell * W ..], W = ceil(prod(nblk) / 32) words)
// and counts of cells [c0, c1); params[cell * ncomp * 10 ..] on the device.
// Returns 0, -1 on bad arguments, -5 on a HIP error.  Asynchronous.
int vg_masks(const int32_t *nblk, const double *vmin, const double *dv, double thresh, int32_t vbuffer,
             int32_t ncomp, double kb_over_mp, double two_pi_15, unsigned long long seed, const double *params,
             long long c0, long long c1, uint32_t *masks, int32_t *counts, void *stream)
{
    Geom g;
    if (geom(&g, nblk, vmin, dv, thresh, vbuffer, ncomp, kb_over_mp, two_pi_15, seed) || c1 < c0 || !params ||
        !masks || !counts)
        return -1;
    if (c1 == c0) return 0;
    hipLaunchKernelGGL(k_masks, dim3((unsigned)(c1 - c0)), dim3(WG), 2 * g.W * sizeof(uint32_t),
                       (hipStream_t)stream, g, params, c0, masks, counts);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// Block ids of cells [c0, c1) at ids[offsets[cell] ..], ascending.
int vg_ids(const uint32_t *masks, int32_t W, const long long *offsets, long long c0, long long c1, int32_t *ids,
           void *stream)
{
    if (W < 1 || c1 < c0 || !masks || !offsets || !ids) return -1;
    if (c1 == c0) return 0;
    hipLaunchKernelGGL(k_ids, dim3((unsigned)(c1 - c0)), dim3(WG), 0, (hipStream_t)stream, masks, W, c0, offsets,
                       ids);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// FP64 values of the blocks of cells [c0, c1) into out[(offsets[cell] + k -
// offsets[c0]) * 64 + lane].
int vg_values(const int32_t *nblk, const double *vmin, const double *dv, double thresh, int32_t vbuffer,
              int32_t ncomp, double kb_over_mp, double two_pi_15, unsigned long long seed, const double *params,
              const long long *offsets, const int32_t *ids, long long c0, long long c1, long long base,
              double *out, void *stream)
{
    Geom g;
    if (geom(&g, nblk, vmin, dv, thresh, vbuffer, ncomp, kb_over_mp, two_pi_15, seed) || c1 < c0 || !params ||
        !offsets || !ids || !out)
        return -1;
    if (c1 == c0) return 0;
    hipLaunchKernelGGL(k_values, dim3((unsigned)(c1 - c0)), dim3(WG), 0, (hipStream_t)stream, g, params, c0,
                       offsets, ids, base, out);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
