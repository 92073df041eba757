// PPM shear kernel.  Persistent: each wavefront repeatedly takes the next
// (pencil, velocity block) work item from the list built by the planner and
// marches along the pencil, one lane per velocity cell of the block (64 lanes
// = 4x4x4 cells), with the reconstruction state in registers:
//   slope of cell t-1      (Colella & Woodward 1984, eq. 1.7-1.8)
//   face value t-3/2       (eq. 1.6, uniform grid)
//   limited profile t-2    (eq. 1.10)
//   flux through t-5/2     (eq. 1.12; upwind cell chosen by the sign of the
//                           lane's Courant number)
//   new average of t-3  =  old average + F(t-7/2) - F(t-5/2), written in place.
// Each (cell, block) belongs to exactly one item of a shear, so the update is
// in place without a second buffer.  Cells that do not hold the block read as
// zero; blocks created by the planner's growth step read as zero too.
//
// Storage variants:
//   VL_F64 : everything in FP64.
//   VL_F32 / VL_BF16 : values are loaded into FP32; slopes, faces and the
//            limiter run in FP32; the Courant number, flux integral and update
//            in FP64.  The FP64 update of a cell takes the rounding residual
//            carried along the pencil (of either sign) if it holds at least
//            that much, else the carry passes it by unchanged, so no cell is
//            driven negative and positive and negative carries are treated
//            alike; the sum is rounded to the storage type and the difference
//            carried on.  A line's carry starts from the residual its last
//            shear along the same axis left for the block (its sum over the
//            block's 64 velocity cells, kept in FP64 in the axis's ledger
//            store and spread evenly over the lanes) and its final carry,
//            summed over the lanes in a fixed order, is stored there for the
//            next one, so residuals are put back into f rather than
//            accumulating.  The line's stored mass changes only by its final
//            carry minus its starting one, which the item leaves for the FP64
//            mass ledger.
#include "vl_internal.h"
#include "vl_storage.h"

namespace vl {

struct SweepParams {
    int d, sidx, L, WL;
    int e1, e2, lo1, n1, lo2;  // pencil geometry (to tell local pencils)
    double dt;
    double sparse_min;
    const double *lg_old;    // residuals of the last shear along d, per old item
    double *lg_new;          // this shear's, per item
    const int32_t *lg_src;   // per item: its old item or -1
    int64_t lg_cap;          // items of a ledger store (0: no ledger)
};

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t ABSENT = 0xffffffffu;
constexpr int PF = 8;  // cells prefetched ahead of the reconstruction front

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// sum over the wavefront's 64 lanes, the same pairing every time
__device__ __forceinline__ double wave_sum64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double uniform_f64(double v)
{
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The starting carry of each velocity cell of item `it`'s line: 1/64 of the
// residual the last shear along the axis left for the same line and block (0
// if the block was not on the line then).  The 64 equal shares add up to the
// residual exactly; it is returned in `sum` (uniform, in scalar registers).
template <int ST>
__device__ __forceinline__ double take_residual(const SweepParams &sp, int64_t it, double &sum)
{
    double r = 0.0;
    if constexpr (ST != VL_F64) {
        if (it < sp.lg_cap) {
            const int32_t s = (int32_t)uniform_u32((uint32_t)sp.lg_src[it]);
            if (s >= 0) r = uniform_f64(sp.lg_old[s]);
        }
    }
    sum = uniform_f64(r);  // kept in scalar registers for the whole item
    return sum * (1.0 / BLK);
}

// Leave the line's final carry, summed over the lanes in a fixed order, for
// the next shear along the axis, and its change (final minus starting) for
// the mass ledger.
template <int ST>
__device__ __forceinline__ void leave_residual(const Dev &D, const SweepParams &sp, int64_t it, int lane,
                                               double carry, double start_sum)
{
    if constexpr (ST != VL_F64) {
        const double s = wave_sum64(carry);
        if (lane == 0) {
            if (it < sp.lg_cap) sp.lg_new[it] = s;
            D.resid[it] = s - start_sum;
        }
    }
}

// max(0, min(x, y)); in FP32 one median-of-three instruction (x >= 0 here,
// and a zero result takes the sign of the side afterwards, so the sign of a
// zero makes no difference)
template <typename C>
__device__ __forceinline__ C clamp_min0(C x, C y)
{
    if constexpr (std::is_same<C, float>::value)
        return __builtin_amdgcn_fmed3f(0.0f, x, y);
    else
        return fmax((C)0, fmin(x, y));
}

// limited slope of a cell (CW84 eq. 1.7-1.8) from its one-sided differences
// dl, dr and central difference cen: cen limited to twice either one-sided
// difference, zero at an extremum.  In FP32 it is minmod(cen, minmod(2 dl,
// 2 dr)) with minmod(x, y) = median(x, y, 0) (the smaller magnitude when x
// and y share a sign, else zero): two median-of-three instructions, the same
// value as the general form (which FP64 keeps) up to the sign of a zero.
template <typename C>
__device__ __forceinline__ C limited_slope(C dl, C dr, C cen)
{
    if constexpr (std::is_same<C, float>::value) {
        return __builtin_amdgcn_fmed3f(cen, __builtin_amdgcn_fmed3f(2.0f * dl, 2.0f * dr, 0.0f), 0.0f);
    } else {
        const C s2 = copysign((C)2.0, cen);
        const C m = fmax((C)0, fmin(fmin(fabs(cen), s2 * dl), s2 * dr));
        return copysign(m, cen);
    }
}

// the monotonicity limiter's face offset x given the other side's offset y
// (CW84 eq. 1.10 written on the offsets): x limited to twice y, zero unless
// they share a sign (the extremum case); in FP32 minmod(x, 2 y), one
// median-of-three instruction
template <typename C>
__device__ __forceinline__ C limited_offset(C x, C y)
{
    if constexpr (std::is_same<C, float>::value)
        return __builtin_amdgcn_fmed3f(x, 2.0f * y, 0.0f);
    else
        return copysign(clamp_min0(fabs(x), copysign((C)2.0, x) * y), x);
}

// The FP64 update x of a cell (its carry included) in the storage type (a
// negative sum, which only FP32 reconstruction rounding can leave, is stored
// as zero).  nv receives the stored value in FP64, so the caller carries
// x - nv on, which keeps the pencil's mass exact whatever the rounding.  BF16: FP64 -> FP32 to nearest, then FP32 -> BF16 to nearest
// even by the hardware conversion (two roundings; they differ from one
// correct rounding only where the FP32 value lands on a BF16 midpoint).
__device__ __forceinline__ float narrow_f32(double x, double &nv)
{
    const float q = fmaxf((float)x, 0.0f);
    nv = (double)q;
    return q;
}
__device__ __forceinline__ uint16_t narrow_bf16(double x, double &nv)
{
    float t = fmaxf((float)x, 0.0f);
    __asm__("" : "+v"(t));  // keeps the two roundings apart (no fused FP64 -> BF16 rounding)
    const uint16_t h = __builtin_bit_cast(uint16_t, (__bf16)t);
    nv = (double)bf16_to_f32(h);
    return h;
}

// Blocks are read and written through buffer resources made in scalar
// registers (block_rsrc, block_load, block_store), so no vector instruction
// computes addresses in the marches.

// One (pencil, block) item: march along the pencil.  DIR = +1 when every
// lane's Courant number is positive, -1 when every one is negative, 0 when
// the block straddles v = 0 (then the upwind side is chosen per lane).
//
// The reconstruction is Colella & Woodward's, written in forms with fewer
// operations that give the same values:
//  * limited slope: copysign(max(0, min(|c|, 2 s dl, 2 s dr)), c) with
//    c = (a+ - a-)/2 and s = sign(c) (zero unless dl and dr share a sign),
//    in FP32 minmod(c, minmod(2 dl, 2 dr)) (limited_slope);
//  * monotonicity limiter on the face offsets dL = a - aL, dR = aR - a: the
//    two overshoot corrections of the limiter are dL' = min(|dL|, 2|dR|) and
//    dR' = min(|dR|, 2|dL|) (with the sign of the side), the extremum case is
//    dL' = dR' = 0;
//  * flux integral of the parabola over the upwind fraction |c| of the cell,
//    expanded in dL', dR': F = c a + P dR' + Q dL' with
//    P = c (1-c)^2, Q = c^2 (1-c) for c > 0 and P = s^2 (1-s), Q = s (1-s)^2
//    for c = -s < 0.
// Variant "unconditional stores": slots of 8 cells at a time from LDS into
// scalar registers; every iteration stores (to a per-wavefront sink block when
// there is nothing to write), which keeps the compiler's memory counters exact.
template <int ST, int DIR, bool LAST>
__device__ __forceinline__ void march_unc(const Dev &D, const uint32_t *srow, uint8_t *sflag, int L, double c,
                                          int lane, double smin, double &carry, int tb, int te)
{
    using C = typename std::conditional<ST == VL_F64, double, float>::type;  // reconstruction type
    const bool pos = (DIR > 0) ? true : (DIR < 0) ? false : (c > 0.0);
    const double s = fabs(c);
    const double P = pos ? c * (1.0 - c) * (1.0 - c) : s * s * (1.0 - s);
    const double Q = pos ? c * c * (1.0 - c) : s * (1.0 - s) * (1.0 - s);
    constexpr int BS = Storage<ST>::BYTES;
    const uint32_t lane_off = (uint32_t)lane * BS;
    const uint32_t zslot = (uint32_t)D.trash;     // all-zero block: reads of absent cells
    // write-only block for discarded stores, one per wavefront
    const uint32_t sink = (uint32_t)D.trash + 1 +
                          (uint32_t)((blockIdx.x * 4 + (threadIdx.x >> 6)) % NSINK);

    // slots of 8 consecutive cells (raw: slot, slot|NEWFLAG or ABSENT), wave-uniform
    auto slots8 = [&](int t, uint32_t (&o)[PF]) {
        const uint4 v0 = *(const uint4 *)(srow + t);
        const uint4 v1 = *(const uint4 *)(srow + t + 4);
        o[0] = uniform_u32(v0.x); o[1] = uniform_u32(v0.y); o[2] = uniform_u32(v0.z); o[3] = uniform_u32(v0.w);
        o[4] = uniform_u32(v1.x); o[5] = uniform_u32(v1.y); o[6] = uniform_u32(v1.z); o[7] = uniform_u32(v1.w);
    };
    auto fetch = [&](uint32_t raw) -> C {
        const uint32_t sl = (raw & NEWFLAG) ? zslot : raw;  // absent or created this shear: zero
        const char *blk = (const char *)D.pool + (uint64_t)sl * (BLK * BS);
        if constexpr (ST == VL_F64)
            return *(const double *)(blk + lane_off);
        else if constexpr (ST == VL_F32)
            return *(const float *)(blk + lane_off);
        else
            return bf16_to_f32(*(const uint16_t *)(blk + lane_off));
    };

    C a1 = 0, a2 = 0;           // a(t-1), a(t-2)
    double a3d = 0.0;           // a(t-3) in FP64 (last iteration's a(t-2))
    C da_prev = 0;              // slope of cell t-2
    C face_prev = 0;            // face t-5/2
    double Fc_prev = 0.0, Ff_prev = 0.0;
    uint32_t prv[PF], cur[PF], nxt[PF];
    C q[PF];
#pragma unroll
    for (int u = 0; u < PF; u++) prv[u] = ABSENT;
    const int t00 = tb & ~3;  // the slot table is read in aligned groups of 4
    slots8(t00, cur);
#pragma unroll
    for (int u = 0; u < PF; u++) q[u] = fetch(cur[u]);
    for (int t0 = t00; t0 < te; t0 += PF) {
        slots8(t0 + PF, nxt);
#pragma unroll
        for (int u = 0; u < PF; u++) {
            const int t = t0 + u;
            const C a = q[u];
            q[u] = fetch(nxt[u]);
            // slope of cell t-1
            const C dl = a1 - a2, dr = a - a1;
            const C cen = (C)0.5 * (a - a2);
            const C da = limited_slope(dl, dr, cen);
            // face between t-2 and t-1
            const C face = a2 + (C)0.5 * (a1 - a2) - (da - da_prev) * (C)(1.0 / 6.0);
            // limited face offsets of cell t-2
            const C ai = a2;
            const C dL = ai - face_prev, dR = face - ai;
            const double dLp = (double)limited_offset(dL, dR), dRp = (double)limited_offset(dR, dL);
            const double aid = (double)ai;
            const double Fc = fma(P, dRp, fma(Q, dLp, c * aid));
            const double Ff = (DIR > 0) ? Fc_prev : (DIR < 0) ? Fc : (pos ? Fc_prev : Fc);
            // new value of cell t-3, stored unconditionally (to the sink when
            // there is nothing to store) so the memory counters stay exact
            const uint32_t raw3 = (u >= 3) ? cur[u - 3] : prv[u + PF - 3];
            // the march runs in whole groups past te; cells from there on
            // belong to the next segment and are written by its own march
            const bool live = (t >= 6) && (t < L) && (t < te) && (raw3 != ABSENT);
            const uint32_t s3 = live ? (raw3 & ~NEWFLAG) : sink;
            char *dst = (char *)D.pool + (uint64_t)s3 * (BLK * BS);
            double nv;
            if constexpr (ST == VL_F64) {
                nv = a3d + (Ff_prev - Ff);
                *(double *)(dst + lane_off) = nv;
            } else {
                // the carry goes into the cell only if the cell holds at least as much
                const double base = a3d + (Ff_prev - Ff);
                const double cin = (live && fabs(carry) <= base) ? carry : 0.0;
                const double x = base + cin;
                if constexpr (ST == VL_F32)
                    *(float *)(dst + lane_off) = narrow_f32(x, nv);
                else
                    *(uint16_t *)(dst + lane_off) = narrow_bf16(x, nv);
                if (live) carry = (carry - cin) + (x - nv);
            }
            if constexpr (LAST) {
                const unsigned long long any = __ballot(nv >= smin);
                if (t >= 3 && t < te) sflag[t - 3] = any ? 1 : 0;  // same value from every lane
            }
            a3d = aid;
            a2 = a1;
            a1 = a;
            da_prev = da;
            face_prev = face;
            Fc_prev = Fc;
            Ff_prev = Ff;
        }
#pragma unroll
        for (int u = 0; u < PF; u++) {
            prv[u] = cur[u];
            cur[u] = nxt[u];
        }
    }
}


// Variant "conditional stores": the slot of each cell is read from LDS when
// it is fetched (prefetch distance PFV) and kept in scalar registers until
// the cell is written PFV + 3 iterations later; the store is skipped (scalar
// branch) for cells without the block and outside the updated range.
template <int ST, int DIR, bool LAST, int PFV>
__device__ __forceinline__ void march_cond(const Dev &D, const uint32_t *srow, uint8_t *sflag, int L, double c,
                                           int lane, double smin, double &carry, int tb, int te)
{
    static_assert(PFV >= 3, "the written cell's slot comes from the previous group");
    using C = typename std::conditional<ST == VL_F64, double, float>::type;  // reconstruction type
    const bool pos = (DIR > 0) ? true : (DIR < 0) ? false : (c > 0.0);
    const double s = fabs(c);
    const double P = pos ? c * (1.0 - c) * (1.0 - c) : s * s * (1.0 - s);
    const double Q = pos ? c * c * (1.0 - c) : s * (1.0 - s) * (1.0 - s);
    constexpr int BS = Storage<ST>::BYTES;
    const uint32_t lane_off = (uint32_t)lane * BS;
    const uint32_t zslot = (uint32_t)D.trash;

    // a cell's value from its raw slot (wave-uniform): absent or created this
    // shear reads the all-zero block
    auto fetch_raw = [&](uint32_t sl) -> C {
        return block_load<ST>(block_rsrc<ST>(D.pool, (sl & NEWFLAG) ? zslot : sl), lane_off);
    };

    C a1 = 0, a2 = 0;
    double a3d = 0.0;
    C da_prev = 0;
    C face_prev = 0;
    double Fc_prev = 0.0, Ff_prev = 0.0;
    C q[PFV];
    // raw slots of the cells t0 .. t0+PFV-1 (fetched by the previous group or
    // the prologue), of the three cells before them, and of the cells this
    // group fetches
    uint32_t prv[PFV], bef[3], cur[PFV];
#pragma unroll
    for (int u = 0; u < PFV; u++) {
        prv[u] = uniform_u32(srow[tb + u]);
        q[u] = fetch_raw(prv[u]);
    }
#pragma unroll
    for (int i = 0; i < 3; i++) bef[i] = (tb - 3 + i >= 0) ? uniform_u32(srow[tb - 3 + i]) : ABSENT;
    // the slot-table entry of the next iteration's fetch, read from LDS one
    // iteration ahead so its latency is hidden behind a cell's arithmetic
    // (the table is padded with ABSENT past L)
    uint32_t f_next = srow[tb + PFV];
    for (int t0 = tb; t0 < te; t0 += PFV) {
#pragma unroll
        for (int u = 0; u < PFV; u++) {
            const int t = t0 + u;
            cur[u] = uniform_u32(f_next);
            f_next = srow[t + PFV + 1];
            const C a = q[u];
            q[u] = fetch_raw(cur[u]);
            const C dl = a1 - a2, dr = a - a1;
            const C cen = (C)0.5 * (a - a2);
            const C da = limited_slope(dl, dr, cen);
            const C face = a2 + (C)0.5 * (a1 - a2) - (da - da_prev) * (C)(1.0 / 6.0);
            const C ai = a2;
            const C dL = ai - face_prev, dR = face - ai;
            const double dLp = (double)limited_offset(dL, dR), dRp = (double)limited_offset(dR, dL);
            const double aid = (double)ai;
            const double Fc = fma(P, dRp, fma(Q, dLp, c * aid));
            const double Ff = (DIR > 0) ? Fc_prev : (DIR < 0) ? Fc : (pos ? Fc_prev : Fc);
            if (t >= 6 && t < L && t < te) {  // past te: the next segment's march
                const uint32_t sl3 = (u >= 3) ? prv[u - 3] : bef[u];  // cell t - 3
                if (sl3 != ABSENT) {
                    const __amdgpu_buffer_rsrc_t dst = block_rsrc<ST>(D.pool, sl3 & ~NEWFLAG);
                    double nv;
                    if constexpr (ST == VL_F64) {
                        nv = a3d + (Ff_prev - Ff);
                        block_store(dst, lane_off, nv);
                    } else {
                        // the carry goes into the cell only if the cell holds at least as much
                        const double base = a3d + (Ff_prev - Ff);
                        const double cin = (fabs(carry) <= base) ? carry : 0.0;
                        const double x = base + cin;
                        if constexpr (ST == VL_F32)
                            block_store(dst, lane_off, narrow_f32(x, nv));
                        else
                            block_store(dst, lane_off, narrow_bf16(x, nv));
                        carry = (carry - cin) + (x - nv);
                    }
                    if constexpr (LAST) {
                        const unsigned long long any = __ballot(nv >= smin);
                        sflag[t - 3] = any ? 1 : 0;
                    }
                }
            }
            a3d = aid;
            a2 = a1;
            a1 = a;
            da_prev = da;
            face_prev = face;
            Fc_prev = Fc;
            Ff_prev = Ff;
        }
#pragma unroll
        for (int i = 0; i < 3; i++) bef[i] = prv[PFV - 3 + i];
#pragma unroll
        for (int u = 0; u < PFV; u++) prv[u] = cur[u];
    }
}

// shear variants chosen by the autotuner (all give bit-identical results)
//   style 0: conditional stores, style 1: unconditional stores, style 2:
//   conditional stores with the items of a wavefront streamed (the next
//   item's slot table and first cells are loaded during the current item)
//   pf: prefetch distance; minw: minimum waves per SIMD asked of the compiler (0 = default)
struct VariantInfo {
    int style, pf, minw;
};
constexpr VariantInfo VARIANTS[] = {{0, 8, 0}, {0, 8, 6}, {0, 4, 0}, {0, 16, 0}, {1, 8, 0}, {1, 8, 5},
                                   {2, 8, 0}, {0, 4, 8}, {0, 8, 8}, {2, 8, 8}, {0, 4, 6}};
constexpr int NVARIANTS = sizeof(VARIANTS) / sizeof(VARIANTS[0]);

template <int ST, int DIR, bool LAST, int V>
__device__ __forceinline__ void march(const Dev &D, const uint32_t *srow, uint8_t *sflag, int L, double c,
                                      int lane, double smin, double &carry, int tb, int te)
{
    constexpr VariantInfo vi = VARIANTS[V];
    if constexpr (vi.style == 1)
        march_unc<ST, DIR, LAST>(D, srow, sflag, L, c, lane, smin, carry, tb, te);
    else
        march_cond<ST, DIR, LAST, vi.pf>(D, srow, sflag, L, c, lane, smin, carry, tb, te);
}

// Content flags of the last shear for an item: bit t of word t / 32 tells
// whether local cell t of the pencil holds the block with a value >=
// sparse_min after the update.  The words replace the item's presence masks
// (read at the item's start, not needed after it) in one coalesced store; the
// pruning finds them through the item recorded for each list entry.
__device__ __forceinline__ void store_flag_words(const Dev &D, int64_t it, const uint32_t *srow,
                                                 const uint8_t *sflag, int L, int lane)
{
    uint32_t word = 0;
    for (int t0 = 0; t0 < L; t0 += 64) {
        const int t = t0 + lane;
        bool f = false;
        if (t >= H && t < L - H) {
            const uint32_t raw = srow[t];
            f = raw != ABSENT && (raw & ~NEWFLAG) < (uint32_t)D.lcap && sflag[t] != 0;
        }
        const unsigned long long b = __ballot(f);
        const int w = t0 >> 5;
        if (lane == w) word = (uint32_t)b;
        if (lane == w + 1) word = (uint32_t)(b >> 32);
    }
    if (lane < D.wlmax) D.masks[it * D.wlmax + lane] = word;
}

// lowest set bit at position >= from of a MAXWL-word mask, or -1
__device__ __forceinline__ int first_bit(const uint32_t (&v)[MAXWL], int from)
{
#pragma unroll
    for (int w = 0; w < MAXWL; w++) {
        uint32_t x = v[w];
        if (32 * w + 31 < from) x = 0u;
        else if (32 * w < from) x &= ~0u << (from - 32 * w);
        if (x) return 32 * w + __builtin_ctz(x);
    }
    return -1;
}

__device__ __forceinline__ int last_bit(const uint32_t (&v)[MAXWL])
{
#pragma unroll
    for (int w = MAXWL - 1; w >= 0; w--)
        if (v[w]) return 32 * w + 31 - __builtin_clz(v[w]);
    return -1;
}

template <int ST, bool LAST, int V>
__device__ __forceinline__ void sweep_body(const Dev &D, const SweepParams &sp)
{
    __shared__ __align__(16) uint32_t s_slot[4][MAXL + 48];
    __shared__ uint8_t s_flag[4][MAXL + 48];
    __shared__ uint32_t s_seg[4][MAXL / 7 + 2];  // segments of the item: first cell | end << 16
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int d = sp.d, L = sp.L, WL = sp.WL;
    const int64_t nitems = min((int64_t)D.ctl->n_items, D.item_cap);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    uint32_t *srow = s_slot[wv];
    uint32_t *sseg = s_seg[wv];

    for (int64_t it = (int64_t)blockIdx.x * 4 + wv; it < nitems; it += nwaves) {
        const Item item = D.items[it];
        // the lane index and the mask words as values of this item (an empty
        // asm the compiler cannot see through), so the per-lane index
        // arithmetic and the word tests of the slot table below are
        // recomputed per item rather than hoisted out of the loop and kept in
        // registers, which spill at eight waves per SIMD
        int li = lane, wl = WL;
        __asm__ volatile("" : "+v"(li), "+s"(wl));
        // presence of the block along the pencil (wave-uniform), and the
        // starts of gaps of at least 6 cells without it
        uint32_t m[MAXWL], gap[MAXWL];
        // per-cell slot table of this item in LDS: slot, slot|NEWFLAG or ABSENT
        {
            int pre[MAXWL + 1];
            pre[0] = 0;
#pragma unroll
            for (int w = 0; w < MAXWL; w++) {
                m[w] = (w < wl) ? __builtin_amdgcn_readfirstlane(D.masks[it * D.wlmax + w]) : 0u;
                pre[w + 1] = pre[w] + __popc(m[w]);
            }
            if (pre[MAXWL] == 0) {  // empty item: no updated cell, the residual passes on
                double sum;
                const double r = take_residual<ST>(sp, it, sum);
                leave_residual<ST>(D, sp, it, li, r, sum);
                continue;
            }
#pragma unroll
            for (int w = 0; w < MAXWL; w++) {
                const uint32_t a0 = ~m[w], a1 = (w + 1 < MAXWL) ? ~m[w + 1] : ~0u;
                uint32_t r = a0;
#pragma unroll
                for (int k = 1; k < 6; k++) r &= (a0 >> k) | (a1 << (32 - k));
                gap[w] = r & ((m[w] << 1) | (w > 0 ? m[w - 1] >> 31 : 0u));
            }
            const int half = li >> 5, b = li & 31;
#pragma unroll
            for (int w = 0; w < MAXWL; w += 2) {
                if (w < wl) {
                    const uint32_t mw = half ? m[w + 1] : m[w];
                    const int base = half ? pre[w + 1] : pre[w];
                    const int t = 32 * (w + half) + b;
                    if (t < L) {
                        const bool pr = (mw >> b) & 1u;
                        const int rk = base + __popc(mw & ((1u << b) - 1u));
                        srow[t] = pr ? (uint32_t)D.rows[item.rowoff + rk] : ABSENT;
                    }
                }
            }
            for (int t = L + li; t < L + 40; t += 64) srow[t] = ABSENT;
        }
        wave_sync_lds();

        // the block's coordinate along d (the mesh extents passed through an
        // empty asm, so the divisions' reciprocals are formed per item, not
        // kept in registers across items) and the lane's velocity cell in it
        int nb0 = D.nblk[0], nb1 = D.nblk[1];
        __asm__ volatile("" : "+s"(nb0), "+s"(nb1));
        const int bd = (d == 0) ? item.id % nb0 : (d == 1) ? (item.id / nb0) % nb1 : item.id / (nb0 * nb1);
        const int ld = (d == 0) ? (li & 3) : (d == 1) ? ((li >> 2) & 3) : (li >> 4);
        const double c = courant(D, d, 4 * bd + ld, sp.dt);
        const unsigned long long npos = __ballot(c > 0.0), nneg = __ballot(c < 0.0);
        double start_sum;
        double carry = take_residual<ST>(sp, it, start_sum);
        uint8_t *sflag = s_flag[wv];
        // March each segment of cells holding the block: from its first such
        // cell to three past its last (where the last one is written).  Before
        // a segment's first cell at least 6 cells read as zero, so the
        // reconstruction state there is the zero state a march starts from;
        // the rounding carry runs on across segments.
        // The segments are listed in LDS first, so the masks need no
        // registers during the marches.
        int nseg = 0;
        for (int tb = first_bit(m, 0); tb >= 0;) {
            const int g = first_bit(gap, tb + 1);
            const int te = (g >= 0) ? g + 3 : last_bit(m) + 4;
            if (li == 0) sseg[nseg] = (uint32_t)tb | ((uint32_t)te << 16);
            nseg++;
            tb = (g >= 0) ? first_bit(m, g) : -1;
        }
        wave_sync_lds();
        for (int k = 0; k < nseg; k++) {
            const uint32_t v = uniform_u32(sseg[k]);
            const int tb = (int)(v & 0xffffu), te = (int)(v >> 16);
            if (npos == ~0ull)
                march<ST, 1, LAST, V>(D, srow, sflag, L, c, li, sp.sparse_min, carry, tb, te);
            else if (nneg == ~0ull)
                march<ST, -1, LAST, V>(D, srow, sflag, L, c, li, sp.sparse_min, carry, tb, te);
            else
                march<ST, 0, LAST, V>(D, srow, sflag, L, c, li, sp.sparse_min, carry, tb, te);
        }
        if constexpr (LAST) {
            wave_sync_lds();
            store_flag_words(D, it, srow, sflag, L, li);
        }

        // the line's final carry (the ledger takes those of the local pencils)
        leave_residual<ST>(D, sp, it, li, carry, start_sum);
        wave_sync_lds();
    }
}


// ---------------------------------------------------------------------------
// streamed items (style 2)
// ---------------------------------------------------------------------------
// Build the per-cell slot table of item `it` into srow[0 .. L+40).
__device__ __forceinline__ void build_slots(const Dev &D, int64_t it, int64_t nitems, int L, int WL, int lane,
                                            uint32_t *srow)
{
    if (it >= nitems) {
        for (int t = lane; t < L + 40; t += 64) srow[t] = ABSENT;
        return;
    }
    const Item item = D.items[it];
    uint32_t m[MAXWL];
    int pre[MAXWL + 1];
    pre[0] = 0;
#pragma unroll
    for (int w = 0; w < MAXWL; w++) {
        m[w] = (w < WL) ? D.masks[it * D.wlmax + w] : 0u;
        pre[w + 1] = pre[w] + __popc(m[w]);
    }
    const int half = lane >> 5, b = lane & 31;
#pragma unroll
    for (int w = 0; w < MAXWL; w += 2) {
        if (w < WL) {
            const uint32_t mw = half ? m[w + 1] : m[w];
            const int base = half ? pre[w + 1] : pre[w];
            const int t = 32 * (w + half) + b;
            if (t < L) {
                const bool pr = (mw >> b) & 1u;
                const int rk = base + __popc(mw & ((1u << b) - 1u));
                srow[t] = pr ? (uint32_t)D.rows[item.rowoff + rk] : ABSENT;
            }
        }
    }
    for (int t = L + lane; t < L + 40; t += 64) srow[t] = ABSENT;
}

// One item of the stream: cells of X; q holds X's first 8 values on entry and
// the next item's (table Y) first 8 on exit.  build_next() fills Y.
template <int ST, int DIR, bool LAST, typename BUILD>
__device__ __forceinline__ void march_stream(const Dev &D, const uint32_t *X, const uint32_t *Y, uint8_t *sflag,
                                             int L, double c, int lane, double smin, double &carry,
                                             typename std::conditional<ST == VL_F64, double, float>::type (&q)[8],
                                             BUILD build_next)
{
    using C = typename std::conditional<ST == VL_F64, double, float>::type;
    const bool pos = (DIR > 0) ? true : (DIR < 0) ? false : (c > 0.0);
    const double s = fabs(c);
    const double P = pos ? c * (1.0 - c) * (1.0 - c) : s * s * (1.0 - s);
    const double Q = pos ? c * c * (1.0 - c) : s * (1.0 - s) * (1.0 - s);
    constexpr int BS = Storage<ST>::BYTES;
    const uint32_t lane_off = (uint32_t)lane * BS;
    const uint32_t zslot = (uint32_t)D.trash;
    auto fetch = [&](const uint32_t *tab, int t) -> C {
        uint32_t sl = uniform_u32(tab[t]);
        sl = (sl & NEWFLAG) ? zslot : sl;
        const char *blk = (const char *)D.pool + (uint64_t)sl * (BLK * BS);
        if constexpr (ST == VL_F64)
            return *(const double *)(blk + lane_off);
        else if constexpr (ST == VL_F32)
            return *(const float *)(blk + lane_off);
        else
            return bf16_to_f32(*(const uint16_t *)(blk + lane_off));
    };
    C a1 = 0, a2 = 0, da_prev = 0, face_prev = 0;
    double a3d = 0.0, Fc_prev = 0.0, Ff_prev = 0.0;
    const int G = (L + 7) / 8;
    if (G == 1) build_next();
    for (int g = 0; g < G; g++) {
        const bool lastg = (g == G - 1);
        const uint32_t *src = lastg ? Y : X;
        const int fb = lastg ? 0 : 8 * (g + 1);
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int t = 8 * g + u;
            const C a = q[u];
            q[u] = fetch(src, fb + u);
            const C dl = a1 - a2, dr = a - a1;
            const C cen = (C)0.5 * (a - a2);
            const C da = limited_slope(dl, dr, cen);
            const C face = a2 + (C)0.5 * dl - (da - da_prev) * (C)(1.0 / 6.0);
            const C ai = a2;
            const C dL = ai - face_prev, dR = face - ai;
            const double dLp = (double)limited_offset(dL, dR), dRp = (double)limited_offset(dR, dL);
            const double aid = (double)ai;
            const double Fc = fma(P, dRp, fma(Q, dLp, c * aid));
            const double Ff = (DIR > 0) ? Fc_prev : (DIR < 0) ? Fc : (pos ? Fc_prev : Fc);
            if (t >= 6 && t < L) {
                const uint32_t sl3 = uniform_u32(X[t - 3]);
                if (sl3 != ABSENT) {
                    const uint32_t s3 = sl3 & ~NEWFLAG;
                    char *dst = (char *)D.pool + (uint64_t)s3 * (BLK * BS);
                    double nv;
                    if constexpr (ST == VL_F64) {
                        nv = a3d + (Ff_prev - Ff);
                        *(double *)(dst + lane_off) = nv;
                    } else {
                        const double base = a3d + (Ff_prev - Ff);
                        const double cin = (fabs(carry) <= base) ? carry : 0.0;
                        const double x = base + cin;
                        if constexpr (ST == VL_F32)
                            *(float *)(dst + lane_off) = narrow_f32(x, nv);
                        else
                            *(uint16_t *)(dst + lane_off) = narrow_bf16(x, nv);
                        carry = (carry - cin) + (x - nv);
                    }
                    if constexpr (LAST) {
                        const unsigned long long any = __ballot(nv >= smin);
                        sflag[t - 3] = any ? 1 : 0;
                    }
                }
            }
            a3d = aid;
            a2 = a1;
            a1 = a;
            da_prev = da;
            face_prev = face;
            Fc_prev = Fc;
            Ff_prev = Ff;
        }
        if (g == 0 && G > 1) build_next();
    }
}

template <int ST, bool LAST>
__device__ __forceinline__ void sweep_stream(const Dev &D, const SweepParams &sp)
{
    using C = typename std::conditional<ST == VL_F64, double, float>::type;
    __shared__ __align__(16) uint32_t s_tab[4][2][MAXL + 48];
    __shared__ uint8_t s_flg[4][MAXL + 48];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int d = sp.d, L = sp.L, WL = sp.WL;
    const int ld = (d == 0) ? (lane & 3) : (d == 1) ? ((lane >> 2) & 3) : (lane >> 4);
    const int64_t nitems = min((int64_t)D.ctl->n_items, D.item_cap);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    int64_t it = (int64_t)blockIdx.x * 4 + wv;
    if (it >= nitems) return;
    uint32_t *X = s_tab[wv][0], *Y = s_tab[wv][1];
    uint8_t *sflag = s_flg[wv];
    build_slots(D, it, nitems, L, WL, lane, X);
    wave_sync_lds();
    const uint32_t zslot = (uint32_t)D.trash;
    constexpr int BS = Storage<ST>::BYTES;
    C q[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        uint32_t sl = uniform_u32(X[u]);
        sl = (sl & NEWFLAG) ? zslot : sl;
        const char *blk = (const char *)D.pool + (uint64_t)sl * (BLK * BS) + (uint32_t)lane * BS;
        if constexpr (ST == VL_F64)
            q[u] = *(const double *)blk;
        else if constexpr (ST == VL_F32)
            q[u] = *(const float *)blk;
        else
            q[u] = bf16_to_f32(*(const uint16_t *)blk);
    }
    for (; it < nitems; it += nwaves) {
        const int64_t nit = it + nwaves;
        const int32_t id = D.items[it].id;
        const int bd = block_coord(D, d, id);
        const double c = courant(D, d, 4 * bd + ld, sp.dt);
        const unsigned long long npos = __ballot(c > 0.0), nneg = __ballot(c < 0.0);
        double start_sum;
        double carry = take_residual<ST>(sp, it, start_sum);
        auto build = [&]() {
            build_slots(D, nit, nitems, L, WL, lane, Y);
            wave_sync_lds();
        };
        if (npos == ~0ull)
            march_stream<ST, 1, LAST>(D, X, Y, sflag, L, c, lane, sp.sparse_min, carry, q, build);
        else if (nneg == ~0ull)
            march_stream<ST, -1, LAST>(D, X, Y, sflag, L, c, lane, sp.sparse_min, carry, q, build);
        else
            march_stream<ST, 0, LAST>(D, X, Y, sflag, L, c, lane, sp.sparse_min, carry, q, build);
        if constexpr (LAST) {
            wave_sync_lds();
            store_flag_words(D, it, X, sflag, L, lane);
        }
        leave_residual<ST>(D, sp, it, lane, carry, start_sum);  // the line's final carry
        wave_sync_lds();
        uint32_t *tmp = X;
        X = Y;
        Y = tmp;
    }
}

template <int ST, bool LAST, int V>
__global__ __launch_bounds__(256) void k_sweep(Dev D, SweepParams sp)
{
    if (failed(D)) return;  // waves are independent: no barrier to keep
    if constexpr (VARIANTS[V].style == 2)
        sweep_stream<ST, LAST>(D, sp);
    else
        sweep_body<ST, LAST, V>(D, sp);
}

template <int ST, bool LAST, int V, int MINW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MINW))) void k_sweep_occ(Dev D, SweepParams sp)
{
    if (failed(D)) return;
    if constexpr (VARIANTS[V].style == 2)
        sweep_stream<ST, LAST>(D, sp);
    else
        sweep_body<ST, LAST, V>(D, sp);
}

template <typename K>
static dim3 persistent_grid(K kernel)
{
    // exactly the workgroups that fit on the device at once, so every
    // wavefront's share of the static item assignment runs in one round
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || per < 1) per = 1;
    return dim3((unsigned)(per * ncu));
}

template <int ST, bool LAST, int V>
static void launch_variant(const Dev &D, const SweepParams &sp, hipStream_t st)
{
    constexpr VariantInfo vi = VARIANTS[V];
    if constexpr (vi.minw > 0) {
        static const dim3 g = persistent_grid(k_sweep_occ<ST, LAST, V, (vi.minw > 0 ? vi.minw : 1)>);
        hipLaunchKernelGGL((k_sweep_occ<ST, LAST, V, (vi.minw > 0 ? vi.minw : 1)>), g, dim3(256), 0, st, D, sp);
    } else {
        static const dim3 g = persistent_grid(k_sweep<ST, LAST, V>);
        hipLaunchKernelGGL((k_sweep<ST, LAST, V>), g, dim3(256), 0, st, D, sp);
    }
}

template <int ST, bool LAST>
static void launch_st(const Dev &D, const SweepParams &sp, int v, hipStream_t st)
{
    switch (v) {
    case 1: launch_variant<ST, LAST, 1>(D, sp, st); break;
    case 2: launch_variant<ST, LAST, 2>(D, sp, st); break;
    case 3: launch_variant<ST, LAST, 3>(D, sp, st); break;
    case 4: launch_variant<ST, LAST, 4>(D, sp, st); break;
    case 5: launch_variant<ST, LAST, 5>(D, sp, st); break;
    case 6: launch_variant<ST, LAST, 6>(D, sp, st); break;
    case 7: launch_variant<ST, LAST, 7>(D, sp, st); break;
    case 8: launch_variant<ST, LAST, 8>(D, sp, st); break;
    case 9: launch_variant<ST, LAST, 9>(D, sp, st); break;
    case 10: launch_variant<ST, LAST, 10>(D, sp, st); break;
    default: launch_variant<ST, LAST, 0>(D, sp, st); break;
    }
}

int sweep_variants() { return NVARIANTS; }

void launch_sweep(const Dev &D, int d, int sidx, const int lo[3], const int hi[3], double dt, bool last,
                  const LedgerIO &lg, hipStream_t st)
{
    SweepParams sp;
    sp.lg_old = lg.old.res;
    sp.lg_new = lg.nw.res;
    sp.lg_src = lg.src;
    sp.lg_cap = lg.src ? lg.cap : 0;
    sp.d = d;
    sp.sidx = sidx;
    sp.L = D.P[d];
    sp.WL = (sp.L + 31) / 32;
    sp.e1 = (d == 0) ? 1 : 0;
    sp.e2 = (d == 2) ? 1 : 2;
    sp.lo1 = lo[sp.e1];
    sp.n1 = hi[sp.e1] - lo[sp.e1];
    sp.lo2 = lo[sp.e2];
    sp.dt = dt;
    sp.sparse_min = D.sparse_min;
    const int v = (D.sweep_variant[sidx] >= 0 && D.sweep_variant[sidx] < NVARIANTS) ? D.sweep_variant[sidx] : 0;
    switch (D.storage) {
    case VL_F64: last ? launch_st<VL_F64, true>(D, sp, v, st) : launch_st<VL_F64, false>(D, sp, v, st); break;
    case VL_F32: last ? launch_st<VL_F32, true>(D, sp, v, st) : launch_st<VL_F32, false>(D, sp, v, st); break;
    default: last ? launch_st<VL_BF16, true>(D, sp, v, st) : launch_st<VL_BF16, false>(D, sp, v, st); break;
    }
}

// ---------------------------------------------------------------------------
// mass ledger of one shear: the terminal residuals of the local pencils'
// items, summed per pencil over its items (ascending block id) by one
// wavefront, then over the pencils in order by one workgroup; no atomics, so
// the total is the same in every run
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ledger_pencils(Dev D, int e1, int e2, int lo1, int n1, int lo2,
                                                        int64_t npen, double *pen_sum)
{
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= npen || failed(D)) return;
    const int t1 = lo1 + (int)(p % n1), t2 = lo2 + (int)(p / n1);
    const bool local = t1 >= H && t1 < H + D.n[e1] && t2 >= H && t2 < H + D.n[e2];
    double acc = 0.0;
    if (local && p < D.pen_cap) {
        const int64_t first = D.pen_first[p];
        const int64_t cnt = min((int64_t)D.pen_cnt[p], max((int64_t)0, D.item_cap - first));
        for (int64_t k = lane; k < cnt; k += 64) acc += D.resid[first + k];
    }
    acc = wave_sum64(acc);
    if (lane == 0) pen_sum[p] = acc;
}

__global__ __launch_bounds__(1024) void k_sum_fixed(const double *in, int64_t n, double *out)
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

void launch_ledger_sum(const Dev &D, int d, const int lo[3], const int hi[3], double *out, hipStream_t st)
{
    const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    const int n1 = hi[e1] - lo[e1], n2 = hi[e2] - lo[e2];
    const int64_t npen = (int64_t)n1 * n2;
    if (npen <= 0 || D.storage == VL_F64) {
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, D.cell_red, (int64_t)0, out);
        return;
    }
    // per-pencil sums in the scratch of per-cell sums (npen <= padded cells)
    hipLaunchKernelGGL(k_ledger_pencils, dim3((unsigned)((npen + 3) / 4)), dim3(256), 0, st, D, e1, e2, lo[e1],
                       n1, lo[e2], npen, D.pen_sum);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, D.pen_sum, npen, out);
}

}  // namespace vl
