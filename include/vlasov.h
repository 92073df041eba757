/*
 * vlasov.h — C ABI of libvlasov.so: the Vlasov translation solver on one
 * MI355X (gfx950), for one partition padded with a coalesced ghost domain.
 *
 * Method (Battarbee et al., "Coalescing MPI communication in 6D Vlasov
 * simulations: solving ghost domains in Vlasiator"):
 *  - translation = the v . grad_x f term of the Vlasov equation (Section 2,
 *    eq. 1), split into three Cartesian shears done in a fixed order
 *    (Section 2.1);
 *  - each shear is a conservative semi-Lagrangian piecewise-parabolic remap
 *    along pencils of spatial cells with a 2-cell stencil; |v dt / dx| <= 1
 *    so that only face neighbours exchange mass (Section 2.1); PPM variant:
 *    Colella & Woodward (1984) with fourth-order faces and the monotonicity
 *    limiter;
 *  - velocity space is stored sparsely in 4x4x4 blocks that are added and
 *    removed as the distribution evolves (Section 2);
 *  - Ghost Translation (Section 3, 3.1, Fig. 3): one ghost update per step
 *    of a halo 3 cells deep (2-cell stencil + 1 face neighbour, the "full"
 *    GT3 set of Section 3.2); the first two shears are also computed on the
 *    ghost cells that later shears read.  The classical scheme (Section 2.1,
 *    Fig. 1) refreshes the current direction's ghost faces before each shear.
 *
 * Conventions
 *  - Spatial cells: local box n[0] x n[1] x n[2], periodic, x fastest.  The
 *    library allocates the padded box (n + 6 per axis) inside the workspace.
 *  - Velocity mesh: nblk[d] blocks of 4 cells per axis.  Block id
 *    b = bx + nblk[0] * (by + nblk[1] * bz); lane l = ix + 4 iy + 16 iz within
 *    a block; cell-centre velocity v_d = vmin[d] + (4 b_d + i_d + 1/2) dv[d].
 *  - f: phase-space density [s^3 m^-6] as cell volume averages.
 *  - Every call is ordered on the HIP stream given at init.  Only calls that
 *    say so synchronise the stream.
 *  - Ownership: the caller allocates the device workspace
 *    (vl_workspace_bytes) and keeps it alive until vl_destroy; the library
 *    never allocates device memory.  Host input arrays are read during the
 *    call only.  Device output arrays are written in stream order.
 *  - Status: 0 = VL_OK, negative = error (vl_status_string).  On VL_ERR_ARG
 *    and VL_ERR_CFL nothing has been enqueued.  Device-side overflow of a
 *    capacity is recorded on the device and reported as VL_ERR_CAPACITY by
 *    the next call that synchronises; the partition is then invalid and must
 *    be re-initialised with larger capacities.  Work enqueued after the
 *    overflow (steps, graph replays, ghost updates, moments) does nothing on
 *    the device: its outputs are not written.
 *  - A handle is not thread-safe; separate handles on separate streams are
 *    independent.
 */
#ifndef VLASOV_H
#define VLASOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VL_F64 = 0, VL_F32 = 1, VL_BF16 = 2 };          /* storage of f */
enum { VL_COALESCED = 0, VL_PER_SWEEP = 1 };            /* ghost scheme */
enum {
    VL_OK = 0,
    VL_ERR_ARG = -1,          /* bad descriptor, pointer or size */
    VL_ERR_CFL = -2,          /* some |v dt / dx| > 1 (Section 2.1) */
    VL_ERR_CAPACITY = -3,     /* block, list or work-list capacity exceeded */
    VL_ERR_STALE_GHOSTS = -4, /* coalesced step without a ghost update */
    VL_ERR_HIP = -5,          /* a HIP runtime call failed */
    VL_ERR_STATE = -6,        /* partition invalid after an earlier error */
    VL_ERR_SCRATCH = -7,      /* vl_moments_static: the fixed scratch array is too small */
    VL_ERR_SPLIT = -8         /* vl_accelerate: a cell's velocity map cannot be split
                                 into three one-coordinate remaps */
};

/* Partition descriptor (all fields are read by vl_workspace_bytes and
 * vl_init_partition; none may change afterwards). */
typedef struct vl_desc {
    int32_t n[3];         /* local cells per axis, >= 1 each; n[d] + 6 <= 256 */
    int32_t nblk[3];      /* velocity blocks per axis, each <= 1024; product <= 131072 */
    int32_t order[3];     /* shear order, a permutation of {0,1,2}; x->y->z = {0,1,2};
                             the paper's Z->X->Y = {2,0,1} */
    int32_t storage;      /* VL_F64, VL_F32 or VL_BF16 */
    int32_t stencil;      /* PPM stencil half-width; must be 2 (Section 2.1) */
    int32_t gt_level;     /* Ghost Translation level k of VL_COALESCED steps (Section 3.2):
                             shear s recomputes the k ghost layers nearest the local box
                             along the axes swept after it; 3 (GT3) is exact, 1 (GT1) and
                             2 (GT2) leave the outer layers at their ghost-update values */
    int32_t vbuffer;      /* velocity-space buffer kept around content blocks:
                             0, 6 (face neighbours) or 26 (all neighbours) */
    int32_t edges;        /* faces at the simulation edge, bit 2d: low face of axis d,
                             bit 2d+1: high face (0 = periodic or interior everywhere).
                             The ghost layers beyond such a face are boundary cells
                             (Section 2.1): they feed the stencils but are not
                             translated, so no Ghost Translation layers are computed
                             there (Section 3.3); their contents come from the sources
                             given to vl_fill_ghosts_from (vl_fill_ghosts is then an
                             error). */
    double dx[3];         /* spatial cell size [m], > 0 */
    double vmin[3];       /* lower edge of the velocity mesh [m/s] */
    double dv[3];         /* velocity cell size [m/s], > 0 */
    double sparse_min;    /* content threshold [s^3 m^-6]: a block is kept if one of
                             its values is >= sparse_min; <= 0 disables pruning */
    int64_t block_capacity;       /* block slots for local cells (>= blocks at init) */
    int64_t ghost_block_capacity; /* block slots for ghost cells */
} vl_desc;

/* Optional per-step report (vl_translate_step).  Masses are
 * dx dy dz dvx dvy dvz * sum f over the local cells, in FP64. */
typedef struct vl_step_stats {
    double mass_before;   /* local mass before the step */
    double mass_after;    /* local mass held in f after the step */
    double pruned_mass;   /* mass of the blocks removed by pruning */
    double ledger_mass;   /* FP32/BF16 storage: change of the FP64 rounding residual
                             kept outside f in this step (0 for FP64).  Each shear
                             carries the rounding residual along a pencil line; the
                             line's final residual, per velocity block, is kept in
                             FP64 and put back into that line and block at the next
                             shear along the same axis (spread evenly over its 64
                             cells), so mass_before = mass_after + pruned_mass +
                             ledger_mass up to FP64 rounding, and the residual held
                             outside f stays that of the last shear of each axis */
    int64_t local_blocks; /* blocks held by local cells after the step */
    int64_t updated_ps[3];/* phase-space cells written by each shear (sweep order) */
    int64_t read_ps[3];   /* phase-space cells read by each shear */
    int64_t items[3];     /* (pencil, block) work items of each shear */
    uint64_t device_errors; /* capacity overflow bits recorded on the device (0 = none):
                               1 free local slots, 2 ghost slots, 4 cell list,
                               8 work items, 16 work rows, 32 ghost lists,
                               64 local lists, 128 moments scratch */
} vl_step_stats;

typedef struct vl_partition vl_partition;

/* Device workspace the partition needs, in bytes; 0 if the descriptor is
 * invalid.  Covers the block pool (block_capacity + ghost_block_capacity
 * blocks of 64 values), block lists, work lists and counters. */
size_t vl_workspace_bytes(const vl_desc *d);

/* Create a partition and load its local cells (Section 2: f on a sparse
 * velocity mesh).  Host inputs, local cells only, x fastest:
 *   cell_offsets[n0*n1*n2 + 1]  CSR row pointers in blocks (cell_offsets[0] = 0)
 *   block_ids[cell_offsets[end]] ascending ids per cell, 0 <= id < prod(nblk)
 *   f[64 * cell_offsets[end]]    values, lane order within each block
 * dev_workspace: >= vl_workspace_bytes(d) bytes of device memory, 256-byte
 * aligned.  hip_stream: a hipStream_t (NULL = default stream).  Values are
 * converted to the storage type (round to nearest even).  The ghost domain
 * is invalid until vl_fill_ghosts.  f may be NULL: the values are then zero
 * until vl_load_values supplies them.  Synchronises the stream.
 * Errors: VL_ERR_ARG (descriptor, alignment, size, unsorted or out-of-range
 * ids), VL_ERR_CAPACITY (more blocks than block_capacity), VL_ERR_HIP. */
int vl_init_partition(const vl_desc *d, void *dev_workspace, size_t ws_bytes,
                      void *hip_stream, const int64_t *cell_offsets,
                      const int32_t *block_ids, const double *f, vl_partition **out);

/* Values of the initial blocks [first_block, first_block + nblocks) in the
 * CSR order given to vl_init_partition (64 FP64 values per block, lane order,
 * in device memory), converted to the storage type as there.  For states
 * sampled on the device in pieces.  Only before the first translation step
 * (else VL_ERR_STATE); marks the ghost domain stale.  Asynchronous: dev_f
 * must stay valid until the stream has passed this call.
 * Errors: VL_ERR_ARG (range or pointer), VL_ERR_STATE, VL_ERR_HIP. */
int vl_load_values(vl_partition *p, int64_t first_block, int64_t nblocks, const double *dev_f);

/* Coalesced ghost update (Section 3, Fig. 3a): every cell of the padded box
 * outside the local box receives the block list and values of its periodic
 * image.  Once per step, before a VL_COALESCED step.  Asynchronous.
 * VL_ERR_ARG if desc.edges is set (boundary cells need their sources). */
int vl_fill_ghosts(vl_partition *p);

/* Coalesced ghost update from neighbouring partitions (Section 3, Fig. 3a:
 * the one exchange of a Ghost Translation step): every ghost cell of p
 * receives the block list and values of the cell at the same position in the
 * partition that owns it.  nbr[(dx+1) + 3(dy+1) + 9(dz+1)] is the partition
 * displaced by (dx, dy, dz) local boxes, nbr[13] == p; all 27 have the same
 * local box (each side >= 3 cells), velocity mesh and storage, and live on the
 * same device (or are readable from it).  The neighbours' local cells are read
 * on p's stream: the caller orders their previous steps before this call and
 * this call before their next steps.  The partition keeps these sources for
 * its per-sweep face refreshes and its graph-recorded ghost updates.  Beyond
 * a simulation edge (desc.edges) the source is a partition that is never
 * stepped, whose cells hold the boundary cells' fixed contents.
 * Asynchronous.
 * Errors: VL_ERR_ARG (mismatch, NULL, nbr[13] != p), VL_ERR_STATE, VL_ERR_HIP. */
int vl_fill_ghosts_from(vl_partition *p, vl_partition *const *nbr);

/* One translation step: three shears in desc.order (Section 2.1), each a PPM
 * remap of every velocity cell along its spatial pencils with Courant number
 * v dt / dx[d], followed by block pruning of the local cells.
 *   mode VL_COALESCED: Ghost Translation; needs vl_fill_ghosts since the
 *        last step (else VL_ERR_STALE_GHOSTS).
 *   mode VL_PER_SWEEP: classical per-direction ghost refresh (Fig. 1), from
 *        the sources of the last vl_fill_ghosts_from if there was one
 *        (required when desc.edges is set), else from periodic images.
 * Both modes give the same local result bit for bit (in FP32/BF16 storage
 * for a partition that stays in one mode: a coalesced step also carries the
 * rounding residuals of the ghost lines it translates, which a per-sweep step
 * does not translate).  The ghost domain is stale afterwards.  dt > 0 [s].  stats: optional host output; if non-NULL
 * the call synchronises and also reports device-side errors.
 * Errors: VL_ERR_ARG, VL_ERR_CFL (checked on the host before launch),
 * VL_ERR_STALE_GHOSTS, VL_ERR_CAPACITY (with stats), VL_ERR_STATE, VL_ERR_HIP. */
int vl_translate_step(vl_partition *p, double dt, int32_t mode, vl_step_stats *stats);

/* Acceleration step: the Lorentz-force term of the Vlasov equation (Section 2,
 * eq. 1, the velocity-space half of the split step, whose solver Section 2
 * names as SLICE-3D).  Per local cell, in the cell's fields E, B, constant
 * over the step, every velocity moves along its exact characteristic: the
 * affine map v' = A v + c with A the rotation by -qm |B| dt about B/|B| and c
 * the E x B drift's part plus the acceleration qm (E.b) dt b along b (with
 * B = 0: v' = v + qm E dt).  The map is applied as three one-coordinate maps
 * in slice_order (a permutation of {0,1,2}, NULL = x, y, z), each setting one
 * velocity coordinate to its final value: a conservative remap of every
 * velocity column along that axis, cell i receiving the mass of its pre-image
 * under the CW84 parabolas of the column (the spatial remap's slopes, faces
 * and limiter).  Mass moved beyond the velocity mesh is lost.  The cell's
 * block set becomes its old blocks plus every block holding a nonzero value,
 * then the end-of-step pruning (sparse_min, vbuffer) as after a translation
 * step.  Computed in FP64 from any storage; the result is rounded to the
 * storage type (no rounding carry).
 *   dev_fields: device, 6 doubles per local cell (Ex, Ey, Ez [V/m],
 *               Bx, By, Bz [T]), x fastest, read only during the call.
 *   qm: charge-to-mass ratio [C/kg]; dt > 0 [s].
 *   stats: optional host output (mass before and after, pruned mass, local
 *          blocks; no ledger); if non-NULL the call synchronises again.
 * The call synchronises once to check the maps: if some cell's map cannot be
 * split (a step's own coefficient not positive, e.g. a rotation of half a
 * turn or more) it returns VL_ERR_SPLIT with f unchanged.  Velocity meshes of
 * more than 64 blocks along an axis are not supported (VL_ERR_ARG).  The
 * ghost domain is stale afterwards.
 * Errors: VL_ERR_ARG, VL_ERR_SPLIT, VL_ERR_CAPACITY (with stats), VL_ERR_STATE,
 * VL_ERR_HIP. */
int vl_accelerate(vl_partition *p, double dt, double qm, const double *dev_fields, const int32_t *slice_order,
                  vl_step_stats *stats);

/* nsteps whole steps, each recorded once into a HIP graph and replayed: in
 * VL_COALESCED mode the coalesced ghost update followed by the three shears
 * and pruning (Section 3.2: one ghost update, then the translations in
 * order); in VL_PER_SWEEP mode the per-direction refreshes and shears.  Each
 * step gives the same state bit for bit as vl_fill_ghosts (coalesced mode)
 * plus vl_translate_step.  The graphs are cached per starting list region
 * and, in FP32/BF16 storage, per rotation of the per-line ledger stores (a
 * step swaps them, repeating every four steps), and re-recorded when dt,
 * mode, shear variant or Courant override change;
 * recording uses a private stream, replays go to the partition's stream.
 * The recorded ghost update uses the sources of the last vl_fill_ghosts_from
 * if there was one (required when desc.edges is set), else periodic images.
 * Asynchronous: device-side errors surface at the next synchronising call.
 * The ghost domain is stale afterwards.  nsteps >= 0.
 * Errors: VL_ERR_ARG, VL_ERR_CFL, VL_ERR_STATE, VL_ERR_HIP. */
int vl_graph_step(vl_partition *p, double dt, int32_t mode, int32_t nsteps);

/* Velocity moments of the local cells, FP64 (paper silent; textbook
 * definitions): n = dv^3 sum f; V = dv^3 sum f v / n;
 * P_ab = m_p dv^3 sum f (v_a - V_a)(v_b - V_b), m_p = 1.67262192e-27 kg.
 * Device outputs, local cells x fastest: dev_n[ncell], dev_V3[3*ncell],
 * dev_P6[6*ncell] in the order xx, yy, zz, xy, xz, yz (any may be NULL).
 * host_total_mass: optional; sum n dx dy dz, synchronises if non-NULL. */
int vl_moments(vl_partition *p, double *dev_n, double *dev_V3, double *dev_P6,
               double *host_total_mass);

/* vl_moments for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * kernels and outputs, with their scratch (the per-cell chunk table and
 * masses, the partial sums of cells split over several wavefronts, two
 * counters) in a fixed device array of 64 MiB that the library holds on every
 * device it runs on until the process ends; nothing is allocated.  dev_n,
 * dev_V3, dev_P6 as in vl_moments (any may be NULL); dev_total_mass: optional
 * device double receiving sum n dx dy dz.  Asynchronous; never synchronises.
 * The array is shared by all partitions on a device and keeps the last
 * call's contents (the counters are cleared by each call): calls that
 * overlap on one device race and give wrong results.  Bit-identical to
 * vl_moments whenever its split of the cells fits the array (cells are split
 * into more blocks per wavefront otherwise).
 * Errors: VL_ERR_SCRATCH (more local cells than the array can describe,
 * about 5 million), VL_ERR_ARG, VL_ERR_STATE, VL_ERR_HIP. */
int vl_moments_static(vl_partition *p, double *dev_n, double *dev_V3, double *dev_P6,
                      double *dev_total_mass);

/* Number of blocks held by the local cells.  Synchronises. */
int vl_local_block_count(vl_partition *p, int64_t *out);

/* Copy the local cells to host memory as CSR (ids ascending per cell, values
 * converted to FP64): cell_offsets[ncell+1], block_ids[cap_blocks],
 * f[64*cap_blocks].  VL_ERR_ARG if cap_blocks is too small.  Synchronises.
 * The per-line rounding ledger of FP32/BF16 storage is not part of the
 * exported state: a partition initialised from it starts with an empty
 * ledger (its stored mass is what f holds). */
int vl_export_state(vl_partition *p, int64_t *cell_offsets, int32_t *block_ids, double *f,
                    int64_t cap_blocks);

/* As vl_export_state for the local cells listed in cells[0..ncells) (local
 * x-fastest indices), in that order.  Synchronises. */
int vl_export_cells(vl_partition *p, const int64_t *cells, int64_t ncells,
                    int64_t *cell_offsets, int32_t *block_ids, double *f, int64_t cap_blocks);

/* Test hook: replace the Courant numbers by table[d * stride + j] for
 * velocity index j along axis d (|values| <= 1), e.g. to drive exact integer
 * shifts; NULL restores v dt / dx.  Synchronises. */
int vl_set_courant_override(vl_partition *p, const double *table, int32_t stride);

/* Diagnostics: copy the device book-keeping counters to out[0..n) (n <= 32):
 * [0] free-ring head, [1] free-ring tail, [2] free-ring limit, [3] ghost slots
 * used, [4] ghost list entries used, [5..6] local list entries used (regions
 * 0, 1), [7] work items, [8] work rows, [9] work counter, [10] error bits,
 * [11..13] updated, [14..16] read phase-space cells, [17..19] items per shear
 * of the last step, [20] local list region in use, [21] updated and [22] read
 * phase-space cells summed over all shears since init.  Synchronises. */
int vl_counters(vl_partition *p, uint64_t *out, int32_t n);

/* Diagnostics: kernel timing with HIP events recorded on the partition's
 * stream around every launch of the ghost update, planner, shear, pruning,
 * moment and acceleration kernels, for up to max_launches launches after
 * vl_profile_start.
 * vl_profile_stop synchronises and returns, per class (0 ghost update,
 * 1 planner, 2 shears (all), 3 pruning, 4 moments, 5/6/7 first/second/third
 * shear of the step, 8 acceleration remaps), the summed milliseconds ms[9]
 * and the launch counts launches[9], then stops recording. */
int vl_profile_start(vl_partition *p, int32_t max_launches);
int vl_profile_stop(vl_partition *p, double *ms, int64_t *launches);

/* Autotuner (Section 2.1's shear, kernel shapes only): runs steps_per_variant
 * x (number of compiled variants) real translation steps (each with its ghost
 * update in VL_COALESCED mode, taken as vl_graph_step takes it: from the
 * sources of the last vl_fill_ghosts_from if there was one, which must exist
 * when desc.edges is set, else from periodic images): first one step with every variant of the
 * shear kernel (store scheme, prefetch depth, occupancy target), then rounds
 * over the variants within 25 % of the best mean time on some shear, until
 * the steps are spent.  Each shear launch is timed with HIP events on the
 * partition's stream and taken per phase-space cell the shear read and
 * updated (the lists grow from step to step, and the variants tried first
 * would otherwise look faster); for each of the three shears of the order
 * the variant with the lowest mean of that time on it is kept (the third shear, which also
 * records the blocks' content flags, has kernels of its own with other
 * register needs).  All variants compute bit-identical results, so the state
 * advances exactly as with ordinary steps.  best[3] receives the chosen
 * variant of the first, second and third shear; ms_out (optional, ms_cap
 * entries) the mean milliseconds per step of all three shears with each
 * variant.  Synchronises.  Errors as vl_translate_step (VL_ERR_STALE_GHOSTS
 * when desc.edges is set and no sources were given). */
int vl_autotune(vl_partition *p, double dt, int32_t mode, int32_t steps_per_variant, int32_t best[3],
                double *ms_out, int32_t ms_cap);

/* Select one shear-kernel variant (0 .. number of variants - 1) for all
 * three shears.  VL_ERR_ARG outside that range. */
int vl_set_variant(vl_partition *p, int32_t variant);

/* Select the variant of each shear of the order (first, second, third);
 * VL_ERR_ARG (nothing changed) if any is outside 0 .. number of variants - 1. */
int vl_set_shear_variants(vl_partition *p, const int32_t variants[3]);

/* The variants in use for the three shears; *count (optional) receives the
 * number of compiled variants.  Does not touch the device. */
int vl_get_shear_variants(const vl_partition *p, int32_t variants[3], int32_t *count);

/* Wait for the partition's stream and report device-side errors. */
int vl_sync(vl_partition *p);

/* Release the host-side handle (the workspace stays the caller's). */
void vl_destroy(vl_partition *p);

const char *vl_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* VLASOV_H */
