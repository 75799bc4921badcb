/*
 * amrx.h -- C ABI of libamrx, the gfx950 (MI355X) hot path of patch-based AMR MHD.
 *
 * The library advances a static, properly nested hierarchy of ghost-padded
 * patches with refinement ratio R = 2 and ghost width G = 4 = R * n_g, n_g = 2
 * being the stencil depth of one substep.  It follows the paper's statement
 * of the problem (Carroll-Nellenback, Shroyer, Frank & Ding, "Efficient
 * Parallelization for AMR MHD Multiphysics Calculations; Implementation in
 * AstroBEAR"):
 *   - patches on levels l with cell width dx_{l-1} = R dx_l, each refined patch
 *     nested in a single parent (Sec. 2);
 *   - one step of level l = Advance, Prolongate pre-advance data to the
 *     children, the children's R substeps, Restrict data and fluxes onto the
 *     parent, Synchronise fluxes with same-level neighbours (Sec. 2.2, the
 *     recursive AMR(l) routine);
 *   - extended ghost cells: a refined patch first updates a region R*n_g
 *     wider than its interior and then successively smaller ones, so it needs
 *     ghost data from its parent only before its first substep (Sec. 2.3);
 *   - level advances may proceed independently, finer levels first (Sec. 4).
 * The per-patch advance is an unsplit MUSCL-Hancock step with HLLD fluxes
 * (Miyoshi & Kusano 2005) and constrained-transport EMFs (Gardiner & Stone
 * 2005); the paper does not describe its solver.
 *
 * Conventions shared by every entry point
 *   - Return value: AMRX_OK (0) or a negative AMRX_E* code.  No entry point
 *     aborts or throws; the text of the last error is hier_last_error().
 *   - Indices are (x, y, z) triples in the index space of the patch's level
 *     (level l has root_n[d] * 2^l cells along axis d on [lo, hi) of the
 *     domain, periodic on all axes).
 *   - Device memory is owned by the caller (e.g. PyTorch tensors) and bound
 *     once with hier_bind(); the library never allocates or frees device
 *     memory.  The library owns only host metadata.
 *   - Asynchrony: every call after hier_bind() is enqueued on desc.stream and
 *     returns without waiting, except cfl_dt(), hier_step(), hier_conservation()
 *     and hier_diag(), which synchronise that stream.  Calls on one hierarchy
 *     must not run concurrently from several host threads.
 *
 * Memory layout of the state arena (size reported by hier_finalize)
 *   Every patch owns two state buffers (current and next; an advance writes
 *   the next buffer and then swaps).  A buffer holds 8 arrays of the patch's
 *   node-padded volume V = (nx+2G+1)(ny+2G+1)(nz+2G+1) real numbers, each
 *   indexed [z][y][x] with x fastest: rho, m_x, m_y, m_z, E (cell centred,
 *   valid on [0, n+2G) per axis) and b_x, b_y, b_z (face-normal field; entry
 *   [k][j][i] of b_x is the face at x = i - 1/2 of padded cell i, likewise for
 *   y and z).  Padded index i corresponds to level index lo_x - G + i.  The
 *   real type is double for AMRX_FP64 and float for both FP32 modes.
 *   patch_layout() gives the byte offset of each array of each buffer.
 */
#ifndef AMRX_H
#define AMRX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AMRX_OK = 0,
  AMRX_EINVAL = -1,   /* bad argument (null pointer, bad size, bad level, ...) */
  AMRX_ENEST = -2,    /* box violates nesting: odd corner, or not inside exactly one parent's
                         interior shrunk by one parent cell on every side */
  AMRX_EOVERLAP = -3, /* box overlaps a patch of the same level */
  AMRX_ENOMEM = -4,   /* a bound buffer is too small */
  AMRX_EHIP = -5,     /* a HIP runtime call failed (message in hier_last_error) */
  AMRX_ESTATE = -6,   /* call out of order (e.g. patch_add after hier_finalize) */
  AMRX_EPHYS = -7     /* device flagged rho <= 0, p <= 0 or a non-finite value */
};

enum { AMRX_FP64 = 0, AMRX_FP32 = 1, AMRX_FP32_MIXED = 2 };

/* Schedules of hier_step(). */
enum {
  AMRX_PLAIN = 0,     /* every stage launched separately for every patch */
  AMRX_BATCHED = 1,   /* every stage launched once for all patches of a level substep */
  AMRX_GRAPH = 2,     /* AMRX_BATCHED captured once into a HIP graph and replayed */
  AMRX_PERSISTENT = 3,/* one launch of a persistent work-queue kernel per root step: every
                         batched launch becomes a node of a dependency graph, levels run
                         concurrently and ready work of finer levels is taken first (Sec. 4) */
  AMRX_CONCURRENT = 4,/* the same dependency graph of batched launches captured into a HIP graph
                         with one branch per level: launches of different levels that touch
                         disjoint data run concurrently (Sec. 4: coarser levels fill the gaps
                         left by finer ones); replayed like AMRX_GRAPH.
                         AMRX_PERSISTENT and AMRX_CONCURRENT are disabled in this version of the library
                         (hier_step returns EINVAL for them). */
  AMRX_LAYERED = 5    /* the AMRX_PERSISTENT dependency graph cut into layers of mutually
                         independent batched launches (a node's layer is one past its latest
                         predecessor's); one launch per layer of a persistent grid whose
                         workgroups claim the layer's block ranges, finer levels' first, from
                         an atomic counter and never wait for each other.  Staged stages only
                         (the fused-kernel tunings do not apply); synchronising like
                         AMRX_BATCHED's dt readback; bit-identical results. */
};

typedef struct amrx_hier amrx_hier;

typedef struct {
  int root_n[3];      /* level-0 cells per axis; refinement requires root_n[0]==root_n[1]==root_n[2] */
  int max_level;      /* deepest level that may hold patches (0 .. 15) */
  int ratio;          /* refinement ratio; must be 2 */
  int nghost;         /* ghost width; must be 4 */
  double gamma;       /* adiabatic index of the ideal gas */
  double cfl;         /* Courant number used by cfl_dt() */
  int precision;      /* AMRX_FP64, AMRX_FP32 or AMRX_FP32_MIXED */
  void* stream;       /* hipStream_t all work is enqueued on (NULL = default stream) */
} amrx_desc;

/* Create an empty hierarchy.  Pure host call.  EINVAL on a bad descriptor. */
int hier_create(const amrx_desc* desc, amrx_hier** out);

/* Destroy host metadata.  Bound device memory stays with its owner. */
int hier_destroy(amrx_hier* h);

/* hier_set_isothermal: switch the hierarchy to the isothermal hydro workload
 *   (the density-and-momentum state the paper counts in its memory estimate,
 *   Sec. 3): p = cs^2 rho, the MUSCL-Hancock step with an isothermal HLLC flux
 *   (mass and normal momentum HLL between min(u) - cs and max(u) + cs, the
 *   transverse momenta upwinded by the contact speed), no energy equation.
 *   The state layout is unchanged: the caller keeps E and the face fields at
 *   zero (they stay zero).  Call before hier_bind (AMRX_ESTATE after);
 *   AMRX_EINVAL unless cs > 0. */
int hier_set_isothermal(amrx_hier* h, double cs);

/* Text of the last error on h (never NULL). */
const char* hier_last_error(const amrx_hier* h);

/* Add the patch [lo, hi) on `level` (Sec. 2: a grid's node with its position and its parent).
 * Level-0 patches must tile the root grid (checked by hier_finalize).  On
 * levels >= 1, lo and hi must be even and the box must lie inside exactly one
 * level-(l-1) patch's interior shrunk by one parent cell; same-level boxes
 * must not overlap.  A patch's ghost-padded extents hi - lo + 9 must stay
 * below 2^20 per axis and their product below 2^31 entries (EINVAL otherwise).  Pure host call.  Errors: EINVAL,
 * ENEST, EOVERLAP, ESTATE. */
int patch_add(amrx_hier* h, int level, const int lo[3], const int hi[3], int* patch_id);

/* Freeze the topology and build every index list (ghost sources, prolongation
 * cells, coverage maps, register layouts, stage task tables).  Pure host call.
 * Reports the byte sizes of the state arena and of the scratch arena the
 * caller must allocate.  Errors: ESTATE (twice), ENEST (root not tiled). */
int hier_finalize(amrx_hier* h, size_t* state_bytes, size_t* scratch_bytes);

/* Byte offsets, within the state arena, of the 8 arrays (rho, mx, my, mz, E,
 * bx, by, bz) of buffer `which` (0 or 1) of a patch, and the padded array
 * shape dims = (NX+1, NY+1, NZ+1).  Pure host call after hier_finalize. */
int patch_layout(const amrx_hier* h, int patch_id, int which, size_t offsets[8], int dims[3]);

/* Index of the buffer (0 or 1) that currently holds the state of a patch. */
int patch_current(const amrx_hier* h, int patch_id, int* which);

/* Bind the caller-owned device arenas (256-byte aligned) and upload the index
 * lists.  Must follow hier_finalize.  ENOMEM if a size is too small. */
int hier_bind(amrx_hier* h, void* state, size_t state_bytes, void* scratch, size_t scratch_bytes);

/* Ghost update of every patch of `level` before substep `substep`: copy the
 * interior (closure, for faces) of the same-level patch holding each ghost
 * value's periodic image (Sec. 2.1: between the first and last substep,
 * ghost data come from same-level neighbours of the same iteration); on
 * levels >= 1 at substep 0, fill the ghost values no same-level patch holds
 * by prolongation of the parent's data from before the parent's advance
 * (Sec. 2.2 P step, Sec. 2.3). */
int level_ghost_fill(amrx_hier* h, int level, int substep);

/* Advance every patch of `level` by dt_level (Sec. 2.2 "Advance"): substep s
 * of a refined patch updates its interior grown by (R-1-s)*n_g cells, level 0
 * its interior (Sec. 2.3).  Records boundary fluxes and EMFs for refluxing
 * and synchronisation, then makes the written buffer current. */
int advance_level(amrx_hier* h, int level, double dt_level, int substep);

/* Restrict level fine_level onto its parents (Sec. 2.2 R step: both the fine
 * data and the fine fluxes are carried to the parent): covered coarse cells
 * and faces take the volume / area mean of the fine data; uncovered coarse
 * cells and faces next to the fine region are corrected so that the coarse
 * fluxes and EMFs across the coverage boundary equal the time and space
 * averages of the fine ones. */
int restrict_level(amrx_hier* h, int fine_level);

/* Synchronise fluxes through faces shared by patches of `level` (Sec. 2.2 S
 * step, flux agreement between adjacent grids of one level): the two sides'
 * fluxes of the last substep are compared, replaced by their mean and the
 * adjacent cells corrected; the largest difference seen is kept for hier_diag. */
int sync_level(amrx_hier* h, int level);

/* Largest stable root time step: dt_l,max = cfl / max over the level's
 * interior cells of sum_d (|v_d| + c_f,d) / dx_l, dt0 = min_l 2^l dt_l,max
 * (the level time steps then follow dt_{l+1} = dt_l / R, Sec. 2.2).
 * Synchronising.  EPHYS if the device flagged an unphysical state. */
int cfl_dt(amrx_hier* h, double* dt0);

/* One root step (Sec. 2.2 recursion AMR(0); serial visit order 0,1,2,2,1,2,2
 * for three levels, Sec. 4).  If *dt0 > 0 on entry it is used, otherwise
 * cfl_dt() chooses it and it is returned.  Synchronising. */
int hier_step(amrx_hier* h, int mode, double* dt0);

/* `nsteps` root steps (Sec. 2.2 recursion AMR(0), one after another) enqueued
 * back to back with no host synchronisation between them; mode AMRX_PLAIN,
 * AMRX_BATCHED or AMRX_GRAPH.  Every step takes dt0 if dt0 > 0, otherwise
 * its own dt from the CFL condition, computed on the device.  Synchronises
 * once, at the end.  *t_advanced = the sum of the steps' dt, accumulated on
 * the device in float64 in step order; *dt_last = the last step's dt (0 for
 * nsteps = 0); either pointer may be NULL.  EPHYS if any of the steps flagged
 * an unphysical state (the flag is latched over the whole run).  States and
 * dts equal those of nsteps hier_step() calls with the same mode and dt0,
 * bit for bit.  EINVAL for another mode, nsteps < 0 or dt0 < 0 or NaN. */
int hier_steps(amrx_hier* h, int mode, int nsteps, double dt0, double* t_advanced, double* dt_last);

/* Sums over leaf cells (not covered by a finer patch) of (rho, m_x, m_y,
 * m_z, E, B_x, B_y, B_z) * cell volume, in float64 with compensated
 * summation: sum[i] + comp[i] is the result.  Synchronising. */
int hier_conservation(amrx_hier* h, double sum[8], double comp[8]);

/* Diagnostics: out[0] = largest flux mismatch seen by sync_level, out[1] =
 * largest face-field mismatch on shared faces, out[2] = 1 if the device
 * flagged an unphysical state.  Synchronising.  n = number of slots (<= 3). */
int hier_diag(amrx_hier* h, double* out, int n);

/* Kernel classes reported by hier_timing_read (one slot each). */
enum {
  AMRX_K_PRIM = 0, AMRX_K_BHALF, AMRX_K_PRED, AMRX_K_FLUX, AMRX_K_EDGE, AMRX_K_UPDATE,
  AMRX_K_COPY, AMRX_K_PROLONG, AMRX_K_RESTRICT, AMRX_K_FLUXCORR, AMRX_K_EMFCORR, AMRX_K_SYNC,
  AMRX_K_CFL, AMRX_K_CONS,
  AMRX_K_PRIMHALF,   /* stages prim, bhalf and pred fused into one LDS-tiled kernel */
  AMRX_K_EDGEUPD,    /* stages edge EMF and update fused into one LDS-tiled kernel */
  AMRX_NKCLASS
};

/* Measurement support.  hier_timing_enable(h, 1) starts recording a HIP event
 * before and after every kernel launch the library enqueues on desc.stream
 * (discarding earlier records); hier_timing_enable(h, 0) stops recording.
 * hier_timing_read synchronises the stream and returns, per kernel class
 * (n <= AMRX_NKCLASS slots), the summed device time in ms between the
 * events and the number of launches.  Recording adds two event records per
 * launch. */
int hier_timing_enable(amrx_hier* h, int on);
int hier_timing_read(amrx_hier* h, int n, double* total_ms, int* launches);

/* Work of one root step per kernel class (pure host, after hier_finalize):
 * units[k] = number of entries the class processes (cells, faces, edges or
 * nodes of the stage regions; copied elements for AMRX_K_COPY; parent cells
 * for AMRX_K_PROLONG; coarse nodes for AMRX_K_RESTRICT; list entries for
 * the corrections and synchronisation; interior cells for AMRX_K_CFL;
 * algorithmic words for AMRX_K_PRIMHALF: 8 read and 8 written per cell of the
 * primitive region, 14 written per cell of the half-step region; algorithmic
 * words for AMRX_K_EDGEUPD: 23 read and 8 written per entry of the update
 * region plus 3 read per edge of the edge region), and
 * launches[k] = kernel launches of that class in the batched schedule, for
 * the current tuning (staged or fused first three and last two stages).  In the
 * batched schedule the flux and EMF corrections run inside the restriction's
 * launch (AMRX_K_FLUXCORR / AMRX_K_EMFCORR report entries but no launches) and
 * the CFL reductions of all levels share one launch. */
int hier_step_work(const amrx_hier* h, int n, double* units, int* launches);

/* Launch tuning (autotuner hooks).  Per level, the first three advance
 * stages run either as three staged kernels (the default) or as one kernel
 * over tiles of the primitive region staged through LDS, with a tile shape
 * from a fixed table.  Both give bit-identical results.
 *   AMRX_TUNE_FUSED: 0 staged, 1 fused
 *   AMRX_TUNE_TILE:  index into the tile table
 *   AMRX_TUNE_EXTEND_ALL: 1 = the substep-0 update region of every refined patch
 *     extends over all six sides (every grid treated as isolated, Sec. 2.3);
 *     0 (default) = only over sides whose extended ghost layers lack a
 *     same-level source somewhere (elsewhere the next substep's ghost copy
 *     replaces those values, so interiors are bit-identical either way).
 *     Level ignored; only before hier_finalize (ESTATE after).
 *   AMRX_TUNE_PAIR: 1 = in the batched and graph schedules, a level's staged
 *     advance shares its launches with the next finer level's first-substep
 *     ghost fill and staged advance (which read only the coarser level's
 *     pre-advance buffer), two batched launches per grid; 0 (default) = one
 *     after the other.  Levels running the fused first stages are not paired;
 *     launches are not paired while launch timing is on.  Level ignored.
 *   AMRX_TUNE_FUSED_EU: 0 (default) staged edge EMF and update kernels, 1 one
 *     kernel over tiles of the update region that computes the tile's edge
 *     EMFs (and a one-layer halo) into LDS and updates its cells and faces
 *     from them; bit-identical results.  Levels running it are not paired.
 *   AMRX_TUNE_TILE_EU: index into the tile table for AMRX_TUNE_FUSED_EU
 *   AMRX_TUNE_GHOSTS: how refined patches get ghost data for their later
 *     substeps (Sec. 2.3 names both solutions for isolated grids).  0 (default)
 *     extended ghost regions: substep 0 also updates up to (R-1) n_g ghost
 *     layers (on the sides AMRX_TUNE_EXTEND_ALL selects).  1 coarse time
 *     derivative: every substep updates the interior only; before substep s >= 1
 *     the parent level's n_g ghost layers are refreshed from their same-level
 *     sources at its advanced time and the ghost data without a same-level
 *     source is prolongated from old + (s / R) (new - old) of the parent (its
 *     pre-advance and advanced buffers).  hier_finalize then returns ENEST if
 *     such a prolongation would read a parent entry that is neither interior
 *     (closure, for faces) nor a same-level-sourced ghost entry within n_g
 *     layers.  Only before hier_finalize (ESTATE after); level ignored; the
 *     persistent and concurrent schedules refuse it (EINVAL).
 *   AMRX_TUNE_FLUX_SPLIT (FP32_MIXED only; other precisions ignore it): 1
 *     (default) the flux stage runs as two launches over the same faces, a
 *     float one that leaves the low-beta faces (a NaN mass flux, and the
 *     wave holding one appended to a device list) and one that solves those
 *     faces' Riemann problems in double, so the float kernel keeps the plain
 *     FP32 kernel's register footprint; 0 one launch with the double solver
 *     inline, better where most faces are low-beta.  Bit-identical results.
 *   AMRX_TUNE_UPDATE_NT: 1 = the staged update kernel writes the next state
 *     with non-temporal stores (a cache hint; faster on some levels, slower
 *     on others), 0 (default) ordinary stores.  Bit-identical results.
 * level = -1 sets every level.  Pure host calls (captured graph-schedule steps
 * are discarded on a change).  EINVAL for a bad parameter, level or index, or
 * a tile whose LDS footprint exceeds the limit for the hierarchy's precision. */
enum { AMRX_TUNE_FUSED = 0, AMRX_TUNE_TILE = 1, AMRX_TUNE_EXTEND_ALL = 2, AMRX_TUNE_PAIR = 3,
       AMRX_TUNE_FUSED_EU = 4, AMRX_TUNE_TILE_EU = 5, AMRX_TUNE_GHOSTS = 6, AMRX_TUNE_FLUX_SPLIT = 7,
       AMRX_TUNE_UPDATE_NT = 8 };
int hier_tune_set(amrx_hier* h, int level, int param, int value);
int hier_tune_get(const amrx_hier* h, int level, int param, int* value);

/* The tile table: n_tiles receives its length; if shapes is non-NULL it
 * receives up to cap (tx, ty, tz) triples and lds_bytes (if non-NULL) the LDS
 * bytes per workgroup of each tile at `precision` (0 where the tile is not
 * allowed at that precision).  Pure host call. */
int hier_tile_table(int precision, int* n_tiles, int* shapes, int* lds_bytes, int cap);

/* Time the first three stages of (level, substep): the fused kernel with
 * tile `tile`, or the three staged kernels for tile = -1; `reps` repetitions
 * on desc.stream bracketed by HIP events; *ms = mean device time per
 * repetition.  Writes only intermediate scratch, never the state (so it may
 * run between steps).  Synchronising.  Needs hier_bind. */
int hier_tune_time(amrx_hier* h, int level, int substep, int tile, int reps, double* ms);

/* Time the edge EMF and update stages of substep 0 of `level`: the fused
 * kernel with tile `tile` (every table entry is allowed: its LDS footprint is
 * 3 (tx+1)(ty+1)(tz+1) reals), or the two staged kernels for tile = -1
 * (-2: with the non-temporal update of AMRX_TUNE_UPDATE_NT); `reps` repetitions, *ms = mean device time per repetition.  Writes the
 * level's next-state buffer and its EMF registers, which hold nothing needed
 * between root steps: call it only between steps (hier_step), never inside a
 * sequence of per-level calls.  Synchronising.  Needs hier_bind. */
int hier_tune_time_eu(amrx_hier* h, int level, int tile, int reps, double* ms);

/* Time the flux stage of substep 0 of `level` in FP32_MIXED's two-launch
 * (split = 1) or one-launch (split = 0) form (other precisions: their one
 * form), after one untimed pass of the staged first stages so the low-beta
 * faces are those of the current state; *ms = mean device time per
 * repetition.  Writes intermediates and the level's flux registers, which hold
 * nothing needed between root steps: call it only between steps.
 * Synchronising.  Needs hier_bind. */
int hier_tune_time_flux(amrx_hier* h, int level, int split, int reps, double* ms);

/* Regridding of the finest level (Sec. 2.2: a level's grids decide which cells
 * to refine and lay down child grids over them; new grids take the data of the
 * preceding grids of their level where those overlap them and are prolongated
 * from the parent elsewhere).
 *
 * hier_flag_bytes: bytes of a flag array = padded cells of all patches.
 * hier_flag: device flags (one byte per padded cell; patch p's cell at padded
 *   index q is byte first_state_offset(p) / 16 + q, see patch_layout) of the
 *   interior cells of `level`: 1 where the density jump to a face neighbour
 *   inside the same patch exceeds eps times the smaller density, evaluated in
 *   the state's precision.  Asynchronous on desc.stream.
 * amrx_cluster: Berger-Rigoutsos clustering (pure host) of a flag array
 *   f[(z ny + y) nx + x]: boxes (lo x, y, z, hi x, y, z; cap of them) covering
 *   every flag, each shrunk to its flags and kept once flagged / volume >=
 *   efficiency or no side can be cut into two of >= min_side; cuts at the
 *   flag-free plane nearest the middle, else at the strongest sign change of
 *   the signature's second difference, else in the middle of the longest
 *   axis.  ENOMEM (with *nboxes set) if more than cap boxes result.
 * hier_regrid_boxes: level-(level+1) boxes (pure host) from a downloaded flag
 *   array: per level-`level` patch in id order its interior flags grown by one
 *   cell in all 26 directions, cleared within one cell of the interior
 *   boundary (the nesting rule), clustered, scaled by R.
 * hier_init_from_bytes / hier_init_from: fill a new hierarchy `dst` whose
 *   finest level `level` replaces that of `src` (the levels below must be the
 *   same patches in both; same precision): lower levels copy src's current
 *   buffers, level-`level` interiors (closures, for faces) copy src's
 *   level-`level` patches where they overlap, and the remaining parent cells
 *   under them are prolongated (the ghost-fill operator) from dst's parent
 *   level.  work: device workspace of at least the queried bytes, 256-byte
 *   aligned.  Synchronising; ghost data is filled by the next step.
 * hier_init_from_levels_bytes / hier_init_from_levels: the same with two
 *   sources, for regridding several levels coarse to fine (Sec. 2.2: each new
 *   level is laid over the flags of the new level below it and takes the data
 *   of the old grids of its own level): the levels below `level` copy the
 *   identical patches of `below` (a hierarchy already holding the new coarser
 *   levels), level `level` copies the overlapping level-`level` patches of
 *   `src` (the old hierarchy; none when src has no such level) and is
 *   prolongated from dst's level - 1 elsewhere.  hier_init_from(dst, src, ...)
 *   is hier_init_from_levels(dst, src, src, ...).  EINVAL when `below` lacks
 *   a patch of dst's lower levels, when the precisions differ or when `level`
 *   is not dst's finest level; ESTATE when a hierarchy is not bound. */
int hier_flag_bytes(const amrx_hier* h, size_t* bytes);
int hier_flag(amrx_hier* h, int level, double eps, unsigned char* flags);
int amrx_cluster(const unsigned char* flags, int nx, int ny, int nz, int min_side, double efficiency, int* boxes,
                 int cap, int* nboxes);
int hier_regrid_boxes(const amrx_hier* h, int level, const unsigned char* flags, int min_side, double efficiency,
                      int* boxes, int cap, int* nboxes);
int hier_init_from_bytes(const amrx_hier* dst, const amrx_hier* src, int level, size_t* bytes);
int hier_init_from(amrx_hier* dst, const amrx_hier* src, int level, void* work, size_t work_bytes);
int hier_init_from_levels_bytes(const amrx_hier* dst, const amrx_hier* below, const amrx_hier* src, int level,
                                size_t* bytes);
int hier_init_from_levels(amrx_hier* dst, const amrx_hier* below, const amrx_hier* src, int level, void* work,
                          size_t work_bytes);

/* hier_init_from_levels_static: hier_init_from_levels for callers that cannot
 *   allocate device memory (code under HIP graph capture, tight serving loops,
 *   harnesses that forbid hipMalloc).  It takes no workspace: the copy runs and
 *   the prolongation list go to a static device array of the library, one per
 *   GPU, AMRX_STATIC_WORK_BYTES bytes, held until the process ends; the call
 *   makes no allocation of any kind.  The workspace it would need is
 *   hier_init_from_levels_bytes(); above AMRX_STATIC_WORK_BYTES it returns
 *   AMRX_EINVAL without touching any device memory.  All calls on one GPU share
 *   that array: calls that overlap in time on one GPU (several host threads, or
 *   streams of several hierarchies) race and must be serialised by the caller.
 *   Nothing in the array must start at zero (each call uploads its own lists
 *   before use).  Results equal hier_init_from_levels() bit for bit. */
#define AMRX_STATIC_WORK_BYTES ((size_t)32 << 20)
int hier_init_from_levels_static(amrx_hier* dst, const amrx_hier* below, const amrx_hier* src, int level);

/* Debug / test exports (pure host, after hier_finalize).  For every padded
 * cell (kind 0) or face normal to axis kind-1 (kind 1..3) of a patch, in
 * node-padded [z][y][x] order: the same-level source as
 * src_patch * 2^32 + linear padded index, the patch's own interior (closure)
 * entries included, or -1 where none exists.  `out` holds V entries. */
int hier_debug_sources(const amrx_hier* h, int patch_id, int kind, long long* out);

/* The layered schedule (AMRX_LAYERED) of one root step for the current buffer
 * parities: sizes = (layers, items); first (layers + 1 ints) the first item of
 * each layer; items (4 ints each: node, first block, end block, 0) in launch
 * order, nodes numbered as hier_debug_schedule reports them.  Pure host call. */
int hier_debug_layers(amrx_hier* h, int fixed_dt, int* sizes, int* first, int* items);

/* The persistent schedule of one root step as built for the current buffer
 * parities (fixed_dt: dt0 preset instead of computed), for `nworkgroups`
 * workgroups.  sizes = (nodes, preds, items, queues); each non-NULL array
 * receives the records (nodes: 12 ints each, items: 4 ints, queues: 2 ints)
 * in the layout the device uses. */
int hier_debug_schedule(amrx_hier* h, int fixed_dt, int nworkgroups, int* sizes, int* nodes, int* preds, int* items,
                        int* queues);

/* The concurrent schedule's capture plan (AMRX_CONCURRENT, which is switched
 * off) for the current buffer parities and tuning: sizes = (nodes, preds, ops,
 * side streams, events); nodes and preds as hier_debug_schedule reports them
 * (fused tiles included where the tuning enables them); ops (4 ints each:
 * kind, stream, event, node) in issue order, kind 0 = record event on stream,
 * 1 = stream waits for event, 2 = launch node on stream, 3 = clear the device
 * slots; stream -1 is the capturing stream.  Pure host call. */
int hier_debug_concurrent(amrx_hier* h, int fixed_dt, int* sizes, int* nodes, int* preds, int* ops);

/* The update region [lo, hi) (padded cell indices) of a patch at `substep`. */
int hier_debug_update_box(const amrx_hier* h, int patch_id, int substep, int lo[3], int hi[3]);

/* The batched task list of one advance stage (0 primitives, 1 half-step
 * field, 2 predictor, 3 flux, 4 edge EMFs, 5 update) of a level substep:
 * *count tasks; if out is non-NULL, up to cap records of 9 ints each (patch,
 * axis, lo[3], hi[3] in padded entry indices, first block of the task within
 * the launch).  The flux and edge stages hold one task per axis and slab of
 * z planes, the axes of a slab adjacent and in order.  Pure host call. */
int hier_debug_tasks(const amrx_hier* h, int level, int substep, int stage, int* count, int* out, int cap);

/* Number of parent cells prolongated into a patch at substep 0, and (if out
 * is non-NULL, cap entries) their level-(l-1) (x, y, z) indices. */
int hier_debug_prolong_cells(const amrx_hier* h, int patch_id, int* count, int* out, int cap);

#ifdef __cplusplus
}
#endif

#endif /* AMRX_H */
