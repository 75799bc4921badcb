// Internal layout shared by the host bookkeeping (hier.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AMRX_G 4        // ghost width = ratio * stencil depth
#define AMRX_R 2        // refinement ratio
#define AMRX_NG 2       // stencil depth of one substep
#define AMRX_MAXLEV 16
#define AMRX_BLOCK 256  // threads per block of the stage kernels (4 wavefronts)

// Intermediates of the staged advance, per patch, in units of the patch's
// node-padded volume V.  Quantities consumed as whole records are interleaved
// per entry (read with 16-byte vector loads); quantities consumed one
// component at a time are plain arrays.
#define AMRX_NSCR 49
enum {
  SCR_W = 0,     // 8 per cell, interleaved: primitives at t^n (rho, vx, vy, vz, p, Bx, By, Bz)
  SCR_DU = 8,    // 8 per cell, interleaved: Hancock half-step increments of the 8 conserved components
  SCR_F4 = 16,   // 3 axes x 4 per face, interleaved: momentum and energy fluxes (m_x, m_y, m_z, E)
  SCR_F0 = 28,   // 3 arrays: mass flux through the faces normal to each axis
  SCR_FE = 31,   // 3 axes x 2 arrays: face EMF along (d+2)%3, face EMF along (d+1)%3
  SCR_EC = 37,   // 3 arrays: cell EMFs at t^n
  SCR_BH = 40,   // 3 arrays: face-normal field at t^{n+1/2}
  SCR_ER = 43,   // 3 arrays: cell reference EMFs at t^{n+1/2}
  SCR_E = 46     // 3 arrays: edge EMFs
};

struct PatchDev {
  int n[3];          // interior cells per axis
  int dim[3];        // node-padded array dims (n + 2G + 1)
  long long vol;     // dim[0]*dim[1]*dim[2]
  long long st[2];   // element offsets of state buffers 0 / 1 (8 arrays of vol each)
  long long scr;     // element offset of the AMRX_NSCR intermediate arrays
  long long freg;    // register-element offset of fine face registers: blocks acc, lo, last
  long long fsize;   // entries of one fine face register block
  long long ereg;    // register-element offset of fine edge registers: blocks acc, lo
  long long esize;   // entries of one fine edge register block
  long long creg;    // coarse-side face registers (parent's fluxes on this patch's box surface)
  long long cereg;   // coarse-side edge registers
  long long cov;     // int offset of the coverage map (child id per padded cell), -1 if childless
  int level;
  int parent;
  int lo[3];         // level index of the first interior cell
  int has_children;
  double dx;         // cell width
};

// A region of one patch processed by a stage kernel (padded indices, half-open).
struct Task {
  int patch;
  int axis;
  int lo[3];
  int hi[3];
  double inv0, inv1;  // 1 / (hi[0] - lo[0]) and 1 / (hi[1] - lo[1]): entry index -> (i, j, k) without integer division
};

// A run of consecutive padded entries (along x) copied from a same-level patch.
struct Run {
  int dst_patch, dst_lin, src_patch, src_lin;
  int len;   // entries in the run
  int kind;  // 0: the 5 cell arrays, 1..3: face array of axis kind-1
  int off;   // first element of the run within its list (prefix sum of len)
  int pad;
};

// One parent cell prolongated into a fine patch's ghost region.
struct Pro {
  int patch;   // fine patch
  int c[3];    // coarse cell relative to the fine padded origin (fine padded index = 2*c)
  int pidx;    // parent padded linear index of that coarse cell
  int flags;   // bit 2*d+s: the coarse face (axis d, side s) already holds same-level fine data
};

// A run of consecutive state entries copied from one hierarchy's arena to another's (regridding).
struct XRun {
  long long src, dst;  // offsets in reals of the two arenas
  long long off;       // first element of the run within its list (prefix sum of lengths)
};

// An entry of the correction lists of a parent patch.
struct Corr {
  int patch;   // parent
  int axis;    // face axis (EMF correction), unused for cells
  int lin;     // padded linear index of the cell / face
};

// A boundary face of patch a shared with patch b (same level, possibly a periodic image of a).
struct SyncPair {
  int a, b, axis, a_side;
  int a_reg, b_reg;        // offsets inside one fine face register block (component 0)
  int a_face, b_face;      // padded linear indices of the face in a and b
  int a_cell;              // padded linear index of a's interior cell adjacent to the face
};

// ---------------------------------------------------------------------------
// register layouts on a box surface (used with the fine sizes n or the coarse
// sizes n/2); identical on host and device
// ---------------------------------------------------------------------------
__host__ __device__ inline void other_axes(int d, int& a1, int& a2) {
  a1 = d == 0 ? 1 : 0;
  a2 = d == 2 ? 1 : 2;
}

// Face register: axis d, side s (0 low, 1 high), component c (0..4), transverse t1 (along a1), t2 (along a2).
__host__ __device__ inline long long face_reg_size(const int n[3]) {
  return 10LL * (n[1] * (long long)n[2] + n[0] * (long long)n[2] + n[0] * (long long)n[1]);
}
__host__ __device__ inline long long face_reg_index(const int n[3], int d, int s, int c, int t1, int t2) {
  long long base = 0;
  for (int e = 0; e < d; ++e) {
    int b1, b2;
    other_axes(e, b1, b2);
    base += 10LL * n[b1] * n[b2];
  }
  int a1, a2;
  other_axes(d, a1, a2);
  return base + ((long long)(s * 5 + c) * n[a2] + t2) * n[a1] + t1;
}

// Edge register for edges along e; (a, b) = ((e+1)%3, (e+2)%3).  Plane "pa": the
// box face normal to a (side s), entries (ib in [0, n_b], ie in [0, n_e)); plane
// "pb": the box face normal to b (side s), entries (ia in [0, n_a], ie).
__host__ __device__ inline long long edge_reg_size(const int n[3]) {
  long long t = 0;
  for (int e = 0; e < 3; ++e) {
    int a = (e + 1) % 3, b = (e + 2) % 3;
    t += 2LL * n[e] * (n[a] + n[b] + 2);
  }
  return t;
}
__host__ __device__ inline long long edge_reg_base(const int n[3], int e) {
  long long base = 0;
  for (int f = 0; f < e; ++f) {
    int a = (f + 1) % 3, b = (f + 2) % 3;
    base += 2LL * n[f] * (n[a] + n[b] + 2);
  }
  return base;
}
__host__ __device__ inline long long edge_reg_pa(const int n[3], int e, int s, int ib, int ie) {
  int b = (e + 2) % 3;
  return edge_reg_base(n, e) + ((long long)s * (n[b] + 1) + ib) * n[e] + ie;
}
__host__ __device__ inline long long edge_reg_pb(const int n[3], int e, int s, int ia, int ie) {
  int a = (e + 1) % 3, b = (e + 2) % 3;
  return edge_reg_base(n, e) + 2LL * (n[b] + 1) * n[e] + ((long long)s * (n[a] + 1) + ia) * n[e] + ie;
}

// ---------------------------------------------------------------------------
// kernel launchers (kernels.hip); all enqueue on `stream`, return hipError_t
// ---------------------------------------------------------------------------
struct DevCtx {
  void* state;            // state arena
  void* rscr;             // real intermediates
  void* reg;              // registers (double for FP64 / mixed, float for FP32)
  const PatchDev* patches;
  const Task* tasks;
  const int* blk;         // per-task first block (prefix)
  const int* tbl;         // per task list (indexed by its first task): offset of the list's block table in b2t
  const int* b2t;         // block tables: task of every block of a list (one entry per block)
  const Run* runs;
  const int* run_blk;     // per copy block: index (within the list) of the run holding its first element
  const Pro* pros;
  const Corr* fcorrs;     // flux-correction entries (uncovered parent cells)
  const Corr* ecorrs;     // EMF-correction entries (uncovered parent faces)
  const SyncPair* syncs;
  int* cov;               // coverage maps
  unsigned long long* slots;  // reduction / diagnostic slots
  double* partials;       // per-block conservation partials
  int* lbflag;            // FP32_MIXED flux: count + list of the waves whose faces were left to the low-beta pass
  int precision;
  double gamma;
  int iso;                // isothermal hydro workload: p = cs2 * rho, HLLC fluxes, no energy, zero field
  double cs2;             // isothermal sound speed squared
  hipStream_t stream;
};

enum { STAGE_PRIM = 0, STAGE_BHALF, STAGE_PRED, STAGE_FLUX, STAGE_EDGE, STAGE_UPDATE, NSTAGE };

// slot indices in DevCtx::slots
// SLOT_DT holds the root time step dt0 (double bits); level l uses dt0 * 2^-l.
// SLOT_SCHED is set when a persistent workgroup gave up waiting for work.
enum { SLOT_PHYS = 0, SLOT_SYNC_F = 1, SLOT_SYNC_B = 2, SLOT_DT = 3, SLOT_SCHED = 4, SLOT_SMAX = 8 /* + level */,
       NSLOT = 8 + AMRX_MAXLEV };
// accumulators of a run of root steps (hier_steps), after the slots: k_clear_slots leaves them alone
enum { ACC_PHYS = NSLOT, ACC_TIME = NSLOT + 1, ACC_STEPS = NSLOT + 2, NSLOT_ALL = NSLOT + 3 };

// ---------------------------------------------------------------------------
// persistent schedule of one root step: nodes (one batched launch's worth of
// blocks each) with predecessor lists, and per-level queues of items (block
// ranges of a node) in program order; finer queues are served first
// ---------------------------------------------------------------------------
enum { OP_CFL = 0, OP_DT, OP_COPY, OP_PROLONG, OP_PRIM, OP_BHALF, OP_PRED, OP_FLUX, OP_EDGE, OP_UPDATE, OP_RESTRICT,
       OP_FCORR, OP_ECORR, OP_SYNC,
       OP_FUSEDA, /* fused first three stages (aux: tile index); host-launched schedules only */
       OP_FUSEDB  /* fused edge EMF and update stages (aux: tile index); host-launched schedules only */ };

struct Node {
  int op, level, substep, cur, aux;        // aux: parent parity (prolong), coarse parity (restrict, corrections)
  int first, n, blk_first, nblk, nelem;    // list parameters of the equivalent batched launch
  int pred_first, npred;                   // predecessors in the schedule's pred array
};

struct Item {
  int node, b0, b1, pad;                   // blocks [b0, b1) of a node
};

struct Queue {
  int first, len;                          // items of one level, in program order
};

struct Sched {
  const Node* nodes;
  const int* preds;
  const Item* items;
  const Queue* queues;
  int nq;
  int* heads;                              // per queue: next unclaimed item
  int* done;                               // per node: completed blocks
};

hipError_t launch_stage(const DevCtx& c, int stage, int task_first, int ntask, int blk_first, int nblk,
                        int cur, int level, int substep);
// The update stage's kernel over a task list; nt: the next state written with non-temporal stores.
hipError_t launch_update(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, bool nt);
// The flux stage; FP32_MIXED: split = float pass + low-beta pass, otherwise one pass with the
// double Riemann solver inline (other precisions ignore it).
hipError_t launch_flux(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int substep,
                       bool split);
hipError_t launch_set_dt(const DevCtx& c, double dt0);
hipError_t launch_dt_from_cfl(const DevCtx& c, int nlev, double cfl);
hipError_t launch_copy(const DevCtx& c, int run_first, int nrun, int blk_first, int nblk, int nelem, int cur);
// fused stages 1-3 over tiles of tx x ty x tz cells of the primitive region (one block per tile)
#define AMRX_FUSED_LDS_MAX 65536
size_t fused_a_lds_bytes(int precision, int tx, int ty, int tz);
size_t fused_b_lds_bytes(int precision, int tx, int ty, int tz);
hipError_t launch_fused_b(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int substep, int tx,
                          int ty, int tz);
int fused_a_threads(int tx, int ty, int tz);
hipError_t launch_fused_a(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int tx, int ty,
                          int tz);
// Prolongation from the parent's buffer old_parent, or for w > 0 from old + w (new - old) with the
// advanced buffer new_parent.
hipError_t launch_prolong(const DevCtx& c, int first, int n, int cur_fine, int old_parent, int new_parent, double w);
hipError_t launch_restrict(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk, int cur_fine,
                           int cur_coarse);
hipError_t launch_flux_corr(const DevCtx& c, int first, int n, int cur_coarse);
hipError_t launch_emf_corr(const DevCtx& c, int first, int n, int cur_coarse);
hipError_t launch_sync(const DevCtx& c, int first, int n, int cur);
hipError_t launch_cfl(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk, int cur, int level);
hipError_t launch_conservation(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk,
                               const int* cur_of_level);
hipError_t launch_clear_slots(const DevCtx& c);
hipError_t launch_clear_acc(const DevCtx& c);
hipError_t launch_step_acc(const DevCtx& c);
// every level's CFL reduction in one launch; level l takes blocks [grid0[l], grid0[l + 1])
struct CflLevels {
  int nlev;
  int first[AMRX_MAXLEV], n[AMRX_MAXLEV], nblk[AMRX_MAXLEV], cur[AMRX_MAXLEV];
  int grid0[AMRX_MAXLEV + 1];
};
// blocks of one level's CFL reduction (a grid-stride loop covers the rest; one atomic per block)
inline int cfl_grid(int nblk) { return nblk < 2048 ? nblk : 2048; }
// CFL of all levels (block maxima into the partials) followed by the dt0 reduction into SLOT_DT
hipError_t launch_cfl_all(const DevCtx& c, const CflLevels& L, double cfl);
// restriction of a fine level with both corrections of its parents, one launch
hipError_t launch_restrict_corr(const DevCtx& c, int rfirst, int rn, int rnblk, int ffirst, int fn, int efirst, int en,
                                int cur_fine, int cur_coarse);
hipError_t launch_persistent(const DevCtx& c, const Sched& sc, int nnodes, int nworkgroups, int nlev, double cfl);
// two independent batched launches in one grid (supported combinations only)
bool pair_supported(int op_a, int op_b);
hipError_t launch_pair(const DevCtx& c, const Node& a, const Node& b);
// op: the single operation of every node of the layer, 64 * (a + 1) + b for a layer of the two
// operations a < b with a specialised kernel (layer2_supported), or -1 for other layers
bool layer2_supported(int oa, int ob);
hipError_t launch_layer(const DevCtx& c, const Node* nodes, const Item* items, int first, int n, int* counter,
                        int nworkgroups, int nlev, double cfl, int op);
hipError_t launch_clear_ints(const DevCtx& c, int* p, int n);
hipError_t launch_flag(const DevCtx& c, int first, int n, int nblk, int cur, double eps, unsigned char* flags);
hipError_t launch_xcopy(int precision, hipStream_t s, const void* src, void* dst, const XRun* runs, int nrun,
                        long long nelem);
int layer_blocks_per_cu(int precision);
int persistent_blocks_per_cu(int precision);
// device address of the library's static workspace on device `dev` (AMRX_STATIC_WORK_BYTES bytes,
// looked up once per device with that device current), or null with the HIP error in *err
#define AMRX_MAX_DEVICES 64
void* static_work_ptr(int dev, hipError_t* err);
