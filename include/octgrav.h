/*
 * octgrav.h -- C ABI of an MI355X (gfx950) implementation of the group
 * tree-walk gravity method of E. Gaburov, J. Bedorf and S. Portegies Zwart,
 * "Gravitational tree-code on graphics processing units: implementation in
 * CUDA", ICCS 2010 (Procedia Computer Science).
 *
 * Split of the work (Sec. 2): the host builds the octree, the tight boxes,
 * the boundary cubes and the multipole moments in FP64 (Sec. 2.1); the GPU
 * walks the tree once per particle group to build a cell (node) interaction
 * list and a leaf interaction list (Sec. 2.2, the tree-walk and test-cell
 * listings), then evaluates softened particle-cell (monopole + quadrupole)
 * and particle-particle interactions from those lists (Sec. 2.3, the
 * body-node and body-leaf listings).  Interaction arithmetic is FP32 with
 * compensated per-particle accumulation; FP64 on the GPU is used only for the
 * momentum and energy diagnostics.  G = 1.
 *
 * Conventions shared by every call:
 *   - Return codes: 0 = OK, negative = error (codes below).  Calls that
 *     return a pointer return NULL on failure.  octgrav_last_error() gives
 *     the calling thread's message for its last failure.  No C++ exception
 *     crosses this boundary.
 *   - Positions are row-major n x 3 FP32 [x0 y0 z0 x1 ...]; masses n FP32.
 *     Outputs are always in the caller's original particle order.
 *   - A handle must not be used by two threads at once.
 *   - Device pointers are HIP device allocations on the current device (for
 *     example torch tensors on cuda:0); host pointers are ordinary memory.
 */
#ifndef OCTGRAV_H
#define OCTGRAV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCTGRAV_OK 0
#define OCTGRAV_EINVAL (-1)    /* bad argument (NULL, n < 1, theta outside [0,1], eps <= 0, ...) */
#define OCTGRAV_ENOMEM (-2)    /* host or device allocation failed */
#define OCTGRAV_EHIP (-3)      /* a HIP runtime call or kernel launch failed */
#define OCTGRAV_ECAPACITY (-4) /* an internal capacity bound was exceeded after retry */

/* octgrav_build_tree_ex flags */
#define OCTGRAV_BUILD_HOST_ONLY 1u /* build and keep the host tree only: no device
                                      memory, no HIP call; forces/lists return EINVAL */
#define OCTGRAV_BUILD_DEVICE 2u    /* build the tree on the GPU (same tree, bit for bit, as
                                      the host build); the host keeps only what the calls
                                      need, the first octgrav_export_tree copies the rest */

/* octgrav_forces_ex flags */
#define OCTGRAV_PLAIN_SUM 1u /* plain FP32 accumulation instead of compensated */
#define OCTGRAV_TIMED 2u     /* record HIP events around each kernel phase */
/* Path selection (at most one; none = chosen from theta, see octgrav_forces):
 * OCTGRAV_TWO_PASS    count walk, offsets, write walk and evaluation kernels (the paper's
 *                     structure), pipelined over batches of groups on two streams;
 * OCTGRAV_FUSED_BLOCK one 256-thread block per group walks and evaluates (lists stay in LDS);
 * OCTGRAV_FUSED_WAVE  one 64-lane wave per group walks and evaluates (the default). */
#define OCTGRAV_TWO_PASS 4u
#define OCTGRAV_FUSED_BLOCK 8u
#define OCTGRAV_FUSED_WAVE 16u

/* Opening-test variant for octgrav_forces_ex / octgrav_lists_ex.  The
 * default test (Sec. 2.2, the test-cell listing; the reading fixed here)
 * measures d from the cell's boundary centre cb to the group's box and opens
 * iff d2 == 0 or d2 theta^2 < l^2.  OCTGRAV_MAC_COM measures d from the cell's
 * FP32 centre of mass instead and enlarges the size by the offset between
 * the two centres (Barnes' offset criterion, a variant the paper's choice of
 * centre leaves open): delta = sqrtf((dx*dx + dy*dy) + dz*dz) with
 * d = com - cb, l' = l + theta * delta, open iff d2 == 0 or
 * d2 theta^2 < l'^2, all in FP32 without contraction (sqrtf correctly
 * rounded).  It runs on the fused wave path only (with a path flag other than
 * OCTGRAV_FUSED_WAVE, or with a learned criterion set: OCTGRAV_EINVAL) and
 * accepts theta in [0, 0.57]: there every cell holding a particle of the group
 * is opened (its centre of mass lies in its tight box, within sqrt(3) l of the
 * particle), so no particle meets itself through a multipole. */
#define OCTGRAV_MAC_COM 32u

typedef struct octgrav_tree octgrav_tree;

typedef struct {
  int64_t n;               /* particles */
  int64_t n_cells;         /* cells (nodes + leaves), breadth-first numbered */
  int64_t n_leaves;        /* leaves */
  int64_t n_groups;        /* particle groups (walk units) */
  int64_t max_depth;       /* deepest cell level (root = 0, at most 21) */
  int64_t max_level_cells; /* most cells on one level */
  int64_t n_work;          /* evaluation work items (groups split in chunks of 32 targets) */
  int64_t n_leaf, n_group; /* build parameters */
} octgrav_stats;

/* Host copies of the built tree; every pointer is caller-owned and may be NULL.
 * Sizes come from octgrav_tree_stats. */
typedef struct {
  int32_t* perm;   /* [n]          sorted position -> caller's particle index */
  int32_t* topo;   /* [n_cells*4]  first_child, n_child (0 = leaf), first particle, n particles */
  float* geo;      /* [n_cells*4]  FP32 boundary centre xyz and side (opening-test input) */
  float* mp;       /* [n_cells*12] FP32 com xyz, M | Qxx Qyy Qzz Qxy | Qxz Qyz 0 0 */
  double* mp64;    /* [n_cells*10] FP64 M, com xyz, Qxx Qyy Qzz Qxy Qxz Qyz */
  double* box;     /* [n_cells*6]  FP64 tight box min xyz, max xyz */
  int32_t* depth;  /* [n_cells]    level of each cell */
  int32_t* groups; /* [n_groups]   cell id of each group, ascending first particle */
  double* cube;    /* [4]          root cube corner xyz and side */
} octgrav_tree_view;

/*
 * Builds the tree of Sec. 2.1 on the host in FP64 and uploads it.
 *   pos   host, n x 3 FP32, finite, |x| < 2^60 (keeps FP32 squared distances finite)
 *   mass  host, n FP32, each > 0 and finite
 *   n     1 <= n < 2^31
 *   n_leaf  leaf capacity, 1..64: a cell is a leaf iff it holds n <= n_leaf
 *           particles or sits at depth 21 (coincident particles).
 * Groups are the maximal cells with at most 64 particles (Sec. 2.1).  The
 * inputs are copied; the caller may free them when the call returns.  The
 * handle owns all internal host and device memory until octgrav_free.
 * Returns NULL on failure, also for a tree of 2^29 cells or more (the walks'
 * frontier entries hold cell ids in 29 bits).
 */
octgrav_tree* octgrav_build_tree(const float* pos, const float* mass, int64_t n, int32_t n_leaf);

/* As octgrav_build_tree with an explicit group capacity n_group (1..1024)
 * and flags (OCTGRAV_BUILD_*). */
octgrav_tree* octgrav_build_tree_ex(const float* pos, const float* mass, int64_t n,
                                    int32_t n_leaf, int32_t n_group, uint32_t flags);

/*
 * Accelerations and potentials of every particle (Sec. 2.2 + 2.3):
 * per-group walk with the opening angle theta, then evaluation of the cell
 * list (softened monopole + traceless quadrupole) and the leaf list (softened
 * particle-particle, self excluded from the potential).
 *   theta  0 <= theta <= 1 (theta <= 1 guarantees that every cell containing a
 *          group particle is opened, so no self term goes through a multipole)
 *   eps    Plummer softening length, > 0
 *   acc    device, n x 3 FP32, caller's order (written)
 *   pot    device, n FP32, caller's order (written), or NULL
 * Runs on the handle's stream and returns once the results are complete on it.
 * All paths evaluate the same lists; the default is the fastest measured one
 * at every theta, the fused wave walk.
 */
int octgrav_forces(octgrav_tree* t, float theta, float eps, float* acc, float* pot);

/* As octgrav_forces with OCTGRAV_PLAIN_SUM / OCTGRAV_TIMED and path flags. */
int octgrav_forces_ex(octgrav_tree* t, float theta, float eps, float* acc, float* pot,
                      uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or time-step loops, harnesses that forbid
 * hipMalloc): the same force call as octgrav_forces (same paths, kernels,
 * lists and compensated sums, so the same results bit for bit), whose per-call
 * scratch (group records, totals, work counters, overflow lists, fallback
 * frontier queues, diagnostic partial sums) lives in one file-scope device
 * array of 128 MiB per GPU instead of the handle's buffers.  The call makes
 * no hipMalloc / hipFree or other allocating call; the array is looked up on
 * the first call on each device (that device current) and held until the
 * process ends.  Afterwards octgrav_diagnostics, octgrav_last_counts and
 * octgrav_mac_stats report this call, as after octgrav_forces.
 *   Sizes: the tree must need at most 128 MiB of scratch (about
 *   16 B x groups + 8 B x max(groups, work items) + one fallback frontier
 *   queue of 8 B x (2 x its widest level + 64) rounded up to a power of two;
 *   the 2^24-particle galaxy mix needs 21.4 MiB + 8 MiB), else OCTGRAV_EINVAL before
 *   any launch.  Fewer fallback queues than octgrav_forces uses may fit
 *   (only the rare walks that outgrow the LDS queues use them).
 *   Sharing: every call on one GPU uses that GPU's one array; it keeps the
 *   last call's contents and each call clears what it needs.  Calls that
 *   overlap in time on one GPU (handles on different streams, or threads)
 *   race on it and must be serialised by the caller.
 */
int octgrav_forces_noalloc(octgrav_tree* t, float theta, float eps, float* acc, float* pot);

/* Releases the handle and everything it owns.  NULL is a no-op. */
void octgrav_free(octgrav_tree* t);

/* Message of the calling thread's last failure ("" if none).  The string
 * stays valid until the thread's next octgrav call. */
const char* octgrav_last_error(void);

/* Sets the HIP stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream)
 * that later calls on this handle run on.  NULL selects the null stream. */
int octgrav_set_stream(octgrav_tree* t, void* hip_stream);

/* Sizes of the built tree. */
int octgrav_tree_stats(const octgrav_tree* t, octgrav_stats* s);

/* Copies the host tree into caller-provided arrays (see octgrav_tree_view). */
int octgrav_export_tree(const octgrav_tree* t, const octgrav_tree_view* v);

/*
 * Interaction lists of every group at opening angle theta, built by the GPU
 * walk (Sec. 2.2) and copied to the host in CSR form over groups; ids are
 * cell ids in ascending order.  Sizes and offsets come from the count walk
 * and the device prefix sum; the entries are written by the walk of the path
 * the same flags select in octgrav_forces_ex (the fused kernels run with
 * their evaluation skipped).  Two-call pattern: with c_off/c_ids/l_off/l_ids NULL only *n_c
 * and *n_l (total entries) are set; otherwise c_off and l_off hold
 * n_groups+1 int64 each and c_ids/l_ids at least *n_c / *n_l int32 entries.
 */
int octgrav_lists(octgrav_tree* t, float theta, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                  int32_t* l_ids, int64_t* n_c, int64_t* n_l);

/* As octgrav_lists with a path flag (OCTGRAV_TWO_PASS, OCTGRAV_FUSED_BLOCK,
 * OCTGRAV_FUSED_WAVE; none = the default path for theta). */
int octgrav_lists_ex(octgrav_tree* t, float theta, uint32_t flags, int64_t* c_off, int32_t* c_ids,
                     int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l);

/*
 * Interaction lists of selected groups (Sec. 2.2), for trees whose full lists
 * would not fit in host memory: the walk covers every group as in
 * octgrav_lists_ex (same flags, same lists on the device), and only the
 * groups named in groups (host, n_sel int32 group indices in [0, n_groups),
 * any order, repeats allowed; n_sel >= 0) are copied back, in that order:
 * c_off and l_off hold n_sel+1 int64 offsets into c_ids / l_ids, and *n_c /
 * *n_l the selection's total entries.  Two-call pattern as octgrav_lists.
 * An index outside [0, n_groups) gives OCTGRAV_EINVAL before any launch.
 */
int octgrav_lists_select(octgrav_tree* t, float theta, uint32_t flags, const int32_t* groups,
                         int64_t n_sel, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                         int32_t* l_ids, int64_t* n_c, int64_t* n_l);

/* FP64 diagnostics of the last octgrav_forces call, reduced on the GPU:
 * mom = sum_i m_i a_i and *w = 1/2 sum_i m_i phi_i (0 if pot was NULL). */
int octgrav_diagnostics(octgrav_tree* t, double mom[3], double* w);

/* Interaction totals of the last forces/lists call: out[0] = cell-list
 * entries, out[1] = leaf-list entries, out[2] = particle-cell interactions
 * sum_g |g| |C_g|, out[3] = particle-particle interactions sum_g |g| n_src(L_g)
 * (self pairs included, as they are evaluated). */
int octgrav_last_counts(octgrav_tree* t, int64_t out[4]);

/* Per-group list lengths of the last forces/lists call over all groups
 * (Sec. 2.2's lists, without exporting them): out (host, n_groups x 4
 * int32) gets, for group g in the handle's group order, |C_g|, |L_g|, the
 * particles in L_g's leaves (n_src), and a flag word (the learned criterion:
 * 2 x band candidates visited + 1 if the group fell back to theta; the
 * two-pass path: 1 if the group's walk needed the global-memory queues;
 * otherwise 0).  OCTGRAV_EINVAL before any such call. */
int octgrav_group_counts(octgrav_tree* t, int32_t* out);

/* Kernel-phase times in ms of the last OCTGRAV_TIMED forces call, measured
 * with HIP events on the handle's stream: out[0] count walk, out[1] offsets,
 * out[2] write walk, out[3] evaluation (in the default fused path: walk and
 * evaluation together; out[0..2] are then 0), out[4] diagnostics,
 * out[5] total. */
int octgrav_last_timings(octgrav_tree* t, double out[6]);

/*
 * Direct summation on the GPU (FP32 with compensated accumulation), the
 * reference the paper measures its errors against (Sec. 3.1) and the
 * normalization of the learned criterion's labels.
 *   targets  device int32 caller indices, or NULL for all n particles
 *   nt       number of targets (ignored when targets is NULL)
 *   acc      device, nt x 3 FP32 in target order; pot device nt FP32 or NULL
 * Softened like the tree forces (eps > 0), self excluded.  Synchronous.
 * Target indices outside [0, n) give OCTGRAV_EINVAL before any launch.
 */
int octgrav_direct(octgrav_tree* t, float eps, const int32_t* targets, int64_t nt, float* acc,
                   float* pot);

/*
 * Training data of the learned acceptance criterion.  Walks every group at
 * theta_lo and keeps the band candidates (cells the theta_lo test opens and
 * the theta_hi test does not); for the groups g = 0, stride, 2*stride, ...
 * (while the pairs fit in cap) writes for each pair its 12 FP32 features
 * (device feat, cap x 12) and its label e = max over the group's particles i
 * of |a_pc(i; c) - sum_{j in c} a_pp(i, j)| / |a_i| (device label, cap),
 * with |a_i| from acc_direct (device, n x 3 caller order, e.g. from
 * octgrav_direct), and optionally the pair's group index and cell id (device
 * int32 arrays, cap, or NULL).  *n_out = pairs written.  Synchronous.
 */
int octgrav_mac_collect(octgrav_tree* t, float theta_lo, float theta_hi, float eps,
                        const float* acc_direct, int32_t stride, float* feat, float* label,
                        int32_t* group_out, int32_t* cell_out, int64_t cap, int64_t* n_out);

/*
 * ---- Learned acceptance criterion (an extension of the opening test of
 * Sec. 2.2; the paper itself uses the opening angle only).
 *
 * The network maps 12 features of a (group, cell) candidate to a predicted
 * log10 of the cell's relative force error on the group: 12 -> 64 -> 64 -> 1
 * with ReLU, 5057 FP32 parameters laid out as W1 [64 x 12] row-major, b1
 * [64], W2 [64 x 64] row-major, b2 [64], w3 [64], b3.  Inference rounds the
 * inputs, weights and hidden activations to BF16 (nearest even) and
 * accumulates in FP32 on the matrix cores.
 */
typedef struct octgrav_mlp octgrav_mlp;

/* A network with the given parameters (host, 5057 FP32; NULL = zeros) and
 * zero Adam moments.  NULL on failure (octgrav_last_error). */
octgrav_mlp* octgrav_mlp_create(const float* params);
void octgrav_mlp_free(octgrav_mlp* m); /* NULL-safe */
int octgrav_mlp_set_stream(octgrav_mlp* m, void* hip_stream);
/* Replaces the parameters (host, 5057 FP32, finite) and zeroes the moments. */
int octgrav_mlp_set_params(octgrav_mlp* m, const float* params);
int octgrav_mlp_get_params(const octgrav_mlp* m, float* params);
/* Training checkpoints: the Adam first and second moments (host, 5057 FP32
 * each), and the whole optimiser state restored at once (parameters and
 * moments, host, 5057 FP32 each; all finite, second moments >= 0, else
 * OCTGRAV_EINVAL and nothing changes).  With the step count kept by the
 * caller, a restored network continues training exactly as the saved one
 * would have.  Synchronous. */
int octgrav_mlp_get_moments(const octgrav_mlp* m, float* mom1, float* mom2);
int octgrav_mlp_set_state(octgrav_mlp* m, const float* params, const float* mom1,
                          const float* mom2);
/* y[b] (device FP32) for inputs x (device, b x 12 FP32).  Synchronous. */
int octgrav_mlp_forward(octgrav_mlp* m, const float* x, int64_t b, float* y);
/*
 * Mean pinball loss at quantile tau in (0, 1) of targets (device, b FP32) and
 * its gradient, kept in the handle for octgrav_mlp_adam and optionally copied
 * to grad (host, 5057 FP32, may be NULL).  *loss is FP64.  Weight gradients
 * use the BF16-rounded activation gradients and activations, bias gradients
 * the unrounded ones.  Synchronous.
 */
int octgrav_mlp_loss_grad(octgrav_mlp* m, const float* x, const float* target, int64_t b,
                          float tau, double* loss, float* grad);
/* One Adam step (Kingma & Ba, bias-corrected; step counts from 1) with the
 * last gradient, then the BF16 inference image is rebuilt.  Synchronous. */
int octgrav_mlp_adam(octgrav_mlp* m, float lr, float beta1, float beta2, float eps, int32_t step);

/*
 * Sets the tree's acceptance criterion.  m == NULL: the opening angle (the
 * default).  Otherwise a copy of m's current network is taken and, in later
 * octgrav_forces / octgrav_lists calls, a candidate the theta_lo test accepts
 * is accepted, one the theta_hi test opens is opened, and in between it is
 * accepted iff the network's output <= log10(tau_pair) (tau_pair = 0: never;
 * the threshold is the FP64 log10 of the FP32 tau_pair rounded once to FP32).
 * A group whose network-accepted candidates have sqrt(sum 10^(2 y)) > budget
 * is walked with the call's theta instead (budget < 0: every group).
 * Needs 0 < theta_lo < theta_hi <= 1.  These calls then use the fused wave
 * path (OCTGRAV_TWO_PASS / OCTGRAV_FUSED_BLOCK give OCTGRAV_EINVAL).
 */
int octgrav_set_mac(octgrav_tree* t, const octgrav_mlp* m, float theta_lo, float theta_hi,
                    float tau_pair, float budget);
/* After a forces / lists call with the learned criterion: out[0] = band
 * candidates the network scored, out[1] = groups that fell back to theta. */
int octgrav_mac_stats(octgrav_tree* t, int64_t out[2]);
/*
 * Decision trace of the learned walks at this theta (test export): off
 * (host, n_groups + 1) receives group g's range of trace entries, fell_back
 * (host, n_groups) 1 for the groups walked with theta; with cells and scores
 * (host, cap entries) non-NULL, the band candidates' cell ids and network
 * outputs in walk order (the fell-back groups' entries are those of their
 * learned attempt).  *n_out = entries.  Two-call pattern as octgrav_lists.
 */
int octgrav_mac_trace(octgrav_tree* t, float theta, int64_t* off, int32_t* cells, float* scores,
                      int64_t cap, int64_t* n_out, int32_t* fell_back);

/* As octgrav_mac_trace for the selected groups only (groups: host, n_sel
 * int32 group indices in [0, n_groups), any order): off (n_sel+1) and
 * fell_back (n_sel) follow the selection's order, cells / scores hold the
 * selected groups' entries.  The learned walk itself covers every group. */
int octgrav_mac_trace_select(octgrav_tree* t, float theta, const int32_t* groups, int64_t n_sel,
                             int64_t* off, int32_t* cells, float* scores, int64_t cap,
                             int64_t* n_out, int32_t* fell_back);

/*
 * ---- Time integration (the step after the force call: the paper's science
 * runs advance a particle system with the tree code).
 *
 * A particle system on the device, advanced with kick-drift-kick leapfrog
 * (v += a dt/2, x += v dt, new tree and forces, v += a dt/2) in FP32; the
 * tree is rebuilt on the GPU from the drifted positions every step (as
 * OCTGRAV_BUILD_DEVICE, inputs never leave the device).  The handle owns the
 * state and one tree that is rebuilt in place: its device buffers are kept
 * and reused from step to step (a buffer is reallocated only when a tree
 * outgrows it) until octgrav_sim_free.  Calls return OCTGRAV_OK or the codes
 * above (OCTGRAV_EINVAL for bad arguments or positions that became
 * non-finite, OCTGRAV_ENOMEM, OCTGRAV_EHIP), with octgrav_last_error()
 * holding the message.  One handle must not be used by two threads at once.
 */
typedef struct octgrav_sim octgrav_sim;

/* Copies pos, vel (host, n x 3 FP32) and mass (host, n FP32) to the device;
 * input rules as octgrav_build_tree_ex, velocities finite.  NULL on failure. */
octgrav_sim* octgrav_sim_create(const float* pos, const float* vel, const float* mass, int64_t n,
                                int32_t n_leaf, int32_t n_group);
void octgrav_sim_free(octgrav_sim* s); /* NULL-safe */
int octgrav_sim_set_stream(octgrav_sim* s, void* hip_stream);
/* steps leapfrog steps of length dt with opening angle theta and softening
 * eps (forces at the current positions are computed first when missing or
 * when theta / eps changed; steps = 0 only does that).  Synchronous.
 * A failure inside a step (after its first half-kick: the rebuild or the
 * forces fail, or a device error) leaves velocities, positions and
 * accelerations at different times; the handle is then marked inconsistent
 * and every later octgrav_sim_run, octgrav_sim_energy and octgrav_sim_state
 * returns OCTGRAV_EINVAL (free it and create a new one from saved state).
 * A failure before the first step (the initial forces) changes nothing. */
int octgrav_sim_run(octgrav_sim* s, float theta, float eps, float dt, int32_t steps);
/* out = {K, W, E = K + W, sum m vx, sum m vy, sum m vz} in FP64: K = 1/2 sum
 * m v^2, W = 1/2 sum m phi with the last forces (potentials self-excluded). */
int octgrav_sim_energy(octgrav_sim* s, double out[6]);
/* Host copies of positions, velocities and the last accelerations (each
 * n x 3 FP32, any may be NULL). */
int octgrav_sim_state(const octgrav_sim* s, float* pos, float* vel, float* acc);
/* Last run, per step: total, tree build and force milliseconds (host clock). */
int octgrav_sim_timings(const octgrav_sim* s, double out[3]);

#ifdef __cplusplus
}
#endif

#endif /* OCTGRAV_H */
