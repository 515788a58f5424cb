/*
 * bard.h -- C ABI of the MI355X (gfx950) batched rigid-body dynamics library.
 *
 * One call evaluates a kinematic tree for B independent configurations
 * ("instances") at once: forward kinematics, the geometric Jacobian, inverse
 * dynamics (RNEA), the joint-space mass matrix (CRBA), forward dynamics (ABA),
 * a fused RNEA + CRBA + Jacobian chain, and vector-Jacobian products of RNEA and
 * FK.  The algorithms are Featherstone's recursions that the paper restructures
 * for batched GPU evaluation (Sec. 3); the joint transforms use precomputed
 * Rodrigues constants (Sec. 3.2, eqs. (2)-(5)), traversals go level by level
 * (Sec. 3.3, eq. (6)) and Jacobian columns are built directly (Sec. 3.4, eq. (7)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns a bard_status (0 on success, negative on error)
 *   and never aborts or throws.  bard_last_error() returns a thread-local
 *   message for the last failure.  Argument and topology errors are detected on
 *   the host before any launch; an asynchronous device fault surfaces as
 *   BARD_E_DEVICE on a later call.
 * Memory: model arrays given to bard_model_create are host arrays, copied (the
 *   caller keeps ownership).  Every operator I/O pointer is a DEVICE pointer
 *   owned by the caller; the library never frees or retains it past the call.
 *   Operators launch asynchronously on `stream` (a hipStream_t, NULL = the
 *   default stream).  Device memory the library owns is allocated once, on
 *   first use, never per call: the model's tables on the first call on a
 *   device, an end-effector set's table on its first Jacobian or chain call,
 *   the reduction buffer of bard_rnea_vjp on its first call with
 *   inertia_bar, workspace tiers on their first use.  Those first uses also
 *   copy synchronously.  bard_model_upload does the model's part ahead of
 *   time; a call that would allocate while `stream` is being captured into a
 *   HIP graph returns BARD_E_CAPTURE and launches nothing.
 * Layout: each operator takes `L`, an array with one bard_layout per array
 *   argument, in the order the arguments appear (inputs first, as listed in the
 *   operator's comment).  Element k of instance b of an array lives at
 *   base[b * stride_b + k * stride_k], where k is the flattened per-instance
 *   index (row-major over the per-instance shape).  L == NULL means every array
 *   is instance-minor ("SoA"): stride_b = 1, stride_k = B.  Strides are in
 *   elements and must be >= 1.
 * Scalars: `dtype` selects float or double for every floating array of a call.
 * Spatial conventions: joint axes are unit vectors in the joint frame (they are
 *   normalised at create).  Free joints use q = [x y z qx qy qz qw] (the
 *   quaternion is normalised on read), velocity = body-frame twist [v; w], and
 *   the generalised force of a free joint is the body-frame wrench [f; n].
 *   Gravity is a world-frame vector (default {0, 0, -9.81}).
 *   Jacobian rows are [linear; angular] (eq. (7)).  BARD_WORLD gives the
 *   velocity of the body-fixed point at the world origin (the p x w form of
 *   eq. (7)); BARD_LOCAL_WORLD_ALIGNED gives the velocity of the end-effector
 *   origin, in world axes.
 * Poses: 3x4 row-major [R | p] per body, the body frame in the world frame.
 * B == 0 is a no-op returning BARD_OK.
 */
#ifndef BARD_H
#define BARD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bard_model* bard_model_t;
typedef struct bard_ws* bard_ws_t;
typedef struct bard_plan* bard_plan_t;

typedef enum {
  BARD_OK = 0,
  BARD_E_ARG = -1,         /* bad pointer, size, stride or enum value */
  BARD_E_TOPOLOGY = -2,    /* parent[i] >= i, bad joint type, free joint not at a root, zero axis */
  BARD_E_INERTIA = -3,     /* mass <= 0 or COM inertia not positive definite */
  BARD_E_NOMEM = -4,       /* device or host allocation failed (create calls only) */
  BARD_E_DEVICE = -5,      /* a HIP call failed, or an earlier asynchronous fault */
  BARD_E_CAPACITY = -6,    /* batch larger than a workspace/plan capacity, or model too large */
  BARD_E_UNSUPPORTED = -7, /* valid request the library does not implement */
  BARD_E_CAPTURE = -8,     /* the call would allocate or copy synchronously while its stream is
                              captured into a HIP graph (run it once before capturing, or call
                              bard_model_upload) */
  BARD_E_STATE = -9        /* a call that allocates nothing found state it needs missing (the model
                              not yet uploaded to the current device) */
} bard_status;

typedef enum { BARD_F32 = 0, BARD_F64 = 1 } bard_dtype;
typedef enum { BARD_REVOLUTE = 0, BARD_PRISMATIC = 1, BARD_FREE = 2, BARD_FIXED = 3 } bard_joint;
typedef enum { BARD_WORLD = 0, BARD_LOCAL_WORLD_ALIGNED = 1 } bard_frame;

typedef struct {
  int64_t stride_b; /* elements between instance b and b+1 */
  int64_t stride_k; /* elements between per-instance entries k and k+1 */
} bard_layout;

/* Human-readable name of a status code (static storage). */
const char* bard_status_str(int status);
/* Detail of the last error raised on the calling thread ("" if none). */
const char* bard_last_error(void);
/* Library version string, e.g. "bard 0.1 gfx950". */
const char* bard_version(void);

/* ---------------------------------------------------------------- model ----
 * Build an immutable model (the paper's parse-once model, Fig. 1 / Sec. 3).
 *   n_bodies   number of bodies, 1..BARD_MAX_BODIES (64)
 *   parent     [n] parent index, -1 for a body attached to the world; parent[i] < i
 *   joint_type [n] bard_joint; BARD_FREE only on body 0 with parent -1;
 *              BARD_FIXED is rejected with BARD_E_UNSUPPORTED
 *   axis       [n][3] joint axis in the joint frame (normalised here; ignored for FREE)
 *   X_tree     [n][3][4] row-major [R_pre | t_pre]: pose of joint i's frame in
 *              the parent body frame; the body frame is the joint frame after
 *              the joint motion
 *   inertia    [n][10] m, h = m*c (3), then I_xx I_xy I_yy I_xz I_yz I_zz of the
 *              rotational inertia about the body-frame origin
 * The host-side compile (level schedule, Rodrigues constants of eqs. (2)-(3),
 * tables) happens here; device constants are uploaded on the first operator
 * call on a device, or by bard_model_upload.  Errors: BARD_E_ARG, BARD_E_TOPOLOGY, BARD_E_INERTIA,
 * BARD_E_UNSUPPORTED, BARD_E_NOMEM.  *out is set only on success. */
int bard_model_create(int32_t n_bodies, const int32_t* parent, const int32_t* joint_type,
                      const double* axis, const double* X_tree, const double* inertia,
                      bard_model_t* out);
/* Set the world-frame gravity vector (host array of 3). Default {0, 0, -9.81}. */
int bard_model_set_gravity(bard_model_t model, const double* g);
/* Sizes of a model. Any output pointer may be NULL. */
int bard_model_info(bard_model_t model, int32_t* nq, int32_t* nv, int32_t* n_bodies, int32_t* depth);
/* Level schedule chosen by the compiler: lanes per instance and levels. */
int bard_model_schedule(bard_model_t model, int32_t* lanes_per_instance, int32_t* levels);
/* Host-side evaluation of one joint's parent-to-child transform from the Rodrigues
 * constants (eqs. (4)-(5)), in FP64, for testing the compile step without a GPU.
 * out_R: [3][3] row-major, out_t: [3].  Free joints take q as 7 values. */
int bard_model_joint_transform(bard_model_t model, int32_t body, const double* q, double* out_R,
                               double* out_t);
/* Upload ahead of time what the first operator calls on the current device
 * would upload: the model's tables, and if n_ee > 0 the table of the
 * end-effector set ee_body (a HOST array of n_ee body indices, as passed to
 * bard_jacobian / bard_chain), and with flags = BARD_UPLOAD_ADJOINT the
 * reduction buffer of bard_rnea_vjp.  Synchronous and idempotent; after it,
 * calls with that model (and end-effector set) on this device allocate
 * nothing and may be captured into a HIP graph.  Call it outside any capture.
 * Errors: BARD_E_ARG, BARD_E_NOMEM, BARD_E_DEVICE, BARD_E_CAPTURE. */
#define BARD_UPLOAD_ADJOINT 1
int bard_model_upload(bard_model_t model, int32_t n_ee, const int32_t* ee_body, int32_t flags);
int bard_model_destroy(bard_model_t model);
/* ------------------------------------------------- specialised kernels ----
 * The fused chain of bard_chain (RNEA + CRBA + Jacobian) written for one
 * tree: the model compiler emits HIP source in which every model constant is
 * a literal and the traversal is unrolled body by body (the generated,
 * model-specific kernels Sec. 2 cites as prior art), and hipRTC compiles it
 * for gfx950 at run time.  Four forms, 64 instances per workgroup, one lane
 * per instance:
 *   split (default): a tree with branches is cut into its trunk (the bodies
 *     with two or more children and their ancestors) and limbs (the chains
 *     hanging off it); each wave of the workgroup computes the trunk's
 *     kinematics and then whole limbs, and after one barrier one wave sums the
 *     trunk.  A tree that is a single chain runs as one wave.
 *   whole (BARD_SPEC_WHOLE): one wave walks the whole tree; fewer
 *     instructions in all, so it can win once the batch fills the device.
 *   dual (BARD_SPEC_DUAL): split, and each group of 64 instances runs as two
 *     workgroups of the launch: one computes the torques (kinematics, body
 *     forces, subtree forces), the other the mass matrix and the Jacobians
 *     (kinematics, composite inertias).  Each computes the kinematics it
 *     needs, so the instructions per wave drop and twice the compute units
 *     take part; for small batches.  Refused (BARD_E_UNSUPPORTED) when no
 *     split plan fits in LDS.
 *   triple (BARD_SPEC_TRIPLE): as dual with three workgroups per 64
 *     instances: torques, mass matrix, Jacobians (the last needs only the
 *     kinematics and has no barrier).  Refused as dual is.
 *
 * specialize: compiles the kernel of one form for (dtype, end-effector set
 * ee_body [n_ee, host], frame) and loads it on the current device (once; later
 * calls only change the routing).  flags: BARD_SPEC_ROUTE -- bard_chain calls
 * with these arguments on this device then launch this kernel for every batch
 * (and not the other form); without it, this form takes no calls.  Results
 * agree with the generic kernel's within the tolerance contract, not bitwise
 * (different summation order).  BARD_SPEC_COMPILE_ONLY -- generate and
 * compile only, needing no GPU, and keep nothing (a check that the
 * generator's output compiles).  BARD_SPEC_WHOLE, BARD_SPEC_DUAL,
 * BARD_SPEC_TRIPLE -- that form (at most one of them).  Uploads
 * the model's tables as bard_model_upload does; synchronous; call it outside
 * any graph capture.  The kernels are unloaded by bard_model_destroy.
 * Errors: BARD_E_ARG, BARD_E_DEVICE (a hipRTC compile or module load failed;
 * bard_last_error holds the compiler log), BARD_E_NOMEM, BARD_E_UNSUPPORTED
 * (trees deeper than 32 or with more than 1500 dof-ancestor pairs, whose
 * generated code would take minutes to compile: the generic kernel serves
 * them).  Routed calls whose per-instance byte offset into an array reaches
 * 4 GiB run the generic kernel (the generated code addresses with 32-bit
 * lane offsets). */
#define BARD_SPEC_ROUTE 1
#define BARD_SPEC_COMPILE_ONLY 2
#define BARD_SPEC_WHOLE 4
#define BARD_SPEC_DUAL 8
#define BARD_SPEC_TRIPLE 16
int bard_model_specialize(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                          bard_frame frame, int32_t flags);
/* Resources of a loaded specialised kernel (form by flags: 0,
 * BARD_SPEC_WHOLE, BARD_SPEC_DUAL or BARD_SPEC_TRIPLE) on the current device: registers per lane, scratch bytes
 * per lane (spills), hipRTC compile time, the batch tiers routed to it (bit k
 * for tier k: [0, 4096), [4096, 16384), [16384, 65536), [65536, inf)) and
 * waves per workgroup.  Any output may be NULL.  BARD_E_STATE if none is
 * loaded for these arguments. */
int bard_model_specialized_info(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                bard_frame frame, int32_t flags, int32_t* vgprs, int32_t* scratch_bytes,
                                double* compile_seconds, int32_t* routed_tiers, int32_t* waves);
/* Choose between the generic chain kernel and the specialised forms by
 * timing: compiles and loads the forms if needed (split, dual and triple;
 * whole too when the tree splits over several waves), times every candidate on scratch arrays (allocated here and
 * freed before returning) at B = 1024, 4096, 16384 and 65536 on `stream`, and
 * routes each batch tier (as in bard_model_specialized_info; the tier of
 * 1024 covers every batch below 4096) to the fastest.  *min_batch receives
 * the smallest batch any specialised form takes (0, 4096, 16384 or 65536),
 * or -1.  Synchronous; not under graph capture (BARD_E_CAPTURE).  A later
 * bard_model_specialize call resets the routing.  Errors: as
 * bard_model_specialize, BARD_E_NOMEM, BARD_E_CAPTURE. */
int bard_chain_autotune(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                        bard_frame frame, void* stream, int64_t* min_batch);
/* The generated source text of one form (flags: 0, BARD_SPEC_WHOLE,
 * BARD_SPEC_DUAL or BARD_SPEC_TRIPLE; NUL-terminated, truncated to cap - 1 bytes); *len receives its full length.
 * Host only. */
int bard_model_specialized_source(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                  bard_frame frame, int32_t flags, char* buf, int64_t cap, int64_t* len);

/* Inverse dynamics alone written for one tree in the same way (Sec. 3.3's
 * RNEA, the torque code of the chain kernels: poses and velocities forward,
 * body forces, subtree forces back, tau_i = s_i . F_i), for RL loops that
 * call bard_rnea only.  flags: BARD_SPEC_ROUTE (bard_rnea calls without a
 * workspace and without an inertia override then launch it, at every
 * batch), BARD_SPEC_COMPILE_ONLY (compile only, no GPU needed),
 * BARD_SPEC_WHOLE (one wave over the whole tree instead of the split form).
 * Routing one form takes the calls from the other.  Results agree with the
 * generic kernel's within the tolerance contract, not bitwise.
 * Errors: as bard_model_specialize (trees deeper than 32: BARD_E_UNSUPPORTED). */
int bard_model_specialize_rnea(bard_model_t model, bard_dtype dtype, int32_t flags);
/* Resources of the loaded inverse-dynamics kernel of the form flags selects
 * (0 or BARD_SPEC_WHOLE), as bard_model_specialized_info.  BARD_E_STATE if
 * none is loaded. */
int bard_model_specialized_rnea_info(bard_model_t model, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                     int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                     int32_t* waves);
/* Its generated source (flags 0 or BARD_SPEC_WHOLE), as
 * bard_model_specialized_source.  Host only. */
int bard_model_specialized_rnea_source(bard_model_t model, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                       int64_t* len);
/* The joint-space mass matrix alone written for one tree in the same way
 * (Sec. 3's CRBA: poses forward, composite inertias back, M_ij = s_i . Ic_j
 * s_j over each dof's ancestors, the structural zeros from tables, by extra
 * workgroups for instance-minor 16-byte-aligned outputs); routes bard_crba
 * calls without a workspace.  Flags, errors and the two companions as for
 * the inverse-dynamics kernel above. */
int bard_model_specialize_crba(bard_model_t model, bard_dtype dtype, int32_t flags);
int bard_model_specialized_crba_info(bard_model_t model, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                     int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                     int32_t* waves);
int bard_model_specialized_crba_source(bard_model_t model, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                       int64_t* len);
/* The world pose of every body alone (FK, Sec. 3.1 tier 3) written for one
 * tree in the same way; routes bard_fk calls without a workspace.  Flags,
 * errors and the two companions as above. */
int bard_model_specialize_fk(bard_model_t model, bard_dtype dtype, int32_t flags);
int bard_model_specialized_fk_info(bard_model_t model, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                   int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                   int32_t* waves);
int bard_model_specialized_fk_source(bard_model_t model, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                     int64_t* len);
/* The Jacobians of n_ee end-effector bodies (host array ee_body) in
 * `frame` alone written for one tree in the same way (eq. (7) columns from
 * each path joint's world axis and position, the off-path rows from tables);
 * routes bard_jacobian calls with the same end effectors and frame and
 * without a workspace.  Flags, errors and the two companions as above. */
int bard_model_specialize_jacobian(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                   bard_frame frame, int32_t flags);
int bard_model_specialized_jacobian_info(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                         bard_frame frame, int32_t flags, int32_t* vgprs, int32_t* scratch_bytes,
                                         double* compile_seconds, int32_t* routed_tiers, int32_t* waves);
int bard_model_specialized_jacobian_source(bard_model_t model, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                           bard_frame frame, int32_t flags, char* buf, int64_t cap, int64_t* len);

/* The forward dynamics of bard_aba written for one tree in the same way (one
 * wave per 64 instances over the whole tree, constants as literals; the
 * articulated-body algorithm's three passes of Sec. 3, in the base frame as
 * the generic kernel computes them): passes 1 and 2 in one depth-first walk
 * holding only the current path's state, pass 3 with what each body's
 * articulated solve leaves (U / D and the scaled bias) and its kinematics
 * recomputed.
 * specialize_aba: compile and load (flags BARD_SPEC_ROUTE: bard_aba calls of
 * this dtype on this device then launch it at every batch;
 * BARD_SPEC_COMPILE_ONLY: compile only, no GPU).  Errors as
 * bard_model_specialize; BARD_E_UNSUPPORTED for trees deeper than 16.
 * aba_info: resources and routed batch tiers of the loaded kernel.
 * aba_autotune: times the generic and the specialised kernel at B = 1024,
 * 4096, 16384, 65536 and routes each tier to the faster; *min_batch as for
 * bard_chain_autotune.  aba_source: the generated text.  Routed calls whose
 * per-instance byte offset into an array reaches 4 GiB run the generic
 * kernel. */
int bard_model_specialize_aba(bard_model_t model, bard_dtype dtype, int32_t flags);
int bard_model_specialized_aba_info(bard_model_t model, bard_dtype dtype, int32_t* vgprs, int32_t* scratch_bytes,
                                    double* compile_seconds, int32_t* routed_tiers);
int bard_aba_autotune(bard_model_t model, bard_dtype dtype, void* stream, int64_t* min_batch);
int bard_model_specialized_aba_source(bard_model_t model, bard_dtype dtype, char* buf, int64_t cap, int64_t* len);

/* ------------------------------------------------------------ workspace ----
 * A workspace holds cached state of one stream for up to max_batch instances
 * (Sec. 3.1's tiered lazy evaluation, extended to dynamics results), in
 * tiers keyed by caller version tags:
 *   BARD_TIER_KINEMATICS (q_tag): the world pose of every body, every joint's
 *     motion subspace and the base origin.  A call whose components were all
 *     computed for its q_tag and B loads them instead of computing them (FK,
 *     Jacobian and CRBA then skip the level sweep; RNEA keeps only the
 *     velocity and acceleration propagation); otherwise it computes them and
 *     stores what it computed.  Used by bard_fk, bard_jacobian, bard_rnea and
 *     bard_crba.
 *   BARD_TIER_MASS (q_tag): M(q).  bard_crba on a hit copies the cached
 *     matrix into its output instead of launching the tree traversal; on a
 *     miss it computes M and copies it into the tier.
 *   BARD_TIER_BIAS (q_tag, qd_tag): the bias forces b = RNEA(q, qd, 0).
 *     bard_rnea without an inertia override and with both tags non-zero, on a
 *     hit of both this tier and the mass tier, returns tau = M qdd + b (RNEA
 *     is affine in qdd with slope M) from one bandwidth-bound pass instead of
 *     the traversal; when b is missing it computes tau and b in one traversal
 *     and stores b (not on trees of depth 32 or more, which take the
 *     pointer-jumping kinematics: there b is not cached).  The cached path
 *     rounds differently: its error is bounded like ABA's backward error,
 *     atol + rtol (|tau| + |M| |qdd| + |b|) in the infinity norm.
 * bard_aba and bard_chain accept a workspace for argument checks only.  Equal
 * non-zero tags promise equal contents; the library never inspects inputs to
 * check.  Each tier (4 or 8 bytes x rows x max_batch; rows = 12 n_bodies +
 * 6 nv + 3, nv*nv and nv) is allocated on the first call that uses it, on the
 * workspace's device (that of its first use); a workspace serves one stream
 * at a time.  Changing the model's gravity invalidates the bias tier.
 * Errors: BARD_E_ARG, BARD_E_NOMEM. */
#define BARD_TIER_KINEMATICS 1
#define BARD_TIER_MASS 2
#define BARD_TIER_BIAS 4
int bard_ws_create(bard_model_t model, bard_dtype dtype, int64_t max_batch, bard_ws_t* out);
int bard_ws_destroy(bard_ws_t ws);
/* policy: the OR of the BARD_TIER_* bits in use (default BARD_TIER_KINEMATICS;
 * 0: the workspace is not used and every call computes everything).  Whether
 * reloading cached state beats recomputing it depends on the tree and the
 * batch; the policy is the knob that chooses.
 * Errors: BARD_E_ARG (NULL workspace, unknown bits). */
int bard_ws_set_policy(bard_ws_t ws, int32_t policy);
/* Counters of the tier decisions taken so far, per tier in the order
 * kinematics, mass, bias (arrays of 3; either may be NULL): a hit reused the
 * tier, a miss computed (and stored) its contents.  A call counts once per
 * tier it consults.  Errors: BARD_E_ARG. */
int bard_ws_stats(bard_ws_t ws, uint64_t* hits, uint64_t* misses);

/* ------------------------------------------------------------ operators ----
 * q_tag / qd_tag: caller version tags of q and qd for the workspace; 0 =
 * unknown (always recompute).  Only bard_rnea's bias tier uses qd_tag. */

/* FK (world pose of every body, Sec. 3.1 tier 3).
 * Arrays (L order): q [nq] in, poses [n_bodies*12] out. */
int bard_fk(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, void* poses,
            const bard_layout* L, uint64_t q_tag, int64_t B, void* stream);

/* Geometric Jacobian of n_ee end-effector bodies (eq. (7)); zeros off the
 * root-to-body path.  ee_body is a HOST array of body indices.
 * Arrays: q [nq] in, J [n_ee*6*nv] out (per end effector a 6 x nv block). */
int bard_jacobian(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, int32_t n_ee,
                  const int32_t* ee_body, bard_frame frame, void* J, const bard_layout* L,
                  uint64_t q_tag, int64_t B, void* stream);

/* Standalone FK and Jacobian of one kinematic chain (Sec. 3.1: path-only
 * functions for a root-to-end-effector chain).  Visits only the bodies on the
 * path from ee_body's root to ee_body, uses no workspace and caches nothing.
 * Below 65,536 instances 4 or 16 lanes share an instance's path (segments
 * combined by a scan across lanes); from there one lane walks it (the
 * environment variable BARD_PATH_LANES = 1 or 16 pins either form).  pose and J hold the
 * same values (up to rounding) as the ee_body block of bard_fk's poses and
 * of bard_jacobian's J for the one end effector ee_body.
 * Arrays (L order, three entries): q [nq] in; pose [12] out, the 3x4
 * [R | p] of ee_body (NULL: not computed); J [6*nv] out, the eq. (7)
 * columns of the dofs on the path and zeros elsewhere (NULL: not computed).
 * At least one of pose and J is given.
 * Errors: BARD_E_ARG (NULL model or q, no output, ee_body outside
 * 0..n_bodies-1, bad frame or stride), BARD_E_CAPTURE (first use of the model
 * on a device while capturing), BARD_E_DEVICE. */
int bard_path_kinematics(bard_model_t model, bard_dtype dtype, const void* q, int32_t ee_body, bard_frame frame,
                         void* pose, void* J, const bard_layout* L, int64_t B, void* stream);

/* Inverse dynamics tau = M(q) qdd + C(q, qd) qd + g(q) (RNEA, Sec. 3.3).
 * inertia_override: NULL or a DEVICE array [n_bodies][10] (same dtype, shared by
 * all instances) replacing the model's inertial parameters.
 * Arrays: q [nq], qd [nv], qdd [nv] in, tau [nv] out. */
int bard_rnea(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd,
              const void* qdd, const void* inertia_override, void* tau, const bard_layout* L,
              uint64_t q_tag, uint64_t qd_tag, int64_t B, void* stream);

/* Joint-space mass matrix M(q) by the composite-rigid-body algorithm, one of
 * the operators the paper restructures (Sec. 3; its composite-inertia update
 * is the 6x6 congruence Sec. 3.5 names as the cost of CRBA and ABA, which the
 * base-frame kernels here replace by plain sums).  Both triangles are
 * written from one value, so M is bitwise symmetric.
 * Arrays: q [nq] in, M [nv*nv] out (row-major). */
int bard_crba(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, void* M,
              const bard_layout* L, uint64_t q_tag, int64_t B, void* stream);

/* Forward dynamics qdd = M(q)^-1 (tau - C(q, qd) qd - g(q)) by the
 * articulated-body algorithm (Sec. 3), whose three passes (velocities root to
 * leaves, articulated inertias and bias forces leaves to root, accelerations
 * root to leaves) Sec. 4.1 names as the reason its rounding error exceeds
 * that of RNEA and CRBA.  A free root solves its 6x6 articulated system by
 * Cholesky factorisation.
 * Arrays: q [nq], qd [nv], tau [nv] in, qdd [nv] out. */
int bard_aba(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd,
             const void* tau, void* qdd, const bard_layout* L, uint64_t q_tag, uint64_t qd_tag,
             int64_t B, void* stream);

/* Fused RNEA + CRBA + Jacobian: one forward and one backward sweep per
 * instance sharing the per-body transforms.  The paper evaluates the three
 * operators separately (its "full" pipeline chains them); this fused form and
 * its throughput metric (evaluations of all three per second) are this
 * library's addition.  Results equal the three separate operators up to
 * rounding.  Arrays: q [nq], qd [nv], qdd [nv] in; tau [nv], M [nv*nv],
 * J [n_ee*6*nv] out. */
int bard_chain(bard_model_t model, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd,
               const void* qdd, int32_t n_ee, const int32_t* ee_body, bard_frame frame, void* tau,
               void* M, void* J, const bard_layout* L, int64_t B, void* stream);

/* ------------------------------------------------------------- adjoints ----
 * Vector-Jacobian products: the gradients Sec. 4.3 takes through RNEA with
 * respect to the state and the inertial parameters (system identification),
 * and the FK gradient of the functional mode (Sec. 3.5).  Both run as one
 * level sweep and subtree sums in the world frame (the gradient for q_j is
 * s_j . W_j, W_j a sum over the subtree of body j), with no stored tape.
 * A free root's q_bar has 7 entries: position (zero for rnea_vjp, which does
 * not depend on it) and quaternion [x y z w]; the quaternion is normalised on
 * read, so its gradient is orthogonal to q (the change of q along itself
 * changes nothing).
 *
 * rnea_vjp: given tau_bar, writes per instance q_bar = (dtau/dq)^T tau_bar
 * [nq], qd_bar [nv] and qdd_bar [nv]; if inertia_bar != NULL, also the
 * gradient with respect to the [n_bodies][10] inertial parameters (the layout
 * of bard_model_create), summed over the batch.  inertia_bar is a dense
 * DEVICE array of the call's dtype, overwritten; the batch sum is accumulated
 * in FP64 in a fixed order (two stages: per-workgroup sums over a fixed grid,
 * then a fixed-order sum of those), so results are identical run to run.
 * inertia_override (nullable, device [n_bodies][10]) replaces the model's
 * parameters as in bard_rnea.
 * Arrays (L order): q, qd, qdd, tau_bar in; q_bar, qd_bar, qdd_bar out
 * (inertia_override and inertia_bar take no layout).
 * Scratch: a call with inertia_bar != NULL uses a per-model, per-device FP64
 * buffer of 2048 * n_bodies * 10 values, allocated on the first such call;
 * such calls on one model and device must not overlap (different streams
 * included).
 * Errors: BARD_E_ARG (NULL array, bad stride), BARD_E_NOMEM, BARD_E_CAPACITY,
 * BARD_E_DEVICE. */
int bard_rnea_vjp(bard_model_t model, bard_dtype dtype, const void* q, const void* qd,
                  const void* qdd, const void* inertia_override, const void* tau_bar, void* q_bar,
                  void* qd_bar, void* qdd_bar, void* inertia_bar, const bard_layout* L, int64_t B,
                  void* stream);
/* rnea_vjp_noalloc: bard_rnea_vjp for callers that cannot allocate device
 * memory -- code being captured into a HIP graph, tight serving or training
 * loops, harnesses that forbid allocation.  Same arguments, outputs, layouts
 * and kernels (its results are bitwise those of bard_rnea_vjp on the same
 * device), but it calls no allocating routine: the model must already be on
 * the current device (bard_model_upload, or any earlier operator call there),
 * else BARD_E_STATE and nothing is launched; and the per-workgroup
 * inertial-parameter sums go to a file-scope device array of 2048 * 64 * 10
 * FP64 values (10 MiB), one per GPU the library runs on, held until the
 * process ends.  That array is shared by every call on a GPU and keeps the
 * last call's contents (every workgroup overwrites its own sums before they
 * are read, so nothing needs clearing): calls with inertia_bar != NULL that
 * overlap on one GPU -- other streams, other models, other threads -- race
 * and must be serialised by the caller.  A request whose sums would not fit
 * returns BARD_E_CAPACITY (not reachable with n_bodies <= 64).
 * Errors: as bard_rnea_vjp, plus BARD_E_STATE. */
int bard_rnea_vjp_noalloc(bard_model_t model, bard_dtype dtype, const void* q, const void* qd,
                          const void* qdd, const void* inertia_override, const void* tau_bar,
                          void* q_bar, void* qd_bar, void* qdd_bar, void* inertia_bar,
                          const bard_layout* L, int64_t B, void* stream);
/* fk_vjp: given poses_bar (per body the 3x4 row-major [R_bar | p_bar] of the
 * bard_fk output), writes q_bar [nq] = (d poses / dq)^T poses_bar.
 * Arrays (L order): q, poses_bar [n_bodies*12] in; q_bar out.
 * Errors: as bard_rnea_vjp. */
int bard_fk_vjp(bard_model_t model, bard_dtype dtype, const void* q, const void* poses_bar,
                void* q_bar, const bard_layout* L, int64_t B, void* stream);
/* crba_vjp: given M_bar (per instance an nv x nv cotangent, row-major), writes
 * q_bar [nq] = d<M_bar, M(q)>/dq, the derivatives of the mass matrix that
 * analytical forward-dynamics derivatives and trajectory optimisation need
 * (Sec. 2 names analytical dynamics derivatives as prior art; Sec. 5 names
 * trajectory optimisation as the next use of the differentiable operators).
 * One traversal: the CRBA sweeps, then per dof and per body the sensitivities
 * of <M_bar, M> to each motion subspace and composite inertia, gathered over
 * subtrees as for rnea_vjp.  Only the symmetric part of M_bar matters (M is
 * symmetric).  A free root's seven entries are zero: with the root velocity
 * in the root's body frame, M does not depend on the root's pose.
 * Arrays (L order): q [nq], M_bar [nv*nv] in; q_bar [nq] out.
 * Errors: BARD_E_ARG, BARD_E_CAPACITY (the tile's on-chip state does not fit,
 * e.g. FP64 on trees of about 30 bodies or more), BARD_E_DEVICE,
 * BARD_E_CAPTURE. */
int bard_crba_vjp(bard_model_t model, bard_dtype dtype, const void* q, const void* M_bar, void* q_bar,
                  const bard_layout* L, int64_t B, void* stream);
/* aba_vjp: reverse-mode product of forward dynamics qdd = ABA(q, qd, tau)
 * (the analytical derivatives of forward dynamics).  Differentiating
 * RNEA(q, qd, qdd) = tau gives dqdd = M^-1 (dtau - dRNEA/dq dq - dRNEA/dqd dqd),
 * so for the cotangent qdd_bar: tau_bar = M^-1 qdd_bar (the articulated-body
 * sweeps with no velocity and no gravity), and q_bar, qd_bar are the RNEA
 * adjoint at (q, qd, qdd) for the cotangent -tau_bar.  qdd must be the
 * forward-dynamics result for (q, qd, tau).
 * Arrays (L order): q [nq], qd [nv], qdd [nv], qdd_bar [nv] in; q_bar [nq],
 * qd_bar [nv], tau_bar [nv] out.  Two launches on `stream`.
 * Errors: as bard_rnea_vjp. */
int bard_aba_vjp(bard_model_t model, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
                 const void* qdd_bar, void* q_bar, void* qd_bar, void* tau_bar, const bard_layout* L,
                 int64_t B, void* stream);

/* ---------------------------------------------------- multi-tree plans ----
 * A plan evaluates several models, each with its own batch size, in one
 * launch over a list of work items (model, tile of instances).  The paper
 * evaluates one robot per call and notes that small trees leave per-launch
 * overhead dominant (Sec. 5); batching uneven trees into one launch is this
 * library's addition for that regime.  Items are ordered longest first,
 * so the hardware workgroup dispatcher, which hands out workgroups in order,
 * acts as a longest-processing-time work queue.
 *
 * op_mask: bit 0 RNEA, bit 1 CRBA, bit 2 Jacobian.  The Jacobian of a model
 * covers its tip end effectors: its leaves of greatest depth, at most four,
 * ties to the lowest body index (bard_plan_ee lists them), in BARD_WORLD.
 * io: per model 6 DEVICE pointers q, qd, qdd, tau, M, J, every array
 * instance-minor [K][batch] (the default layout of the operators); pointers
 * an op_mask does not need may be NULL.
 * bard_plan_run: the first run of a configuration launches directly; later
 * runs replay one HIP graph captured from it.  When io changes, the new
 * pointers are copied to the plan's device descriptor in stream order, so the
 * graph is never recaptured.  A plan runs on the device of its first run and
 * on one stream at a time.  Preparing a configuration (first run, first run
 * after bard_plan_configure or bard_plan_autotune) synchronizes the device.
 * bard_plan_autotune: times every valid configuration (tile 8, 16 or 32 instances;
 * fusion 0 = one launch for all models, 1 = one launch per model, 2 = one
 * launch per operator, 3 = one launch of a kernel generated for the plan's
 * trees; item order 0 = longest first, 1 = model order; lanes
 * per instance at the model's minimum or twice that) on
 * zero-filled scratch arrays for about budget_ms, keeps the fastest and
 * records it in a JSON cache (file $BARD_TUNE_CACHE, else
 * $HOME/.cache/bard_plan_tune.json) keyed by the GPU, dtype, op_mask, tree
 * topologies and batches; bard_plan_create applies a cached choice.
 * Errors: BARD_E_ARG, BARD_E_NOMEM, BARD_E_CAPACITY (a tree does not fit the
 * tile's on-chip staging), BARD_E_DEVICE. */
int bard_plan_create(const bard_model_t* models, int32_t n_models, const int64_t* batch,
                     uint32_t op_mask, bard_dtype dtype, bard_plan_t* out);
int bard_plan_autotune(bard_plan_t plan, void* stream, int32_t budget_ms);
/* bard_plan_run on a stream the caller is capturing into a HIP graph: the
 * plan must have run before (eagerly) with the same io; the call then records
 * its kernel launches into the caller's graph (BARD_E_CAPTURE otherwise). */
int bard_plan_run(bard_plan_t plan, const void* const* io, void* stream);
int bard_plan_destroy(bard_plan_t plan);
/* Pin a configuration (what bard_plan_autotune chooses): tile 8, 16 or 32,
 * fusion 0..3, order 0..1 as above, lanes 0 or 1 (twice the lanes per
 * instance of the level sweep when 1: each instance's bodies spread over
 * more lanes, so a tile occupies more waves).  Fusion 0 and 1 need op_mask to
 * be one operator or all three.  A configuration whose sweep needs more than
 * 8 waves is refused by the first run with BARD_E_CAPACITY.
 * Fusion 3 (all three operators only; tile and order are ignored): the
 * model compiler emits one kernel holding every tree's model-specialised
 * chain code (as bard_model_specialize does for one model: every constant a
 * literal, one lane per instance, the dual form where a tree has limbs),
 * compiled with hipRTC on the plan's first run in this configuration (which
 * may take seconds); its workgroups take the trees' 64-instance groups,
 * trees of larger nv first; each tree is split over at most 8 waves (lanes
 * 0) or 4 (lanes 1: narrower workgroups, two of which fit a CU where one of
 * 8 waves did).  bard_plan_autotune always includes both when the plan has
 * all three operators and does not count their compilation against
 * budget_ms. */
int bard_plan_configure(bard_plan_t plan, int32_t tile, int32_t fusion, int32_t order, int32_t lanes);
/* Current configuration; from_cache = 1 if it came from the tuning cache. */
int bard_plan_get_config(bard_plan_t plan, int32_t* tile, int32_t* fusion, int32_t* order, int32_t* lanes,
                         int32_t* from_cache);
/* The generated source of the plan's fusion-3 kernel for its current lanes
 * setting (NUL-terminated into buf when cap > 0; *len its length without
 * the NUL); compile_only = 1 also compiles it for gfx950 with hipRTC (no GPU
 * needed) and reports a failure as BARD_E_DEVICE.  Errors: BARD_E_ARG, BARD_E_UNSUPPORTED (op_mask not all
 * three operators), BARD_E_DEVICE. */
int bard_plan_specialized_source(bard_plan_t plan, int32_t compile_only, char* buf, int64_t cap, int64_t* len);
/* Resources of the plan's fusion-3 kernel once built (any argument may be
 * NULL): registers per lane, scratch bytes per lane, waves per workgroup,
 * workgroups per launch and the seconds its generation and compilation took
 * (0 when the code object came from an earlier plan with the same source).
 * Errors: BARD_E_ARG, BARD_E_STATE (not built yet). */
int bard_plan_specialized_info(bard_plan_t plan, int32_t* vgprs, int32_t* scratch_bytes, int32_t* waves,
                               int64_t* workgroups, double* compile_s);
/* Tip end effectors of model `model_index` (ee_body: room for 4 entries). */
int bard_plan_ee(bard_plan_t plan, int32_t model_index, int32_t* n_ee, int32_t* ee_body);

#ifdef __cplusplus
}
#endif

#endif /* BARD_H */
