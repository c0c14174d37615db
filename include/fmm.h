/*
 * fmm.h -- C ABI of libfmm.so, an MI355X (gfx950) implementation of the
 * Cartesian Fast Multipole Method and the multipolar Barnes-Hut method of
 * Pepper & Fangohr, "fmmgen: Automatic Code Generation of Operators for
 * Cartesian Fast Multipole and Barnes-Hut Methods" (arXiv 2005.12351).
 *
 * What is computed (Section 2): the potential phi(x_i) = sum_{j != i} of the
 * field of point sources of order m (0 monopole, 1 dipole, 2 quadrupole,
 * 3 octupole) with the Coulomb kernel 1/|x_i - x_j| (Eq. 1, no 1/(4 pi)
 * factor), and the field E = -grad phi.  Physical moments: phi = q/r,
 * phi = mu.r/r^3, phi = 1/2 sum_ij Q_ij d_i d_j (1/r),
 * phi = -1/6 sum_ijk O_ijk d_i d_j d_k (1/r) with r = x_target - x_source
 * (each the order-m term of the multipole series of a charge cloud with
 * moments sum q x^m).
 *
 * Method (Section 3.2): an adaptive octree split while a cell holds more than
 * ncrit particles, P2M at the leaves (Eq. 3, Eq. 5), M2M upward (Eq. 4), then
 *   FMM: dual-tree traversal with the acceptance test (r_A + r_B) < theta R
 *        (Eq. 13), stored interaction lists, M2L (Eq. 8), L2L, L2P (Eq. 9-10)
 *        and direct P2P over the near-field lists;
 *   BH:  per-particle traversal with r_A < theta |x - z_A| (Eq. 12), M2P
 *        (Eq. 6) for accepted cells and P2P at unaccepted leaves.
 * Cell radius r = half the cell side; expansion centre = geometric centre.
 *
 * Conventions of every entry point:
 *  - All particle arrays are DEVICE pointers of the context's device, owned
 *    by the caller, IEEE double, C-contiguous:
 *      pos      n x 3   (x, y, z)
 *      moments  n       (order 0: q)
 *               n x 3   (order 1: mu_x, mu_y, mu_z)
 *               n x 6   (order 2: Q_xx, Q_xy, Q_xz, Q_yy, Q_yz, Q_zz, symmetric Q)
 *      phi      n       output potential, caller's particle order
 *      field    n x 3   output field, caller's particle order
 *  - Calls are stream-ordered on the context's stream and return before the
 *    GPU work finishes; inputs must stay valid and outputs untouched until the
 *    stream is synchronised.  fmm_build_tree is the exception: it reads the
 *    positions back to the host and returns after the tree is resident.
 *    The library orders nothing against the caller's other streams: work
 *    that produces an input must be complete or ordered before the call on
 *    the context's stream (e.g. an event recorded on the producer's stream
 *    and waited on by the context's stream), and work that consumes an output
 *    must be ordered after the call the same way.
 *  - Every entry point returns FMM_OK or an error code; no C++ exception
 *    crosses the ABI.  Arguments are checked before any GPU work is queued.
 *    fmm_last_error() returns a thread-local text for the last failure.
 *  - The library owns fmm_ctx and fmm_tree objects and all device memory they
 *    hold; free them with the matching *_destroy call.
 *  - A context and its trees are used from one host thread at a time;
 *    different contexts may be used from different threads at once (the
 *    serving loop gives each slot its own).  Results do not depend on how
 *    many host threads a build gets.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_ctx fmm_ctx;
typedef struct fmm_tree fmm_tree;

enum {
    FMM_OK = 0,
    FMM_EINVAL = 1,    /* bad argument; nothing was queued */
    FMM_ENOMEM = 2,    /* device or host allocation failed / over the budget */
    FMM_EDEVICE = 3,   /* a HIP call failed */
    FMM_ESTATE = 4,    /* call out of order (e.g. evaluate before upward) */
    FMM_EBUSY = 5,     /* serving: request not finished yet */
    FMM_ETIMEOUT = 6   /* serving: wait timed out */
};

enum { FMM_POT = 1, FMM_FIELD = 2, FMM_GRAD = 4 };   /* output bit mask (FMM_GRAD: fmm_evaluate_grad only) */
enum { FMM_METHOD_FMM = 0, FMM_METHOD_BH = 1 };
enum { FMM_M2L_FULL = 0, FMM_M2L_HARMONIC = 1 };   /* see fmm_ctx_set_m2l_basis */
enum { FMM_M2L_ENGINE_VALU = 0, FMM_M2L_ENGINE_MFMA = 1, FMM_M2L_ENGINE_AUTO = 2 };   /* see fmm_ctx_set_m2l_engine */
enum {
    FMM_PREC_FP64 = 0,   /* every operator in IEEE double on the GPU */
    FMM_PREC_MIXED = 1   /* M2L, M2P and P2P in FP32 (P2P compensated),
                            P2M, M2M, L2L, L2P in FP64 */
};

#define FMM_P_MAX 10     /* largest expansion order p compiled in */

/* Source order codes.  0, 1, 2, 3: every particle is a charge, a dipole, a
 * quadrupole or an octupole.  FMM_MIXED | mask: several orders in one system
 * (mask bit k: order k present, e.g. FMM_MIXED | 3 for charges with dipoles);
 * each moment row then holds the present orders' moments in ascending order,
 * [q | mu | Qxx Qxy Qxz Qyy Qyz Qzz | Oxxx Oxxy Oxxz Oxyy Oxyz Oxzz Oyyy
 * Oyyz Oyzz Ozzz], and the expansions start at the lowest order present
 * (Section 2: the multipole series of a point source of order s starts at
 * order s; a system's series is the sum of its sources'). */
#define FMM_MIXED 16

/* Context on HIP device `device`; `hip_stream` is a hipStream_t (NULL: the
 * library creates its own, non-blocking).  Calls that capture graphs need a
 * stream other than the legacy default stream.  `hbm_budget_bytes` bounds
 * the device memory the serving loop admits (0: 80% of the free memory at
 * creation).  The context keeps device memory for reuse, each part up to
 * min(budget / 8, 4 GiB): the blocks of destroyed trees (handed to later
 * trees of the same size class) and the scratch arena of tree builds; both
 * are released with the context.  Creating a context also sets the release
 * threshold of the device's default stream-ordered memory pool to keep
 * freed memory mapped for reuse (process-wide; memory freed to that pool is
 * not returned to the driver before the process ends).  A context is used
 * by one host thread at a time. */
int fmm_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, fmm_ctx **out);
/* Destroys the context after its device work has finished.  Trees of this
 * context that are still alive lose their device memory; fmm_tree_destroy
 * remains valid on them (and is then the only call they accept). */
int fmm_ctx_destroy(fmm_ctx *ctx);

/* Device bytes one tree of this context may hold (0, the default: no limit).
 * A tree allocation beyond it fails with FMM_ENOMEM, as one the device
 * refuses does: the call returns FMM_ENOMEM with nothing queued that reads
 * the missing buffers, the tree keeps no half-built expansion set, and a
 * later fmm_upward / fmm_run whose buffers fit sets it up again (with any
 * parameters, the failed call's previous ones included). */
int fmm_ctx_set_tree_limit(fmm_ctx *ctx, size_t bytes);

/* Octree, Morton order and (for FMM) interaction lists of n particles
 * (Section 3.2).  n >= 1, ncrit >= 1, 0 < theta < 1; method FMM_METHOD_FMM or
 * FMM_METHOD_BH (for BH, theta is the acceptance parameter of Eq. 12 used by
 * fmm_evaluate).  The root box is the cube of side W = the largest extent of
 * the positions, with corner at the componentwise minimum. */
int fmm_build_tree(fmm_ctx *ctx, const double *pos, int64_t n, int ncrit, double theta,
                   int method, fmm_tree **out);

/* Upward pass: P2M at the leaves (Eq. 5 with the source tensor
 * S_n = (-1)^|n| T_n / n! of the physical moment T) and M2M towards the root
 * (Eq. 4), expansion order p; for FMM trees also the near field (direct
 * sums over the P2P lists, Section 3.2) into library-owned storage, since it
 * depends only on the moments.  order: a source order code (0, 1, 2, 3 or
 * FMM_MIXED | mask, see above) with lowest order s; s+1 <= p <= FMM_P_MAX
 * for FMM, max(s,1) <= p <= FMM_P_MAX for BH.  `moments`: device, n x w FP64
 * row-major (w = 1, 3, 6, 10 for one order, the sum of the present orders'
 * widths for several), caller-owned, read only by the work this call queues
 * on the context stream (a sorted copy is kept). */
int fmm_upward(fmm_ctx *ctx, fmm_tree *tree, int order, const double *moments, int p,
               int precision);

/* Far field (M2L, L2L, L2P or, for BH, the whole per-particle traversal
 * with M2P and direct sums) plus the near field summed by fmm_upward, at
 * every particle, written in the caller's particle order.  `outputs` is a mask of FMM_POT / FMM_FIELD; phi (n) and field
 * (n x 3) must be non-NULL for the requested outputs.  FMM_ESTATE if
 * fmm_upward has not run on this tree. */
int fmm_evaluate(fmm_ctx *ctx, fmm_tree *tree, int outputs, double *phi, double *field);

/* fmm_evaluate plus the field gradient (Section 2: derivatives of the
 * potential of order |k| from the local expansion, here k = e_i + e_j).
 * `outputs` may add FMM_GRAD; grad (n x 6, caller order, device FP64)
 * receives G_ij = d_i E_j = -d_i d_j phi as xx, xy, xz, yy, yz, zz: the
 * second derivatives of the local expansion, -(1/r^3) sum_{|n| <= p-s-2}
 * eta^n/n! L~_{n+e_i+e_j}, plus the closed-form gradients of the near-field
 * pairs (computed by an extra near-field pass in this call, in the tree's
 * precision).  phi and field as for fmm_evaluate and bit-identical to it.
 * FMM trees need p - s >= 2 (below that the truncated expansion has no
 * second derivative; a finite difference of it would be zero too):
 * FMM_EINVAL otherwise, FMM_ESTATE before fmm_upward.  The near-field
 * gradient buffer (48 bytes per particle) is allocated on the first call.
 * Barnes-Hut trees (any p the tree accepts): each accepted cell adds
 * -(1/r^3) sum_m M~_m D_{m+e_i+e_j}(u) (the second derivatives of the M2P of
 * Eq. 6, u = (x - z_A)/r, r the cell's half side), each unaccepted leaf the
 * pairs' closed forms, in one traversal that also writes phi and field
 * (equal to fmm_evaluate's up to the rounding of the tree's precision: the
 * kernel is a separately compiled variant). */
int fmm_evaluate_grad(fmm_ctx *ctx, fmm_tree *tree, int outputs, double *phi, double *field, double *grad);

/* fmm_evaluate_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same outputs, from the same kernels, but the near-field gradient of an
 * FMM tree (48 bytes per particle) goes to a static device array that the
 * library holds on every device it runs on until the process ends, so the
 * call makes no hipMalloc/hipFree or other allocating call, and it launches
 * the kernels one by one instead of capturing a graph.  Limit: FMM trees of
 * at most 262 144 (2^18) particles when FMM_GRAD is requested (12 MiB of
 * scratch); larger ones get FMM_EINVAL (use fmm_evaluate_grad).  Barnes-Hut
 * trees use no scratch and have no limit.  Every call on a device shares that
 * device's array: calls that overlap on one device (from several contexts or
 * streams) race and give wrong gradients; each call writes every particle's
 * six values before reading them, so nothing carries over between calls.
 * The tree's own buffers come from fmm_build_tree and fmm_upward, which
 * allocate as usual. */
int fmm_evaluate_grad_noalloc(fmm_ctx *ctx, fmm_tree *tree, int outputs, double *phi, double *field,
                              double *grad);

/* Derivatives of the potential of order K = 1, 2 or 3 at every particle
 * (Section 2: the derivatives of order |k| from the local expansion, Eq. 10,
 * plus the same derivatives of the near-field pair potentials,
 * sum_{|m|=s} S_m D_{m+k}(x_i - x_j)).  out: device, n x (K+1)(K+2)/2 FP64,
 * caller's particle order; the columns are d^k phi for the multi-indices of
 * order K in the index order (n_x descending, then n_y): K = 1 gives -E,
 * K = 2 gives -G of fmm_evaluate_grad, K = 3 the ten third derivatives
 * d_i d_j d_l phi = -d_i d_j E_l.  Computed in FP64 from the tree's
 * expansions (in MIXED precision the FMM locals come from the FP32 M2L) and
 * its sorted FP64 moments.  FMM trees: K <= p - s (the truncated local
 * expansion has no derivative of higher order).  Barnes-Hut trees: Eq. 6
 * differentiated K times for every cell the particle accepts (Eq. 12, own
 * cell never accepted) plus the pairs of the unaccepted leaves, any p.
 * FMM_EINVAL for other K, FMM_ESTATE before fmm_upward. */
int fmm_evaluate_derivs(fmm_ctx *ctx, fmm_tree *tree, int K, double *out);

/* Tree sizes: info[0..9] = n, ncells, nlevels, nleaves, n_m2l, n_p2p,
 * n_m2l_classes, n_m2l_tiles, n_m2l_slots_used (tile lanes x union entries),
 * device bytes held. */
int fmm_tree_info(const fmm_tree *tree, int64_t *info);

/* fmm_upward followed by fmm_evaluate, with the same arguments, results and
 * errors, queued as one launch sequence (one captured graph when graphs are
 * on): the near field then overlaps the whole far field and is joined only
 * before the final L2P.  The tree keeps the upward state afterwards, so
 * fmm_evaluate may follow. */
int fmm_run(fmm_ctx *ctx, fmm_tree *tree, int order, const double *moments, int p, int precision,
            int outputs, double *phi, double *field);

/* Copy the canonical tree to HOST arrays (any pointer may be NULL), sized by
 * fmm_tree_info: geom[4] = lo_x, lo_y, lo_z, W; key[n] Morton keys of the
 * sorted particles; perm[n] input index of sorted particle i; per cell
 * (level-major, ascending key): level, ix[3] integer cell coordinates,
 * first, count (sorted particle range), parent (-1 at the root), child0,
 * nchild; CSR interaction lists per target cell, sources sorted ascending:
 * m2l_ptr[ncells+1], m2l_src[n_m2l], p2p_ptr[ncells+1], p2p_src[n_p2p].
 * When the M2L schedule was made on the device the M2L lists live there
 * only: asking for them synchronises the context stream. */
int fmm_tree_export(const fmm_tree *tree, double *geom, uint64_t *key, int64_t *perm,
                    int32_t *level, int32_t *ix, int64_t *first, int64_t *count,
                    int64_t *parent, int64_t *child0, int32_t *nchild, int64_t *m2l_ptr,
                    int64_t *m2l_src, int64_t *p2p_ptr, int64_t *p2p_src);

int fmm_tree_destroy(fmm_tree *tree);

/* Text of the last error on the calling thread ("" if none). */
const char *fmm_last_error(void);

/* Near field (P2P) on a second stream beside the far field.  `on`:
 * FMM_OVERLAP_OFF (default): every kernel runs on the context stream, one
 * after the other, so the per-kernel timings below measure each kernel alone;
 * FMM_OVERLAP_WHOLE: the whole near field beside the whole far field;
 * FMM_OVERLAP_SPLIT: in fmm_run, half the near field (by cost) beside the
 * upward M2M levels, joined before the M2L, the other half after the M2L
 * beside the combine and L2L, joined before the L2P, so that it never
 * competes with the M2L (fmm_upward alone runs the whole near field);
 * FMM_OVERLAP_TAIL: in fmm_run, the whole near field after the M2L, beside
 * the combine and L2L, joined before the L2P (fmm_upward alone runs it as
 * OFF does).  FMM_EINVAL for other values. */
enum { FMM_OVERLAP_OFF = 0, FMM_OVERLAP_WHOLE = 1, FMM_OVERLAP_SPLIT = 2, FMM_OVERLAP_TAIL = 3 };
int fmm_ctx_set_overlap(fmm_ctx *ctx, int on);

/* Replay HIP graphs (default on): the kernel sequence of fmm_upward and of
 * fmm_evaluate is captured the first time a tree sees a given argument set
 * (moments / output pointers, order, p, precision) and replayed afterwards,
 * which removes the per-kernel launch cost.  Graphs are never used while
 * profiling is enabled.  Off: kernels are launched one by one. */
int fmm_ctx_set_graphs(fmm_ctx *ctx, int on);

/* Basis of the M2L contraction of FMM trees and of the M2P of Barnes-Hut
 * trees (Eq. 8, Eq. 6 and the Discussion's irreducible representation).  FMM_M2L_FULL contracts every Cartesian
 * component.  FMM_M2L_HARMONIC (default) uses that the derivative tensor of
 * 1/r is harmonic (D_{k+2e_x} + D_{k+2e_y} + D_{k+2e_z} = 0): each multipole
 * is folded once onto its components with m_z <= 1, the contraction runs on
 * those and yields the local components with n_z <= 1, and the remaining
 * local components follow from the same identity.  Order l then carries
 * 2l+1 components instead of (l+1)(l+2)/2 (at p = 8, s = 1: 1 284
 * multiply-adds per list entry instead of 2 838).  Barnes-Hut M2P likewise
 * contracts the folded row and forms only the derivatives with k_z <= 2.
 * In exact arithmetic both bases give the same results; they differ by
 * rounding only.  Takes effect at the
 * next fmm_upward / fmm_run of a tree.  FMM_EINVAL for another value. */
int fmm_ctx_set_m2l_basis(fmm_ctx *ctx, int basis);

/* Units that run the M2L contraction (Eq. 8) of MIXED-precision FMM trees in
 * the harmonic basis.  FMM_M2L_ENGINE_MFMA: the matrix cores, one
 * v_mfma_f32_4x4x1 per (multipole coefficient, four local outputs) for 64
 * target cells at once, FP32 products with FP32 accumulation as on the
 * vector units; FMM_M2L_ENGINE_VALU: the vector units, one FMA per term;
 * FMM_M2L_ENGINE_AUTO (default): the matrix cores for p >= 8, where they
 * were measured faster, the vector units below.  Both compute the same sums
 * (they round differently only through the order of the FP32 additions).
 * FP64 trees and the full basis always use the vector units.  Takes effect
 * at the next fmm_upward / fmm_run of a tree.  FMM_EINVAL for another
 * value. */
int fmm_ctx_set_m2l_engine(fmm_ctx *ctx, int engine);

/* Where fmm_build_tree makes the M2L schedule of FMM trees (Section 3.3:
 * the M2L of every target of every list, grouped for the kernel): targets
 * 64 to a tile in (level, position in the parent, same-level neighbourhood,
 * list length) order; per tile the sorted distinct pair geometries
 * ((z_B - z_A) / r_B, r_A / r_B), each one derivative tensor for all 64
 * lanes; class ids the ranks of the geometries among all tiles'; per
 * (entry, lane) the source cell or the zero row.  FMM_SCHEDULE_DEVICE:
 * built on the GPU after the interaction lists, without their round trip
 * through the host; when a tile holds more than 4096 distinct geometries or
 * a packed key would overflow the build takes the host code instead.
 * FMM_SCHEDULE_HOST: built by the host threads.  FMM_SCHEDULE_AUTO
 * (default): the device (measured faster for every tree size, from a few
 * thousand list entries on), the host where the device cannot.  All give
 * the same schedule, entry for entry.  Takes effect for trees
 * built afterwards.  FMM_EINVAL for another value. */
enum { FMM_SCHEDULE_HOST = 0, FMM_SCHEDULE_DEVICE = 1, FMM_SCHEDULE_AUTO = 2 };
int fmm_ctx_set_m2l_schedule(fmm_ctx *ctx, int where);

/* The M2L schedule of an FMM tree, to HOST arrays (any pointer may be NULL)
 * sized by fmm_tree_info (classes info[6], tiles info[7], slots info[8]):
 * tile_cell[64 tiles] target cell of each lane or -1; tile_uoff[tiles+1]
 * entry range of each tile; ucls[slots/64] class id of each entry (ascending
 * within a tile); usrc[slots] source cell of each (entry, lane), ncells
 * where the lane lacks the class; cls_geom[4 classes] the class geometry
 * (three offsets in units of r_B, then r_A / r_B); *where the schedule's
 * builder (FMM_SCHEDULE_DEVICE or _HOST).  Synchronises the context stream.
 * FMM_EINVAL for a Barnes-Hut tree. */
int fmm_tree_m2l_schedule(const fmm_tree *tree, int32_t *tile_cell, int32_t *tile_uoff, int32_t *ucls,
                          int32_t *usrc, double *cls_geom, int *where);

/* Per-kernel device timing.  When enabled, every kernel launch is bracketed
 * by HIP events on the stream it runs on.  fmm_profile_read synchronises and
 * writes, for up to `cap` kernel kinds, the kind name (static string), the
 * summed milliseconds and the launch count; returns the number of kinds. */
int fmm_profile_enable(fmm_ctx *ctx, int on);
int fmm_profile_reset(fmm_ctx *ctx);
int fmm_profile_read(fmm_ctx *ctx, const char **names, double *ms, int64_t *launches, int cap);

/* Algorithmic work of the last fmm_evaluate on a tree (for roofline
 * accounting): w[0] = M2L list entries, w[1] = M2L FLOPs (2 per
 * multiply-add of the contraction in the basis in use), w[2] = P2P pairs,
 * w[3] = P2P FLOPs, w[4] = M2P (cell, particle) pairs, w[5] = M2P FLOPs
 * (contraction plus derivative tensor, in the basis in use), w[6] = M2L
 * input and output bytes (one multipole and one local row per cell),
 * w[7] = P2P input and output bytes.  For Barnes-Hut trees
 * the traversal kernel counts its accepted cells and direct pairs itself;
 * reading them synchronises the context stream. */
int fmm_work_counts(const fmm_tree *tree, double *w);

/* ---------------------------------------------------------------- serving
 * Continuous batching: requests are admitted while their device footprint
 * fits the context budget and a stream slot is free; admitted requests run
 * tree build, upward pass and evaluation concurrently on separate HIP
 * streams and release their memory when done.  The caller owns the request's
 * buffers (device pointers, as above) until the request completes. */
typedef struct {
    const double *pos;       /* n x 3, device */
    const double *moments;   /* n x {1,3,6}, device */
    double *phi;             /* n or NULL, device */
    double *field;           /* n x 3 or NULL, device */
    int64_t n;
    int order, p, ncrit, method, precision, outputs;
    double theta;
} fmm_request;

enum { FMM_REQ_QUEUED = 0, FMM_REQ_RUNNING = 1, FMM_REQ_DONE = 2, FMM_REQ_FAILED = 3 };

/* Start the server with `max_concurrent` (1..64) worker slots, each with its
 * own context and stream.  Admission is in arrival order: the oldest queued
 * request starts when a slot is free and its estimated footprint fits in the
 * budget minus the footprints of the running requests.  One slot per
 * hardware queue of the process (4 by default) serves best: more slots
 * share queues, and a slot then waits behind another's kernels at each of
 * its tree build's read-backs.  Each slot's tree-build arena is allocated
 * here (64 MB, at most min(budget / 8, 4 GiB)), so that the first requests
 * do not pay for it. */
int fmm_serve_start(fmm_ctx *ctx, int max_concurrent);
/* Queue a request (copied); FMM_ENOMEM if its footprint exceeds the whole
 * budget, FMM_EINVAL for bad parameters (nothing is queued then).  The
 * request runs on the server's own streams, which are not ordered after any
 * stream of the caller: its inputs must be complete on the device when
 * fmm_submit is called (e.g. the producer stream synchronised), and its
 * outputs are complete once fmm_wait returns FMM_OK or fmm_poll reports
 * FMM_REQ_DONE. */
int fmm_submit(fmm_ctx *ctx, const fmm_request *req, uint64_t *ticket);
int fmm_poll(fmm_ctx *ctx, uint64_t ticket, int *state);
/* Block until the request is done (timeout_s < 0: no limit); FMM_ETIMEOUT
 * if it is not done in time, the request's own error code if it failed. */
int fmm_wait(fmm_ctx *ctx, uint64_t ticket, double timeout_s);
/* t[0] submit, t[1] admitted, t[2] done, in seconds since fmm_serve_start;
 * bytes[0] estimated footprint used for admission, bytes[1] device bytes the
 * request actually held. */
int fmm_request_times(fmm_ctx *ctx, uint64_t ticket, double *t, int64_t *bytes);
/* Worker-side phases of a finished request, seconds since fmm_serve_start:
 * t[0] tree and lists built, t[1] results on the device (after the stream
 * synchronisation); the device memory is released between t[1] and done.
 * Zero for a fake context or a request that has not run. */
int fmm_request_phases(fmm_ctx *ctx, uint64_t ticket, double *t);
/* stats[0..6] = budget, bytes admitted now, peak bytes admitted, running
 * requests, peak running, queued requests, slots. */
int fmm_serve_stats(fmm_ctx *ctx, int64_t *stats);
/* Stop accepting requests, finish the queued and running ones, join the
 * workers (also done by fmm_ctx_destroy). */
int fmm_serve_stop(fmm_ctx *ctx);

/* A context without a device whose server runs the scheduling and admission
 * logic with a simulated executor (each request waits ns_per_particle * n
 * nanoseconds and touches no memory).  Only the serving entry points accept
 * it; it exists to test the scheduler on machines without a GPU. */
int fmm_ctx_create_fake(size_t budget_bytes, double ns_per_particle, fmm_ctx **out);

#ifdef __cplusplus
}
#endif
#endif
