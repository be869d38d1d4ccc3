/*
 * oc.h -- C ABI of the MI355X overset connectivity library.
 *
 * The library computes the two data-parallel steps of overset domain
 * connectivity for curved quadratic grids (Crabill, Witherden & Jameson,
 * "A Parallel Direct Cut Algorithm for High-Order Overset Methods"):
 *
 *   hole cutting      Sec. 4.2 (Parallel Direct Cut) and Sec. 2.1 step 1:
 *                     every element of a grid is classified against closed
 *                     cutting surfaces as hole, fringe or field;
 *   point connectivity Sec. 4.3 and Sec. 2.1 step 2: each receptor point is
 *                     located in a donor element and its reference
 *                     coordinates are found by Newton inversion of the
 *                     isoparametric map (eq. reftophys, eq. ref-update).
 *
 * General rules
 *   - Every function returns an oc_status (0 = OC_OK, < 0 = error) and never
 *     aborts; oc_last_error() returns a thread-local message for the last
 *     failure of the calling thread.
 *   - Registration calls take HOST pointers; the library copies what it needs
 *     to device memory and the caller keeps ownership of its arrays.
 *   - Compute calls (oc_cut*, oc_fringe_points, oc_donor_search) take DEVICE
 *     pointers for bulk inputs and outputs and are ordered on the context's
 *     stream (oc_set_stream).  Poses are 12 host doubles
 *     {R00,R01,R02,R10,R11,R12,R20,R21,R22,tx,ty,tz} applied as x' = R x + t.
 *   - Results are deterministic: identical inputs give identical bits.
 *   - Floating point: element/face/donor boxes, bins and the box filter are
 *     FP32 with outward rounding (no true candidate is ever dropped); every
 *     decision (intersection, side, containment) is taken in FP64.
 *   - One context owns one device; a context is not thread safe.
 */
#ifndef OC_H
#define OC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oc_ctx oc_ctx;
typedef struct oc_slot oc_slot;
typedef int32_t oc_status;

enum {
    OC_OK = 0,
    OC_EINVAL = -1,    /* bad handle, size, pointer or argument */
    OC_ENOMEM = -2,    /* device or host allocation failed */
    OC_EDEVICE = -3,   /* HIP runtime error */
    OC_ENOTFOUND = -4, /* unknown grid / surface id */
    OC_EBUDGET = -5,   /* the context's HBM budget would be exceeded */
    OC_EGEOM = -6,     /* invalid geometry (open or inverted surface, inverted element) */
    OC_ECAPACITY = -7, /* an output buffer is too small */
    OC_ETIMEDOUT = -8, /* oc_wait: the request has not finished yet */
    OC_ESTARTED = -9   /* oc_cancel: the request is already on the device or finished */
};

/* int8 blanking values (hole map values are not reused: hole 0, field 1,
 * fringe -1; fringe = artificial-boundary element of Sec. 4.2) */
enum { OC_HOLE = 0, OC_FIELD = 1, OC_FRINGE = -1 };

/* Cutting-surface kinds (Sec. 3 and Sec. 4: near-body grids are cut by
 * solid walls, off-body grids by overset boundaries).  Elements intersected
 * by a WALL surface become holes; elements intersected by an OVERSET surface
 * stay field (they are needed for overlap). */
enum { OC_SURF_WALL = 0, OC_SURF_OVERSET = 1 };

/* Per-element face tags, face order (-xi, +xi, -eta, +eta, -zeta, +zeta). */
enum { OC_FACE_INTERIOR = 0, OC_FACE_WALL = 1, OC_FACE_OVERSET = 2, OC_FACE_FARFIELD = 3 };

/* Fixed constants of the method (not configurable: results depend on them). */
#define OC_TOL_HIT 1e-7      /* triangle pairs closer than this intersect (Alg. cp1/cp2) */
#define OC_NEWTON_MAXIT 10   /* Newton iteration limit (Sec. 4.3) */
#define OC_NEWTON_CLAMP 0.01 /* iterates clamped to [-1-c, 1+c] (Sec. 4.3) */
#define OC_CONTAIN_TOL 1e-10 /* contained if max|xi| <= 1 + tol */

typedef struct oc_config {
    int32_t device;         /* HIP device ordinal */
    int32_t surf_bins;      /* cut-surface bins per axis; 0 = automatic */
    double donor_bin_scale; /* donor bin edge / mean element extent; 0 = 0.5 */
    int64_t hbm_budget;     /* device bytes the context may hold; 0 = no limit */
    const char *tune_cache; /* tuning file applied at creation (NULL = none): text lines
                               "exact_waves N", "filter_block N", "donor_waves N" and
                               "bin_factor C F" (surfaces of 2^C .. 2^(C+1)-1 faces get
                               F times the automatic bins per axis, F in (0, 1]), as
                               written by the autotuner; '#' starts a comment.  An
                               unreadable file or a bad line is OC_EINVAL. */
} oc_config;

/* Statistics of the last oc_cut / oc_cut_multi call (host copy; the call
 * synchronises the context stream). */
typedef struct oc_cut_info {
    int64_t n_elem;       /* elements classified */
    int64_t n_inbox;      /* elements whose box meets a surface box */
    int64_t n_near;       /* elements with at least one candidate face */
    int64_t n_far;        /* in-box elements without candidates (ray parity) */
    int64_t n_hit;        /* elements intersected by a surface */
    int64_t n_hole;       /* hole elements */
    int64_t n_cand_pairs; /* element x face pairs passing the FP32 box filter */
    int64_t n_side;       /* near elements not intersected: their side comes from the
                             nearest-face search (over 512 of them in one call: one
                             wavefront per element, else an 8-wavefront group each) */
} oc_cut_info;

/* Statistics of the last oc_donor_search call (host copy; synchronises). */
typedef struct oc_donor_info {
    int64_t n_points;  /* points searched */
    int64_t n_newton;  /* Newton solves run (candidates whose box holds the point) */
    int64_t n_iter;    /* Newton iterations run in total */
    int64_t n_orphan;  /* points without a donor */
    int64_t n_overflow;/* points whose candidates did not fit the pair capacity and
                          were solved one candidate at a time in ascending id */
} oc_donor_info;

/* Create / destroy a context on cfg->device (cfg may be NULL: device 0,
 * automatic bins, no budget).  *ctx receives an opaque handle. */
oc_status oc_create(oc_ctx **ctx, const oc_config *cfg);
oc_status oc_destroy(oc_ctx *ctx);
const char *oc_last_error(void);

/* Stream for all later compute calls (a hipStream_t; NULL = default stream). */
oc_status oc_set_stream(oc_ctx *ctx, void *hip_stream);

/* Host or device memory.  The arrays given to the plain (non-slot) calls
 * below -- registration inputs, oc_cut / oc_cut_multi / oc_cut_posed
 * outputs, oc_donor_search and oc_fringe_points inputs and outputs -- may
 * be host or device memory: the pointer's attributes decide (device and
 * managed memory are used in place; anything else is host memory, staged
 * through device memory the context keeps, and the call then synchronises
 * the context stream).  Device inputs are read in the context stream's
 * order.  The slot calls take device memory only. */

/* Register a grid of quadratic 27-node hexahedra (eq. reftophys with K = 2).
 *   nodes     [n_nodes*3] FP64 xyz, host or device
 *   conn      [n_elem*27] int32, lexicographic a+3b+9c over reference nodes
 *             {-1,0,1}^3, host; every id in [0, n_nodes)
 *   face_tags [n_elem*6] int8 OC_FACE_* or NULL (all interior/boundary)
 * Face adjacency is derived from shared corner node ids.  The grid is fixed
 * in its registration frame; motion is given per call by a pose.
 * Errors: OC_EINVAL (sizes, ids), OC_EGEOM (non-positive Jacobian at an
 * element centre), OC_ENOMEM / OC_EBUDGET. */
oc_status oc_register_grid(oc_ctx *ctx, const double *nodes, int64_t n_nodes, const int32_t *conn,
                           int64_t n_elem, const int8_t *face_tags, int32_t *grid_id);

/* Register a closed cutting surface of 9-node quadratic quads (Sec. 4.2:
 * each face is split into 2x2 linear quads of two triangles each, along the
 * diagonal from lattice node (m,n) to (m+1,n+1)).
 *   nodes [n_nodes*3] FP64, conn [n_face*9] int32 (a+3b), host or device,
 *   outward normal = d/dxi x d/deta.
 *   kind  OC_SURF_WALL or OC_SURF_OVERSET
 * Errors: OC_EGEOM if the triangulation is not closed and consistently
 * oriented or encloses a non-positive volume. */
oc_status oc_register_cut_surface(oc_ctx *ctx, const double *nodes, int64_t n_nodes, const int32_t *conn,
                                  int64_t n_face, int32_t kind, int32_t *surf_id);

/* Direct cut of a grid by one posed surface (Sec. 4.2).  iblank_out: int8
 * [n_elem] (host or device) receiving OC_HOLE / OC_FIELD / OC_FRINGE.  An element is a
 * hole if the surface (wall) intersects it -- some element/surface triangle
 * pair closer than OC_TOL_HIT -- or if it lies inside the surface.  Fringe =
 * field element sharing a face with a hole, or carrying an OVERSET face tag
 * (artificial boundary of Sec. 4.2).  iblank_out must be 4-byte aligned. */
oc_status oc_cut(oc_ctx *ctx, int32_t grid_id, int32_t surf_id, const double pose[12], int8_t *iblank_out);

/* Union of holes over n_surf posed surfaces (Sec. 4.2: union over cutting
 * boundaries), then one fringe layer.  poses: n_surf*12 host doubles.
 * n_surf = 0 gives the fringe layer of OVERSET-tagged faces only. */
oc_status oc_cut_multi(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses,
                       int32_t n_surf, int8_t *iblank_out);
/* oc_cut_multi with the grid moving too: grid_pose and poses are world-frame
 * rigid poses (host FP64), and each surface is cut at inverse(grid_pose)
 * after its own pose (R = Rg^T Rs, t = Rg^T ts - Rg^T tg), the rigid-motion
 * composition of Sec. 4.3 done by the library. */
oc_status oc_cut_posed(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *surf_ids,
                       const double *poses, int32_t n_surf, int8_t *iblank_out);

/* Warm-started cut of a moving surface (the per-time-step recut of Sec. 3):
 * prev_iblank (device, not aliasing iblank_out) is this grid's iblank from
 * oc_cut of the same single surface at prev_pose.  Elements whose box grown
 * by the sweep bound (oc_sweep_bound) meets no face box keep their previous
 * hole/field status; all others are recomputed.  The result equals a cold
 * oc_cut at pose. */
oc_status oc_cut_warm(oc_ctx *ctx, int32_t grid_id, int32_t surf_id, const double pose[12], const double prev_pose[12],
                      const int8_t *prev_iblank, int8_t *iblank_out);
/* Largest distance a point of the surface travels from pose_a to pose_b:
 * rotation angle of R_b R_a^T times the largest node radius plus |t_b - t_a|. */
oc_status oc_sweep_bound(oc_ctx *ctx, int32_t surf_id, const double pose_a[12], const double pose_b[12], double *out);

/* The paper's filtered cut (Sec. 4.2; Alg. cp0, bboxdix, cp1, cp2), for
 * comparison with oc_cut_multi: per element whose box meets a surface's box,
 * the nf1 (N_F^1, 1..32) faces of smallest approximate distance (box distance
 * in the element's corner OBB frame plus 1/100 of the centroid distance), of
 * those the nf2 (N_F^2, 1..16, <= nf1) of smallest linear first-pass
 * distance over the three element faces at the corner nearest the face
 * centroid, then the lattice triangles at that corner: a pair closer than
 * 1e-7 is a hit, else the nearest pair's face normal gives the side (the tie
 * rule of the exact cut).  Holes are united over the surfaces, then one
 * fringe layer.  poses: host FP64 [n_surf*12].  Synchronises once per
 * surface; *n_listed (may be NULL) receives the number of (surface,
 * element) pairs examined. */
oc_status oc_cut_filtered(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses, int32_t n_surf,
                          int32_t nf1, int32_t nf2, int8_t *iblank_out, int64_t *n_listed);

/* The cut with the curved faces resolved to level k (Sec. 4.2, the closing
 * paragraph on linearising the curved faces): every surface face is split
 * into k x k quadratic sub-faces (the face map of eq. reftophys on the
 * sub-squares of [-1,1]^2, points on a face edge evaluated from the edge's
 * lower-id node so neighbouring faces share them) and every element whose
 * control-net box meets the refined surface's face boxes into k^3 quadratic
 * sub-elements; each sub-element is cut as an element is by oc_cut, and an
 * element is a hole when one of its sub-elements is.  The triangulations of
 * level k lie within M / (4 k^2) of the curved faces (M bounds the second
 * derivatives of the face map); k = 1 is oc_cut_multi.  Union of holes
 * over the n_surf surfaces, then one fringe layer.  poses: host FP64
 * [n_surf*12]; 1 <= k <= 8; iblank_out device int8 [n_elem], 4-byte
 * aligned.  Synchronises; scratch on the context grows with k^3 times the
 * near elements (81 doubles each).  *n_near (may be NULL) receives the
 * number of (surface, element) items refined. */
oc_status oc_cut_refined(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses, int32_t n_surf,
                         int32_t k, int8_t *iblank_out, int64_t *n_near);

oc_status oc_last_cut_info(oc_ctx *ctx, oc_cut_info *info);

/* Blanking of one time step of a moving grid, with unblanking (Sec. 3,
 * Alg. unblank, steps 3-7).  The grid is cut by its n_surf surfaces (all of
 * one kind) at the poses of time t (poses_t) and of t + dt (poses_tp), host
 * FP64 [n_surf*12] each.  The new holes are, for WALL surfaces, the cells
 * that are holes at t or at t + dt (a cell about to enter the wall is a hole
 * now); for OVERSET surfaces, the cells that are holes at both (a cell is
 * not blanked before it is known to be unneeded).  iblank_out (device int8
 * [n_elem]) receives the new blanking with one fringe layer around its
 * holes and overset-tagged faces fringe.  The cells to unblank -- holes of
 * prev_iblank (the previous step's blanking, device, not aliasing
 * iblank_out) that are not holes of the new one -- are written to
 * unblank_out (device int32 [cap], ascending ids) and counted in
 * *n_unblank (host; synchronises).  OC_ECAPACITY if cap is too small
 * (*n_unblank is set); OC_EINVAL if the surfaces mix kinds.  At most 127
 * surfaces.  Their interior points come from oc_element_points and their
 * donors from oc_donor_search. */
oc_status oc_unblank(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, int32_t n_surf, const double *poses_t,
                     const double *poses_tp, const int8_t *prev_iblank, int8_t *iblank_out, int32_t *unblank_out,
                     int64_t cap, int64_t *n_unblank);
/* Receptor points of listed elements (Alg. unblank step 8: the interior
 * points of the cells to unblank): 27 Gauss-Legendre points per element of
 * elems (device int32 [n], any order), order a+3b+9c, mapped by
 * eq. reftophys and posed by grid_pose, into points_out (device FP64
 * [27*n*3]); src_out (device int32 [27*n], may be NULL) receives each
 * point's element.  An id outside [0, n_elem) yields NaN points and
 * source -1 (the ids are checked on the device, not the host). */
oc_status oc_element_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *elems, int64_t n,
                            double *points_out, int32_t *src_out);

/* Artificial-boundary (AB) faces (Sec. 2, step 1; Sec. 4.2, last
 * paragraph): the faces of kept (field or fringe) elements of iblank (device
 * int8 [n_elem]) whose neighbour across is a hole, and the OVERSET-tagged
 * faces of kept elements (a near-body grid's outer boundary, where the AB
 * method exchanges data).  Each face is named from its kept side, id =
 * 6 e + f with f in the order -xi, +xi, -eta, +eta, -zeta, +zeta; ids are
 * written ascending into faces_out (device int32 [cap]).  *n_out (host)
 * receives their number (synchronises); OC_ECAPACITY if cap is too small. */
oc_status oc_ab_faces(oc_ctx *ctx, int32_t grid_id, const int8_t *iblank, int32_t *faces_out, int64_t cap,
                      int64_t *n_out);
/* Flux points of faces (Sec. 2, step 2: the receptor points of the AB
 * method): m x m points per face id of faces (device int32 [n]).  The face's
 * own reference axis is at -1 (even f) or +1 (odd f); the two other axes, in
 * increasing axis order, take nodes1d[a] and nodes1d[b] (host FP64 [m],
 * 1 <= m <= 8, distinct), point a + m b.  Mapped by eq. reftophys and posed
 * by grid_pose into points_out (device FP64 [n*m*m*3]); src_out (device int32
 * [n*m*m], may be NULL) receives each point's face id.  An id outside
 * [0, 6 n_elem) gives NaN points and source -1. */
oc_status oc_face_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *faces, int64_t n,
                         const double *nodes1d, int32_t m, double *points_out, int32_t *src_out);
/* Interpolation weights (Sec. 2, step 3): for n receptor points with donor
 * ids donors (device int32 [n]) and reference coordinates ref (device FP64
 * [n*3], as oc_donor_search writes them), the m^3 values of the tensor
 * Lagrange basis through nodes1d (host FP64 [m], 1 <= m <= 8, distinct) at
 * the point's reference location, weight a + m b + m^2 c =
 * (l_a(xi) l_b(eta)) l_c(zeta), l_a(s) = prod_{j != a} (s - z_j)/(z_a - z_j)
 * with the factors taken in j order, into weights_out (device FP64
 * [n*m^3]).  Orphans (donor < 0) get NaN weights. */
oc_status oc_interp_weights(oc_ctx *ctx, const int32_t *donors, const double *ref, int64_t n, const double *nodes1d,
                            int32_t m, double *weights_out);

/* One request of a cut batch: grid grid_id cut by n_surf posed surfaces
 * (union of holes, as oc_cut_multi) into its own iblank_out (device int8
 * [n_elem], 4-byte aligned; no two requests of a batch may share one). */
typedef struct oc_cut_req {
    int32_t grid_id;
    int32_t n_surf;
    const int32_t *surf_ids; /* host [n_surf] */
    const double *poses;     /* [n_surf*12]: host memory for oc_cut_batch,
                                device memory (8-byte aligned) for oc_slot_cut_batch */
    int8_t *iblank_out;
} oc_cut_req;

/* Cut a batch of independent requests (Sec. 4.2 applied to many grids and
 * bodies at once).  Every stage of the cut is one launch for the whole
 * batch: face and element launches are flattened over the requests, the
 * exact stages take work items from batch-wide lists, so instances of very
 * different sizes share the device.  Each request's iblank equals what
 * oc_cut_multi gives for it alone.  At most 254 poses per batch (no limit
 * on a slot, oc_slot_cut_batch).
 * oc_last_cut_info then reports totals over the batch. */
oc_status oc_cut_batch(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req);

/* ---------------------------------------------------------- cut service
 * Requests served as they arrive (the serving case of Sec. 5: many grids and
 * bodies, each request one cut of Sec. 4.2).  oc_submit takes one request,
 * copies its surface ids and host poses, and returns a ticket at once; the
 * request is ordered after the work enqueued on the context stream
 * (oc_set_stream) before the call.  It runs on a service slot of its own (a
 * slot sized for it, with its own stream), so requests submitted while
 * others run share the device.  A request is admitted as soon as an idle
 * service slot covers it, or a new one fits within the context's HBM budget
 * and the slot limit (OC_TUNE_SERVICE_SLOTS); idle slots that do not cover
 * it are released to make room, least recently used first.  A request that
 * cannot be admitted yet waits without holding back later requests that
 * can; queued requests are tried in submission order whenever oc_submit,
 * oc_wait or oc_service_info is called.
 *   oc_submit: OC_EINVAL for a bad request or an iblank_out that is the
 *   output of a request not yet waited for; OC_EBUDGET when the request does
 *   not fit in the budget even with every service slot released (no ticket
 *   is issued then).  iblank_out must stay allocated and untouched until
 *   oc_wait has returned for the ticket.
 *   oc_wait: blocks until the request has finished (timeout_ms < 0), or for
 *   at most timeout_ms milliseconds (0 = poll).  OC_OK: iblank_out holds the
 *   result, equal bit for bit to oc_cut_multi's; OC_ETIMEDOUT: not finished
 *   yet, the ticket stays valid; any other status is the request's own
 *   failure.  A ticket is forgotten once oc_wait has returned anything but
 *   OC_ETIMEDOUT (OC_ENOTFOUND after that, and for tickets never issued).
 * One host thread per context: the service is not thread safe.  Queued
 * requests are dropped and service slots released by oc_destroy. */
typedef oc_cut_req oc_request;
oc_status oc_submit(oc_ctx *ctx, const oc_request *req, uint64_t *ticket);
oc_status oc_wait(oc_ctx *ctx, uint64_t ticket, int32_t timeout_ms);

/* Cancel a request of the cut service that has not been admitted yet: it is
 * taken out of the queue, its ticket is forgotten (oc_wait then returns
 * OC_ENOTFOUND) and its iblank_out is left untouched and free for reuse.
 * OC_ESTARTED if the request is already on the device or has finished (its
 * result must be retired with oc_wait), OC_ENOTFOUND for an unknown
 * ticket.  Queued requests behind it are admitted as usual. */
oc_status oc_cancel(oc_ctx *ctx, uint64_t ticket);

typedef struct oc_service_stats {
    int32_t slots;        /* service slots held */
    int32_t running;      /* requests on the device */
    int32_t queued;       /* requests waiting for admission */
    int32_t finished;     /* finished, not yet waited for */
    int32_t peak_running; /* most requests on the device at once so far */
    int32_t pad;
    int64_t slot_bytes;   /* device bytes of the service slots */
} oc_service_stats;
oc_status oc_service_info(oc_ctx *ctx, oc_service_stats *info);

/* Receptor points: 27 Gauss-Legendre points (3x3x3 tensor, order a+3b+9c)
 * per FRINGE element of iblank, in ascending element id, mapped by
 * eq. reftophys and posed by grid_pose into the world frame.
 *   iblank      int8 [n_elem], host or device
 *   points_out  FP64 [cap*3] xyz, host or device
 *   src_out     int32 [cap] source element of each point (may be NULL), host
 *               or device
 *   n_out       host: number of points (27 * fringe elements)
 * Synchronises the stream.  OC_ECAPACITY if cap is too small (n_out is set). */
oc_status oc_fringe_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int8_t *iblank,
                           double *points_out, int64_t cap, int64_t *n_out, int32_t *src_out);

/* Donor search (Sec. 4.3).  points: FP64 [n*3] world frame.  Each
 * point is mapped into the donor grid's registration frame by the inverse
 * of grid_pose, candidates are the elements whose Bernstein control-net box
 * contains it, and Newton iterations from xi = 0 (at most OC_NEWTON_MAXIT,
 * clamped to [-1-OC_NEWTON_CLAMP, 1+OC_NEWTON_CLAMP]) decide containment;
 * the lowest-id containing element is the donor.
 *   donor_out int32 [n]   (-1 = orphan)
 *   ref_out   FP64 [n*3]  reference coordinates (NaN for orphans)
 * points, donor_out and ref_out: host or device. */
oc_status oc_donor_search(oc_ctx *ctx, int32_t donor_grid_id, const double grid_pose[12], const double *points,
                          int64_t n, int32_t *donor_out, double *ref_out);

oc_status oc_last_donor_info(oc_ctx *ctx, oc_donor_info *info);

/* oc_donor_search without any allocation, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight
 * serving loops, hosts that forbid allocation after start-up).  Same
 * arguments, layout, stream (the context's) and results as oc_donor_search
 * (donor ids equal; reference coordinates equal to the last bits unless a
 * point has more candidate boxes than oc_donor_search's pair capacity
 * holds, and always within 1e-10).  Its scratch is one fixed device array
 * of the library (under 48 MiB, one per device, held from the first
 * oc_create on that device until the process ends) sized for at most
 * oc_noalloc_max_points() points: a larger n returns OC_EINVAL (split the
 * points: each is searched on its own).  Every call on a device shares that
 * array and leaves its contents behind; the call writes every part it reads
 * first, so no clearing is needed, but calls that overlap in time on one
 * device (two streams, two contexts, two threads) race and give wrong
 * results: order them.  oc_last_donor_info and oc_timing do not cover this
 * call.  No hipMalloc, hipFree or other allocation is made. */
oc_status oc_donor_search_noalloc(oc_ctx *ctx, int32_t donor_grid_id, const double grid_pose[12],
                                  const double *points, int64_t n, int32_t *donor_out, double *ref_out);
/* the largest n oc_donor_search_noalloc accepts */
oc_status oc_noalloc_max_points(int64_t *n);

/* ------------------------------------------------------------------ slots
 * A slot is the per-request scratch of the compute calls (element lists,
 * posed surface copies and bins, counters) plus the stream they run on.
 * The oc_cut / oc_fringe_points / oc_donor_search calls above use the
 * context's default slot, which grows on demand.  A slot made with
 * oc_slot_create reserves everything up front for the listed grids and
 * surfaces (OC_EBUDGET if the context's HBM budget would be exceeded), its
 * calls never allocate, never synchronise and take poses and point counts in
 * device memory, so several slots can run at once on different streams and a
 * sequence of slot calls can be captured in a HIP graph and replayed.  Calls
 * on one slot must not overlap in time. */
/* points_cap: largest point count of one donor search on this slot */
oc_status oc_slot_create(oc_ctx *ctx, const int32_t *grid_ids, int32_t n_grids, const int32_t *surf_ids,
                         int32_t n_surfs, int64_t points_cap, oc_slot **slot);
/* A slot sized for batches shaped like reqs (grid and surface ids are read;
 * poses and outputs are ignored): any batch whose summed grid elements x
 * surfaces, faces, bins, cuts and requests do not exceed those of reqs. */
oc_status oc_slot_create_batch(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req, int64_t points_cap,
                               oc_slot **slot);
oc_status oc_slot_destroy(oc_slot *slot);
oc_status oc_slot_set_stream(oc_slot *slot, void *hip_stream);
/* device bytes reserved by the slot */
oc_status oc_slot_bytes(oc_slot *slot, int64_t *bytes);
/* oc_cut_multi on a slot; poses_dev: device FP64 [n_surf*12] (8-byte aligned) */
oc_status oc_slot_cut(oc_slot *slot, int32_t grid_id, const int32_t *surf_ids, const double *poses_dev,
                      int32_t n_surf, int8_t *iblank_out);
/* oc_cut_posed on a slot: grid_pose_dev device FP64 [12], poses_dev device
 * FP64 [n_surf*12] (world frame, 8-byte aligned); the composition runs on
 * the slot stream into the slot's pose slots (capturable). */
oc_status oc_slot_cut_posed(oc_slot *slot, int32_t grid_id, const double *grid_pose_dev, const int32_t *surf_ids,
                            const double *poses_dev, int32_t n_surf, int8_t *iblank_out);
/* oc_cut_batch on a slot; every request's poses are in device memory */
oc_status oc_slot_cut_batch(oc_slot *slot, const oc_cut_req *reqs, int32_t n_req);
/* oc_cut_warm on a slot; sweep from oc_sweep_bound for the two poses */
oc_status oc_slot_cut_warm(oc_slot *slot, int32_t grid_id, int32_t surf_id, const double *pose_dev, double sweep,
                           const int8_t *prev_iblank, int8_t *iblank_out);
/* oc_fringe_points on a slot; pose_dev: device FP64 [12]; the number of
 * points (27 per fringe element) is written to the device int32 *n_dev;
 * at most cap points are written. */
oc_status oc_slot_fringe_points(oc_slot *slot, int32_t grid_id, const double *pose_dev, const int8_t *iblank,
                                double *points_out, int64_t cap, int32_t *n_dev, int32_t *src_out);
/* oc_donor_search on a slot for min(*n_dev, cap) points (n_dev may be NULL:
 * cap points); pose_dev: device FP64 [12]. */
oc_status oc_slot_donor_search(oc_slot *slot, int32_t donor_grid_id, const double *pose_dev, const double *points,
                               int64_t cap, const int32_t *n_dev, int32_t *donor_out, double *ref_out);
/* oc_unblank on a slot: poses_dev is device FP64 [2*n_surf*12], the poses
 * of t followed by those of t + dt; the number of cells to unblank goes to
 * the device int32 *n_dev (no synchronisation; at most cap ids written).
 * The overset rule (surfaces of kind OC_SURF_OVERSET) needs a slot that may
 * grow (the context's own), the wall rule none. */
oc_status oc_slot_unblank(oc_slot *slot, int32_t grid_id, const int32_t *surf_ids, int32_t n_surf,
                          const double *poses_dev, const int8_t *prev_iblank, int8_t *iblank_out, int32_t *unblank_out,
                          int64_t cap, int32_t *n_dev);
/* oc_element_points on a slot for the first *n_dev ids of elems (device
 * count); at most cap points written; their number (27 per element) goes
 * to the device int32 *n_points_dev (may be NULL). */
oc_status oc_slot_element_points(oc_slot *slot, int32_t grid_id, const double *pose_dev, const int32_t *elems,
                                 const int32_t *n_dev, int64_t cap, double *points_out, int32_t *n_points_dev,
                                 int32_t *src_out);
/* oc_ab_faces on a slot: at most cap ids written; their number goes to the
 * device int32 *n_dev (no synchronisation). */
oc_status oc_slot_ab_faces(oc_slot *slot, int32_t grid_id, const int8_t *iblank, int32_t *faces_out, int64_t cap,
                           int32_t *n_dev);
/* oc_face_points on a slot for min(*n_faces_dev, faces_cap) faces
 * (n_faces_dev may be NULL: faces_cap); pose_dev: device FP64 [12]; at most
 * cap points written; their number (m*m per face) goes to the device int32
 * *n_points_dev (may be NULL). */
oc_status oc_slot_face_points(oc_slot *slot, int32_t grid_id, const double *pose_dev, const int32_t *faces,
                              const int32_t *n_faces_dev, int64_t faces_cap, const double *nodes1d, int32_t m,
                              double *points_out, int64_t cap, int32_t *n_points_dev, int32_t *src_out);
/* oc_interp_weights on a slot for min(*n_dev, cap) points (n_dev may be
 * NULL: cap points). */
oc_status oc_slot_interp_weights(oc_slot *slot, const int32_t *donors, const double *ref, const int32_t *n_dev,
                                 int64_t cap, const double *nodes1d, int32_t m, double *weights_out);
/* counters of the slot's last cut / donor search (synchronise the slot stream) */
oc_status oc_slot_cut_info(oc_slot *slot, oc_cut_info *info);
oc_status oc_slot_donor_info(oc_slot *slot, oc_donor_info *info);

/* Per-kernel device timing with HIP events recorded on the context stream.
 * oc_timing(ctx, 1) starts collecting (and clears), oc_timing(ctx, 0) stops.
 * oc_timing_report writes a JSON object {"kernel": [total_ms, launches], ...}
 * into buf (synchronises the stream). */
oc_status oc_timing(oc_ctx *ctx, int32_t enable);
oc_status oc_timing_report(oc_ctx *ctx, char *buf, int64_t buf_len);

/* Tuning knobs.  They change speed only, never results.
 *   OC_TUNE_SURF_BINS    arg = surface id; value = cap on its bins per axis
 *                        (1 .. the cap chosen at registration; 0 restores
 *                        that cap).  Coarser bins hold more faces each.
 *                        A slot reserves bins for the caps in force when it
 *                        is created and refuses a later cut needing more
 *                        (OC_EINVAL); lowering a cap never does that.
 *   OC_TUNE_EXACT_WAVES  arg unused; value = wavefronts launched for each of
 *                        the persistent exact-stage kernels (0 = 8192).
 *   OC_TUNE_SERVICE_SLOTS arg unused; value = most slots the cut service
 *                        keeps, hence most requests running at once
 *                        (1 .. 64, 0 = 4).
 *   OC_TUNE_DONOR_WAVES  arg unused; value = most wavefronts launched for
 *                        each donor-search kernel (0 = as many as the
 *                        points and pairs ask for).  A lower cap leaves
 *                        room on the device for work running beside the
 *                        search on another stream.
 *   OC_TUNE_DONOR_PAIRS  arg unused; value = most (point, element) pairs one
 *                        donor search keeps for its batched Newton solves
 *                        (0 = the slot's capacity, 8 per point); the points
 *                        whose pairs fall beyond it are solved one candidate
 *                        at a time in ascending id (same donors).
 *   OC_TUNE_FILTER_BLOCK arg unused; value = threads per block of the
 *                        element-box filter (64, 128, 256, 512 or 1024, four
 *                        elements per thread; 0 = 256).
 *   OC_TUNE_POINT_TILES  arg unused; value = most tiles of the fringe list
 *                        (4096 elements each) for which every block of the
 *                        receptor-point kernel forms the tiles' offsets
 *                        itself from their counts (1 .. 2048, 0 = 2048);
 *                        larger grids take a scan launch for them.
 *   OC_TUNE_SIDE_LIST    arg unused; value = most faces one wavefront of the
 *                        side search lists in its second stage for the tie
 *                        stage (1 .. 64, 0 = 64); an element with more faces
 *                        within its bound walks the bins again (same result).
 *   OC_TUNE_HBM_BUDGET   arg unused; value = the context's HBM budget in
 *                        bytes (0 = none), as oc_config.hbm_budget; later
 *                        allocations are held to it, memory already held is
 *                        kept (registration needs transient room beyond
 *                        what it keeps, so a budget can be set after it).
 * value = -1 changes nothing and returns the value in force (a query).
 * *applied (may be NULL) receives the value in force afterwards. */
enum {
    OC_TUNE_SURF_BINS = 1,
    OC_TUNE_EXACT_WAVES = 2,
    OC_TUNE_SERVICE_SLOTS = 3,
    OC_TUNE_HBM_BUDGET = 4,
    OC_TUNE_DONOR_WAVES = 5,
    OC_TUNE_DONOR_PAIRS = 6,
    OC_TUNE_FILTER_BLOCK = 7,
    OC_TUNE_POINT_TILES = 8,
    OC_TUNE_SIDE_LIST = 9
};
oc_status oc_tune(oc_ctx *ctx, int32_t knob, int32_t arg, int64_t value, int64_t *applied);

/* The check word of a checked build (liboc_checked.so, compiled with
 * OC_CHECKED): its bin walks, pair lists and candidate records validate
 * every index against the array it reads; a violation sets a bit (1 surface
 * bin range, 2 surface record's face, 4 donor bin range, 8 donor record's
 * element, 16 pair's element) and the access is skipped, so the kernels
 * report bad offsets instead of faulting.  Product builds skip the checks
 * and leave the word at zero.  Waits for the device; clear != 0 resets the
 * word; *checked (may be NULL) receives 1 for a checked build. */
oc_status oc_check_word(oc_ctx *ctx, uint32_t *word, int32_t clear, int32_t *checked);

/* Device bytes currently held by the context. */
oc_status oc_memory_used(oc_ctx *ctx, int64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* OC_H */
