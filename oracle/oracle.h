/*
 * Plain FP64 CPU oracle for the overset direct cut and donor search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this code: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP library.
 *
 * Conventions (all arrays row-major, caller-owned):
 *   grid nodes   [n_nodes*3] xyz,  conn [n_elem*27] lexicographic a+3b+9c
 *   surface      [n_snodes*3] xyz, conn [n_face*9] lexicographic a+3b,
 *                outward normal d/dxi x d/deta
 *   pose         12 doubles {R row-major, t}: x' = R x + t
 *   status       0 = hole, 1 = field (per surface, before fringe marking)
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Distance between two triangles (9 doubles each); closest points out. */
double orc_tri_tri(const double *A, const double *B, double *pa, double *pb);
/* Signed solid angle of triangle (a,b,c) seen from p (Van Oosterom-Strackee). */
double orc_solid_angle(const double *p, const double *a, const double *b, const double *c);
/* Quadratic isoparametric map and Jacobian J[i*3+j] = dx_i/dxi_j. */
void orc_q2_eval(const double *X, const double *xi, double *x, double *J);
/* Newton inversion of one element; returns 1 if the point is contained. */
int orc_newton(const double *X, const double *xp, int maxit, double *xi_out, int *iters_out);
/* Face neighbours from shared corner ids: nbr[e*6+f] = element or -1. */
int orc_face_neighbors(const int32_t *conn, int64_t n_elem, int32_t *nbr);
/* Winding number of element e's closed boundary at point p. */
double orc_element_winding(const double *nodes, const int32_t *conn, int64_t e, const double *p);
/* The 48 boundary triangles of element e (48*9 doubles). */
void orc_element_tris(const double *nodes, const int32_t *conn, int64_t e, double *tris);

/* Classify selected elements against one posed surface.
 * sel == NULL means all elements.  brute != 0 disables every acceleration.
 * Outputs (per selected element, any may be NULL):
 *   status  0 hole / 1 field for this surface
 *   hit     1 if the element intersects (or encloses) the surface
 *   dstar   global minimum element-surface distance (0 when hit)
 *   nsign   nearest-face side: +1 outside, -1 inside, 0 when hit
 *   wind    generalised winding number at the element's first node
 *   psign   nearest-face side of the element's first node (0 when hit) */
int orc_cut_surface(const double *gnodes, const int32_t *gconn, int64_t n_elem,
                    const int64_t *sel, int64_t n_sel,
                    const double *snodes, int64_t n_snodes, const int32_t *sconn, int64_t n_face,
                    const double *pose, int kind, int brute, int n_threads,
                    int8_t *status, int8_t *hit, double *dstar, int8_t *nsign, double *wind, int8_t *psign);

/* 27 Gauss points per listed element, mapped and posed (n*27*3 doubles). */
int orc_fringe_points(const double *gnodes, const int32_t *gconn, const int64_t *elems, int64_t n,
                      const double *pose, double *pts);

/* Donor search of world-frame points in a posed grid.  donor -1 = orphan. */
int orc_donor_search(const double *gnodes, const int32_t *gconn, int64_t n_elem, const double *pose,
                     const double *pts, int64_t n, int brute, int maxit, int n_threads,
                     int32_t *donor, double *xi, int32_t *iters, int32_t *n_cand);

/* The paper's filtered cut (Sec. 4.2; Alg. cp0, bboxdix, cp1, cp2): per
 * element near the surface's box, the nf1 faces of smallest approximate
 * distance, the nf2 of those with the smallest linear first-pass distance,
 * then the lattice triangles at the kept corner; hit if any pair is closer
 * than 1e-7, else the side of the nearest pair's face normal.  status: 0
 * hole, 1 field; hit (may be NULL): 1 where a second-pass pair hit. */
int orc_cut_heuristic(const double *gnodes, const int32_t *gconn, int64_t n_elem, const double *snodes,
                      int64_t n_snodes, const int32_t *sconn, int64_t n_face, const double *pose, int kind, int nf1,
                      int nf2, int n_threads, int8_t *status, int8_t *hit);
/* element OBB of Alg. cp0: centroid[3], axes R[9] (rows), extents[6] */
void orc_hx_obb(const double *X, double *obb);
/* Alg. bboxdix */
double orc_hx_bbox_dist(const double *B1, const double *B2);
/* the two kept lists of the filtered cut for one element X (27 x 3) */
int orc_hx_lists(const double *X, const double *snodes, const int32_t *sconn, int64_t n_face, const double *pose,
                 int nf1, int nf2, int64_t *l1, double *d1, int64_t *l2, double *d2, int32_t *c2);

#ifdef __cplusplus
}
#endif

#endif
