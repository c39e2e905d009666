/*
 * FP64 CPU oracle for the AIR reconstruction path (arXiv 1310.1434).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct
 * implementation used to check the GPU library.  Only the test suite, the
 * smoke entry and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header or table with the GPU library.
 *
 * What it computes (paper, Methods, Eqs. (1)-(5) and the split Bregman
 * L2 step of the Methods; Materials for the framelet regulariser):
 *   A          Joseph ray-driven X-ray transform (2D, parallel or flat fan beam)
 *   A^T        its exact transpose, in scatter form
 *   C = k R    per-view Ram-Lak ramp filtration, R symmetric Toeplitz
 *   A'^T = A^T C   the filtered adjoint (Methods, text before Eq. (5))
 *   W, W^T     one-level undecimated piecewise-linear tensor framelet
 *   CG_n       n conjugate-gradient steps on M = A^T C A + mu I
 *   solve      split Bregman for min ||P(AX-Y)||^2 + lambda ||W X||_1
 *              (and the L2 case, Eq. (5))
 * Everything is float64.  All arrays are row-major: images [n][n] (row j,
 * column i), sinograms [n_views][n_bins], framelet coefficients [9][n][n]
 * with band = 3*m_y + m_x.
 *
 * Parity unpinned: the full split-Bregman solve at the benchmark sizes.  The
 * paper prints no intermediate values; it is pinned only through its parts
 * (closed forms, invariants and optimality conditions in the CPU tests).
 */
#ifndef AIR_ORACLE_H
#define AIR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t beam;          /* 0 = parallel, 1 = fan beam, flat detector */
    int32_t n;             /* image n x n */
    double pixel;          /* pixel side, mm */
    int32_t n_views;
    int32_t n_bins;
    const double* cosv;    /* [n_views] view cosines (host) */
    const double* sinv;    /* [n_views] view sines (host) */
    double bin;            /* detector pitch, mm */
    double sod;            /* source to isocentre, mm (fan) */
    double sdd;            /* source to detector, mm (fan) */
    int32_t ramp;          /* filtration C: bits 0-3 window (0 Ram-Lak, 1 Shepp-Logan, 2 Hann),
                              bit 4 symmetric cosine weighting (fan beam) */
} orc_geom;

typedef struct {
    double lambda;         /* framelet weight, or the L2 weight when reg = 1 */
    double mu;             /* Bregman penalty (reg = 0), or the step of Eq. (6) (reg = 2) */
    int32_t n_outer;       /* Bregman (reg = 0) or forward-backward (reg = 2) iterations */
    int32_t n_cg;          /* CG steps per L2 sub-problem */
    int32_t reg;           /* 0 = tensor framelet (split Bregman), 1 = L2, Eq. (5),
                              2 = tensor framelet by forward-backward splitting, Eq. (6) */
    int32_t filter;        /* 1 = AIR (A^T C), 0 = plain IR (A^T) */
} orc_params;

int  orc_num_threads(void);
void orc_set_threads(int n);

/* Per-ray index tables, [n_views * n_bins]: axis 0 = x-driven, 1 = y-driven;
 * lo/hi = first/last driving index with -1 < t < n (brute-force scan), or
 * (0, -1) for a ray that misses the image. */
int orc_tables(const orc_geom* g, int8_t* axis, int32_t* lo, int32_t* hi);

int orc_project(const orc_geom* g, const double* x, double* y);          /* y = A x   */
int orc_backproject(const orc_geom* g, const double* y, double* x);      /* x = A^T y */
void orc_ramp_taps(int32_t n_bins, double* r);                           /* Ram-Lak r[0..n_bins-1] */
int  orc_ramp_taps_kind(int32_t kind, int32_t n_bins, double* r);        /* window `kind` */
int  orc_ramp_weights(const orc_geom* g, double* w);                     /* cosine weights [n_bins] */
int orc_ramp(const orc_geom* g, const double* y, double* yf);            /* yf = C y  */
int orc_filtered_backproject(const orc_geom* g, const double* y, double* x, int32_t filter);
int orc_framelet(int32_t n, const double* x, double* z);                 /* z = W x   */
int orc_framelet_adjoint(int32_t n, const double* z, double* x);         /* x = W^T z */
void orc_shrink(int32_t n, const double* v, double t, double* d);        /* bands 1..8 */
int orc_apply_normal(const orc_geom* g, const double* x, double mu, int32_t filter, double* out);
int orc_cg(const orc_geom* g, const double* rhs, double mu, int32_t filter, int32_t n_iter, double* x);
int orc_solve(const orc_geom* g, const double* y, const orc_params* p, double* x, double* resid,
              double* b_out);

#ifdef __cplusplus
}
#endif
#endif
