/*
 * FP64 CPU oracle of the differentiable edge-sampling path tracer.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. The product path never links it.
 * It shares no code with the HIP implementation: it has its own Philox, its
 * own intersection code and BVH, its own edge hierarchy and a tape-based
 * reverse-mode differentiator for the interior term.
 *
 * What it computes (thesis Ch. 5, Method): for a triangle scene, a pinhole
 * camera, a seed and a sample count, the Monte Carlo image estimate of the
 * pixel integral (eq. first, eq. gradient_monte_carlo, box pixel filter) and
 * the gradient sum_p dL/dI_p * dI_p/dPhi, split by the product rule
 * (eq. redner_product_rule) into
 *   - the interior term: reverse mode through each sample with its
 *     integration variables held fixed,
 *   - the primary boundary term: screen-space edge samples (eq. mc), and
 *   - the secondary boundary term: direction-space edge samples at every path
 *     vertex (Secondary visibility; eq. dirac_3d_edge rewritten in the
 *     direction measure), with edges drawn from the edge hierarchy
 *     (Importance Sampling the Edges, Edge selection).
 */
#ifndef DIFFRT_ORACLE_H
#define DIFFRT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t num_vertices, num_triangles;
    const float*   vertices;      /* [V][3] */
    const int32_t* indices;       /* [T][3] */
    const float*   albedo;        /* [T] */
    const float*   emission;      /* [T] */
    const float*   normals;       /* [V][3] or NULL (flat shading) */
    int32_t emission_two_sided;
    float   background;
    const double* vertices64;     /* [V][3] or NULL: FP64 override (finite-difference pins) */
    const double* albedo64;       /* [T] or NULL: FP64 override */
} orc_scene;

typedef struct {
    float position[3], look_at[3], up[3];
    float fov_y_deg, near_clip;
    int32_t width, height;
    int32_t win_x0, win_y0, win_x1, win_y1;   /* pixel window [x0,x1) x [y0,y1) */
    const double* params64;       /* [9] or NULL: FP64 override of position, look_at, up */
} orc_camera;

typedef struct {
    int32_t  spp, max_depth;
    uint64_t seed;
    uint32_t view_id;
    int32_t  interior, primary_edges, secondary_edges;   /* term switches (1 = on) */
    int32_t  use_bvh;            /* 0 = brute-force intersection */
    int32_t  exclude_flagged;    /* 1 = drop units with near-tie decisions */
    int32_t  num_threads;        /* <= 0: one */
    const uint8_t* unit_mask;    /* [M] or NULL; 0 = unit skipped */
    /* Direction record/replay for finite-difference pins of the interior term:
     * 1 = record the main path's sampled world directions and solid-angle
     * factors into dir_log, 2 = replay them instead of sampling. [M][64]. */
    int32_t dir_mode;
    double* dir_log;
    /* Proposal mixture: edge_pdf[E] is a distribution over all edges (edge ids
     * as orc_edges numbers them); an edge is drawn from it with probability
     * mix and from the plain sampler otherwise, and every sample is weighted
     * by the mixture pdf. mix_terms: bit 0 = primary edges, bit 1 = secondary
     * edges. mix = 0 or edge_pdf = NULL: plain sampling. */
    const double* edge_pdf;
    double  mix;
    int32_t mix_terms;
    /* Geometry buffer instead of radiance (0 = radiance): the value of one
     * channel at the first camera hit, 0 on a miss: 1-3 world position x/y/z,
     * 4-6 shading normal x/y/z (facing the ray), 7 albedo. Gradients: interior
     * term of that value and the primary boundary term (no secondary term). */
    int32_t aov;
    /* Point on a secondary edge: 0 = uniform in the edge parameter t, 1 = in
     * proportion to the clamped cosine with the shading normal in the
     * arc-length measure of its direction (closed-form inverse). */
    int32_t edge_t_mode;
    /* Secondary edge selection: 0 or 1 = one descent of the hierarchy, its
     * pdf in the weight; M in 2..64 = M samples distributed down the
     * hierarchy in proportion to importance, one of the leaves reached kept
     * by weighted reservoir sampling (weight W / (M imp) in place of 1/pdf).
     * Not with a secondary proposal mixture. */
    int32_t edge_candidates;
    /* Next event estimation for edges: with probability enee (in [0, 1); 0 =
     * off) the secondary edge sample comes from the billboard strategy (a
     * light point, the billboards the segment to it crosses, one chosen by
     * importance), otherwise from the hierarchy; every sample is weighted by
     * the mixture density. enee_width: billboard width (0 = 2% of the mean
     * absolute deviation of the vertex positions, L2 over the coordinates).
     * Uniform edge points, one descent, no secondary proposal mixture. */
    double  enee;
    double  enee_width;
} orc_options;

typedef struct {
    double* image;               /* [Hw][Ww] or NULL */
    const double* d_image;       /* [Hw][Ww]; NULL = no gradients */
    double* d_vertices;          /* [V][3] */
    double* d_albedo;            /* [T] */
    double* d_camera;            /* [9]: position, look_at, up */
    double* mass_vertices;       /* [V][3] rounding scale: sum of |per-sample contribution| (boundary samples
                                    scaled by (|f+| + |f-|) / |f+ - f-|), or NULL */
    double* mass_albedo;         /* [T] or NULL */
    double* mass_camera;         /* [9] or NULL */
    uint8_t* unit_flags;         /* [M] or NULL: 1 = a decision was within rounding of a tie */
    int64_t* stats;              /* [8] or NULL: rays, flagged units, edge samples used, ... */
    double* edge_stats;          /* [E] or NULL: per edge, sum over its boundary samples (primary and
                                    secondary) of P * |c|^2, P the probability with which the edge was
                                    drawn, c the sample's contribution to the edge's two endpoints */
    double* edge_stats_mass;     /* [E] or NULL: the same sum with each term scaled by its contribution's
                                    rounding scale (as in the mass arrays) */
} orc_outputs;

/* Error codes (0 = ok). */
enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENONMANIFOLD = 2, ORC_EDEPTH = 3 };

int  orc_render(const orc_scene* s, const orc_camera* c, const orc_options* o, orc_outputs* out);

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Diagnostic counters of near-tie flags by reason (see oracle.cpp). */
void orc_tie_reasons(int64_t out[24], int32_t reset);

/* Unique undirected edges: rows (va, vb, f0, f1), va < vb, f1 = -1 on a boundary. */
int  orc_edges(const orc_scene* s, int32_t* num_edges, int32_t* rows /* [E][4] or NULL */);

/* Closest hit for n rays (origin, direction, tmin, tmax). tri = -1 on a miss. */
int  orc_closest_hit(const orc_scene* s, int32_t n, const double* o, const double* d,
                     double tmin, double tmax, int32_t use_bvh, int32_t* tri, double* t);

/* Edge hierarchy for camera c: full distribution of the sampled edge at shading
 * point p with normal n. pdf[E] (0 for edges never reached) and the probability
 * that the descent ends at a node whose children both have zero importance. */
int  orc_edge_tree_pdf(const orc_scene* s, const orc_camera* c, const double p[3],
                       const double n[3], double* pdf, double* p_fail);

/* Probability that one descent ends at each of the given edges (the product of
 * branch probabilities along each edge's root-to-leaf path). */
int  orc_edge_tree_pdf_of(const orc_scene* s, const orc_camera* c, const double p[3],
                          const double n[3], int32_t count, const int32_t* edges, double* pdf);
/* Stratified multi-sample descent with reservoir selection from (p, n):
 * count draws, draw i taking its uniforms from u[i*ustride ...] in order (one
 * per split, one per leaf reached); edge[i] = kept edge or -1, weight[i] =
 * W / (M imp) of the kept edge (0 when none). ORC_EINVAL if a draw needs
 * more than ustride uniforms. */
int  orc_edge_tree_select(const orc_scene* s, const orc_camera* c, const double p[3], const double n[3],
                          int32_t M, int32_t count, const double* u, int32_t ustride, int32_t* edge,
                          double* weight);
/* One descent per row of u (u[i][0] = root uniform, u[i][1..64] = level uniforms). */
int  orc_edge_tree_sample(const orc_scene* s, const orc_camera* c, const double p[3],
                          const double n[3], int32_t count, const double* u,
                          int32_t* edge, double* pdf);

/* The clamped-cosine edge-point sampler for one shading point (p, n) and edge
 * (v0, v1): t[i] and its density pdf_t[i] for each uniform u[i] (t = -1,
 * pdf_t = 0 when there is no sample), and the density at a given t. */
int    orc_edge_t_cosine(const double p[3], const double n[3], const double v0[3], const double v1[3], int32_t count,
                         const double* u, double* t, double* pdf_t);
double orc_edge_t_cosine_pdf(const double p[3], const double n[3], const double v0[3], const double v1[3], double t);

/* Next event estimation for edges at shading point p (normal n, on triangle
 * tri or -1), billboards of full width `width`:
 *  - the default width of the scene;
 *  - count draws of the billboard strategy alone, draw i from Philox stream
 *    (i, 0, 32; seed): edge (-1: none), strip coordinates (t, s), and 1 in
 *    flags[i] (may be NULL) when a decision was within rounding of a tie;
 *  - its density in dt ds at given (edge, t, s);
 *  - count draws of the mixture with the hierarchy of camera c (probability
 *    alpha for the billboards; streams (i, 0, 2) and (i, 0, 33); seed): edge
 *    (-1: none), t and the mixture density in (e, t). */
double orc_edge_nee_width(const orc_scene* s);
int    orc_edge_nee_sample(const orc_scene* s, const double p[3], const double n[3], int32_t tri, double width,
                           int32_t count, uint64_t seed, int32_t* edge, double* t, double* sv, uint8_t* flags);
int    orc_edge_nee_pdf(const orc_scene* s, const double p[3], const double n[3], int32_t tri, double width,
                        int32_t count, const int32_t* edge, const double* t, const double* sv, double* pdf);
int    orc_edge_nee_mix_sample(const orc_scene* s, const orc_camera* c, const double p[3], const double n[3],
                               int32_t tri, double width, double alpha, int32_t count, uint64_t seed,
                               int32_t* edge, double* t, double* pdf);

/* Secondary boundary factor in both measures for one edge point (for the
 * identity test between the thesis's area form and the direction form).
 * Inputs: shading point p, edge v0 v1, parameter t, and a plane (point m0,
 * normal nm) behind the edge standing for the surface the edge projects onto.
 * Outputs (each a 9-vector: d/dv0, d/dv1, d/dp):
 *   area_form: grad_alpha / |grad_m alpha| * |J_m| / |n_m x n_h| (eq. dirac_3d_edge,
 *              eq. alpha_3d with m held fixed, J_m from the appendix derivation),
 *   dir_form : grad_beta / |v0' x v1'| * |e x w^| / |w| (direction measure). */
void orc_secondary_forms(const double p[3], const double v0[3], const double v1[3], double t,
                         const double m0[3], const double nm[3],
                         double area_form[9], double dir_form[9]);

#ifdef __cplusplus
}
#endif
#endif
