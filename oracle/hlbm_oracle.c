/*
 * hlbm_oracle.c -- plain, slow FP64 CPU reference of one HLBM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no source, table or helper with the HIP
 * library: its velocity ordering, storage order (f[cell][i], push streaming,
 * separate collide and stream passes) and every formula are written here from
 * the paper (Marquardt, Hafen, Krause, arXiv 2312.14172, Sec. 3).
 *
 * Conventions (lattice units, Sec. 3.1):
 *   cell (x,y,z) has centre (x+1/2, y+1/2, z+1/2) and index x + nx*(y + ny*z);
 *   bc[k] = 0 periodic, 1 half-way bounce-back walls at 0 and n_k;
 *   f is the post-streaming state at integer time t.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* ---------------------------------------------------------------------------
 * D3Q19 velocity set and weights (Sec. 3.1, velocity-set and weight equations).
 * This file's own order: rest; +x,+y,+z,-x,-y,-z; then the twelve diagonals.
 * ------------------------------------------------------------------------- */
static const int C[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {-1, 0, 0},  {0, -1, 0}, {0, 0, -1},
    {1, 1, 0},  {1, -1, 0}, {1, 0, 1},  {1, 0, -1},  {0, 1, 1},  {0, 1, -1},
    {-1, -1, 0}, {-1, 1, 0}, {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1}};

static double W[Q];
static int OPP[Q];
static int tables_ready = 0;

static void init_tables(void) {
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        int c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
        /* weights: 1/3 rest, 1/18 axis, 1/36 diagonal */
        W[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        OPP[i] = -1;
        for (int j = 0; j < Q; ++j)
            if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2]) OPP[i] = j;
    }
    tables_ready = 1;
}

void orc_tables(int *c, double *w, int *opp) {
    init_tables();
    for (int i = 0; i < Q; ++i) {
        for (int k = 0; k < 3; ++k) c[3 * i + k] = C[i][k];
        w[i] = W[i];
        opp[i] = OPP[i];
    }
}

/* ---------------------------------------------------------------------------
 * Configuration and particle records (this file's own declarations).
 * ------------------------------------------------------------------------- */
typedef struct {
    int n[3];
    int bc[3];
    double tau;      /* relaxation time, tau = 3 nu + 1/2 (relaxation eq.) */
    double eps;      /* smooth-boundary width of the indicator, 1/2 in the paper */
    double rho_f;    /* fluid density used in the buoyancy term */
    double g[3];     /* gravity vector */
    double af[3];    /* fluid body acceleration (Poiseuille / sphere-array drag) */
    int coupling;    /* 0: HLBM (EDM source), 1: partially saturated method */
} ocfg;

enum { SH_SPHERE = 0, SH_ROUNDED_CUBE = 1, SH_SPHEROID = 2, SH_MESH = 3 };

typedef struct {
    double X[3];   /* centre of mass */
    double q[4];   /* unit quaternion (w,x,y,z), body -> world */
    double U[3];   /* translational velocity */
    double W[3];   /* angular velocity, world frame */
    double m;      /* mass; <= 0 holds the particle fixed */
    double V;      /* volume (buoyancy) */
    double I[3];   /* principal moments of inertia, body frame */
    double prm[3]; /* shape parameters */
    int32_t shape;
    int32_t flags;
} opart;

/* ---------------------------------------------------------------------------
 * Equilibrium (Sec. 3.1, Maxwell-Boltzmann equation), c_s^2 = 1/3.
 * ------------------------------------------------------------------------- */
void orc_feq(double rho, const double *u, double *feq) {
    init_tables();
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
        feq[i] = W[i] * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* ---------------------------------------------------------------------------
 * Signed distance functions, negative inside (Sec. 3.2, indicator paragraph).
 * p is in the particle's body frame.
 * reading: the paper's experiments use spheres only; the rounded cube and the
 * spheroid use the exact Euclidean distance.
 * ------------------------------------------------------------------------- */

/* Distance from (y0,y1), y0,y1 >= 0, to the ellipse (u/e0)^2 + (v/e1)^2 = 1
 * with e0 >= e1.  Unsigned.  The nearest point satisfies x_k = e_k^2 y_k /
 * (t + e_k^2) for the root t of G(t) = sum_k (e_k y_k/(t+e_k^2))^2 - 1, which
 * is bracketed by [e1 y1 - e1^2, |(e0 y0, e1 y1)| - e1^2] and found by plain
 * bisection. */
static double ellipse_dist_sorted(double e0, double e1, double y0, double y1) {
    if (y1 > 0.0) {
        if (y0 > 0.0) {
            double lo = e1 * y1 - e1 * e1;
            double hi = sqrt(e0 * e0 * y0 * y0 + e1 * e1 * y1 * y1) - e1 * e1;
            for (int it = 0; it < 400; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double a0 = e0 * y0 / (mid + e0 * e0);
                double a1 = e1 * y1 / (mid + e1 * e1);
                double G = a0 * a0 + a1 * a1 - 1.0;
                if (G > 0.0) lo = mid; else hi = mid;
            }
            double t = 0.5 * (lo + hi);
            double x0 = e0 * e0 * y0 / (t + e0 * e0);
            double x1 = e1 * e1 * y1 / (t + e1 * e1);
            return sqrt((x0 - y0) * (x0 - y0) + (x1 - y1) * (x1 - y1));
        }
        return fabs(y1 - e1); /* on the minor axis */
    }
    /* on the major axis */
    double num = e0 * e0 - e1 * e1;
    if (e0 * y0 < num) {
        double x0 = e0 * e0 * y0 / num;
        double r = x0 / e0;
        double x1 = e1 * sqrt(fmax(0.0, 1.0 - r * r));
        return sqrt((x0 - y0) * (x0 - y0) + x1 * x1);
    }
    return fabs(y0 - e0);
}

static double sdf_spheroid(double a, double b, const double *p) {
    /* symmetry axis = body x, semi-axis a; the other two semi-axes are b */
    double y0 = fabs(p[0]);
    double y1 = sqrt(p[1] * p[1] + p[2] * p[2]);
    double inside = (y0 / a) * (y0 / a) + (y1 / b) * (y1 / b) - 1.0;
    double d = (a >= b) ? ellipse_dist_sorted(a, b, y0, y1) : ellipse_dist_sorted(b, a, y1, y0);
    return inside <= 0.0 ? -d : d;
}

static double sdf_rounded_cube(double h, double rc, const double *p) {
    /* Minkowski sum of a cube with half-extent h - rc and a ball of radius rc */
    double core = h - rc;
    double qx = fabs(p[0]) - core, qy = fabs(p[1]) - core, qz = fabs(p[2]) - core;
    double ox = fmax(qx, 0.0), oy = fmax(qy, 0.0), oz = fmax(qz, 0.0);
    double outside = sqrt(ox * ox + oy * oy + oz * oz);
    double inside = fmin(fmax(qx, fmax(qy, qz)), 0.0);
    return outside + inside - rc;
}

/* Closed triangle mesh (one per run), vertices in the body frame at unit
 * scale, triangles counter-clockwise seen from outside: g_mesh[t][v][k]. */
static double *g_mesh = NULL;
static int g_mesh_nt = 0;

void orc_set_mesh(const double *tri, int nt) {
    free(g_mesh);
    g_mesh = (double *)malloc(sizeof(double) * 9 * (size_t)(nt > 0 ? nt : 1));
    memcpy(g_mesh, tri, sizeof(double) * 9 * (size_t)nt);
    g_mesh_nt = nt;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* squared distance from q to the segment [a, b] */
static double seg_dist2(const double *q, const double *a, const double *b) {
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, aq[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
    double t = dot3(aq, ab) / dot3(ab, ab);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    double d[3] = {aq[0] - t * ab[0], aq[1] - t * ab[1], aq[2] - t * ab[2]};
    return dot3(d, d);
}

/* squared distance from q to the triangle (a, b, c): the foot of the
 * perpendicular onto the plane if its barycentric coordinates are all
 * non-negative, else the nearest of the three edges */
static double tri_dist2(const double *q, const double *a, const double *b, const double *c) {
    double e0[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e1[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]};
    double aq[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
    double nn = dot3(n, n);
    double h = dot3(aq, n) / nn;
    double f[3] = {aq[0] - h * n[0], aq[1] - h * n[1], aq[2] - h * n[2]}; /* foot - a */
    /* barycentric coordinates of the foot: f = u e0 + v e1 */
    double d00 = dot3(e0, e0), d01 = dot3(e0, e1), d11 = dot3(e1, e1);
    double f0 = dot3(f, e0), f1 = dot3(f, e1);
    double den = d00 * d11 - d01 * d01;
    double u = (d11 * f0 - d01 * f1) / den, v = (d00 * f1 - d01 * f0) / den;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) return h * h * nn;
    double d = seg_dist2(q, a, b);
    d = fmin(d, seg_dist2(q, b, c));
    return fmin(d, seg_dist2(q, c, a));
}

/* solid angle of the triangle seen from q (Van Oosterom and Strackee 1983) */
static double tri_solid_angle(const double *q, const double *a, const double *b, const double *c) {
    double A[3] = {a[0] - q[0], a[1] - q[1], a[2] - q[2]};
    double B[3] = {b[0] - q[0], b[1] - q[1], b[2] - q[2]};
    double Cc[3] = {c[0] - q[0], c[1] - q[1], c[2] - q[2]};
    double la = sqrt(dot3(A, A)), lb = sqrt(dot3(B, B)), lc = sqrt(dot3(Cc, Cc));
    double bxc[3] = {B[1] * Cc[2] - B[2] * Cc[1], B[2] * Cc[0] - B[0] * Cc[2], B[0] * Cc[1] - B[1] * Cc[0]};
    double num = dot3(A, bxc);
    double den = la * lb * lc + dot3(A, B) * lc + dot3(A, Cc) * lb + dot3(B, Cc) * la;
    return 2.0 * atan2(num, den);
}

/* Mesh at scale s: unsigned distance = the least distance to a triangle;
 * inside where the generalised winding number (summed solid angles / 4 pi)
 * exceeds 1/2. */
static double sdf_mesh(double s, const double *p) {
    double q[3] = {p[0] / s, p[1] / s, p[2] / s};
    double d2 = 1e300, omega = 0.0;
    for (int t = 0; t < g_mesh_nt; ++t) {
        const double *a = g_mesh + 9 * t, *b = a + 3, *c = a + 6;
        d2 = fmin(d2, tri_dist2(q, a, b, c));
        omega += tri_solid_angle(q, a, b, c);
    }
    double d = s * sqrt(d2);
    return omega > 2.0 * M_PI ? -d : d;
}

double orc_sdf(int shape, const double *prm, const double *p) {
    switch (shape) {
    case SH_SPHERE: return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - prm[0];
    case SH_ROUNDED_CUBE: return sdf_rounded_cube(prm[0], prm[1], p);
    case SH_SPHEROID: return sdf_spheroid(prm[0], prm[1], p);
    case SH_MESH: return sdf_mesh(prm[0], p);
    default: return 1e300;
    }
}

/* Largest distance of the surface from the centre of mass (for a mesh the
 * caller stores it in prm[1]: scale times the largest vertex radius). */
double orc_circumradius(int shape, const double *prm) {
    switch (shape) {
    case SH_SPHERE: return prm[0];
    case SH_ROUNDED_CUBE: return sqrt(3.0) * (prm[0] - prm[1]) + prm[1];
    case SH_SPHEROID: return fmax(prm[0], prm[1]);
    case SH_MESH: return prm[1];
    default: return 0.0;
    }
}

/* Trigonometric indicator B(d_s) (Sec. 3.2, level-set equation).
 * reading: the printed cosine argument has an unbalanced parenthesis; it is
 * read as cos^2( (pi/2) (d/eps + 1/2) ), which is continuous with the outer
 * pieces (1 at d = -eps/2, 0 at d = +eps/2). */
double orc_indicator(double d, double eps) {
    if (d <= -0.5 * eps) return 1.0;
    if (d >= 0.5 * eps) return 0.0;
    double c = cos(0.5 * M_PI * (d / eps + 0.5));
    return c * c;
}

/* ---------------------------------------------------------------------------
 * Geometry helpers
 * ------------------------------------------------------------------------- */
static void quat_to_rot(const double *q, double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* Separation of cell centre from the particle centre, minimum image on
 * periodic axes (reading: torque lever arm and u_p(x) use it). */
static void cell_offset(const ocfg *cfg, const opart *P, int ix, int iy, int iz, double *d) {
    int idx[3] = {ix, iy, iz};
    for (int k = 0; k < 3; ++k) {
        double v = (idx[k] + 0.5) - P->X[k];
        if (cfg->bc[k] == 0) v -= cfg->n[k] * nearbyint(v / cfg->n[k]);
        d[k] = v;
    }
}

static double particle_sdf_at(const opart *P, const double *d) {
    double R[3][3], pb[3];
    quat_to_rot(P->q, R);
    for (int k = 0; k < 3; ++k) pb[k] = R[0][k] * d[0] + R[1][k] * d[1] + R[2][k] * d[2];
    return orc_sdf(P->shape, P->prm, pb);
}

/* rigid-body velocity at offset d (Sec. 3.2, below the velocity-difference eq.) */
static void rigid_velocity(const opart *P, const double *d, double *u) {
    u[0] = P->U[0] + P->W[1] * d[2] - P->W[2] * d[1];
    u[1] = P->U[1] + P->W[2] * d[0] - P->W[0] * d[2];
    u[2] = P->U[2] + P->W[0] * d[1] - P->W[1] * d[0];
}

static long cell_index(const ocfg *cfg, int x, int y, int z) {
    return (long)x + (long)cfg->n[0] * ((long)y + (long)cfg->n[1] * z);
}

/* Map an integer coordinate onto the lattice; returns 0 if it lies past a wall. */
static int wrap_coord(const ocfg *cfg, int k, int v, int *out) {
    int n = cfg->n[k];
    if (v >= 0 && v < n) { *out = v; return 1; }
    if (cfg->bc[k] != 0) return 0;
    *out = ((v % n) + n) % n;
    return 1;
}

/* Cells whose centre lies within `reach` of the particle centre along each
 * axis, as an integer range [lo, hi]; wrapped later. */
static void cell_range(const opart *P, int k, double reach, int *lo, int *hi) {
    *lo = (int)ceil(P->X[k] - reach - 0.5);
    *hi = (int)floor(P->X[k] + reach - 0.5);
}

/* ---------------------------------------------------------------------------
 * Lattice-wide passes
 * ------------------------------------------------------------------------- */
long orc_ncells(const ocfg *cfg) { return (long)cfg->n[0] * cfg->n[1] * cfg->n[2]; }

/* f = f^eq(rho, u) at every cell; rho, u may be NULL for rest (rho=1, u=0). */
void orc_equilibrium_field(const ocfg *cfg, const double *rho, const double *u, double *f) {
    init_tables();
    long N = orc_ncells(cfg);
    for (long x = 0; x < N; ++x) {
        double uu[3] = {0, 0, 0}, r = 1.0;
        if (rho) r = rho[x];
        if (u) { uu[0] = u[x]; uu[1] = u[N + x]; uu[2] = u[2 * N + x]; }
        orc_feq(r, uu, f + Q * x);
    }
}

/* Bare moments (Sec. 3.1): rho = sum f_i, rho u = sum c_i f_i.  u is three planes. */
void orc_moments(const ocfg *cfg, const double *f, double *rho, double *u) {
    long N = orc_ncells(cfg);
#pragma omp parallel for schedule(static) if (N >= 4096)
    for (long x = 0; x < N; ++x) {
        double r = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
            r += f[Q * x + i];
            for (int k = 0; k < 3; ++k) j[k] += C[i][k] * f[Q * x + i];
        }
        rho[x] = r;
        for (int k = 0; k < 3; ++k) u[k * N + x] = j[k] / r;
    }
}

/* Collision with EDM source at one cell (collide, BGK and EDM equations):
 *   rho, u from f;  du = B (u_s - u) + (1 - B) a_f;
 *   f*_i = f_i - (f_i - feq_i(rho,u))/tau + feq_i(rho,u+du) - feq_i(rho,u).
 * reading: the fluid velocity entering du and feq is the bare moment of the
 * pre-collision populations; a_f is a body acceleration applied through the
 * same exact-difference source outside the solid. */
void orc_collide_cell(const ocfg *cfg, const double *f, double B, const double *us, double *fs) {
    init_tables();
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int k = 0; k < 3; ++k) j[k] += C[i][k] * f[i];
    }
    double u[3], du[3], ud[3];
    for (int k = 0; k < 3; ++k) u[k] = j[k] / rho;
    for (int k = 0; k < 3; ++k) {
        du[k] = B * (us[k] - u[k]) + (1.0 - B) * cfg->af[k];
        ud[k] = u[k] + du[k];
    }
    double feq[Q], feqd[Q];
    orc_feq(rho, u, feq);
    orc_feq(rho, ud, feqd);
    for (int i = 0; i < Q; ++i) {
        double omega = -(f[i] - feq[i]) / cfg->tau;
        double S = feqd[i] - feq[i];
        fs[i] = f[i] + omega + S;
    }
}

/* Weight of the solid collision in the partially saturated method (Noble and
 * Torczynski 1998, whose family of methods Sec. 3.2 names as a possible host
 * of the decomposition): B_n = B (tau - 1/2) / ((1 - B) + (tau - 1/2)), with
 * the solid fraction B of the cell. */
double orc_psm_weight(double B, double tau) {
    return B * (tau - 0.5) / ((1.0 - B) + (tau - 0.5));
}

/* Partially saturated collision at one cell:
 *   rho, u from f;  B_n = orc_psm_weight(B, tau);
 *   Omega^s_i = f_opp(i) - feq_opp(i)(rho, u) + feq_i(rho, u_s) - f_i
 *   f*_i = f_i - (1 - B_n)(f_i - feq_i(rho, u))/tau + B_n Omega^s_i
 *          + (1 - B_n) (feq_i(rho, u + a_f) - feq_i(rho, u)).
 * reading: the solid fraction and solid velocity are those of the HLBM
 * coupling (B = min(1, sum B_p), u_s the B-weighted particle velocity); a
 * fluid body acceleration a_f acts on the fluid part through the
 * exact-difference source. */
void orc_collide_cell_psm(const ocfg *cfg, const double *f, double B, const double *us, double *fs) {
    init_tables();
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int k = 0; k < 3; ++k) j[k] += C[i][k] * f[i];
    }
    double u[3], ua[3];
    for (int k = 0; k < 3; ++k) {
        u[k] = j[k] / rho;
        ua[k] = u[k] + cfg->af[k];
    }
    double feq[Q], feqs[Q], feqa[Q];
    orc_feq(rho, u, feq);
    orc_feq(rho, us, feqs);
    orc_feq(rho, ua, feqa);
    const double Bn = orc_psm_weight(B, cfg->tau);
    for (int i = 0; i < Q; ++i) {
        const int o = OPP[i];
        const double omega_s = f[o] - feq[o] + feqs[i] - f[i];
        fs[i] = f[i] - (1.0 - Bn) * (f[i] - feq[i]) / cfg->tau + Bn * omega_s + (1.0 - Bn) * (feqa[i] - feq[i]);
    }
}

void orc_collide(const ocfg *cfg, const double *f, const double *B, const double *us, double *fs) {
    long N = orc_ncells(cfg);
#pragma omp parallel for schedule(static) if (N >= 4096)
    for (long x = 0; x < N; ++x) {
        double uu[3] = {us[x], us[N + x], us[2 * N + x]};
        if (cfg->coupling == 1)
            orc_collide_cell_psm(cfg, f + Q * x, B[x], uu, fs + Q * x);
        else
            orc_collide_cell(cfg, f + Q * x, B[x], uu, fs + Q * x);
    }
}

/* Streaming f_i(x + c_i, t+1) = f*_i(x, t) (stream equation), push form.
 * reading: a population whose target lies past a wall returns to its own cell
 * in the opposite direction (half-way bounce-back for resting walls). */
void orc_stream(const ocfg *cfg, const double *fs, double *fn) {
    init_tables();
    int nx = cfg->n[0], ny = cfg->n[1], nz = cfg->n[2];
    long N = orc_ncells(cfg);
#pragma omp parallel for schedule(static) if (N >= 4096)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long s = cell_index(cfg, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    int t[3], ok = 1;
                    int v[3] = {x + C[i][0], y + C[i][1], z + C[i][2]};
                    for (int k = 0; k < 3; ++k) ok &= wrap_coord(cfg, k, v[k], &t[k]);
                    if (ok) fn[Q * cell_index(cfg, t[0], t[1], t[2]) + i] = fs[Q * s + i];
                    else fn[Q * s + OPP[i]] = fs[Q * s + i];
                }
            }
}

/* ---------------------------------------------------------------------------
 * Fluid -> particle: momentum exchange (Sec. 3.2, MEA, force and torque eqs.)
 *   F_h(x) = sum_i (c_i - u_p(x)) f_i(x + c_i, t) + (c_i + u_p(x)) f_ibar(x, t)
 * summed over the cells whose centre is inside the particle (d_s <= 0).
 * reading: as printed, F_h is the momentum handed to the fluid; the force on
 * the particle is its negative.  The sum over i covers both terms; i = 0
 * contributes nothing.  A direction whose neighbour lies past a wall is
 * skipped.  The lever arm is the minimum-image offset.
 * ------------------------------------------------------------------------- */
void orc_mea(const ocfg *cfg, int np, const opart *P, const double *f, double *F, double *T) {
    init_tables();
    for (int p = 0; p < np; ++p) {
        double Fp[3] = {0, 0, 0}, Tp[3] = {0, 0, 0};
        double reach = orc_circumradius(P[p].shape, P[p].prm) + 1.0;
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) cell_range(&P[p], k, reach, &lo[k], &hi[k]);
        for (int a = lo[2]; a <= hi[2]; ++a)
            for (int b = lo[1]; b <= hi[1]; ++b)
                for (int c = lo[0]; c <= hi[0]; ++c) {
                    int x[3];
                    if (!wrap_coord(cfg, 0, c, &x[0]) || !wrap_coord(cfg, 1, b, &x[1]) ||
                        !wrap_coord(cfg, 2, a, &x[2]))
                        continue;
                    double d[3];
                    cell_offset(cfg, &P[p], x[0], x[1], x[2], d);
                    if (particle_sdf_at(&P[p], d) > 0.0) continue; /* not in x_b */
                    double up[3];
                    rigid_velocity(&P[p], d, up);
                    long xs = cell_index(cfg, x[0], x[1], x[2]);
                    double Fh[3] = {0, 0, 0};
                    for (int i = 1; i < Q; ++i) {
                        int y[3], ok = 1;
                        for (int k = 0; k < 3; ++k) ok &= wrap_coord(cfg, k, x[k] + C[i][k], &y[k]);
                        if (!ok) continue;
                        long ys = cell_index(cfg, y[0], y[1], y[2]);
                        double fin = f[Q * ys + i];       /* f_i(x + c_i, t) */
                        double fout = f[Q * xs + OPP[i]]; /* f_ibar(x, t) */
                        for (int k = 0; k < 3; ++k)
                            Fh[k] += (C[i][k] - up[k]) * fin + (C[i][k] + up[k]) * fout;
                    }
                    double tq[3] = {d[1] * Fh[2] - d[2] * Fh[1], d[2] * Fh[0] - d[0] * Fh[2],
                                    d[0] * Fh[1] - d[1] * Fh[0]};
                    for (int k = 0; k < 3; ++k) { Fp[k] -= Fh[k]; Tp[k] -= tq[k]; }
                }
        for (int k = 0; k < 3; ++k) { F[3 * p + k] = Fp[k]; T[3 * p + k] = Tp[k]; }
    }
}

/* ---------------------------------------------------------------------------
 * External force and equations of motion (Sec. 2.2, Newton and Euler eqs.;
 * gravity and buoyancy of Sec. 5.1), dt = 1, FP64.
 * reading: semi-implicit Euler; F_total = F_p + (m - rho_f V) g;
 * the rotation is advanced in the body frame,
 *   w_b <- w_b + I^-1 (T_b - w_b x (I w_b)),
 * and the orientation by the exponential map q <- q (x) exp(w_b / 2).
 * Fixed particles (m <= 0) are left untouched.
 * ------------------------------------------------------------------------- */
static void quat_mul(const double *a, const double *b, double *o) {
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

void orc_apply_eom(const ocfg *cfg, int np, opart *P, const double *F, const double *T) {
    for (int p = 0; p < np; ++p) {
        opart *s = &P[p];
        if (s->m <= 0.0) continue;
        double Ft[3];
        for (int k = 0; k < 3; ++k) Ft[k] = F[3 * p + k] + (s->m - cfg->rho_f * s->V) * cfg->g[k];
        for (int k = 0; k < 3; ++k) {
            s->U[k] += Ft[k] / s->m;
            s->X[k] += s->U[k];
            if (cfg->bc[k] == 0) s->X[k] -= cfg->n[k] * floor(s->X[k] / cfg->n[k]);
        }
        double R[3][3];
        quat_to_rot(s->q, R);
        double wb[3], tb[3];
        for (int k = 0; k < 3; ++k) {
            wb[k] = R[0][k] * s->W[0] + R[1][k] * s->W[1] + R[2][k] * s->W[2];
            tb[k] = R[0][k] * T[3 * p + 0] + R[1][k] * T[3 * p + 1] + R[2][k] * T[3 * p + 2];
        }
        double Iw[3] = {s->I[0] * wb[0], s->I[1] * wb[1], s->I[2] * wb[2]};
        double gyro[3] = {wb[1] * Iw[2] - wb[2] * Iw[1], wb[2] * Iw[0] - wb[0] * Iw[2],
                          wb[0] * Iw[1] - wb[1] * Iw[0]};
        for (int k = 0; k < 3; ++k) wb[k] += (tb[k] - gyro[k]) / s->I[k];
        double ang = sqrt(wb[0] * wb[0] + wb[1] * wb[1] + wb[2] * wb[2]);
        double dq[4] = {1, 0, 0, 0};
        if (ang > 0.0) {
            double sh = sin(0.5 * ang) / ang;
            dq[0] = cos(0.5 * ang);
            dq[1] = sh * wb[0]; dq[2] = sh * wb[1]; dq[3] = sh * wb[2];
        }
        double qn[4];
        quat_mul(s->q, dq, qn);
        double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
        for (int k = 0; k < 4; ++k) s->q[k] = qn[k] / nq;
        quat_to_rot(s->q, R);
        for (int k = 0; k < 3; ++k) s->W[k] = R[k][0] * wb[0] + R[k][1] * wb[1] + R[k][2] * wb[2];
    }
}

/* ---------------------------------------------------------------------------
 * Contact (an addition: the paper runs without a contact model and names one
 * only by citation, Sec. 2.2, Sec. 3.2 and Sec. 5.3).
 *
 * Sphere pairs -- reading: the short-range repulsion of Glowinski, Pan,
 * Hesla, Joseph and Periaux (J. Comput. Phys. 169, 2001).  Two spheres whose
 * centres are closer than R_p + R_q + zeta repel along the line of centres
 * with
 *     F_pq = k ((R_p + R_q + zeta - d) / zeta)^2 (X_p - X_q) / d,
 * and a wall acts on a sphere like its mirror image (centre distance
 * d' = 2 h, h the distance of the centre from the wall):
 *     F_pw = k_w ((2 R_p + zeta - d') / zeta)^2, directed away from the wall.
 *
 * Pairs with a non-spherical particle, and such particles at walls -- reading:
 * the same repulsion written as a volume law and evaluated on surface nodes
 * against the partner's signed distance (nodes probing a level set, as in the
 * level-set discrete element method of Kawamoto, Ando, Viggiani and Andrade,
 * J. Mech. Phys. Solids 91, 2016).  Grow both bodies by zeta/2; the volume of
 * their overlap is V = 1/2 (int_{dP} delta_q dA + int_{dQ} delta_p dA), with
 * delta_q(s) = max(0, zeta - d_q(s)) the depth of a surface point s of P in
 * the grown Q, and the force on P is
 *     F_P = k V / (pi R_eff zeta^2),  R_eff = R_P R_Q / (R_P + R_Q),
 * R the volume-equivalent radius, spread over the surface points along the
 * partner's outward normal grad d:
 *     F_P = K [ sum_{s in P} 1/2 a_s delta_q(s) grad d_q(s)
 *             - sum_{s in Q} 1/2 a_s delta_p(s) grad d_p(s) ],
 *     T_P = K [ sum_{s in P} (s - X_P) x (...) - sum_{s in Q} (s - X_P) x (...) ],
 * K = k / (pi R_eff zeta^2).  For two spheres V = pi R_eff h^2 to leading
 * order in the penetration h = R_p + R_q + zeta - d, so the law reduces to the
 * sphere law above.  A wall acts like the mirror image: delta_w(s) =
 * max(0, zeta - 2 h_s) with h_s the distance of s from the wall, V =
 * sum_s a_s delta_w(s), R_eff = R_P / 2, K_w = k_w / (pi (R_P / 2) zeta^2),
 * along the wall normal (for a sphere again the sphere law).
 * Surface nodes: M directions of a Fibonacci lattice on the unit sphere
 * (z_m = 1 - (2 m + 1) / M, azimuth m times the golden angle pi (3 - sqrt 5)),
 * the surface point on the ray from the centre by bisection of the signed
 * distance on [0, R_circ] (the bodies are star-shaped about their centre),
 * outward normal n the normalised gradient of the signed distance (central
 * differences, step 1e-5), area weight a = (4 pi / M) t^2 / (u . n) (the
 * surface element of a star-shaped body per solid angle).
 * Separations are minimum images on periodic axes; the state is that of time
 * t (the one the momentum exchange reads); force and torque are added to the
 * hydrodynamic ones in the equations of motion.  Sums run over q = 0, 1, ...,
 * np-1 (nodes of P, then nodes of Q), then the walls axis by axis (lower wall
 * first).
 * ------------------------------------------------------------------------- */
static double g_contact_range = 0.0, g_contact_k = 0.0, g_contact_kw = 0.0;
static int g_contact_nodes = 1024;

void orc_set_contact(double range, double k, double kw) {
    g_contact_range = range;
    g_contact_k = k;
    g_contact_kw = kw;
}

/* number of surface nodes per particle (1024 unless a test changes it) */
void orc_set_contact_nodes(int M) { g_contact_nodes = M > 0 ? M : 1024; }

static double inscribed_radius(const opart *P) {
    switch (P->shape) {
    case SH_SPHERE: return P->prm[0];
    case SH_ROUNDED_CUBE: return P->prm[0];
    case SH_SPHEROID: return fmin(P->prm[0], P->prm[1]);
    case SH_MESH: return P->prm[2];
    default: return 0.0;
    }
}

static double vol_radius(const opart *P) { return cbrt(3.0 * P->V / (4.0 * M_PI)); }

/* normalised central-difference gradient of the body-frame signed distance */
static void sdf_normal(const opart *P, const double *b, double *g) {
    const double h = 1e-5;
    double nn = 0.0;
    for (int k = 0; k < 3; ++k) {
        double bp[3] = {b[0], b[1], b[2]}, bm[3] = {b[0], b[1], b[2]};
        bp[k] += h;
        bm[k] -= h;
        g[k] = (orc_sdf(P->shape, P->prm, bp) - orc_sdf(P->shape, P->prm, bm)) / (2.0 * h);
        nn += g[k] * g[k];
    }
    nn = sqrt(nn);
    for (int k = 0; k < 3; ++k) g[k] /= nn;
}

/* Surface node m of M: body-frame position b, body-frame outward normal n,
 * area weight a. */
static void surface_node(const opart *P, int m, int M, double *b, double *n, double *a) {
    const double z = 1.0 - (2.0 * m + 1.0) / M, r = sqrt(fmax(0.0, 1.0 - z * z));
    const double ph = m * (M_PI * (3.0 - sqrt(5.0)));
    const double u[3] = {r * cos(ph), r * sin(ph), z};
    double lo = 0.0, hi = orc_circumradius(P->shape, P->prm);
    for (int it = 0; it < 60; ++it) {
        const double t = 0.5 * (lo + hi), p[3] = {t * u[0], t * u[1], t * u[2]};
        if (orc_sdf(P->shape, P->prm, p) < 0.0) lo = t; else hi = t;
    }
    const double t = 0.5 * (lo + hi);
    for (int k = 0; k < 3; ++k) b[k] = t * u[k];
    sdf_normal(P, b, n);
    *a = (4.0 * M_PI / M) * t * t / (u[0] * n[0] + u[1] * n[1] + u[2] * n[2]);
}

static void rot_apply(double R[3][3], const double *v, double *o) {
    for (int k = 0; k < 3; ++k) o[k] = R[k][0] * v[0] + R[k][1] * v[1] + R[k][2] * v[2];
}
static void rot_apply_t(double R[3][3], const double *v, double *o) {
    for (int k = 0; k < 3; ++k) o[k] = R[0][k] * v[0] + R[1][k] * v[1] + R[2][k] * v[2];
}
static void add_cross(const double *r, const double *f, double s, double *T) {
    T[0] += s * (r[1] * f[2] - r[2] * f[1]);
    T[1] += s * (r[2] * f[0] - r[0] * f[2]);
    T[2] += s * (r[0] * f[1] - r[1] * f[0]);
}

/* Node sums of one side: the nodes of A (centre at the origin) probing the
 * grown B (centre at e); adds sign * K/2 a delta grad d_B to F and
 * sign * (lever + node) x (...) to T, lever = offset of A's centre from the
 * particle whose force is summed. */
static void node_side(const opart *A, const opart *B, const double *e, double zeta, double K, double sign,
                      const double *lever, double *F, double *T) {
    double RA[3][3], RB[3][3];
    quat_to_rot(A->q, RA);
    quat_to_rot(B->q, RB);
    const int M = g_contact_nodes;
    for (int m = 0; m < M; ++m) {
        double b[3], n[3], a, s[3], y[3], yb[3];
        surface_node(A, m, M, b, n, &a);
        rot_apply(RA, b, s);
        for (int k = 0; k < 3; ++k) y[k] = s[k] - e[k];
        rot_apply_t(RB, y, yb);
        const double d = orc_sdf(B->shape, B->prm, yb);
        if (!(d < zeta)) continue;
        double gb[3], g[3], f[3], r[3];
        sdf_normal(B, yb, gb);
        rot_apply(RB, gb, g);
        const double w = 0.5 * K * a * (zeta - d);
        for (int k = 0; k < 3; ++k) {
            f[k] = w * g[k];
            F[k] += sign * f[k];
            r[k] = lever[k] + s[k];
        }
        add_cross(r, f, sign, T);
    }
}

void orc_contact_forces(const ocfg *cfg, int np, const opart *P, double range, double k, double kw,
                        double *Fc, double *Tc) {
    for (int p = 0; p < np; ++p) {
        double acc[3] = {0.0, 0.0, 0.0}, tor[3] = {0.0, 0.0, 0.0};
        if (range > 0.0) {
            const double rcp = orc_circumradius(P[p].shape, P[p].prm);
            for (int q = 0; q < np; ++q) {
                if (q == p) continue;
                double dx[3];
                for (int a = 0; a < 3; ++a) {
                    dx[a] = P[p].X[a] - P[q].X[a];
                    if (cfg->bc[a] == 0) dx[a] -= cfg->n[a] * round(dx[a] / cfg->n[a]);
                }
                const double d = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
                if (P[p].shape == SH_SPHERE && P[q].shape == SH_SPHERE) {
                    const double reach = P[p].prm[0] + P[q].prm[0] + range;
                    if (!(d < reach) || d == 0.0) continue;
                    const double s = (reach - d) / range;
                    for (int a = 0; a < 3; ++a) acc[a] += k * s * s * dx[a] / d;
                    continue;
                }
                if (!(d < rcp + orc_circumradius(P[q].shape, P[q].prm) + range) || k == 0.0) continue;
                const double Rp = vol_radius(&P[p]), Rq = vol_radius(&P[q]);
                const double K = k / (M_PI * (Rp * Rq / (Rp + Rq)) * range * range);
                const double e[3] = {-dx[0], -dx[1], -dx[2]}, zero[3] = {0.0, 0.0, 0.0};
                /* nodes of p in the grown q: force on p along grad d_q */
                node_side(&P[p], &P[q], e, range, K, 1.0, zero, acc, tor);
                /* nodes of q in the grown p: force on q along grad d_p, minus
                 * that on p; q's nodes sit at e + node from p's centre */
                const double me[3] = {dx[0], dx[1], dx[2]};
                node_side(&P[q], &P[p], me, range, K, -1.0, e, acc, tor);
            }
            for (int a = 0; a < 3; ++a) {
                if (cfg->bc[a] == 0 || kw == 0.0) continue;
                if (P[p].shape == SH_SPHERE) {
                    const double Rp = P[p].prm[0];
                    const double dlo = 2.0 * P[p].X[a], dhi = 2.0 * (cfg->n[a] - P[p].X[a]);
                    const double reach = 2.0 * Rp + range;
                    if (dlo < reach) {
                        const double s = (reach - dlo) / range;
                        acc[a] += kw * s * s;
                    }
                    if (dhi < reach) {
                        const double s = (reach - dhi) / range;
                        acc[a] -= kw * s * s;
                    }
                    continue;
                }
                if (!(P[p].X[a] < rcp + 0.5 * range || cfg->n[a] - P[p].X[a] < rcp + 0.5 * range)) continue;
                const double Kw = kw / (M_PI * 0.5 * vol_radius(&P[p]) * range * range);
                double R[3][3];
                quat_to_rot(P[p].q, R);
                const int M = g_contact_nodes;
                for (int side = 0; side < 2; ++side) {
                    for (int m = 0; m < M; ++m) {
                        double b[3], n[3], w, s[3];
                        surface_node(&P[p], m, M, b, n, &w);
                        rot_apply(R, b, s);
                        const double pos = P[p].X[a] + s[a];
                        const double h = side == 0 ? pos : cfg->n[a] - pos;
                        const double delta = range - 2.0 * h;
                        if (!(delta > 0.0)) continue;
                        double f[3] = {0.0, 0.0, 0.0};
                        f[a] = (side == 0 ? 1.0 : -1.0) * Kw * w * delta;
                        acc[a] += f[a];
                        add_cross(s, f, 1.0, tor);
                    }
                }
            }
        }
        for (int a = 0; a < 3; ++a) {
            Fc[3 * p + a] = acc[a];
            if (Tc) Tc[3 * p + a] = tor[a];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Particle -> lattice: indicator and solid velocity fields (Sec. 3.2).
 * reading (overlap of smoothed regions, not covered by the paper):
 *   S0 = sum_p B_p, S1 = sum_p B_p u_p(x); B = min(1, S0), u_s = S1 / S0.
 * Cells farther than R_circ + eps/2 from the centre have d_s >= eps/2 and
 * B = 0, so only that box is visited.
 * ------------------------------------------------------------------------- */
void orc_coupling(const ocfg *cfg, int np, const opart *P, double *B, double *us) {
    long N = orc_ncells(cfg);
    double *S0 = (double *)calloc((size_t)N, sizeof(double));
    double *S1 = (double *)calloc((size_t)N * 3, sizeof(double));
    for (int p = 0; p < np; ++p) {
        double reach = orc_circumradius(P[p].shape, P[p].prm) + 0.5 * cfg->eps;
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) cell_range(&P[p], k, reach, &lo[k], &hi[k]);
        for (int a = lo[2]; a <= hi[2]; ++a)
            for (int b = lo[1]; b <= hi[1]; ++b)
                for (int c = lo[0]; c <= hi[0]; ++c) {
                    int x[3];
                    if (!wrap_coord(cfg, 0, c, &x[0]) || !wrap_coord(cfg, 1, b, &x[1]) ||
                        !wrap_coord(cfg, 2, a, &x[2]))
                        continue;
                    double d[3];
                    cell_offset(cfg, &P[p], x[0], x[1], x[2], d);
                    double ds = particle_sdf_at(&P[p], d);
                    if (ds >= 0.5 * cfg->eps) continue;
                    double Bp = orc_indicator(ds, cfg->eps), up[3];
                    rigid_velocity(&P[p], d, up);
                    long xs = cell_index(cfg, x[0], x[1], x[2]);
                    S0[xs] += Bp;
                    for (int k = 0; k < 3; ++k) S1[k * N + xs] += Bp * up[k];
                }
    }
    for (long x = 0; x < N; ++x) {
        B[x] = S0[x] < 1.0 ? S0[x] : 1.0;
        for (int k = 0; k < 3; ++k) us[k * N + x] = S0[x] > 0.0 ? S1[k * N + x] / S0[x] : 0.0;
    }
    free(S0);
    free(S1);
}

/* ---------------------------------------------------------------------------
 * One time step in the order of the paper's time-step algorithm (Sec. 4.2,
 * Algorithm 1):
 * MEA -> external force (and contact, when set) -> equations of motion ->
 * EDM coupling -> collide -> stream.  The communication and assignment steps have nothing to do on one
 * address space.  F_last/T_last receive the hydrodynamic force and torque of
 * the last MEA.  Returns 0.
 * ------------------------------------------------------------------------- */
int orc_run(const ocfg *cfg, int np, opart *P, double *f, int nsteps, double *Flast, double *Tlast) {
    init_tables();
    long N = orc_ncells(cfg);
    double *fs = (double *)malloc(sizeof(double) * Q * (size_t)N);
    double *B = (double *)malloc(sizeof(double) * (size_t)N);
    double *us = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *F = (double *)calloc((size_t)(np > 0 ? np : 1) * 3, sizeof(double));
    double *T = (double *)calloc((size_t)(np > 0 ? np : 1) * 3, sizeof(double));
    double *Fc = (double *)calloc((size_t)(np > 0 ? np : 1) * 3, sizeof(double));
    double *Tc = (double *)calloc((size_t)(np > 0 ? np : 1) * 3, sizeof(double));
    const int contact = g_contact_range > 0.0 && (g_contact_k != 0.0 || g_contact_kw != 0.0);
    for (int s = 0; s < nsteps; ++s) {
        orc_mea(cfg, np, P, f, F, T);
        if (contact) {
            /* the equations of motion take F + F_contact and T + T_contact;
             * F and T stay the hydrodynamic ones that are reported */
            orc_contact_forces(cfg, np, P, g_contact_range, g_contact_k, g_contact_kw, Fc, Tc);
            for (int i = 0; i < 3 * np; ++i) {
                Fc[i] = F[i] + Fc[i];
                Tc[i] = T[i] + Tc[i];
            }
            orc_apply_eom(cfg, np, P, Fc, Tc);
        } else {
            orc_apply_eom(cfg, np, P, F, T);
        }
        orc_coupling(cfg, np, P, B, us);
        orc_collide(cfg, f, B, us, fs);
        orc_stream(cfg, fs, f);
    }
    if (Flast && nsteps > 0) memcpy(Flast, F, sizeof(double) * 3 * np);
    if (Tlast && nsteps > 0) memcpy(Tlast, T, sizeof(double) * 3 * np);
    free(fs); free(B); free(us); free(F); free(T); free(Fc); free(Tc);
    return 0;
}

/* Reported fields: bare rho and u, the physical velocity u_phys = u + du/2
 * with du from the current particles (EDM: du = B (u_s - u) + (1 - B) a_f;
 * partially saturated method: the velocity change of its collision per unit
 * density, du = B_n (u_s - u) + (1 - B_n) a_f), and B. */
void orc_fields(const ocfg *cfg, int np, const opart *P, const double *f, double *rho, double *u,
                double *uphys, double *B) {
    long N = orc_ncells(cfg);
    double *Bt = (double *)malloc(sizeof(double) * (size_t)N);
    double *us = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    orc_moments(cfg, f, rho, u);
    orc_coupling(cfg, np, P, Bt, us);
    for (long x = 0; x < N; ++x) {
        const double Bw = cfg->coupling == 1 ? orc_psm_weight(Bt[x], cfg->tau) : Bt[x];
        for (int k = 0; k < 3; ++k) {
            double du = Bw * (us[k * N + x] - u[k * N + x]) + (1.0 - Bw) * cfg->af[k];
            uphys[k * N + x] = u[k * N + x] + 0.5 * du;
        }
        if (B) B[x] = Bt[x];
    }
    free(Bt);
    free(us);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
