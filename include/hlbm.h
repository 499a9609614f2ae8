/*
 * hlbm.h -- C ABI of the MI355X (gfx950) HLBM hot path.
 *
 * The library advances a D3Q19 BGK lattice Boltzmann fluid coupled to resolved
 * rigid particles with the homogenized lattice Boltzmann method (HLBM) of
 * Marquardt, Hafen and Krause, "A novel particle decomposition scheme to
 * improve parallel performance of fully resolved particulate flow
 * simulations" (arXiv 2312.14172):
 *   - fluid: D3Q19 velocity set, BGK collision, streaming with dt = dx = 1
 *     (Sec. 3.1, collide/stream/BGK/relaxation/equilibrium equations);
 *   - particle -> fluid: trigonometric indicator B(d_s) of the signed
 *     distance, velocity difference du = B (u_p(x) - u_f) and the
 *     exact-difference source S_i = feq(rho, u + du) - feq(rho, u)
 *     (Sec. 3.2, level-set, velocity-difference and source equations);
 *   - fluid -> particle: momentum exchange summed over the cells whose centre
 *     is inside the particle, force and torque (Sec. 3.2, MEA, force and
 *     torque equations);
 *   - Newton-Euler equations with gravity and buoyancy (Sec. 2.2, Sec. 5.1),
 *     and optionally a contact force and torque (hlbm_set_contact);
 *   - in the order of the paper's time-step algorithm (Sec. 4.2, Algorithm 1); its
 *     communication and assignment steps have nothing to do on one GPU.
 *
 * Units are lattice units throughout.  Cell (x, y, z) has its centre at
 * (x + 1/2, y + 1/2, z + 1/2); cell index = x + nx * (y + ny * z).
 *
 * Conventions for every call:
 *   - return 0 on success or a negative HLBM_E* code; hlbm_last_error()
 *     returns a message for the calling thread's last failure;
 *   - no C++ exception crosses this ABI;
 *   - the caller owns every buffer it passes; the library keeps no pointer to
 *     a caller buffer after the call returns, except the device workspace
 *     handed to hlbm_init, which must stay allocated until hlbm_destroy;
 *   - the library allocates no device memory; everything lives in the
 *     caller's workspace;
 *   - all device work is queued on cfg.stream (NULL = the default stream);
 *     calls that return data synchronise that stream and report any error a
 *     kernel raised since the last such call;
 *   - a context is used by one host thread at a time.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define HLBM_OK 0
#define HLBM_EINVAL (-1)       /* bad argument or configuration */
#define HLBM_ENOMEM (-2)       /* workspace too small */
#define HLBM_EDEVICE (-3)      /* a HIP call failed */
#define HLBM_ESTATE (-4)       /* call not valid in the current state */
#define HLBM_EUNSTABLE (-5)    /* non-finite / non-positive density, |u| > 0.3, or a
                                  particle left the domain through a wall */
#define HLBM_EUNSUPPORTED (-6) /* a capacity of the library was exceeded */

/* boundary type per axis */
#define HLBM_BC_PERIODIC 0
#define HLBM_BC_WALL 1 /* resting half-way bounce-back walls at 0 and n */

/* population storage / arithmetic */
/* Every format stores the relative deviation K (f_i - w_i) / w_i of each
 * population from its lattice weight (Sec. 3.1 weights). */
#define HLBM_FP64 0  /* FP64 storage and arithmetic, K = 1 */
#define HLBM_FP32 1  /* FP32 arithmetic, FP32 storage, K = 1 */
#define HLBM_FP16S 2 /* FP32 arithmetic, FP16 storage, K = 256 */

/* particle -> fluid coupling of the collision (hlbm_config.coupling) */
#define HLBM_COUPLING_HLBM 0 /* BGK with the exact-difference source (Sec. 3.2) */
#define HLBM_COUPLING_PSM 1  /* partially saturated collision of Noble and Torczynski
                                (1998), the method family Sec. 3.2 names as a host of
                                the scheme: where B > 0,
                                f*_i = f_i - (1 - B_n)(f_i - feq_i(rho, u))/tau
                                       + B_n (f_opp(i) - feq_opp(i)(rho, u)
                                              + feq_i(rho, u_s) - f_i)
                                       + (1 - B_n)(feq_i(rho, u + a_f) - feq_i(rho, u)),
                                B_n = B (tau - 1/2) / ((1 - B) + (tau - 1/2)); the
                                particle force stays the momentum exchange's
                                (Sec. 4.2, Algorithm 1) */

/* particle shapes (body-frame parameters in hlbm_particle.param) */
#define HLBM_SPHERE 0       /* param[0] = radius */
#define HLBM_ROUNDED_CUBE 1 /* param[0] = half-extent h, param[1] = corner radius
                               (cube of half-extent h - r_c dilated by r_c) */
#define HLBM_SPHEROID 2     /* param[0] = semi-axis a along body x,
                               param[1] = the two equal semi-axes */
#define HLBM_MESH 3         /* param[0] = scale of the context's closed triangle
                               mesh (hlbm_set_mesh; body frame = mesh frame,
                               whose axes must be principal axes of inertia);
                               param[1], param[2] are replaced by the library
                               with scale x (largest vertex radius, least
                               distance of the surface from the origin) */

/* field selection for hlbm_get_fields */
#define HLBM_FIELD_RHO 1u    /* rho = sum_i f_i                              (1 plane) */
#define HLBM_FIELD_U 2u      /* bare u = sum_i c_i f_i / rho                 (3 planes) */
#define HLBM_FIELD_U_PHYS 4u /* u + du/2 with du from the current particles  (3 planes);
                                with HLBM_COUPLING_PSM du = B_n (u_s - u) + (1 - B_n) a_f */
#define HLBM_FIELD_SOLID 8u  /* B = min(1, sum_p B_p)                        (1 plane) */

typedef struct hlbm_config {
    int32_t nx, ny, nz;   /* lattice size, each >= 1 */
    int32_t bc[3];        /* HLBM_BC_* per axis */
    int32_t precision;    /* HLBM_FP64 | HLBM_FP32 | HLBM_FP16S */
    int32_t max_particles;/* capacity, >= 0 */
    double tau;           /* BGK relaxation time > 1/2; nu = (tau - 1/2) / 3 */
    double eps;           /* indicator smoothing width (the paper uses 1/2), > 0 */
    double rho_f;         /* fluid density used in the buoyancy term */
    double gravity[3];    /* gravity vector g (e.g. {0, 0, -1e-5}) */
    double fluid_accel[3];/* body acceleration of the fluid outside the solid */
    void *stream;         /* hipStream_t, NULL = default stream */
    int32_t learned;      /* 1: reserve memory for learned indicators (networks,
                             training samples, per-particle distance tables) */
    int32_t learned_samples; /* training + held-out sample capacity (0 = 1.2e6) */
    double learned_max_circumradius; /* largest circumradius of a particle that
                             may use a learned indicator (sizes the tables) */
    int32_t max_mesh_triangles; /* capacity of the HLBM_MESH shape's mesh, >= 0 */
    int32_t coupling;     /* HLBM_COUPLING_HLBM (0) or HLBM_COUPLING_PSM */
} hlbm_config;

typedef struct hlbm_particle {
    double pos[3];     /* centre of mass */
    double quat[4];    /* unit quaternion (w, x, y, z), body -> world */
    double vel[3];     /* velocity of the centre of mass */
    double omega[3];   /* angular velocity, world frame */
    double mass;       /* > 0; <= 0 holds the particle fixed at its state */
    double volume;     /* volume (> 0), used for buoyancy and the contact stiffness */
    double inertia[3]; /* principal moments of inertia in the body frame, > 0 */
    double param[3];   /* shape parameters, see HLBM_SPHERE etc. */
    int32_t shape;     /* HLBM_SPHERE | HLBM_ROUNDED_CUBE | HLBM_SPHEROID | HLBM_MESH */
    int32_t flags;     /* reserved, must be 0 */
} hlbm_particle;

typedef struct hlbm_ctx hlbm_ctx;

/* Bytes of device workspace hlbm_init needs for cfg (two population buffers,
 * particle records, tile lists, partial-force records and a staging area of
 * 4 doubles per cell for field transfers).  Returns HLBM_EINVAL for an
 * invalid configuration. */
int hlbm_workspace_size(const hlbm_config *cfg, size_t *bytes);

/* Create a context over a device workspace of at least hlbm_workspace_size
 * bytes (any alignment; 256-byte alignment is used internally).  The fluid
 * starts at rest (f_i = w_i, Sec. 3.1 weights), with no particles.  The
 * configuration is copied.  On failure *out is NULL. */
int hlbm_init(const hlbm_config *cfg, void *d_workspace, size_t bytes, hlbm_ctx **out);

/* Release the host-side context; the workspace is the caller's to free. */
int hlbm_destroy(hlbm_ctx *ctx);

/* Replace the particle set with n host records (copied).  The records are
 * the particle data of Sec. 4.2 (communication of particle data: position,
 * orientation, velocity, angular
 * velocity, shape).  Checks: n <= max_particles; finite values; unit
 * quaternion (|q| within 1e-6 of 1, renormalised); inertia > 0; volume > 0;
 * positive shape parameters; a particle's reach (circumradius + max(eps/2, sqrt 2) + 1)
 * below half of every periodic extent; centres inside the domain on wall
 * axes; circumradius below about 27 cells (the tile binning's limit). */
int hlbm_set_particles(hlbm_ctx *ctx, int32_t n, const hlbm_particle *host);

/* Set the fluid to equilibrium f_i = feq_i(rho, u) (Sec. 3.1) from host
 * arrays rho[ncells] and u[3][ncells] (x-fastest planes); rho == NULL means
 * rho = 1 and u == NULL means u = 0. */
int hlbm_set_fields(hlbm_ctx *ctx, const double *rho, const double *u);

/* Queue nsteps >= 0 time steps on the stream.  Each step: momentum exchange
 * force and torque on every particle (Sec. 3.2) -> gravity and buoyancy ->
 * Newton-Euler update in FP64 -> particle-to-lattice coupling with the
 * updated particles -> fused collide and stream with the exact-difference
 * source.  Asynchronous: errors raised inside kernels are reported by the
 * next hlbm_get_* call.  Runs are bitwise reproducible on a given GPU: every
 * sum runs in a fixed order (lists filled by atomic appends are ranked by
 * particle index before they are summed; no floating-point atomics). */
int hlbm_step(hlbm_ctx *ctx, int32_t nsteps);

/* Set the closed triangle mesh of HLBM_MESH particles: vertices[nv][3] in
 * the body frame at unit scale (FP32), triangles[nt][3] vertex indices,
 * counter-clockwise seen from outside, enclosing the origin (the centre of
 * mass).  Copied to the device.  The signed distance of a point is its least
 * distance to a triangle, negative where the generalised winding number of
 * the mesh exceeds 1/2; it feeds the indicator (Sec. 3.2 level-set
 * equation) and the momentum exchange's inside test, like the closed-form
 * distances of the other shapes.  The paper points to such irregular shapes
 * (Sec. 5.4) as where the cost of the distance grows; the learned indicator
 * (hlbm_train_indicator with HLBM_MESH) replaces it there.  Call before
 * hlbm_set_particles (HLBM_ESTATE if particles are set); HLBM_EUNSUPPORTED
 * above cfg.max_mesh_triangles; HLBM_EINVAL for bad indices, non-finite
 * vertices, or a mesh that does not wind once around the origin. */
int hlbm_set_mesh(hlbm_ctx *ctx, const float *vertices, int32_t nv, const int32_t *triangles, int32_t nt);

/* Replace the fluid body acceleration of the configuration (the fluid
 * outside the solid, as in hlbm_config.fluid_accel) for the steps queued
 * after this call.  It stands in for a mean pressure gradient: Sec. 5.1
 * drives a periodic suspension with a pressure gradient, updated as the
 * settling proceeds, that keeps the net volume flux at zero.  Stream-ordered
 * (takes effect with the next hlbm_step); non-finite values are rejected
 * with HLBM_EINVAL and leave the acceleration unchanged. */
int hlbm_set_fluid_accel(hlbm_ctx *ctx, const double accel[3]);

/* Particle contact, off by default.  Sec. 2.2 lets contact forces enter the
 * particles' equations of motion next to the hydrodynamic ones; Sec. 3.2
 * leaves the cited contact model (one for arbitrary convex shapes) out on
 * purpose, and Sec. 5.3 names the missing contact model as the likely cause
 * of the overestimated settling velocities at high volume fractions, without
 * giving a model.  Spheres: the short-range repulsion of Glowinski et al.
 * (J. Comput. Phys. 169, 2001): spheres whose centres are closer than
 * R_p + R_q + range repel along the line of centres with stiffness *
 * ((R_p + R_q + range - d) / range)^2 (minimum image on periodic axes), and a
 * wall pushes a sphere whose centre is at distance h with wall_stiffness *
 * ((2 R + range - 2 h) / range)^2 (its mirror image).  Pairs with a
 * non-spherical particle (and such particles at walls): the same repulsion
 * written as a volume law, stiffness * V / (pi R_eff range^2) with V the
 * overlap of the two bodies grown by range / 2, evaluated on 1024 surface
 * nodes of each body against the partner's signed distance and applied at
 * the nodes along the partner's normal, so that it also exerts a torque
 * (R_eff = R_p R_q / (R_p + R_q) from volume-equivalent radii; R_p / 2 and
 * the mirror image at a wall); for two spheres it reduces to the law above
 * to leading order in the penetration.  The force and torque act on the
 * state of the step's momentum exchange and are added to the hydrodynamic
 * ones in the equations of motion (hlbm_get_forces still reports the
 * hydrodynamic force and torque alone).  Pairs are found by testing all
 * n^2 pairs below 4096 particles and on a grid of the particle centres from
 * there on; a particle may have at most 64 partners whose bounding spheres
 * come within the range (64 non-spherical pairs below 4096 particles), and a
 * step with more fails with HLBM_EUNSUPPORTED (checked when the step's
 * results are read).  Stream-ordered like hlbm_set_fluid_accel; range = 0 or
 * both stiffnesses 0 turn it off.  HLBM_EINVAL for negative or non-finite
 * values. */
int hlbm_set_contact(hlbm_ctx *ctx, double range, double stiffness, double wall_stiffness);

/* Copy to host the hydrodynamic force F[n][3] and torque T[n][3] on each
 * particle from the last completed step's momentum exchange (zero before the
 * first step): the force is minus the sum of the MEA momentum F_h over the
 * cells whose centre is inside the particle, the torque minus the sum of
 * (x_b - X_p) x F_h (Sec. 3.2, MEA, total-force and torque equations; the
 * sign reads F_h as the momentum given to the fluid).  Optionally also the
 * current particle records.  Any pointer may be NULL.  Synchronises the
 * stream. */
int hlbm_get_forces(hlbm_ctx *ctx, double *F, double *T, hlbm_particle *state);

/* Write the fields selected by mask as planes of ncells values each, in the
 * order rho, u (3), u_phys (3), B, to out: FP64 values for dtype ==
 * HLBM_FP64, FP32 (rounded to nearest) for dtype == HLBM_FP32; out is host
 * memory if out_on_device == 0, else device memory on the context's device,
 * and must hold (planes x ncells) values of the chosen type.  The fields are
 * the moments of the current state (Sec. 3.1: rho = sum f_i, rho u = sum c_i
 * f_i of the post-streaming populations at the current integer time),
 * u_phys = u + du/2 with du of Sec. 3.2's velocity-difference equation from
 * the current particles and fluid acceleration, and B, the indicator of
 * Sec. 3.2's level-set equation combined over particles as min(1, sum B_p).
 * HLBM_EINVAL for an empty or unknown mask or another dtype.  Synchronises
 * the stream. */
int hlbm_get_fields(hlbm_ctx *ctx, uint32_t mask, int32_t dtype, void *out, int32_t out_on_device);

/* Volume flux of the current state: mean_u_phys[3] = the mean of u_phys over
 * all cells, mean_fluid_u_phys[3] = its mean over the pure-fluid cells
 * (B = 0; zero if there are none) and *fluid_cells their number (host
 * pointers, each may be NULL).  Summed in FP64 in a fixed order on the
 * device (bitwise reproducible).  Sec. 5.1 sets the periodic suspension's
 * pressure gradient so that the net volume flux vanishes; the fluid-cell mean
 * gives the settling velocity relative to the fluid.  Synchronises the
 * stream. */
int hlbm_get_mean_velocity(hlbm_ctx *ctx, double *mean_u_phys, double *mean_fluid_u_phys, int64_t *fluid_cells);

/* Measurement hooks: from hlbm_profile_begin on, every collide-and-stream
 * launch of hlbm_step is bracketed by two HIP events recorded on the
 * context's stream.  hlbm_profile_end synchronises the stream, returns the
 * summed event time in milliseconds and the number of timed launches, and
 * stops timing. */
int hlbm_profile_begin(hlbm_ctx *ctx);
int hlbm_profile_end(hlbm_ctx *ctx, double *collide_ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Learned indicator (not part of the paper; its hook is Sec. 5.4: signed
 * distances of non-spherical shapes cost more per lattice node).  For a shape
 * family (HLBM_ROUNDED_CUBE or HLBM_SPHEROID with a fixed aspect, or HLBM_MESH) a network
 * 3 -> 64 -> 64 -> 64 -> 1 with SiLU activations maps a body-frame point
 * divided by the circumradius R_c to d_s / R_c.  BF16 matrix-core products
 * with FP32 accumulation; FP32 master parameters trained with Adam.  When a
 * family is in HLBM_INDICATOR_LEARNED mode, every step fills a per-particle
 * distance table over each such particle's coupling box: the network is
 * queried on the shell r_in - eps/2 <= |x - X| <= R_c + eps/2 (r_in the
 * inscribed radius), cells nearer the centre count as inside (B = 1), cells
 * farther as outside (B = 0); both the indicator B(d_s) and the inside test
 * d_s <= 0 of the momentum exchange read the table.  Requires cfg.learned = 1.
 *
 * Parameters are one flat float vector of HLBM_MLP_NPARAM entries in the
 * order W1 (64x3, row-major), b1 (64), W2 (64x64), b2, W3 (64x64), b3,
 * W4 (64), b4 (1).
 * ------------------------------------------------------------------------ */
#define HLBM_MLP_NPARAM 8641
#define HLBM_INDICATOR_EXACT 0
#define HLBM_INDICATOR_LEARNED 1

typedef struct hlbm_train_opts {
    int32_t samples;     /* training samples: uniform in the box, or within `band` (band_share) */
    int32_t holdout;     /* held-out samples within `band` (evaluate the gate) */
    int32_t iterations;  /* Adam steps */
    int32_t batch;       /* samples per step */
    double lr;           /* initial learning rate */
    double lr_final;     /* learning rate of the last step (geometric decay) */
    double box;          /* sampling cube half-width, in circumradii (e.g. 1.1) */
    double band;         /* near-surface band half-width, in circumradii */
    double clip;         /* targets clipped to +-clip circumradii */
    double band_share;   /* fraction of training samples drawn within `band` (0..1) */
    double gate_rms;     /* accept if held-out RMS error <= gate_rms ... */
    double gate_max;     /* ... and max error <= gate_max (lattice units at ref size) */
    double ref_circumradius; /* particle size (lattice units) at which the gate is evaluated */
    uint64_t seed;       /* sample generator seed */
} hlbm_train_opts;

typedef struct hlbm_train_report {
    double loss_first;   /* mean-squared loss (normalised units) of the first batch */
    double loss_last;    /* ... and of the last batch */
    double rms_err;      /* held-out RMS |d_net - d| in lattice units at ref size */
    double max_err;      /* held-out max |d_net - d| in lattice units at ref size */
    double train_ms;     /* wall time of sample generation + training */
    int32_t iterations;
    int32_t accepted;    /* 1: gate passed and the family switched to LEARNED */
} hlbm_train_report;

/* Load / read the network parameters of a shape family (host float arrays of
 * HLBM_MLP_NPARAM).  Setting parameters resets the Adam moments. */
int hlbm_mlp_set_params(hlbm_ctx *ctx, int32_t shape, const float *theta);
int hlbm_mlp_get_params(hlbm_ctx *ctx, int32_t shape, float *theta);

/* Network outputs at n normalised points pts[n][3] (host) -> out[n] (host). */
int hlbm_mlp_eval(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, double *out);

/* Gradient of the mean-squared loss mean_s (net(pts_s) - target_s)^2 with
 * respect to the parameters (host double[HLBM_MLP_NPARAM]) and the loss,
 * computed by the training kernels (BF16 products, FP32 accumulation). */
int hlbm_mlp_gradient(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, const double *target,
                      double *grad, double *loss);

/* One training step on n points (host arrays as for hlbm_mlp_gradient):
 * the gradient of the mean-squared loss by the training kernels, then one
 * bias-corrected Adam step (Kingma and Ba 2015; beta1 0.9, beta2 0.999,
 * epsilon 1e-8) with learning rate lr as the step-th update of the family's
 * FP32 moments (reset by hlbm_mlp_set_params and by hlbm_train_indicator).
 * Returns the gradient used (host double[HLBM_MLP_NPARAM], may be NULL) and
 * the loss (may be NULL); the updated parameters are read with
 * hlbm_mlp_get_params.  HLBM_EINVAL for lr <= 0 or step < 1. */
int hlbm_mlp_train_step(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, const double *target,
                        double lr, int32_t step, double *grad, double *loss);

/* The training samples hlbm_train_indicator draws for a shape with
 * parameters param[3] and the given seed: n points uniform in [-box, box]^3
 * of the normalised body frame (the shape scaled to circumradius 1), of which
 * a share band_share is redrawn (up to 64 times) until the exact signed
 * distance is within band; out[n][4] (host) receives x, y, z and the signed
 * distance clipped to +-clip, each rounded to FP32.  n up to the sample
 * capacity. */
int hlbm_mlp_samples(hlbm_ctx *ctx, int32_t shape, const double *param, uint64_t seed, int32_t n, double box,
                     double band, double clip, double band_share, double *out);

/* Train the family's network (starting from its current parameters) on
 * samples of the exact signed distance of a shape with parameters param[3]
 * (lattice units; they fix the aspect), generated on the GPU.  If the
 * held-out errors pass the gate the family switches to LEARNED, otherwise it
 * stays EXACT (the fallback).  Synchronises the stream. */
int hlbm_train_indicator(hlbm_ctx *ctx, int32_t shape, const double *param, const hlbm_train_opts *opts,
                         hlbm_train_report *report);

/* Select HLBM_INDICATOR_EXACT or HLBM_INDICATOR_LEARNED for a shape family.
 * LEARNED needs parameters (set or trained) and an aspect ratio: particles of
 * the family whose aspect differs from the trained one keep the exact path. */
int hlbm_set_indicator(hlbm_ctx *ctx, int32_t shape, int32_t mode);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the gradient of
 * hlbm_mlp_gradient without a context.  All pointers are device memory on
 * the current device: d_theta[HLBM_MLP_NPARAM] the FP32 parameters,
 * d_samples[n][4] FP32 (x, y, z, target) in normalised units, d_grad
 * receives HLBM_MLP_NPARAM + 1 floats: the gradient of the mean-squared loss
 * mean_s (net(x_s) - t_s)^2, then the sum of squared errors.  The work is
 * queued on stream (hipStream_t, NULL = default) and not waited for; nothing
 * is allocated or freed.  The working memory is a fixed array of 2.2 MB per
 * GPU inside the library, so n is limited to 2048 (HLBM_EUNSUPPORTED above);
 * the results equal hlbm_mlp_gradient's for the same inputs (the same
 * kernels and partition).  Calls that overlap on one GPU (on different
 * streams or threads) race on that array.  HLBM_EINVAL for NULL pointers. */
int hlbm_mlp_gradient_noalloc(const float *d_theta, int32_t n, const float *d_samples, float *d_grad, void *stream);

/* Number of particles currently held. */
int hlbm_num_particles(const hlbm_ctx *ctx, int32_t *n);

/* Message for the calling thread's most recent failure ("" if none). */
const char *hlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HLBM_H */
