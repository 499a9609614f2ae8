// hlbm_api.hip -- the C ABI declared in include/hlbm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include <string>
#include <vector>

#include "hlbm_internal.h"
#include "hlbm_mlp.h"

#include <chrono>
#include <mutex>

using namespace hlbm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(HLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// z-layers a particle's momentum-exchange box can span (circumradius <= 27)
constexpr int LMAX_CAP = 56;
// particle count from which the momentum exchange is dispatched XCD-chunked
constexpr int MEA_CHUNKED_MIN = 4096;

size_t pop_bytes(int precision) { return precision == HLBM_FP64 ? 8 : (precision == HLBM_FP32 ? 4 : 2); }

struct Layout {
  size_t fA, fB, parts, order, stage_parts, tcnt[2], tlist[2], partial, contact, status, stage, total;
  size_t cshapes, cdirs, ccand, ccnt;  // node contact: records, node directions, partner lists and counts
  size_t gcount, gfill, gcell, glist, gpos;  // contact pair search (grid of centres)
  // learned indicator (cfg.learned)
  size_t theta[NFAM], mom1[NFAM], mom2[NFAM], packed[NFAM], gpart, gout, pool, epts, eout, tables, mesh;
  size_t band[NFAM];  // band grids (learned or mesh shapes)
  long long pool_cap, table_cap;
};

int validate(const hlbm_config *c) {
  if (!c) return fail(HLBM_EINVAL, "config is NULL");
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(HLBM_EINVAL, "lattice size must be >= 1");
  const long long N = (long long)c->nx * c->ny * c->nz;
  if (N >= (1LL << 31)) return fail(HLBM_EINVAL, "lattice too large (at most 2^31 - 1 cells)");
  for (int k = 0; k < 3; ++k)
    if (c->bc[k] != HLBM_BC_PERIODIC && c->bc[k] != HLBM_BC_WALL)
      return fail(HLBM_EINVAL, "bc[%d] must be HLBM_BC_PERIODIC or HLBM_BC_WALL", k);
  if (c->precision < HLBM_FP64 || c->precision > HLBM_FP16S) return fail(HLBM_EINVAL, "unknown precision");
  if (c->max_particles < 0) return fail(HLBM_EINVAL, "max_particles < 0");
  if (c->max_mesh_triangles < 0) return fail(HLBM_EINVAL, "max_mesh_triangles < 0");
  if (!(c->tau > 0.5) || !isfinite(c->tau)) return fail(HLBM_EINVAL, "tau must be > 1/2 (nu > 0)");
  if (!(c->eps > 0.0) || !isfinite(c->eps)) return fail(HLBM_EINVAL, "eps must be > 0");
  if (!isfinite(c->rho_f)) return fail(HLBM_EINVAL, "rho_f not finite");
  if (c->learned != 0 && c->learned != 1) return fail(HLBM_EINVAL, "learned must be 0 or 1");
  if (c->coupling != HLBM_COUPLING_HLBM && c->coupling != HLBM_COUPLING_PSM)
    return fail(HLBM_EINVAL, "coupling must be HLBM_COUPLING_HLBM or HLBM_COUPLING_PSM");
  if ((c->learned || c->max_mesh_triangles > 0) &&
      !(c->learned_max_circumradius > 0 && c->learned_max_circumradius <= 27.0))
    return fail(HLBM_EINVAL, "learned_max_circumradius must be in (0, 27] (distance tables of learned or mesh shapes)");
  if (c->learned && c->learned_samples < 0) return fail(HLBM_EINVAL, "learned_samples < 0");
  if (c->learned || c->max_mesh_triangles > 0) {
    // the table kernels index a box with FP32 quotients, exact below 2^22 cells
    const double side = floor(2.0 * (c->learned_max_circumradius + 0.5 * c->eps)) + 2;
    if (side * side * side >= 4194304.0)
      return fail(HLBM_EUNSUPPORTED, "distance tables of %.0f^3 cells: learned_max_circumradius + eps/2 too large",
                  side);
  }
  for (int k = 0; k < 3; ++k)
    if (!isfinite(c->gravity[k]) || !isfinite(c->fluid_accel[k]))
      return fail(HLBM_EINVAL, "gravity / fluid_accel not finite");
  return HLBM_OK;
}

Lattice make_lattice(const hlbm_config *c) {
  Lattice L;
  L.nx = c->nx; L.ny = c->ny; L.nz = c->nz;
  for (int k = 0; k < 3; ++k) L.bc[k] = c->bc[k];
  L.ntx = (c->nx + TX - 1) / TX;
  L.nty = (c->ny + TY - 1) / TY;
  L.ntz = (c->nz + TZ - 1) / TZ;
  L.ntiles = L.ntx * L.nty * L.ntz;
  L.N = (long long)c->nx * c->ny * c->nz;
  L.omega = 1.0 / c->tau;
  L.eps = c->eps;
  for (int k = 0; k < 3; ++k) { L.af[k] = c->fluid_accel[k]; L.g[k] = c->gravity[k]; }
  L.rho_f = c->rho_f;
  L.tables = nullptr;
  L.table_cap = 0;
  L.mesh = nullptr;
  L.mesh_nt = 0;
  L.psm = c->coupling == HLBM_COUPLING_PSM ? 1 : 0;
  L.tau_mh = c->tau - 0.5;
  return L;
}

Layout make_layout(const hlbm_config *c, const Lattice &L) {
  Layout y;
  size_t off = 0;
  const size_t pop = align_up((size_t)19 * L.N * pop_bytes(c->precision));
  const size_t np = c->max_particles > 0 ? (size_t)c->max_particles : 1;
  y.fA = off; off += pop;
  y.fB = off; off += pop;
  y.parts = off; off += align_up(np * sizeof(DevParticle));
  y.order = off; off += align_up(np * sizeof(int));
  y.stage_parts = off; off += align_up(np * sizeof(hlbm_particle));
  for (int b = 0; b < 2; ++b) {
    y.tcnt[b] = off; off += align_up((size_t)L.ntiles * sizeof(int));
    y.tlist[b] = off; off += align_up((size_t)L.ntiles * MAXC * sizeof(int));
  }
  y.partial = off; off += align_up(np * LMAX_CAP * 6 * sizeof(double));
  y.contact = off; off += align_up(np * (size_t)CONTACT_MAX_CHUNKS * 3 * sizeof(double));
  y.gcount = off; off += align_up((size_t)(CGRID_MAX + 1) * sizeof(int));
  y.gfill = off; off += align_up((size_t)CGRID_MAX * sizeof(int));
  y.gcell = off; off += align_up(np * sizeof(int));
  y.glist = off; off += align_up(np * sizeof(int));
  y.gpos = off; off += align_up(np * sizeof(double4));
  y.cshapes = off; off += align_up(np * 6 * sizeof(double));
  y.cdirs = off; off += align_up((size_t)CONTACT_NODES * 3 * sizeof(double));
  y.ccand = off; off += align_up(np * CONTACT_CAND * sizeof(int));
  y.ccnt = off; off += align_up(np * sizeof(int));
  y.status = off; off += 256;
  // staging: 4 FP64 planes for host transfers, or the 7-double tile records
  // of the mean-velocity reduction and their sums
  y.stage = off; off += align_up(std::max<size_t>((size_t)4 * L.N, (size_t)7 * L.ntiles + 7) * sizeof(double));
  y.mesh = off; off += align_up((size_t)(c->max_mesh_triangles > 0 ? c->max_mesh_triangles : 1) * 3 * sizeof(float4));
  y.pool_cap = 0;
  y.table_cap = 0;
  const bool tables = c->learned || c->max_mesh_triangles > 0;
  if (c->learned) {
    for (int f = 0; f < NFAM; ++f) {
      y.theta[f] = off; off += align_up(MLP_PARTIAL * sizeof(float));
      y.mom1[f] = off; off += align_up(MLP_PARTIAL * sizeof(float));
      y.mom2[f] = off; off += align_up(MLP_PARTIAL * sizeof(float));
      y.packed[f] = off; off += align_up(MLP_PACKED_BYTES);
    }
    y.gpart = off; off += align_up((size_t)MLP_MAX_BLOCKS * MLP_PARTIAL * sizeof(float));
    y.gout = off; off += align_up(MLP_PARTIAL * sizeof(float));
    y.pool_cap = c->learned_samples > 0 ? c->learned_samples : 1200000;
    y.pool = off; off += align_up((size_t)y.pool_cap * 16);
    y.epts = off; off += align_up((size_t)y.pool_cap * 3 * sizeof(float));
    y.eout = off; off += align_up((size_t)y.pool_cap * sizeof(float));
  }
  if (tables) {
    for (int f = 0; f < NFAM; ++f) {
      y.band[f] = off; off += align_up(BAND_BYTES);
    }
    const long long side = (long long)floor(2.0 * (c->learned_max_circumradius + 0.5 * c->eps)) + 2;
    y.table_cap = side * side * side;
    y.tables = off; off += align_up((size_t)np * y.table_cap * sizeof(float));
  }
  y.total = off + 256;  // slack for aligning the caller's base pointer
  return y;
}

}  // namespace

struct hlbm_ctx {
  hlbm_config cfg;
  Lattice L;
  Layout lay;
  hipStream_t stream;
  char *base;
  void *fA, *fB;
  DevParticle *parts;
  int *order;         // particles in the momentum-exchange visiting order
  int mea_chunked;    // that order is dispatched in XCD-contiguous runs
  hlbm_particle *stage_parts;
  int *tcnt[2], *tlist[2], *status;
  int cur;            // tile-list buffer describing the current particles
  double *partial, *stage;
  double *contact;    // per-chunk sphere contact forces [chunk][n][3]
  double *cshapes;    // contact force and torque of pairs with a non-spherical particle [n][6]
  double *cdirs;      // surface-node directions of that contact [CONTACT_NODES][3]
  int *ccand, *ccnt;  // its partner lists [n][CONTACT_CAND] and counts (zero between steps)
  ContactWork cwork;  // pair-search arrays
  double cwmax;       // largest sphere radius / circumradius of the particles
  bool nonspherical;  // the current particles include non-spherical ones
  ContactParams cparams;
  int lmax;           // z-layers of the largest momentum-exchange box
  int n;
  int bin_cap;        // tiles a particle's coupling box can touch (bin grid width)
  bool binned;        // tile lists describe the current particles
  long long steps_done;
  bool profiling;
  std::vector<hipEvent_t> events;  // start/stop pairs around collide launches
  size_t events_used;
  // learned indicator, index 0: rounded cube, 1: spheroid, 2: mesh
  float *theta[NFAM], *mom1[NFAM], *mom2[NFAM];
  __bf16 *packed[NFAM];
  float *gpart, *gout, *epts, *eout;
  float4 *pool;
  float *tables;
  float *band[NFAM];     // band grid of each family's shape at unit circumradius
  int band_ok[NFAM];     // the grid holds the trained (or, for meshes, the current) shape
  int mode[NFAM];        // HLBM_INDICATOR_EXACT / LEARNED
  int has_params[NFAM];
  double aspect[NFAM];   // param[1] / param[0] of the trained shape, 0 = unknown
  // the mesh of HLBM_MESH particles (unit scale): triangles in the workspace,
  // largest vertex radius and least distance of the surface from the origin
  float4 *mesh;
  double mesh_rc, mesh_rin;
  bool mesh_particles;  // the current particles include HLBM_MESH ones
};

namespace {

int check_status(hlbm_ctx *c) {
  int st = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost));
  if (st) {
    const int zero = 0;
    HIP_TRY(hipMemcpy(c->status, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (st & ST_TILE_OVERFLOW)
      return fail(HLBM_EUNSUPPORTED, "more than %d particles touch one 64x4x4 tile", MAXC);
    if (st & ST_CONTACT_OVERFLOW)
      return fail(HLBM_EUNSUPPORTED, "a non-spherical particle has more than %d contact partners", CONTACT_CAND);
    if (st & ST_WALL_EXIT) return fail(HLBM_EUNSTABLE, "a particle centre left the domain through a wall");
    return fail(HLBM_EUNSTABLE, "non-finite or non-positive density, or |u| > 0.3");
  }
  return HLBM_OK;
}

bool any_learned(const hlbm_ctx *c) {
  if (!c->tables) return false;
  for (int f = 0; f < NFAM; ++f)
    if (c->mode[f] == HLBM_INDICATOR_LEARNED) return true;
  return false;
}

int refresh_tables(hlbm_ctx *c) {
  if (c->n == 0 || !c->tables) return HLBM_OK;
  // exact tables of mesh particles without a network
  if (c->mesh_particles && c->mode[2] != HLBM_INDICATOR_LEARNED)
    HIP_TRY(launch_mesh_table(c->L, c->parts, c->n, c->band_ok[2] ? c->band[2] : nullptr, c->tables,
                              c->lay.table_cap, c->stream));
  if (!any_learned(c)) return HLBM_OK;
  LearnedNets nets;
  for (int f = 0; f < NFAM; ++f) {
    nets.theta[f] = c->theta[f];
    nets.packed[f] = c->packed[f];
    nets.band[f] = c->band_ok[f] ? c->band[f] : nullptr;
  }
  HIP_TRY(launch_mlp_table(c->L, c->parts, c->n, nets, c->tables, c->lay.table_cap, c->stream));
  return HLBM_OK;
}

int mark_learned(hlbm_ctx *c) {
  if (!c->tables || c->n == 0) return HLBM_OK;
  LearnedModes modes;
  for (int f = 0; f < NFAM; ++f) {
    modes.on[f] = c->mode[f] == HLBM_INDICATOR_LEARNED;
    modes.aspect[f] = c->aspect[f];
  }
  HIP_TRY(launch_mark_learned(c->parts, c->n, modes, c->stream));
  return refresh_tables(c);
}

int rebin(hlbm_ctx *c) {
  HIP_TRY(launch_fill_int(c->tcnt[0], 0, c->L.ntiles, c->stream));
  HIP_TRY(launch_fill_int(c->tcnt[1], 0, c->L.ntiles, c->stream));
  HIP_TRY(launch_bin(c->L, c->parts, c->n, c->bin_cap, c->tcnt[c->cur], c->tlist[c->cur], c->status,
                     c->stream));
  c->binned = true;
  return HLBM_OK;
}

}  // namespace

extern "C" {

const char *hlbm_last_error(void) { return g_last_error.c_str(); }

int hlbm_workspace_size(const hlbm_config *cfg, size_t *bytes) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!bytes) return fail(HLBM_EINVAL, "bytes is NULL");
  const Lattice L = make_lattice(cfg);
  *bytes = make_layout(cfg, L).total;
  return HLBM_OK;
}

int hlbm_init(const hlbm_config *cfg, void *d_workspace, size_t bytes, hlbm_ctx **out) {
  if (!out) return fail(HLBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!d_workspace) return fail(HLBM_EINVAL, "workspace is NULL");
  const Lattice L = make_lattice(cfg);
  const Layout lay = make_layout(cfg, L);
  if (bytes < lay.total) return fail(HLBM_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, lay.total);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, d_workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(HLBM_EINVAL, "workspace is not device memory");
  }
  hlbm_ctx *c = new (std::nothrow) hlbm_ctx();
  if (!c) return fail(HLBM_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->L = L;
  c->lay = lay;
  c->stream = (hipStream_t)cfg->stream;
  c->base = (char *)(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
  c->fA = c->base + lay.fA;
  c->fB = c->base + lay.fB;
  c->parts = (DevParticle *)(c->base + lay.parts);
  c->order = (int *)(c->base + lay.order);
  c->stage_parts = (hlbm_particle *)(c->base + lay.stage_parts);
  for (int b = 0; b < 2; ++b) {
    c->tcnt[b] = (int *)(c->base + lay.tcnt[b]);
    c->tlist[b] = (int *)(c->base + lay.tlist[b]);
  }
  c->cur = 0;
  c->partial = (double *)(c->base + lay.partial);
  c->contact = (double *)(c->base + lay.contact);
  c->cshapes = (double *)(c->base + lay.cshapes);
  c->cdirs = (double *)(c->base + lay.cdirs);
  c->ccand = (int *)(c->base + lay.ccand);
  c->ccnt = (int *)(c->base + lay.ccnt);
  c->cwork = ContactWork{(int *)(c->base + lay.gcount), (int *)(c->base + lay.gfill), (int *)(c->base + lay.gcell),
                         (int *)(c->base + lay.glist), (double4 *)(c->base + lay.gpos)};
  c->cwmax = 0.0;
  c->nonspherical = false;
  c->cparams = ContactParams{0.0, 0.0, 0.0, 0};
  c->lmax = 1;
  c->status = (int *)(c->base + lay.status);
  c->stage = (double *)(c->base + lay.stage);
  c->n = 0;
  c->mea_chunked = 0;
  c->binned = false;
  c->bin_cap = 1;
  c->steps_done = 0;
  c->profiling = false;
  c->events_used = 0;
  for (int f = 0; f < NFAM; ++f) {
    c->theta[f] = c->mom1[f] = c->mom2[f] = nullptr;
    c->packed[f] = nullptr;
    c->mode[f] = HLBM_INDICATOR_EXACT;
    c->has_params[f] = 0;
    c->band[f] = nullptr;
    c->band_ok[f] = 0;
    c->aspect[f] = 0.0;
  }
  c->gpart = c->gout = c->epts = c->eout = c->tables = nullptr;
  c->mesh = (float4 *)(c->base + lay.mesh);
  c->mesh_rc = c->mesh_rin = 0.0;
  c->mesh_particles = false;
  c->pool = nullptr;
  if (cfg->learned) {
    for (int f = 0; f < NFAM; ++f) {
      c->theta[f] = (float *)(c->base + lay.theta[f]);
      c->mom1[f] = (float *)(c->base + lay.mom1[f]);
      c->mom2[f] = (float *)(c->base + lay.mom2[f]);
      c->packed[f] = (__bf16 *)(c->base + lay.packed[f]);
    }
    c->gpart = (float *)(c->base + lay.gpart);
    c->gout = (float *)(c->base + lay.gout);
    c->pool = (float4 *)(c->base + lay.pool);
    c->epts = (float *)(c->base + lay.epts);
    c->eout = (float *)(c->base + lay.eout);
  }
  if (cfg->learned || cfg->max_mesh_triangles > 0) {
    c->tables = (float *)(c->base + lay.tables);
    for (int f = 0; f < NFAM; ++f) c->band[f] = (float *)(c->base + lay.band[f]);
    c->L.tables = c->tables;
    c->L.table_cap = lay.table_cap;
  }
  // rest state: every deviation f_i - w_i is zero
  hipError_t e = hipMemsetAsync(c->fA, 0, (size_t)19 * L.N * pop_bytes(cfg->precision), c->stream);
  if (e == hipSuccess) e = launch_fill_int(c->tcnt[0], 0, L.ntiles, c->stream);
  if (e == hipSuccess) e = launch_fill_int(c->tcnt[1], 0, L.ntiles, c->stream);
  if (e == hipSuccess) e = launch_fill_int(c->status, 0, 1, c->stream);
  if (e == hipSuccess) e = launch_fill_int(c->ccnt, 0, std::max(cfg->max_particles, 1), c->stream);
  // surface-node directions of the non-spherical contact: a Fibonacci lattice
  // on the unit sphere, z_m = 1 - (2 m + 1) / M, azimuth m times the golden
  // angle pi (3 - sqrt 5)
  std::vector<double> dirs((size_t)3 * CONTACT_NODES);
  for (int m = 0; m < CONTACT_NODES; ++m) {
    const double z = 1.0 - (2.0 * m + 1.0) / CONTACT_NODES, r = sqrt(std::max(0.0, 1.0 - z * z));
    const double ph = m * (M_PI * (3.0 - sqrt(5.0)));
    dirs[3 * m] = r * cos(ph);
    dirs[3 * m + 1] = r * sin(ph);
    dirs[3 * m + 2] = z;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->cdirs, dirs.data(), sizeof(double) * dirs.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return fail(HLBM_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
  }
  c->binned = true;
  *out = c;
  return HLBM_OK;
}

int hlbm_destroy(hlbm_ctx *ctx) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  delete ctx;
  return HLBM_OK;
}

int hlbm_profile_begin(hlbm_ctx *ctx) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  ctx->profiling = true;
  ctx->events_used = 0;
  return HLBM_OK;
}

int hlbm_profile_end(hlbm_ctx *ctx, double *collide_ms, int64_t *launches) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (!ctx->profiling) return fail(HLBM_ESTATE, "profiling was not started");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  double total = 0.0;
  for (size_t k = 0; k + 1 < ctx->events_used; k += 2) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->events[k], ctx->events[k + 1]));
    total += ms;
  }
  if (collide_ms) *collide_ms = total;
  if (launches) *launches = (int64_t)(ctx->events_used / 2);
  ctx->profiling = false;
  ctx->events_used = 0;
  return HLBM_OK;
}

int hlbm_num_particles(const hlbm_ctx *ctx, int32_t *n) {
  if (!ctx || !n) return fail(HLBM_EINVAL, "NULL argument");
  *n = ctx->n;
  return HLBM_OK;
}

int hlbm_set_particles(hlbm_ctx *ctx, int32_t n, const hlbm_particle *host) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (n < 0 || n > ctx->cfg.max_particles)
    return fail(HLBM_EINVAL, "n = %d outside [0, max_particles = %d]", n, ctx->cfg.max_particles);
  if (n > 0 && !host) return fail(HLBM_EINVAL, "particles is NULL");
  const int nn[3] = {ctx->cfg.nx, ctx->cfg.ny, ctx->cfg.nz};
  int cap = 1, lmax = 1;
  double wmax = 0.0;
  for (int i = 0; i < n; ++i) {
    const hlbm_particle &p = host[i];
    const double *vals[] = {p.pos, p.quat, p.vel, p.omega, p.inertia, p.param};
    const int lens[] = {3, 4, 3, 3, 3, 3};
    for (int a = 0; a < 6; ++a)
      for (int k = 0; k < lens[a]; ++k)
        if (!isfinite(vals[a][k])) return fail(HLBM_EINVAL, "particle %d: non-finite value", i);
    if (!isfinite(p.mass) || !isfinite(p.volume)) return fail(HLBM_EINVAL, "particle %d: non-finite mass", i);
    if (!(p.volume > 0.0)) return fail(HLBM_EINVAL, "particle %d: volume must be > 0", i);
    if (p.shape < HLBM_SPHERE || p.shape > HLBM_MESH) return fail(HLBM_EINVAL, "particle %d: bad shape", i);
    if (p.shape == HLBM_MESH && ctx->L.mesh_nt == 0)
      return fail(HLBM_ESTATE, "particle %d: HLBM_MESH particle but no mesh (hlbm_set_mesh)", i);
    if (p.flags != 0) return fail(HLBM_EINVAL, "particle %d: flags must be 0", i);
    const double qn = sqrt(p.quat[0] * p.quat[0] + p.quat[1] * p.quat[1] + p.quat[2] * p.quat[2] +
                           p.quat[3] * p.quat[3]);
    if (fabs(qn - 1.0) > 1e-6) return fail(HLBM_EINVAL, "particle %d: quaternion not unit", i);
    if (p.mass > 0 && !(p.inertia[0] > 0 && p.inertia[1] > 0 && p.inertia[2] > 0))
      return fail(HLBM_EINVAL, "particle %d: inertia must be > 0", i);
    double rc;
    if (p.shape == HLBM_SPHERE) {
      if (!(p.param[0] > 0)) return fail(HLBM_EINVAL, "particle %d: radius must be > 0", i);
      rc = p.param[0];
    } else if (p.shape == HLBM_ROUNDED_CUBE) {
      if (!(p.param[0] > 0 && p.param[1] >= 0 && p.param[1] <= p.param[0]))
        return fail(HLBM_EINVAL, "particle %d: need h > 0 and 0 <= r_c <= h", i);
      rc = sqrt(3.0) * (p.param[0] - p.param[1]) + p.param[1];
    } else if (p.shape == HLBM_SPHEROID) {
      if (!(p.param[0] > 0 && p.param[1] > 0)) return fail(HLBM_EINVAL, "particle %d: semi-axes must be > 0", i);
      rc = fmax(p.param[0], p.param[1]);
    } else {
      if (!(p.param[0] > 0)) return fail(HLBM_EINVAL, "particle %d: mesh scale must be > 0", i);
      rc = p.param[0] * ctx->mesh_rc;
    }
    wmax = std::max(wmax, rc);
    const double reach = rc + fmax(0.5 * ctx->cfg.eps, sqrt(2.0)) + 1.0;
    for (int k = 0; k < 3; ++k) {
      if (ctx->cfg.bc[k] == HLBM_BC_PERIODIC && 2.0 * reach >= nn[k])
        return fail(HLBM_EINVAL, "particle %d: reach %.3f not below half of periodic extent %d", i, reach, nn[k]);
      if (ctx->cfg.bc[k] == HLBM_BC_WALL && !(p.pos[k] >= 0 && p.pos[k] <= nn[k]))
        return fail(HLBM_EINVAL, "particle %d: centre outside the walls", i);
    }
    // the coupling box spans at most floor(2 (rc + eps/2)) + 1 cells per axis;
    // the binning handles up to MAX_AXIS_TILES tiles of 4 cells per axis
    const int cells = (int)floor(2.0 * (rc + 0.5 * ctx->cfg.eps)) + 2;
    if (cells / TY + 2 > MAX_AXIS_TILES)
      return fail(HLBM_EUNSUPPORTED, "particle %d: circumradius too large for the tile binning", i);
    const int tiles_x = std::min(ctx->L.ntx, cells / TX + 2);
    const int tiles_y = std::min(ctx->L.nty, cells / TY + 2);
    const int tiles_z = std::min(ctx->L.ntz, cells / TZ + 2);
    cap = std::max(cap, tiles_x * tiles_y * tiles_z);
    lmax = std::max(lmax, (int)floor(2.0 * rc) + 2);
    if ((ctx->cfg.learned || p.shape == HLBM_MESH) && p.shape != HLBM_SPHERE &&
        rc > ctx->cfg.learned_max_circumradius)
      return fail(HLBM_EINVAL, "particle %d: circumradius %.3f above learned_max_circumradius (table size)", i, rc);
  }
  if (lmax > LMAX_CAP) return fail(HLBM_EUNSUPPORTED, "circumradius too large");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  // Order in which the momentum-exchange workgroups visit the particles.  Few
  // particles: (z, y, x) order of their centres, slab-major dispatch (the
  // exchange is bound by latency; the resident workgroups spread over the
  // whole lattice).  Many particles: Morton order of the 64 x 16 x 16-cell
  // blocks holding the centres, each XCD on a contiguous run of it, so that
  // particles whose boxes share rows of a population plane are read through
  // one L2 (the exchange is bound by HBM traffic; measured on 11 265
  // particles: 4.8 -> 3.6 GB per step in an LRU model, -9 % time).  Any
  // order gives the same result.
  const bool chunked = n >= MEA_CHUNKED_MIN;
  std::vector<unsigned long long> key(n);
  auto spread = [](unsigned v) {
    unsigned long long r = 0;
    for (int b = 0; b < 21; ++b) r |= (unsigned long long)((v >> b) & 1u) << (3 * b);
    return r;
  };
  for (int i = 0; i < n; ++i) {
    const double *X = host[i].pos;
    const unsigned bx = (unsigned)std::max(0.0, floor(X[0] / 64.0));
    const unsigned by = (unsigned)std::max(0.0, floor(X[1] / 16.0));
    const unsigned bz = (unsigned)std::max(0.0, floor(X[2] / 16.0));
    key[i] = spread(bx) | (spread(by) << 1) | (spread(bz) << 2);
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [host, chunked, &key](int a, int b) {
    if (chunked) return key[a] != key[b] ? key[a] < key[b] : a < b;
    const double *pa = host[a].pos, *pb = host[b].pos;
    if (floor(pa[2]) != floor(pb[2])) return pa[2] < pb[2];
    if (floor(pa[1]) != floor(pb[1])) return pa[1] < pb[1];
    if (pa[0] != pb[0]) return pa[0] < pb[0];
    return a < b;
  });
  // mesh particles carry scale x (largest vertex radius, least surface
  // distance from the centre) in param[1], param[2]
  std::vector<hlbm_particle> staged(host, host + n);
  for (auto &p : staged)
    if (p.shape == HLBM_MESH) {
      p.param[1] = p.param[0] * ctx->mesh_rc;
      p.param[2] = p.param[0] * ctx->mesh_rin;
    }
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(ctx->stage_parts, staged.data(), sizeof(hlbm_particle) * n, hipMemcpyHostToDevice,
                           ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_prepare(ctx->L, ctx->stage_parts, ctx->parts, n, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));  // the host copies above are released on return
  }
  ctx->n = n;
  ctx->mesh_particles = false;
  ctx->nonspherical = false;
  for (int i = 0; i < n; ++i) {
    ctx->mesh_particles |= host[i].shape == HLBM_MESH;
    ctx->nonspherical |= host[i].shape != HLBM_SPHERE;
  }
  ctx->mea_chunked = chunked ? 1 : 0;
  ctx->bin_cap = cap;
  ctx->lmax = lmax;
  ctx->cwmax = wmax;
  int rc = rebin(ctx);
  if (rc) return rc;
  rc = mark_learned(ctx);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return check_status(ctx);
}

int hlbm_set_fields(hlbm_ctx *ctx, const double *rho, const double *u) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  const long long N = ctx->L.N;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const double *drho = nullptr, *du = nullptr;
  if (rho) {
    HIP_TRY(hipMemcpyAsync(ctx->stage, rho, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    drho = ctx->stage;
  }
  if (u) {
    HIP_TRY(hipMemcpyAsync(ctx->stage + N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, ctx->stream));
    du = ctx->stage + N;
  }
  HIP_TRY(launch_set_fields(ctx->cfg.precision, ctx->L, ctx->fA, drho, du, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return HLBM_OK;
}

int hlbm_step(hlbm_ctx *ctx, int32_t nsteps) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(HLBM_EINVAL, "nsteps < 0");
  const int prec = ctx->cfg.precision;
  hipStream_t s = ctx->stream;
  for (int it = 0; it < nsteps; ++it) {
    const int nxt = 1 - ctx->cur;
    if (ctx->n > 0) {
      // momentum exchange on the state of time t, then Newton-Euler -> t+1 and
      // binning of the updated particles into the other tile-list buffer
      // (slabs of 2 z-layers per workgroup for few particles, 4 for many:
      // enough workgroups to fill the chip, few enough to amortise each)
      const int layers = ctx->n >= 1000 ? 4 : 2;
      HIP_TRY(launch_mea(prec, ctx->L, ctx->fA, ctx->parts, ctx->order, ctx->n, ctx->lmax, layers, ctx->mea_chunked,
                         ctx->partial, s));
      if (ctx->cparams.on) {
        // grid cells at least the largest pair reach 2 w_max + range wide
        ContactGrid cg;
        const double reach = 2.0 * ctx->cwmax + ctx->cparams.range;
        const int nn[3] = {ctx->cfg.nx, ctx->cfg.ny, ctx->cfg.nz};
        for (int a = 0; a < 3; ++a) {
          cg.g[a] = std::max(1, std::min(CGRID_AXIS, (int)floor(nn[a] / reach)));
          cg.size[a] = (double)nn[a] / cg.g[a];
        }
        HIP_TRY(launch_contact(ctx->L, ctx->parts, ctx->n, ctx->cparams, cg, ctx->cwork, ctx->contact, ctx->ccand,
                               ctx->ccnt, ctx->status, s));
      }
      const bool shapes = ctx->cparams.on && ctx->nonspherical;
      if (shapes)
        HIP_TRY(launch_contact_shapes(ctx->L, ctx->parts, ctx->n, ctx->cparams, ctx->cdirs, ctx->ccand, ctx->ccnt,
                                      ctx->cshapes, s));
      HIP_TRY(launch_eom_bin(ctx->L, ctx->parts, ctx->n, ctx->lmax, layers, ctx->partial, ctx->cparams,
                             ctx->contact, shapes ? ctx->cshapes : nullptr, ctx->tcnt[nxt], ctx->tlist[nxt],
                             ctx->status, s));
      int rc = refresh_tables(ctx);
      if (rc) return rc;
    }
    const int use = ctx->n > 0 ? nxt : ctx->cur;
    int *clear = ctx->n > 0 ? ctx->tcnt[ctx->cur] : nullptr;
    if (ctx->profiling) {
      while (ctx->events.size() < ctx->events_used + 2) {
        hipEvent_t e;
        // timing-only events: no system-scope fence (no cache writeback and
        // invalidation between the launches they bracket)
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        ctx->events.push_back(e);
      }
      HIP_TRY(hipEventRecord(ctx->events[ctx->events_used], s));
    }
    HIP_TRY(launch_collide(prec, ctx->L, ctx->fA, ctx->fB, ctx->parts, ctx->tcnt[use], ctx->tlist[use], clear,
                           ctx->status, s));
    ctx->cur = use;
    if (ctx->profiling) {
      HIP_TRY(hipEventRecord(ctx->events[ctx->events_used + 1], s));
      ctx->events_used += 2;
    }
    void *t = ctx->fA;
    ctx->fA = ctx->fB;
    ctx->fB = t;
    ctx->steps_done++;
  }
  return HLBM_OK;
}

namespace {
// host geometry of the mesh: least distance of a triangle from the origin and
// the triangle's solid angle seen from the origin
double h_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void h_cross(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
double h_seg_dist2(const double *a, const double *b) {  // from the origin
  const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double t = -h_dot(a, ab) / h_dot(ab, ab);
  t = t < 0 ? 0 : (t > 1 ? 1 : t);
  const double d[3] = {a[0] + t * ab[0], a[1] + t * ab[1], a[2] + t * ab[2]};
  return h_dot(d, d);
}
double h_tri_dist2(const double *a, const double *b, const double *c) {
  const double e0[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e1[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  double n[3];
  h_cross(e0, e1, n);
  const double nn = h_dot(n, n), h = -h_dot(a, n) / nn;
  const double f[3] = {-a[0] - h * n[0], -a[1] - h * n[1], -a[2] - h * n[2]};
  const double d00 = h_dot(e0, e0), d01 = h_dot(e0, e1), d11 = h_dot(e1, e1);
  const double f0 = h_dot(f, e0), f1 = h_dot(f, e1), den = d00 * d11 - d01 * d01;
  const double u = (d11 * f0 - d01 * f1) / den, v = (d00 * f1 - d01 * f0) / den;
  if (u >= 0 && v >= 0 && u + v <= 1) return h * h * nn;
  return std::min(h_seg_dist2(a, b), std::min(h_seg_dist2(b, c), h_seg_dist2(c, a)));
}
double h_solid_angle(const double *a, const double *b, const double *c) {
  double bxc[3];
  h_cross(b, c, bxc);
  const double la = sqrt(h_dot(a, a)), lb = sqrt(h_dot(b, b)), lc = sqrt(h_dot(c, c));
  return 2.0 * atan2(h_dot(a, bxc), la * lb * lc + h_dot(a, b) * lc + h_dot(a, c) * lb + h_dot(b, c) * la);
}
}  // namespace

int hlbm_set_mesh(hlbm_ctx *ctx, const float *vertices, int32_t nv, const int32_t *triangles, int32_t nt) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (!vertices || !triangles) return fail(HLBM_EINVAL, "NULL argument");
  if (ctx->n > 0) return fail(HLBM_ESTATE, "set the mesh before the particles");
  if (nv < 4 || nt < 4) return fail(HLBM_EINVAL, "a closed mesh needs >= 4 vertices and triangles");
  if (nt > ctx->cfg.max_mesh_triangles)
    return fail(HLBM_EUNSUPPORTED, "%d triangles above max_mesh_triangles = %d", nt, ctx->cfg.max_mesh_triangles);
  for (int k = 0; k < 3 * nv; ++k)
    if (!isfinite(vertices[k])) return fail(HLBM_EINVAL, "vertex coordinate %d not finite", k);
  std::vector<float4> tri((size_t)3 * nt);
  double rc = 0.0, rin2 = 1e300, omega = 0.0;
  for (int t = 0; t < nt; ++t) {
    double v[3][3];
    for (int j = 0; j < 3; ++j) {
      const int id = triangles[3 * t + j];
      if (id < 0 || id >= nv) return fail(HLBM_EINVAL, "triangle %d: vertex index %d out of range", t, id);
      for (int k = 0; k < 3; ++k) v[j][k] = (double)vertices[3 * id + k];
      tri[3 * t + j] = make_float4(vertices[3 * id], vertices[3 * id + 1], vertices[3 * id + 2], 0.f);
      rc = std::max(rc, sqrt(h_dot(v[j], v[j])));
    }
    rin2 = std::min(rin2, h_tri_dist2(v[0], v[1], v[2]));
    omega += h_solid_angle(v[0], v[1], v[2]);
  }
  // winding number of the origin: 1 for a closed, outward-oriented mesh around it
  if (!(fabs(omega / (4.0 * M_PI) - 1.0) < 1e-3))
    return fail(HLBM_EINVAL, "the mesh must be closed, enclose the origin and be counter-clockwise seen from outside "
                             "(winding number of the origin %.4f)", omega / (4.0 * M_PI));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpy(ctx->mesh, tri.data(), sizeof(float4) * tri.size(), hipMemcpyHostToDevice));
  ctx->L.mesh = ctx->mesh;
  ctx->L.mesh_nt = nt;
  ctx->mesh_rc = rc;
  ctx->mesh_rin = sqrt(rin2);
  // band grid of the mesh at unit circumradius (scale 1 / rc)
  HIP_TRY(band_grid(HLBM_MESH, 1.0 / rc, 0.0, ctx->mesh, nt, ctx->band[2], ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->band_ok[2] = 1;
  return HLBM_OK;
}

int hlbm_set_fluid_accel(hlbm_ctx *ctx, const double accel[3]) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (!accel) return fail(HLBM_EINVAL, "accel is NULL");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(accel[k])) return fail(HLBM_EINVAL, "fluid acceleration not finite");
  // the lattice descriptor is passed by value at each launch, so the new
  // value applies from the next queued step on
  for (int k = 0; k < 3; ++k) {
    ctx->cfg.fluid_accel[k] = accel[k];
    ctx->L.af[k] = accel[k];
  }
  return HLBM_OK;
}

int hlbm_set_contact(hlbm_ctx *ctx, double range, double stiffness, double wall_stiffness) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (!(isfinite(range) && isfinite(stiffness) && isfinite(wall_stiffness)))
    return fail(HLBM_EINVAL, "contact parameters not finite");
  if (range < 0.0 || stiffness < 0.0 || wall_stiffness < 0.0)
    return fail(HLBM_EINVAL, "contact range and stiffnesses must be >= 0");
  // passed by value at each launch: applies from the next queued step on
  ctx->cparams = ContactParams{range, stiffness, wall_stiffness,
                               range > 0.0 && (stiffness > 0.0 || wall_stiffness > 0.0) ? 1 : 0};
  return HLBM_OK;
}

int hlbm_get_forces(hlbm_ctx *ctx, double *F, double *T, hlbm_particle *state) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  int rc = check_status(ctx);
  if (rc) return rc;
  if (ctx->n == 0) return HLBM_OK;
  std::vector<DevParticle> p(ctx->n);
  HIP_TRY(hipMemcpy(p.data(), ctx->parts, sizeof(DevParticle) * ctx->n, hipMemcpyDeviceToHost));
  for (int i = 0; i < ctx->n; ++i) {
    for (int k = 0; k < 3; ++k) {
      if (F) F[3 * i + k] = p[i].Fh[k];
      if (T) T[3 * i + k] = p[i].Th[k];
    }
    if (state) {
      hlbm_particle &o = state[i];
      for (int k = 0; k < 3; ++k) {
        o.pos[k] = p[i].X[k]; o.vel[k] = p[i].U[k]; o.omega[k] = p[i].W[k];
        o.inertia[k] = p[i].I[k]; o.param[k] = p[i].prm[k];
      }
      for (int k = 0; k < 4; ++k) o.quat[k] = p[i].q[k];
      o.mass = p[i].m;
      o.volume = p[i].V;
      o.shape = p[i].shape;
      o.flags = p[i].flags;
    }
  }
  return HLBM_OK;
}

int hlbm_get_fields(hlbm_ctx *ctx, uint32_t mask, int32_t dtype, void *out, int32_t out_on_device) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (mask == 0 || (mask & ~15u)) return fail(HLBM_EINVAL, "mask must select fields 1|2|4|8");
  if (dtype != HLBM_FP64 && dtype != HLBM_FP32) return fail(HLBM_EINVAL, "dtype must be HLBM_FP64 or HLBM_FP32");
  if (!out) return fail(HLBM_EINVAL, "out is NULL");
  int rc = check_status(ctx);
  if (rc) return rc;
  if (!ctx->binned) {
    rc = rebin(ctx);
    if (rc) return rc;
  }
  const long long N = ctx->L.N;
  const int f32 = dtype == HLBM_FP32 ? 1 : 0;
  const size_t esize = f32 ? sizeof(float) : sizeof(double);
  if (out_on_device) {
    HIP_TRY(launch_fields(ctx->cfg.precision, ctx->L, ctx->fA, ctx->parts, ctx->tcnt[ctx->cur],
                          ctx->tlist[ctx->cur], mask, f32, out, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return check_status(ctx);
  }
  // host output: at most four FP64 planes fit the staging area at a time
  const unsigned bits[4] = {1u, 2u, 4u, 8u};
  const int width[4] = {1, 3, 3, 1};
  long long plane = 0;
  for (int b = 0; b < 4; ++b) {
    if (!(mask & bits[b])) continue;
    HIP_TRY(launch_fields(ctx->cfg.precision, ctx->L, ctx->fA, ctx->parts, ctx->tcnt[ctx->cur],
                          ctx->tlist[ctx->cur], bits[b], f32, ctx->stage, ctx->stream));
    HIP_TRY(hipMemcpyAsync((char *)out + (size_t)plane * N * esize, ctx->stage, esize * N * width[b],
                           hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    plane += width[b];
  }
  return check_status(ctx);
}

int hlbm_get_mean_velocity(hlbm_ctx *ctx, double *mean_u_phys, double *mean_fluid_u_phys, int64_t *fluid_cells) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  int rc = check_status(ctx);
  if (rc) return rc;
  if (!ctx->binned) {
    rc = rebin(ctx);
    if (rc) return rc;
  }
  // tile records in the staging area (ntiles x 7 doubles <= 4 N), sums after them
  double *partial = ctx->stage;
  double *sums = ctx->stage + (size_t)ctx->L.ntiles * 7;
  HIP_TRY(launch_mean_velocity(ctx->cfg.precision, ctx->L, ctx->fA, ctx->parts, ctx->tcnt[ctx->cur],
                               ctx->tlist[ctx->cur], partial, sums, ctx->stream));
  double h[7];
  HIP_TRY(hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  rc = check_status(ctx);
  if (rc) return rc;
  const double N = (double)ctx->L.N;
  for (int k = 0; k < 3; ++k) {
    if (mean_u_phys) mean_u_phys[k] = h[k] / N;
    if (mean_fluid_u_phys) mean_fluid_u_phys[k] = h[6] > 0.0 ? h[3 + k] / h[6] : 0.0;
  }
  if (fluid_cells) *fluid_cells = (int64_t)h[6];
  return HLBM_OK;
}


// ---------------------------------------------------------------------------
// Learned indicator
// ---------------------------------------------------------------------------
static int family(hlbm_ctx *ctx, int32_t shape, int *f) {
  if (!ctx) return fail(HLBM_EINVAL, "ctx is NULL");
  if (!ctx->cfg.learned) return fail(HLBM_ESTATE, "the context was created without cfg.learned");
  if (shape != HLBM_ROUNDED_CUBE && shape != HLBM_SPHEROID && shape != HLBM_MESH)
    return fail(HLBM_EINVAL, "learned indicators exist for HLBM_ROUNDED_CUBE, HLBM_SPHEROID and HLBM_MESH");
  *f = shape - 1;
  return HLBM_OK;
}

// Host-side check that the device regions the training kernels of family f
// write and read lie inside the workspace and do not overlap: parameters,
// Adam moments, packed BF16 tiles (k_mlp_pack writes MLP_PACKED_BYTES), the
// gradient partials of up to MLP_MAX_BLOCKS workgroups, the reduced gradient
// and the sample pool of `samples` entries.
static int check_training_regions(const hlbm_ctx *ctx, int f, long long samples) {
  struct Region {
    const char *name;
    const char *p;
    size_t bytes;
  };
  const Region r[] = {
      {"theta", (const char *)ctx->theta[f], MLP_PARTIAL * sizeof(float)},
      {"mom1", (const char *)ctx->mom1[f], MLP_PARTIAL * sizeof(float)},
      {"mom2", (const char *)ctx->mom2[f], MLP_PARTIAL * sizeof(float)},
      {"packed", (const char *)ctx->packed[f], (size_t)MLP_PACKED_BYTES},
      {"gpart", (const char *)ctx->gpart, (size_t)MLP_MAX_BLOCKS * MLP_PARTIAL * sizeof(float)},
      {"gout", (const char *)ctx->gout, MLP_PARTIAL * sizeof(float)},
      {"pool", (const char *)ctx->pool, (size_t)samples * sizeof(float4)},
  };
  const int nr = (int)(sizeof r / sizeof r[0]);
  const char *lo = ctx->base, *hi = ctx->base + ctx->lay.total - 256;
  if (samples > ctx->lay.pool_cap) return fail(HLBM_EINVAL, "%lld samples above the pool capacity", samples);
  for (int a = 0; a < nr; ++a) {
    if (!r[a].p || r[a].p < lo || r[a].p + r[a].bytes > hi)
      return fail(HLBM_EDEVICE, "training region %s outside the workspace", r[a].name);
    for (int b = 0; b < a; ++b)
      if (r[a].p < r[b].p + r[b].bytes && r[b].p < r[a].p + r[a].bytes)
        return fail(HLBM_EDEVICE, "training regions %s and %s overlap", r[a].name, r[b].name);
  }
  return HLBM_OK;
}

static double circumradius_host(const hlbm_ctx *ctx, int shape, const double *prm) {
  if (shape == HLBM_ROUNDED_CUBE) return sqrt(3.0) * (prm[0] - prm[1]) + prm[1];
  if (shape == HLBM_SPHEROID) return fmax(prm[0], prm[1]);
  if (shape == HLBM_MESH) return prm[0] * ctx->mesh_rc;
  return prm[0];
}

int hlbm_mlp_set_params(hlbm_ctx *ctx, int32_t shape, const float *theta) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (!theta) return fail(HLBM_EINVAL, "theta is NULL");
  for (int k = 0; k < MLP_NPARAM; ++k)
    if (!isfinite(theta[k])) return fail(HLBM_EINVAL, "theta[%d] not finite", k);
  rc = check_training_regions(ctx, f, 0);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->theta[f], theta, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(launch_fill_int((int *)ctx->mom1[f], 0, MLP_PARTIAL, ctx->stream));
  HIP_TRY(launch_fill_int((int *)ctx->mom2[f], 0, MLP_PARTIAL, ctx->stream));
  HIP_TRY(mlp_pack(ctx->theta[f], ctx->packed[f], ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->has_params[f] = 1;
  return refresh_tables(ctx);
}

int hlbm_mlp_get_params(hlbm_ctx *ctx, int32_t shape, float *theta) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (!theta) return fail(HLBM_EINVAL, "theta is NULL");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpy(theta, ctx->theta[f], sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  return HLBM_OK;
}

int hlbm_mlp_eval(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, double *out) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (n < 0 || n > ctx->lay.pool_cap) return fail(HLBM_EINVAL, "n outside [0, %lld]", ctx->lay.pool_cap);
  if (n == 0) return HLBM_OK;
  if (!pts || !out) return fail(HLBM_EINVAL, "NULL buffer");
  if (!ctx->has_params[f]) return fail(HLBM_ESTATE, "no parameters for this family");
  std::vector<float> p((size_t)3 * n), o(n);
  for (long long k = 0; k < 3LL * n; ++k) p[k] = (float)pts[k];
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->epts, p.data(), sizeof(float) * 3 * n, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(mlp_eval(ctx->theta[f], ctx->packed[f], ctx->epts, ctx->eout, n, ctx->stream));
  HIP_TRY(hipMemcpyAsync(o.data(), ctx->eout, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < n; ++k) out[k] = o[k];
  return HLBM_OK;
}

int hlbm_mlp_gradient(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, const double *target,
                      double *grad, double *loss) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (n < 1 || n > ctx->lay.pool_cap) return fail(HLBM_EINVAL, "n outside [1, %lld]", ctx->lay.pool_cap);
  if (!pts || !target || !grad) return fail(HLBM_EINVAL, "NULL buffer");
  if (!ctx->has_params[f]) return fail(HLBM_ESTATE, "no parameters for this family");
  rc = check_training_regions(ctx, f, n);
  if (rc) return rc;
  std::vector<float4> smp(n);
  for (int k = 0; k < n; ++k)
    smp[k] = make_float4((float)pts[3 * k], (float)pts[3 * k + 1], (float)pts[3 * k + 2], (float)target[k]);
  std::vector<float> g(MLP_PARTIAL);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->pool, smp.data(), sizeof(float4) * n, hipMemcpyHostToDevice, ctx->stream));
  const int nb = mlp_grad_blocks(n, MLP_MAX_BLOCKS);
  HIP_TRY(mlp_grad(ctx->theta[f], ctx->packed[f], ctx->pool, n, MLP_MAX_BLOCKS, 2.0f / n, ctx->gpart, ctx->stream));
  HIP_TRY(mlp_reduce_adam(ctx->theta[f], ctx->mom1[f], ctx->mom2[f], ctx->gpart, nb, ctx->gout, 0, 0.f, 1,
                          nullptr, ctx->stream));
  HIP_TRY(hipMemcpyAsync(g.data(), ctx->gout, sizeof(float) * MLP_PARTIAL, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < MLP_NPARAM; ++k) grad[k] = g[k];
  if (loss) *loss = g[MLP_NPARAM] / n;
  return HLBM_OK;
}

int hlbm_mlp_train_step(hlbm_ctx *ctx, int32_t shape, int32_t n, const double *pts, const double *target,
                        double lr, int32_t step, double *grad, double *loss) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (n < 1 || n > ctx->lay.pool_cap) return fail(HLBM_EINVAL, "n outside [1, %lld]", ctx->lay.pool_cap);
  if (!pts || !target) return fail(HLBM_EINVAL, "NULL buffer");
  if (!(lr > 0.0) || !isfinite(lr) || step < 1) return fail(HLBM_EINVAL, "need lr > 0 and step >= 1");
  if (!ctx->has_params[f]) return fail(HLBM_ESTATE, "no parameters for this family");
  rc = check_training_regions(ctx, f, n);
  if (rc) return rc;
  std::vector<float4> smp(n);
  for (int k = 0; k < n; ++k)
    smp[k] = make_float4((float)pts[3 * k], (float)pts[3 * k + 1], (float)pts[3 * k + 2], (float)target[k]);
  std::vector<float> g(MLP_PARTIAL);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->pool, smp.data(), sizeof(float4) * n, hipMemcpyHostToDevice, ctx->stream));
  const int nb = mlp_grad_blocks(n, MLP_MAX_BLOCKS);
  HIP_TRY(mlp_grad(ctx->theta[f], ctx->packed[f], ctx->pool, n, MLP_MAX_BLOCKS, 2.0f / n, ctx->gpart, ctx->stream));
  HIP_TRY(mlp_reduce_adam(ctx->theta[f], ctx->mom1[f], ctx->mom2[f], ctx->gpart, nb, ctx->gout, 1, (float)lr, step,
                          ctx->packed[f], ctx->stream));
  HIP_TRY(hipMemcpyAsync(g.data(), ctx->gout, sizeof(float) * MLP_PARTIAL, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (grad)
    for (int k = 0; k < MLP_NPARAM; ++k) grad[k] = g[k];
  if (loss) *loss = g[MLP_NPARAM] / n;
  return refresh_tables(ctx);
}

int hlbm_mlp_samples(hlbm_ctx *ctx, int32_t shape, const double *param, uint64_t seed, int32_t n, double box,
                     double band, double clip, double band_share, double *out) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (!param || !out) return fail(HLBM_EINVAL, "NULL argument");
  if (n < 1 || n > ctx->lay.pool_cap) return fail(HLBM_EINVAL, "n outside [1, %lld]", ctx->lay.pool_cap);
  if (shape == HLBM_MESH) {
    if (ctx->L.mesh_nt == 0) return fail(HLBM_ESTATE, "no mesh (hlbm_set_mesh)");
    if (!(param[0] > 0)) return fail(HLBM_EINVAL, "bad shape parameters");
  } else if (!(param[0] > 0 && param[1] > 0) || (shape == HLBM_ROUNDED_CUBE && param[1] > param[0])) {
    return fail(HLBM_EINVAL, "bad shape parameters");
  }
  if (!(box > 0 && band > 0 && clip >= band && band_share >= 0 && band_share <= 1))
    return fail(HLBM_EINVAL, "bad box / band / clip / band_share");
  const double Rc = circumradius_host(ctx, shape, param);
  std::vector<float4> h(n);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(mlp_samples(shape, param[0] / Rc, param[1] / Rc, ctx->L.mesh, ctx->L.mesh_nt, seed, n, box, band, clip,
                      band_share, ctx->pool, ctx->stream));
  HIP_TRY(hipMemcpyAsync(h.data(), ctx->pool, sizeof(float4) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < n; ++k) {
    out[4 * k] = h[k].x; out[4 * k + 1] = h[k].y; out[4 * k + 2] = h[k].z; out[4 * k + 3] = h[k].w;
  }
  return HLBM_OK;
}

int hlbm_train_indicator(hlbm_ctx *ctx, int32_t shape, const double *param, const hlbm_train_opts *o,
                         hlbm_train_report *rep) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (!param || !o) return fail(HLBM_EINVAL, "NULL argument");
  if (!ctx->has_params[f]) return fail(HLBM_ESTATE, "set initial parameters first (hlbm_mlp_set_params)");
  if (shape == HLBM_MESH) {
    if (ctx->L.mesh_nt == 0) return fail(HLBM_ESTATE, "no mesh (hlbm_set_mesh)");
    if (!(param[0] > 0)) return fail(HLBM_EINVAL, "bad shape parameters");
  } else if (!(param[0] > 0 && param[1] > 0) || (shape == HLBM_ROUNDED_CUBE && param[1] > param[0])) {
    return fail(HLBM_EINVAL, "bad shape parameters");
  }
  if (o->samples < 64 || o->holdout < 1 || (long long)o->samples + o->holdout > ctx->lay.pool_cap)
    return fail(HLBM_EINVAL, "samples + holdout must fit the sample capacity %lld", ctx->lay.pool_cap);
  if (o->batch < 32 || o->batch > o->samples || o->iterations < 1)
    return fail(HLBM_EINVAL, "need 32 <= batch <= samples and iterations >= 1");
  if (!(o->lr > 0 && o->lr_final > 0 && o->box > 0 && o->band > 0 && o->clip >= o->band &&
        o->band_share >= 0 && o->band_share <= 1))
    return fail(HLBM_EINVAL, "bad learning rate / box / band / clip");
  rc = check_training_regions(ctx, f, (long long)o->samples + o->holdout);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  const double Rc = circumradius_host(ctx, shape, param);
  const double p0 = param[0] / Rc, p1 = param[1] / Rc;
  hipStream_t s = ctx->stream;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(mlp_samples(shape, p0, p1, ctx->L.mesh, ctx->L.mesh_nt, o->seed, o->samples, o->box, o->band, o->clip,
                      o->band_share, ctx->pool, s));
  HIP_TRY(mlp_samples(shape, p0, p1, ctx->L.mesh, ctx->L.mesh_nt, o->seed ^ 0x5bd1e995ull, o->holdout, o->box,
                      o->band, o->clip, 1.0, ctx->pool + o->samples, s));
  HIP_TRY(launch_fill_int((int *)ctx->mom1[f], 0, MLP_PARTIAL, s));
  HIP_TRY(launch_fill_int((int *)ctx->mom2[f], 0, MLP_PARTIAL, s));
  const int nbatches = o->samples / o->batch;
  const int nb = mlp_grad_blocks(o->batch, MLP_MAX_BLOCKS);
  double loss_first = 0, loss_last = 0;
  for (int it = 0; it < o->iterations; ++it) {
    const double frac = o->iterations > 1 ? (double)it / (o->iterations - 1) : 0.0;
    const float lr = (float)(o->lr * pow(o->lr_final / o->lr, frac));
    const float4 *batch = ctx->pool + (size_t)(it % nbatches) * o->batch;
    const bool record = it == 0 || it == o->iterations - 1;
    HIP_TRY(mlp_grad(ctx->theta[f], ctx->packed[f], batch, o->batch, MLP_MAX_BLOCKS, 2.0f / o->batch, ctx->gpart, s));
    HIP_TRY(mlp_reduce_adam(ctx->theta[f], ctx->mom1[f], ctx->mom2[f], ctx->gpart, nb, record ? ctx->gout : nullptr,
                            1, lr, it + 1, ctx->packed[f], s));
    if (record) {
      float sse = 0;
      HIP_TRY(hipMemcpyAsync(&sse, ctx->gout + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      (it == 0 ? loss_first : loss_last) = sse / o->batch;
    }
  }
  // held-out band samples
  std::vector<float4> hold(o->holdout);
  HIP_TRY(hipMemcpyAsync(hold.data(), ctx->pool + o->samples, sizeof(float4) * o->holdout, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<float> pts((size_t)3 * o->holdout), out(o->holdout);
  for (int k = 0; k < o->holdout; ++k) {
    pts[3 * k] = hold[k].x; pts[3 * k + 1] = hold[k].y; pts[3 * k + 2] = hold[k].z;
  }
  HIP_TRY(hipMemcpyAsync(ctx->epts, pts.data(), sizeof(float) * pts.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(mlp_eval(ctx->theta[f], ctx->packed[f], ctx->epts, ctx->eout, o->holdout, s));
  HIP_TRY(hipMemcpyAsync(out.data(), ctx->eout, sizeof(float) * o->holdout, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double ref = o->ref_circumradius > 0 ? o->ref_circumradius : Rc;
  double se = 0, mx = 0;
  for (int k = 0; k < o->holdout; ++k) {
    const double e = fabs((double)out[k] - (double)hold[k].w) * ref;
    se += e * e;
    mx = fmax(mx, e);
  }
  const double rms = sqrt(se / o->holdout);
  const bool ok = isfinite(rms) && rms <= o->gate_rms && mx <= o->gate_max;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) {
    rep->loss_first = loss_first;
    rep->loss_last = loss_last;
    rep->rms_err = rms;
    rep->max_err = mx;
    rep->train_ms = ms;
    rep->iterations = o->iterations;
    rep->accepted = ok ? 1 : 0;
  }
  // band grid of the trained shape (the same normalisation as the samples)
  HIP_TRY(band_grid(shape, p0, p1, ctx->L.mesh, ctx->L.mesh_nt, ctx->band[f], s));
  ctx->band_ok[f] = 1;
  // the mesh family's particles all have param[1] / param[0] = largest vertex radius
  ctx->aspect[f] = shape == HLBM_MESH ? ctx->mesh_rc : param[1] / param[0];
  ctx->mode[f] = ok ? HLBM_INDICATOR_LEARNED : HLBM_INDICATOR_EXACT;
  return mark_learned(ctx);
}

int hlbm_set_indicator(hlbm_ctx *ctx, int32_t shape, int32_t mode) {
  int f, rc = family(ctx, shape, &f);
  if (rc) return rc;
  if (mode != HLBM_INDICATOR_EXACT && mode != HLBM_INDICATOR_LEARNED) return fail(HLBM_EINVAL, "bad mode");
  if (mode == HLBM_INDICATOR_LEARNED && (!ctx->has_params[f] || !(ctx->aspect[f] > 0)))
    return fail(HLBM_ESTATE, "the family has no trained network (hlbm_train_indicator)");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->mode[f] = mode;
  rc = mark_learned(ctx);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return HLBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The surrogate-network gradient without a context and without allocation.
// Its working memory (the packed BF16 weight tiles and the per-workgroup
// gradient partials) is a fixed device array of this library, held by every
// GPU the library runs on until the process ends.  Host code never passes
// the array's name to a kernel: each device's copy is found once, with that
// device current, by hipGetSymbolAddress.
// ---------------------------------------------------------------------------
namespace {
// samples per call: at most NOALLOC_BLOCKS gradient workgroups of 32 samples,
// the partition hlbm_mlp_gradient takes for these sizes
constexpr int NOALLOC_BLOCKS = 64;
constexpr int NOALLOC_MAX_SAMPLES = NOALLOC_BLOCKS * 32;
constexpr size_t NOALLOC_PACKED_OFF = 0;
constexpr size_t NOALLOC_PARTIAL_OFF = ((size_t)MLP_PACKED_BYTES + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_PARTIAL_OFF + (size_t)NOALLOC_BLOCKS * MLP_PARTIAL * sizeof(float);
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mutex;
unsigned char *g_scratch[NOALLOC_MAX_DEVICES] = {};

// The current device's copy of the scratch array (found on first use).
int scratch_for_current_device(unsigned char **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HLBM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(HLBM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch[dev] = (unsigned char *)p;
  }
  *out = g_scratch[dev];
  return HLBM_OK;
}
}  // namespace

extern "C" int hlbm_mlp_gradient_noalloc(const float *d_theta, int32_t n, const float *d_samples, float *d_grad,
                                         void *stream) {
  if (!d_theta || !d_samples || !d_grad) return fail(HLBM_EINVAL, "NULL argument");
  if (n < 1 || n > NOALLOC_MAX_SAMPLES)
    return fail(HLBM_EUNSUPPORTED, "n = %d outside [1, %d] (fixed scratch)", n, NOALLOC_MAX_SAMPLES);
  const int nb = mlp_grad_blocks(n, MLP_MAX_BLOCKS);
  if (nb > NOALLOC_BLOCKS) return fail(HLBM_EUNSUPPORTED, "n = %d needs %d gradient workgroups", n, nb);
  unsigned char *base = nullptr;
  int rc = scratch_for_current_device(&base);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  __bf16 *packed = (__bf16 *)(base + NOALLOC_PACKED_OFF);
  float *partial = (float *)(base + NOALLOC_PARTIAL_OFF);
  HIP_TRY(mlp_pack(d_theta, packed, s));
  HIP_TRY(mlp_grad(d_theta, packed, (const float4 *)d_samples, n, MLP_MAX_BLOCKS, 2.0f / n, partial, s));
  // the reduction alone (no Adam step): parameters and moments are not touched
  HIP_TRY(mlp_reduce_adam(const_cast<float *>(d_theta), nullptr, nullptr, partial, nb, d_grad, 0, 0.f, 1, nullptr, s));
  return HLBM_OK;
}
