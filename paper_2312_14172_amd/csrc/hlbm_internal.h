// hlbm_internal.h -- host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hlbm.h"
#include "hlbm_device.h"

namespace hlbm {

hipError_t launch_prepare(const Lattice &L, const hlbm_particle *in, DevParticle *out, int n, hipStream_t s);
hipError_t launch_fill_int(int *p, int v, int n, hipStream_t s);
// learned-indicator families: 0 rounded cube, 1 spheroid, 2 mesh (shape - 1)
constexpr int NFAM = 3;
struct LearnedModes {
  int on[NFAM];          // family uses its learned indicator
  double aspect[NFAM];   // param[1] / param[0] of the trained shape
};
struct LearnedNets {
  const float *theta[NFAM];
  const __bf16 *packed[NFAM];
  const float *band[NFAM];  // band grid of the trained shape, or NULL
};
hipError_t launch_mark_learned(DevParticle *parts, int n, const LearnedModes &modes, hipStream_t s);
hipError_t launch_mlp_table(const Lattice &L, const DevParticle *parts, int n, const LearnedNets &nets,
                            float *tables, long long cap, hipStream_t s);
// band: band grid of the mesh at unit circumradius, or NULL
hipError_t launch_mesh_table(const Lattice &L, const DevParticle *parts, int n, const float *band, float *tables,
                             long long cap, hipStream_t s);
hipError_t launch_bin(const Lattice &L, const DevParticle *parts, int n, int cap, int *tcnt, int *tlist,
                      int *status, hipStream_t s);
hipError_t launch_mea(int prec, const Lattice &L, const void *A, const DevParticle *parts, const int *order, int n,
                      int lmax, int layers, int chunked, double *partial, hipStream_t s);
// contact: short-range repulsion of range `range`, pair stiffness k,
// wall stiffness kw (on = range > 0 and k or kw nonzero)
struct ContactParams {
  double range, k, kw;
  int on;
};
constexpr int CONTACT_NODES = 1024;
constexpr int CONTACT_CAND = 64;  // partners of one particle within the bounding-sphere range
// pair search: n^2 tests in partner chunks below CONTACT_GRID_MIN particles,
// a grid of the centres from there on
constexpr int CONTACT_GRID_MIN = 4096;
constexpr int CONTACT_TILE = 1024;      // partners staged in LDS at a time
constexpr int CONTACT_MAX_CHUNKS = 64;  // partner chunks = partial sums per particle
// contact records per particle: one per partner chunk, or one with the grid
__host__ __device__ inline int contact_chunks(int n) {
  return n >= CONTACT_GRID_MIN ? 1 : (n < 1 ? 1 : (n > CONTACT_MAX_CHUNKS ? CONTACT_MAX_CHUNKS : n));
}
// uniform grid of particle centres for the contact pair search: g[a] cells of
// size[a] >= the largest pair reach on axis a, at most CGRID_AXIS per axis
constexpr int CGRID_AXIS = 32;
constexpr int CGRID_MAX = CGRID_AXIS * CGRID_AXIS * CGRID_AXIS;
struct ContactGrid {
  int g[3];
  double size[3];
};
// device work arrays of the pair search: gcount[CGRID_MAX + 1] (cell starts),
// gfill[CGRID_MAX], gcell[n], glist[n], gpos[n] (centre and w = R or -R_circ)
struct ContactWork {
  int *gcount, *gfill, *gcell, *glist;
  double4 *gpos;
};
// sphere-pair contact forces out[contact_chunks(n)][n][3] from the state
// before the EoM, and the partner lists cand / ccnt of pairs with a
// non-spherical particle (appended: ccnt must be zero on entry)
hipError_t launch_contact(const Lattice &L, const DevParticle *parts, int n, const ContactParams &c,
                          const ContactGrid &cg, const ContactWork &w, double *out, int *cand, int *ccnt, int *status,
                          hipStream_t s);
// contact of pairs with a non-spherical particle and of such particles with
// walls: out[p] = (F, T); dirs = CONTACT_NODES unit directions (x, y, z);
// cand / ccnt: the partner lists k_contact fills (emptied here)
hipError_t launch_contact_shapes(const Lattice &L, const DevParticle *parts, int n, const ContactParams &c,
                                 const double *dirs, int *cand, int *ccnt, double *out, hipStream_t s);
// shapes: the records of launch_contact_shapes, or NULL
hipError_t launch_eom_bin(const Lattice &L, DevParticle *parts, int n, int lmax, int layers, const double *partial,
                          const ContactParams &c, const double *contact, const double *shapes, int *tcnt, int *tlist,
                          int *status, hipStream_t s);
hipError_t launch_collide(int prec, const Lattice &L, const void *A, void *B, const DevParticle *parts,
                          const int *tcnt, const int *tlist, int *tcnt_clear, int *status, hipStream_t s);
hipError_t launch_set_fields(int prec, const Lattice &L, void *A, const double *rho, const double *u,
                             hipStream_t s);
hipError_t launch_fields(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                         const int *tcnt, const int *tlist, unsigned mask, int out_f32, void *out,
                         hipStream_t s);
// sums of u_phys over all cells, of u_phys over pure-fluid cells and their
// count (7 doubles to out); partial holds ntiles x 7 doubles
hipError_t launch_mean_velocity(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                                const int *tcnt, const int *tlist, double *partial, double *out,
                                hipStream_t s);

}  // namespace hlbm
