/*
 * impm.h -- C ABI of the MI355X IMPM elastomer simulator (libimpm.so).
 *
 * The library simulates the elastomer layer of an optical tactile sensor with
 * the improved Material Point Method of arXiv 2405.02914, Sec. III-A:
 * particle-to-grid (Eq. 1-4), grid velocity and boundary handling (Eq. 5),
 * grid-to-particle (Eq. 6-7), the relative-rest loop of Algorithm 1 (the
 * elastomer held at rest relative to the indenter during slip and rotation),
 * and particle movement (Eq. 8-9).  The indenter is a rigid kinematic body
 * whose pose the caller sets; the output is the elastomer surface height map
 * (Sec. IV-B, the depth data taken from the surface particles).
 *
 * Conventions
 *   Units are SI (m, s, kg, Pa).  Coordinates are slab-local: origin at the
 *   slab's (-x,-y) bottom corner, z up.  Quaternions are body->world (w,x,y,z).
 *   Matrices are 3x3 row-major.  Particles are addressed by id:
 *   id = ((k*Ny + j)*Nx + i)*ppc + (sz*m + sy)*m + sx for cell (i,j,k) and
 *   sub-cell (sx,sy,sz) of the m^3 = ppc stratification.
 *
 * Ownership
 *   The library owns every device buffer it allocates.  The caller owns every
 *   buffer it passes in; the library never frees caller memory and writes an
 *   output buffer only when the call succeeds.  Pointers flagged *_on_device
 *   are device pointers (for example torch tensors on the same HIP device).
 *
 * Streams and errors
 *   All device work is enqueued on the stream given to sim_create (NULL: a
 *   stream the library creates).  sim_step only enqueues; device-side failures
 *   (non-finite state, det F <= 0, a particle moving more than one cell in a
 *   step) are latched on the device and reported as SIM_ENUMERIC by the next
 *   synchronising call (sim_synchronize, sim_read_*, sim_surface_* with a host
 *   output, sim_get_stats).  Every call returns SIM_OK (0) or a negative code;
 *   sim_last_error gives a message for the last failure on that handle.
 *   A sim_t is not thread-safe; distinct handles are independent.
 */
#ifndef IMPM_H
#define IMPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,    /* bad argument or parameter */
    SIM_ENOMEM = -2,    /* device allocation failed */
    SIM_EHIP = -3,      /* a HIP runtime call failed */
    SIM_ENUMERIC = -4,  /* latched device-side numerical failure */
    SIM_ESTATE = -5     /* call not valid in the handle's state */
};

enum { SIM_SHAPE_NONE = 0, SIM_SHAPE_SPHERE = 1, SIM_SHAPE_CAPSULE = 2, SIM_SHAPE_BOX = 3,
       SIM_SHAPE_HEIGHTFIELD = 4 };
enum { SIM_MODE_IMPM = 0, SIM_MODE_PLAIN = 1 };
enum { SIM_OBJECT_COLLIDER = 0, SIM_OBJECT_PARTICLES = 1 };

/* Device error bits reported by sim_get_stats (SIM_ENUMERIC when non-zero). */
enum { SIM_DEV_CFL = 1, SIM_DEV_NONFINITE = 2, SIM_DEV_DETF = 4 };

typedef struct {
    int32_t cells[3];          /* slab cells per axis (Nx, Ny, Nz), each >= 1 */
    int32_t ppc;               /* particles per cell: 1, 8 or 27 (a cube m^3) */
    double dx;                 /* grid spacing W of Eq. 4 and 7 (m), > 0 */
    uint64_t seed;             /* SplitMix64 seed of the particle jitter */
    double E, nu, rho;         /* Young's modulus (Pa), Poisson ratio (0, 0.5), density */
    double dt;                 /* configured substep (s), > 0 */
    int32_t subcycle;          /* executed steps per configured substep (>= 1), each dt/subcycle */
    int32_t pad_lateral;       /* empty cells on each lateral side of the slab (>= 1) */
    int32_t pad_top;           /* empty cells above the slab (>= 1) */
    int32_t pad_bottom;        /* cells below the slab's bottom face (>= 1); nodes with z <= 0 are fixed */
    int32_t band;              /* zero-velocity node band at the lateral and top domain faces */
    int32_t mode;              /* SIM_MODE_IMPM (Algorithm 1) or SIM_MODE_PLAIN (one exchange) */
    int32_t rest_limit;        /* LIMIT of Algorithm 1 (>= 1) */
    double rest_threshold;     /* threshold of the relative-rest test (>= 0) */
    double fixed_z_fraction;   /* particles with rest height < fraction * slab height get v_z = 0 */
    int32_t shape;             /* SIM_SHAPE_* */
    int32_t _pad0;
    double radius;             /* sphere / capsule radius (m) */
    double half_length;        /* capsule: straight half-length along body x (m) */
    double half_extent[3];     /* box half extents (m) */
    double fillet;             /* box edge rounding radius (m), <= min half extent */
    double pose0[7];           /* initial indenter pose: position xyz (m), quaternion wxyz */
    int32_t stress_each_pass;  /* 1: every pass of the loop re-adds the elastic impulse */
    int32_t _pad1;
    /* SIM_SHAPE_HEIGHTFIELD: the solid above the surface z = h(x, y) (body frame)
     * over the disc x^2 + y^2 <= hf_half^2; h is the bilinear interpolation of
     * hf[j * hf_n + i], the height at (-hf_half + i s, -hf_half + j s) with
     * s = 2 hf_half / (hf_n - 1).  2 <= hf_n <= 4096.  The table is caller
     * memory, read and copied by sim_create / sim_batch_create only.  The
     * calibration point x_o is the lowest sample inside the disc. */
    int32_t hf_n;
    int32_t _pad2;
    double hf_half;            /* footprint radius and table half-width (m) */
    const double* hf;          /* hf_n * hf_n heights (m), row-major by y */
    /* How the object acts on the elastomer (Sec. III-A):
     *   SIM_OBJECT_COLLIDER: a rigid collider at the grid -- every node inside the
     *     indenter takes its rigid velocity;
     *   SIM_OBJECT_PARTICLES: the object is represented by particles, as the
     *     paper describes it -- the body-fixed lattice points of spacing dx / m
     *     (m^3 = ppc) inside the indenter, at most object_cap above its lowest
     *     point and (at the initial pose) inside the grid; Algorithm 1 sets their
     *     velocity to the object's motion before every exchange, they join the
     *     particle-to-grid transfer with density object_density and no stress,
     *     they move rigidly with the pose, and x_o is the object's bottom
     *     particle (ties to the one farthest from the body z axis, then the
     *     smallest body (x, y)).  They are internal: the particle calls below
     *     address the elastomer particles only. */
    int32_t object_mode;
    int32_t _pad3;
    double object_density;     /* kg/m^3, > 0 with SIM_OBJECT_PARTICLES */
    double object_cap;         /* m, > 0 with SIM_OBJECT_PARTICLES */
    /* Shaped elastomer (Sec. VI: the shape of the elastomer particle cloud can be
     * adjusted): NULL for the full Nx x Ny x Nz cuboid, else Nx * Ny column
     * heights in cells (row j, column i; each 0..Nz): column (i, j) holds the
     * cells k < columns[j * Nx + i] of the cuboid, so the elastomer keeps its
     * flat bottom and takes any outline and stepped top.  Particle ids then
     * number the kept cells in (k, j, i) order (id = kept cell * ppc + sub);
     * each particle's jitter is that of the same particle of the cuboid.  The
     * surface particles are the top sub-layer of each column's top cell, and
     * the height map's rest height under a pixel is that of its column (0 where
     * the column is empty).  The table is caller memory, copied by sim_create. */
    const uint8_t* columns;
} sim_params;

typedef struct {
    int64_t substeps;          /* configured substeps completed */
    int64_t steps;             /* executed (sub-cycled) steps */
    int64_t passes;            /* exchange passes of Algorithm 1, summed over steps */
    int64_t limit_hits;        /* steps that ended at LIMIT without meeting the test */
    double last_r;             /* last relative-rest ratio |v_e,t - v_o,t| / |v_o,t| */
    int32_t device_error;      /* SIM_DEV_* bits */
    int32_t _pad;
    double pose[7];            /* current commanded indenter pose */
    double xo[3];              /* object calibration point x_o at the current pose */
    int64_t calib_particle;    /* id of the elastomer calibration particle x_e */
} sim_stats;

typedef struct sim_s sim_t;

/* Fill *p with the 16x16x4 mm, dx 0.5 mm sensor and a sphere indenter. */
int sim_params_default(sim_params* p);

/* Build the grid and the jittered particle cloud (Sec. IV-B: the elastomer
 * cuboid and the object at its initial pose; the calibration points x_o, the
 * object's lowest point, and x_e, the nearest elastomer particle, Algorithm 1).
 * hip_stream: a hipStream_t, or NULL for a library-owned stream. */
int sim_create(const sim_params* p, void* hip_stream, sim_t** out);

/* Free every device buffer of the handle (NULL is ignored). */
void sim_destroy(sim_t* s);

/* Target pose reached at the end of the next sim_step (Fig. 2(B) and Sec. III:
 * the motions -- press, slide, rotate -- are simulated step by step until the
 * object reaches its target pose; Sec. IV-B: the object starts centred over
 * the elastomer, and the distance and angle it has moved are measured at its
 * calibration point x_o).  The indenter moves from its current pose at
 * constant linear and angular velocity (linear position interpolation,
 * rotation about one fixed axis); each executed step's pose is the object
 * velocity that Algorithm 1 prescribes.  pos: 3 doubles (m, slab frame);
 * quat_wxyz: 4 doubles, normalised by the call.  Host memory, read during the
 * call only.  SIM_EINVAL on a NULL handle or pointer or a non-finite value;
 * the pose is not changed then. */
int sim_set_indenter_pose(sim_t* s, const double pos[3], const double quat_wxyz[4]);

/* Enqueue n_substeps configured substeps (n_substeps * subcycle executed steps
 * of Algorithm 1). */
int sim_step(sim_t* s, int32_t n_substeps);

/* Wait for enqueued work; return SIM_ENUMERIC if a device error was latched. */
int sim_synchronize(sim_t* s);

/* Surface height map (Sec. IV-B: after the deformation the elastomer surface
 * particles are read out and interpolated into a depth image; Fig. 2(C):
 * interpolating the surface particles' depths gives the 3-D elastomer model).
 * H rows x W columns, row v and column u at the pixel centre
 * ((u+1/2) Lx/W, (v+1/2) Ly/H): slab height + the Shepard-normalised 2-D
 * quadratic B-spline average (pitch = pixel size) of the top surface
 * particles' z displacement; pixels with no particle weight get the slab
 * height.  The paper's small depth perturbation, a meshing workaround, is not
 * applied.  out: W*H floats (row-major by v), caller memory on the host
 * (out_on_device = 0: the call synchronises the stream and reports latched
 * device errors) or on the handle's device (enqueued only).  SIM_EINVAL on a
 * NULL pointer or W, H < 1; out is written only on success. */
int sim_surface_heightmap(sim_t* s, float* out, int32_t W, int32_t H, int32_t out_on_device);

/* The height map of sim_surface_heightmap without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The pixel accumulators live in a
 * fixed library workspace of 512 * 512 pixels (8 MiB per device, held until
 * the process ends) instead of the handle's own buffer; W * H above that is
 * SIM_EINVAL with a message, before any work is enqueued.  out_device: W*H
 * floats of device memory on the handle's device, written by kernels enqueued
 * on the handle's stream (the call does not synchronise; latched device
 * errors surface at the next synchronising call).  Results are bitwise those
 * of sim_surface_heightmap.  Every call on one GPU shares that workspace and
 * clears it first: calls that overlap on one GPU (two streams, or two host
 * threads) race and give undefined maps; serialise them. */
int sim_surface_heightmap_noalloc(sim_t* s, float* out_device, int32_t W, int32_t H);

/* The same interpolation of the full displacement x - X_rest: H*W*3 floats. */
int sim_surface_displacement(sim_t* s, float* out, int32_t W, int32_t H, int32_t out_on_device);

/* Depth of the indenter below the slab's top face along the vertical line
 * through each pixel centre (as for the height map): (H - z_low) * scale, where
 * z_low is the indenter's lowest point on that line at the target pose (the
 * last sim_set_indenter_pose, which the next sim_step reaches; after a step,
 * the current pose) -- the object's "depth data" of Sec. IV-B and the
 * surrogate's main input; -1e9 where
 * the line misses the indenter.  Needs a pose rotated about z only (else
 * SIM_EINVAL).  out: W*H floats, host or device memory. */
int sim_indenter_depthmap(sim_t* s, float* out, int32_t W, int32_t H, double scale, int32_t out_on_device);

int sim_get_stats(sim_t* s, sim_stats* out);
int sim_num_particles(const sim_t* s, int64_t* n);
int sim_grid_dims(const sim_t* s, int32_t nodes[3]);

/* Particle state in id order, host memory; any pointer may be NULL.
 * x: n*3 doubles (m); v: n*3 floats; C: n*9 floats; G = F - I: n*9 floats. */
int sim_read_particles(sim_t* s, double* x, float* v, float* C, float* G);
int sim_write_particles(sim_t* s, const double* x, const float* v, const float* C, const float* G);

/* Rest positions (n*3 doubles) and flags (bit 0 bottom layer, bit 1 surface). */
int sim_read_rest(sim_t* s, double* X, uint8_t* flags);

/* Keep the grid mass M (n_nodes), momentum MG (n_nodes*3) and velocity V
 * (n_nodes*3) of the last pass for sim_read_grid (costs bandwidth). */
int sim_debug_keep_grid(sim_t* s, int32_t on);
int sim_read_grid(sim_t* s, float* M, float* MG, float* V);

/* Replay a pass schedule: the next n executed steps do exactly passes[i]
 * exchanges each (parity runs near the relative-rest threshold). */
int sim_debug_force_passes(sim_t* s, const int32_t* passes, int32_t n);

/* Tile shape (cells per axis) of the binned particle order and the threads per
 * block of the tile kernels (sim_set_tile: 256).  Only the shapes compiled into
 * the library are accepted (SIM_EINVAL lists them).  Default 8 x 4 x 4 / 256. */
int sim_set_tile(sim_t* s, int32_t tx, int32_t ty, int32_t tz);
int sim_set_tile_threads(sim_t* s, int32_t tx, int32_t ty, int32_t tz, int32_t threads);

/* on != 0: each sim_step's launch sequence is captured once as a HIP graph
 * (per sequence length, pass schedule and buffer parity) and replayed; the
 * replay computes exactly what the eager launches compute.  Ignored while
 * sim_profile is on.  Default off. */
int sim_set_graph(sim_t* s, int32_t on);

/* Storage compaction (a layout choice; the method is unchanged).  every_steps > 0:
 * once every_steps executed steps have accumulated, the particle state (cells,
 * flags, id map and the state planes) is moved on the device into the binned
 * order of the next step, round-robin over the stencil base nodes inside each
 * tile.  An eager sim_step call compacts only between its steps or before its
 * first step (a compaction that fell due at the end of the previous call), and
 * there leaves the velocity and affine planes behind unless the sensor has
 * object particles: the call's last step stores them for every elastomer
 * particle.  A graph-replayed or batched call compacts at its end and moves
 * every plane.  Without it, particles that cross tiles
 * leave a tile's data spread over other tiles' cache lines, and neighbouring
 * lanes come to share base nodes.  The results are bitwise those of a run
 * without compaction: the node sums are exact and order-independent.  The
 * storage order itself may differ between runs.  Each compaction synchronises
 * the stream once, copies the state once (about 2 x 105 B per particle), and
 * reports a latched device error (SIM_ENUMERIC) at that point.  The first use allocates a second
 * copy of the state, owned by the handle (SIM_EHIP if that fails).
 * A batch member (sim_batch_get) with compaction set compacts the same way after
 * sim_batch_step calls, on its own stream once the batch's launches are done.
 * every_steps = 0 (the default) turns it off; negative values are SIM_EINVAL. */
int sim_set_compaction(sim_t* s, int32_t every_steps);

/* Time the first-pass fused exchange kernel (grid-to-particle, commit,
 * particle-to-grid) with HIP events on the handle's stream, in eager calls:
 * on = 1 every launch, on = k > 1 the launches of every k-th executed step (a
 * uniform sample; the event markers cost wall time), on = 0 none; negative
 * values are SIM_EINVAL.  sim_profile_read synchronises, returns the summed
 * kernel time (ms) and the number of timed launches since the last read, and
 * resets them. */
int sim_profile(sim_t* s, int32_t on);
int sim_profile_read(sim_t* s, double* ms_total, int64_t* launches);

const char* sim_last_error(const sim_t* s);

/* ---- Batched sensors (many independent sensors advanced together).
 * All sensors of a batch share dt, subcycle and rest_limit and are stepped
 * together: one launch per kernel phase covers every sensor of a tile-shape
 * group (the blocks of a launch map to (sensor, tile) through prefix sums), so
 * a step of the whole batch costs a handful of launches. */
typedef struct sim_batch_s sim_batch_t;

/* params: n records; tiles: n x (tx, ty, tz, threads) or NULL for the default
 * shape (for example from sim_autotune_tile).  hip_stream as for sim_create. */
int sim_batch_create(const sim_params* params, int32_t n, const int32_t* tiles, void* hip_stream,
                     sim_batch_t** out);
void sim_batch_destroy(sim_batch_t* b);
int sim_batch_size(const sim_batch_t* b, int32_t* n);
/* Borrow sensor i (for sim_read_*, sim_get_stats, ...); owned by the batch. */
int sim_batch_get(sim_batch_t* b, int32_t i, sim_t** out);
/* pos: n x 3, quat_wxyz: n x 4; each sensor's target for the next sim_batch_step. */
int sim_batch_set_indenter_poses(sim_batch_t* b, const double* pos, const double* quat_wxyz);
/* Enqueue n_substeps configured substeps of every sensor.  By default the whole
 * launch sequence of the call is one HIP graph launch (captured on first use per
 * sequence length and pass schedule, then replayed). */
int sim_batch_step(sim_batch_t* b, int32_t n_substeps);
/* on = 0: launch the kernels one by one instead of replaying a graph. */
int sim_batch_set_graph(sim_batch_t* b, int32_t on);
/* Which members the following sim_batch_step calls advance: active[i] != 0
 * (n flags, host memory, read during the call; every member is active after
 * sim_batch_create).  For callers that re-solve some sensors of a batch and
 * not others, such as a serving loop whose learned model covers the rest: a
 * member that sits a call out keeps its particles, grid, counters and pose, and
 * its next active call moves the indenter from its last stepped pose to the
 * latest target.  Its kernels' blocks exit at once, so the call costs what its
 * active members cost.  Errors, at the sim_batch_step call: SIM_EINVAL when a
 * member sits out a call of an odd number of executed steps (n_substeps times
 * subcycle: members keep their binned-order parity only over even counts), and
 * SIM_ESTATE when a member sits out the batch's first call.  A call with no
 * active member does nothing. */
int sim_batch_set_active(sim_batch_t* b, const int32_t* active);
int sim_batch_synchronize(sim_batch_t* b);
/* out: n x H x W (heightmaps) or n x H x W x 3 (displacements), host or device. */
int sim_batch_heightmaps(sim_batch_t* b, float* out, int32_t W, int32_t H, int32_t out_on_device);
int sim_batch_displacements(sim_batch_t* b, float* out, int32_t W, int32_t H, int32_t out_on_device);
/* n x H x W indenter depth maps (sim_indenter_depthmap of every sensor). */
int sim_batch_depthmaps(sim_batch_t* b, float* out, int32_t W, int32_t H, double scale, int32_t out_on_device);
const char* sim_batch_last_error(const sim_batch_t* b);

/* Time `steps` executed steps of a sensor with these parameters for every
 * compiled tile shape, in three interleaved rounds, and return the shape whose
 * fastest round is fastest (tx, ty, tz, threads) with that round's time per
 * executed step in ms. */
int sim_autotune_tile(const sim_params* p, int32_t steps, void* hip_stream, int32_t out[4], double* out_ms);

#ifdef __cplusplus
}
#endif

#endif /* IMPM_H */
