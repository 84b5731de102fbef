/*
 * impm_oracle.c -- plain, slow FP64 CPU oracle of the IMPM elastomer substep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg load it (through ctypes).  It shares no header, helper, table or
 * constant with the HIP path.
 *
 * What it computes (arXiv 2405.02914, Sec. III-A "Elastomer Simulation"):
 *   particle-to-grid       Eq. (1)-(4)   grid mass M_i and momentum MG_i = MM_i + ME_i
 *   boundary conditions    Eq. (5)       V_i = MG_i / M_i, boundary nodes zeroed
 *   grid-to-particle       Eq. (6)-(7)   v_p and the affine matrix C_p
 *   relative-rest check    Algorithm 1   repeat the exchange until the calibration
 *                                        particle x_e moves with the object point x_o
 *   particle movement      Eq. (8)-(9)   F_p <- (I + dt C_p) F_p,  x_p <- x_p + dt v_p
 *
 * Readings of the paper where it is silent or garbled (each is listed with its
 * justification in the design notes of the repository):
 *   - the weight w_ip is the quadratic B-spline on the 3x3x3 stencil (the 4/W^2
 *     factor of Eq. (4) and (7) is the inverse of its inertia dx^2/4);
 *   - Eq. (3) carries m_p on the affine term: MM_i = sum w m_p (v_p + C_p (X_i - x_p));
 *   - X_g in Eq. (3)/(4) is the position of the summed node i; Eq. (7) sums V_g;
 *   - S_p is the fixed-corotated Kirchhoff stress tau = 2mu (F-R) F^T + lambda J (J-1) I,
 *     R the rotation of the polar decomposition of F (Newton iteration of Higham 1986);
 *   - the object is either a rigid kinematic collider (every grid node inside the
 *     indenter at the start of the substep takes the rigid velocity, relative
 *     rest), or, as the paper describes it, a set of object particles whose
 *     velocity is set to the object's prescribed motion before every exchange
 *     (Algorithm 1) and which join the particle-to-grid transfer with their own
 *     mass; its shape is a sphere, a capsule rod, a rounded box or a sampled
 *     height field (the solid above a bilinear surface, over a disc footprint);
 *   - the relative-rest test uses the tangential (x,y) velocity 2-vectors,
 *     |v_e,t - v_o,t| <= threshold |v_o,t|, converged at once if |v_o,t| <= 1e-9 m/s;
 *   - F and x are committed once per substep with the final pass's C and v;
 *   - "bottom elastomer particles" are those whose rest height is below
 *     fixed_z_fraction of the slab thickness; PLAIN mode (the paper's "normal" MPM)
 *     does one pass and has no bottom rule.
 *
 * Particle initialisation draws its jitter from SplitMix64 (Steele, Lea, Flood,
 * OOPSLA 2014) used as a counter-based generator: the t-th output of the stream
 * seeded with s is mix(s + t * 0x9E3779B97F4A7C15).  Particle id
 * ((k Ny + j) Nx + i) ppc + (sz m + sy) m + sx sits in cell (i,j,k), sub-cell
 * (sx,sy,sz) of the m^3 stratification; its axis-a offset inside the cell is
 * r_a = fl32((s_a + u) / m) with u the (3 id + a + 1)-th output's top 53 bits
 * scaled to [0,1), and its position is (cell_a + r_a) dx.
 *
 * Coordinates: slab-local metres, origin at the slab's (-x,-y) bottom corner, z up.
 * Grid node (i,j,k) sits at ((i-pl) dx, (j-pl) dx, (k-pb) dx).
 * Compiled with -ffp-contract=off so every expression rounds as written.
 *
 * With one thread (the default) every loop is the plain serial loop above.
 * orc_set_threads(s, T > 1) runs the same steps with OpenMP for timing on many
 * cores: particle loops split into T contiguous ranges, the particle-to-grid
 * sums taken per thread and added node by node in thread order (a fixed
 * order, so a run is reproducible, but it rounds differently from the serial
 * sums at the level of FP64 round-off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- params */

typedef struct {
    int32_t cells[3];
    int32_t ppc;               /* particles per cell, a cube m^3 (1, 8, 27) */
    double dx;
    uint64_t seed;
    double E, nu, rho, dt;
    int32_t subcycle;          /* each configured substep = subcycle steps of dt/subcycle */
    int32_t pad_lateral, pad_top, pad_bottom, band;
    int32_t mode;              /* 0 = IMPM, 1 = PLAIN */
    int32_t rest_limit;        /* LIMIT of Algorithm 1 */
    double rest_threshold;     /* threshold of Algorithm 1 */
    double fixed_z_fraction;
    /* indenter */
    int32_t shape;             /* 0 none, 1 sphere, 2 capsule rod, 3 rounded box, 4 height field */
    int32_t _pad0;
    double radius, half_length, half_extent[3], fillet;
    double pose0[7];           /* position xyz (m), quaternion wxyz body->world */
    int32_t stress_each_pass;  /* 1: every pass of the loop re-adds ME_i (literal Alg. 1) */
    int32_t _pad1;
    /* height field: hf_n x hf_n body-frame heights (row j, column i) sampled at
     * (-hf_half + i step, -hf_half + j step), step = 2 hf_half / (hf_n - 1);
     * copied at creation */
    int32_t hf_n;
    int32_t _pad2;
    double hf_half;
    const double *hf;
    /* object representation: 0 = rigid collider at the grid, 1 = object particles
     * on a body-fixed lattice of spacing dx / m (m^3 = ppc) filling the body up to
     * object_cap above its lowest point, density object_density */
    int32_t object_mode;
    int32_t _pad3;
    double object_density;
    double object_cap;
    /* elastomer shape (Sec. VI: the elastomer particle cloud shaped at will):
     * NULL for the full cuboid, else Nx * Ny column heights in cells (row j,
     * column i, each 0..Nz): column (i, j) holds cells k < columns[j Nx + i],
     * so the slab keeps its flat glued bottom and takes any outline and top */
    const uint8_t *columns;
} orc_params;

typedef struct {
    orc_params P;
    int64_t n;                 /* particles */
    int nn[3];                 /* nodes per axis */
    int64_t n_nodes;
    double *x, *v, *C, *F;     /* n*3, n*3, n*9, n*9 ; 3x3 row-major */
    double *Xrest;             /* n*3 rest positions */
    unsigned char *bottom, *surface;
    double *M, *MG, *V;        /* n_nodes, n_nodes*3, n_nodes*3 */
    double mu, lam, Vp, mp;
    double pos[3], quat[4];    /* current pose */
    double tpos[3], tquat[4];  /* target pose of the next orc_step */
    double po_body[3];         /* x_o in the body frame */
    int64_t e;                 /* calibration particle id */
    int64_t substeps, steps, passes, limit_hits;
    double last_r;
    double min_margin;         /* min |r - threshold| / threshold over every test taken */
    int32_t *forced;           /* forced pass counts (parity replay), may be NULL */
    int64_t n_forced, forced_pos;
    int32_t *pass_log;         /* passes of each executed step, capacity log_cap */
    int64_t log_cap, log_len;
    int32_t error;             /* 1: a stencil left the grid, 2: non-finite state, 3: det F <= 0 */
    double *hf_copy;           /* the height-field table (shape 4) */
    uint8_t *col_copy;         /* the column heights (NULL: the full cuboid) */
    int32_t threads;           /* OpenMP threads of the timing leg (1: the plain serial loops) */
    double *Mt, *MGt;          /* per-thread node sums of the parallel particle-to-grid */
    int64_t n_obj;             /* object particles (object_mode 1) */
    double *obj_body, *obj_x;  /* n_obj*3 body-frame and world positions */
    double m_obj;              /* mass of one object particle */
} orc_sim;

/* ---------------------------------------------------------------- SplitMix64 */

static uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* t-th output (t >= 1) of the SplitMix64 stream seeded with `seed`. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t t) {
    return sm64_mix(seed + t * 0x9E3779B97F4A7C15ULL);
}

static double sm64_unit(uint64_t seed, uint64_t t) {
    return (double)(orc_splitmix64_at(seed, t) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------------- 3x3 helpers */

static double det3(const double *A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse transpose: A^{-T} = cof(A) / det(A) */
static void inv_transpose3(const double *A, double *out) {
    double d = det3(A);
    out[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    out[1] = -(A[3] * A[8] - A[5] * A[6]) / d;
    out[2] = (A[3] * A[7] - A[4] * A[6]) / d;
    out[3] = -(A[1] * A[8] - A[2] * A[7]) / d;
    out[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    out[5] = -(A[0] * A[7] - A[1] * A[6]) / d;
    out[6] = (A[1] * A[5] - A[2] * A[4]) / d;
    out[7] = -(A[0] * A[5] - A[2] * A[3]) / d;
    out[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

/* Rotation factor of the polar decomposition F = R S (det F > 0):
 * Newton iteration R <- (R + R^{-T}) / 2 from R = F (Higham 1986). */
void orc_polar(const double *F, double *R) {
    double X[9], Y[9];
    memcpy(X, F, sizeof(X));
    for (int it = 0; it < 100; ++it) {
        inv_transpose3(X, Y);
        double diff = 0.0, nrm = 0.0;
        for (int k = 0; k < 9; ++k) {
            double nx = 0.5 * (X[k] + Y[k]);
            diff += (nx - X[k]) * (nx - X[k]);
            nrm += nx * nx;
            X[k] = nx;
        }
        if (diff <= 1e-30 * nrm) break;
    }
    memcpy(R, X, sizeof(X));
}

/* Fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + lambda J (J - 1) I. */
void orc_kirchhoff(const double *F, double mu, double lam, double *tau) {
    double R[9];
    orc_polar(F, R);
    double J = det3(F);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += (F[3 * a + c] - R[3 * a + c]) * F[3 * b + c];
            tau[3 * a + b] = 2.0 * mu * s + (a == b ? lam * J * (J - 1.0) : 0.0);
        }
}

/* Elastic energy density of the fixed-corotated model:
 * psi = mu |F - R|^2 + lambda/2 (J - 1)^2. */
static double energy_density(const double *F, double mu, double lam) {
    double R[9];
    orc_polar(F, R);
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += (F[k] - R[k]) * (F[k] - R[k]);
    double J = det3(F);
    return mu * s + 0.5 * lam * (J - 1.0) * (J - 1.0);
}

/* ---------------------------------------------------------------- quaternions */

static void quat_mul(const double *a, const double *b, double *o) {
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

static void quat_to_matrix(const double *q, double *R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void quat_normalize(double *q) {
    double s = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= s;
}

/* Relative rotation from q0 to q1 as (unit axis, angle in [0, pi]). */
static void quat_rel_axis_angle(const double *q0, const double *q1, double *axis, double *angle) {
    double q0c[4] = {q0[0], -q0[1], -q0[2], -q0[3]};
    double r[4];
    quat_mul(q1, q0c, r);
    if (r[0] < 0.0) { r[0] = -r[0]; r[1] = -r[1]; r[2] = -r[2]; r[3] = -r[3]; }
    double s = sqrt(r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    if (s <= 0.0) { axis[0] = 0.0; axis[1] = 0.0; axis[2] = 1.0; *angle = 0.0; return; }
    axis[0] = r[1] / s; axis[1] = r[2] / s; axis[2] = r[3] / s;
    *angle = 2.0 * atan2(s, r[0]);
}

/* ---------------------------------------------------------------- indenter */

/* Height-field indenter: bilinear interpolation of the sampled lower surface
 * at body-frame (x, y); cells outside the table clamp to its edge cells. */
static double hf_height(const orc_params *P, double x, double y) {
    int n = P->hf_n;
    double step = 2.0 * P->hf_half / (double)(n - 1);
    double u = (x + P->hf_half) / step, v = (y + P->hf_half) / step;
    int i0 = (int)floor(u), j0 = (int)floor(v);
    if (i0 < 0) i0 = 0;
    if (i0 > n - 2) i0 = n - 2;
    if (j0 < 0) j0 = 0;
    if (j0 > n - 2) j0 = n - 2;
    double fu = u - (double)i0, fv = v - (double)j0;
    const double *t = P->hf;
    double z0 = (1.0 - fu) * t[j0 * n + i0] + fu * t[j0 * n + i0 + 1];
    double z1 = (1.0 - fu) * t[(j0 + 1) * n + i0] + fu * t[(j0 + 1) * n + i0 + 1];
    return (1.0 - fv) * z0 + fv * z1;
}

/* Signed-distance-like inside test in the body frame (phi <= 0 is inside). */
static double body_phi(const orc_params *P, const double *p) {
    if (P->shape == 1) {
        return p[0] * p[0] + p[1] * p[1] + p[2] * p[2] - P->radius * P->radius;
    } else if (P->shape == 2) {
        double h = P->half_length;
        double t = p[0] < -h ? -h : (p[0] > h ? h : p[0]);
        double qx = p[0] - t;
        return qx * qx + p[1] * p[1] + p[2] * p[2] - P->radius * P->radius;
    } else if (P->shape == 3) {
        double q[3], out2 = 0.0, inmax = -1e300;
        for (int a = 0; a < 3; ++a) {
            q[a] = fabs(p[a]) - (P->half_extent[a] - P->fillet);
            double qp = q[a] > 0.0 ? q[a] : 0.0;
            out2 += qp * qp;
            if (q[a] > inmax) inmax = q[a];
        }
        double inside_part = inmax < 0.0 ? inmax : 0.0;
        return sqrt(out2) + inside_part - P->fillet;
    } else if (P->shape == 4) {
        /* the solid above the sampled surface, over a disc of radius hf_half */
        if (p[0] * p[0] + p[1] * p[1] > P->hf_half * P->hf_half) return 1.0;
        return hf_height(P, p[0], p[1]) - p[2];
    }
    return 1.0; /* no indenter */
}

/* Body-frame lowest point of the indenter, ties broken towards the point
 * farthest from the body z axis, then the lexicographic minimum of (x, y). */
static void body_lowest_point(const orc_params *P, double *p) {
    p[0] = 0.0; p[1] = 0.0; p[2] = 0.0;
    if (P->shape == 1) { p[2] = -P->radius; }
    else if (P->shape == 2) { p[0] = -P->half_length; p[2] = -P->radius; }
    else if (P->shape == 3) {
        p[0] = -(P->half_extent[0] - P->fillet);
        p[1] = -(P->half_extent[1] - P->fillet);
        p[2] = -P->half_extent[2];
    } else if (P->shape == 4) {
        /* the lowest table sample inside the footprint disc */
        int n = P->hf_n;
        double step = 2.0 * P->hf_half / (double)(n - 1);
        double best_z = 0.0, best_r2 = 0.0;
        int found = 0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double x = -P->hf_half + (double)i * step, y = -P->hf_half + (double)j * step;
                double r2 = x * x + y * y;
                if (r2 > P->hf_half * P->hf_half) continue;
                double z = P->hf[j * n + i];
                int better = !found || z < best_z ||
                             (z == best_z && (r2 > best_r2 ||
                                              (r2 == best_r2 && (x < p[0] || (x == p[0] && y < p[1])))));
                if (better) { found = 1; best_z = z; best_r2 = r2; p[0] = x; p[1] = y; p[2] = z; }
            }
    }
}

/* Pose of the indenter for one executed step: centre c, rotation R (body->world),
 * rigid translational velocity vo and angular velocity w over the step. */
typedef struct { double c[3], R[9], vo[3], w[3]; } step_pose;

static void make_step_pose(const orc_sim *s, int64_t j, int64_t N, double h, step_pose *sp) {
    double frac = (double)j / (double)N;
    for (int a = 0; a < 3; ++a) {
        double d = s->tpos[a] - s->pos[a];
        sp->c[a] = s->pos[a] + d * frac;
        sp->vo[a] = d / ((double)N * h);
    }
    double axis[3], ang;
    quat_rel_axis_angle(s->quat, s->tquat, axis, &ang);
    double half = 0.5 * ang * frac;
    double qs[4] = {cos(half), axis[0] * sin(half), axis[1] * sin(half), axis[2] * sin(half)};
    double qj[4];
    quat_mul(qs, s->quat, qj);
    quat_to_matrix(qj, sp->R);
    for (int a = 0; a < 3; ++a) sp->w[a] = axis[a] * ang / ((double)N * h);
}

static int node_inside(const orc_sim *s, const step_pose *sp, const double *X) {
    if (s->P.shape == 0) return 0;
    double d[3] = {X[0] - sp->c[0], X[1] - sp->c[1], X[2] - sp->c[2]};
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = sp->R[a] * d[0] + sp->R[3 + a] * d[1] + sp->R[6 + a] * d[2];
    return body_phi(&s->P, p) <= 0.0;
}

static void rigid_velocity(const step_pose *sp, const double *X, double *out) {
    double r[3] = {X[0] - sp->c[0], X[1] - sp->c[1], X[2] - sp->c[2]};
    out[0] = sp->vo[0] + (sp->w[1] * r[2] - sp->w[2] * r[1]);
    out[1] = sp->vo[1] + (sp->w[2] * r[0] - sp->w[0] * r[2]);
    out[2] = sp->vo[2] + (sp->w[0] * r[1] - sp->w[1] * r[0]);
}

/* ---------------------------------------------------------------- grid geometry */

static void node_pos(const orc_sim *s, int i, int j, int k, double *X) {
    X[0] = (double)(i - s->P.pad_lateral) * s->P.dx;
    X[1] = (double)(j - s->P.pad_lateral) * s->P.dx;
    X[2] = (double)(k - s->P.pad_bottom) * s->P.dx;
}

static int is_boundary_node(const orc_sim *s, int i, int j, int k) {
    int b = s->P.band;
    if (i < b || i > s->nn[0] - 1 - b) return 1;
    if (j < b || j > s->nn[1] - 1 - b) return 1;
    if (k > s->nn[2] - 1 - b) return 1;
    if (k <= s->P.pad_bottom) return 1;   /* the slab's bottom face is fixed */
    return 0;
}

/* Quadratic B-spline stencil of a particle: base node and the 3 weights per axis. */
static void stencil(const orc_sim *s, const double *xp, int *base, double w[3][3]) {
    double off[3] = {(double)s->P.pad_lateral, (double)s->P.pad_lateral, (double)s->P.pad_bottom};
    for (int a = 0; a < 3; ++a) {
        double xg = xp[a] / s->P.dx + off[a];
        int b = (int)floor(xg - 0.5);
        double f = xg - (double)b;
        base[a] = b;
        w[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
        w[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
        w[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
    }
}

static int64_t node_index(const orc_sim *s, int i, int j, int k) {
    return ((int64_t)k * s->nn[1] + j) * s->nn[0] + i;
}

/* ---------------------------------------------------------------- creation */

static int cube_root_ppc(int ppc) {
    for (int m = 1; m <= 8; ++m) if (m * m * m == ppc) return m;
    return -1;
}

/* Body-frame bounding box of the indenter (half-extents about the body axis in
 * x and y; z from the lowest point up to that plus `cap`). */
static void body_box(const orc_params *P, double z_low, double cap, double lo[3], double hi[3]) {
    double hx = 0.0, hy = 0.0;
    if (P->shape == 1) { hx = P->radius; hy = P->radius; }
    else if (P->shape == 2) { hx = P->half_length + P->radius; hy = P->radius; }
    else if (P->shape == 3) { hx = P->half_extent[0]; hy = P->half_extent[1]; }
    else if (P->shape == 4) { hx = P->hf_half; hy = P->hf_half; }
    lo[0] = -hx; hi[0] = hx; lo[1] = -hy; hi[1] = hy;
    lo[2] = z_low; hi[2] = z_low + cap;
}

/* Object particles (object_mode 1): the body-fixed lattice points
 * ((i + 1/2) h, (j + 1/2) h, z_low + (k + 1/2) h), h = dx / m, that lie inside
 * the indenter, at most object_cap above its lowest point, and (at the initial
 * pose) with their whole stencil at least one node inside the grid.  Ordered
 * by k, then j, then i.  Also sets x_o: the lowest object particle, ties to the
 * one farthest from the body z axis, then to the smallest (x, y). */
static void make_object_particles(orc_sim *s, int m) {
    const orc_params *P = &s->P;
    double low[3];
    body_lowest_point(P, low);
    double h = P->dx / (double)m;
    double lo[3], hi[3];
    body_box(P, low[2], P->object_cap, lo, hi);
    int64_t ni = (int64_t)ceil(hi[0] / h), nj = (int64_t)ceil(hi[1] / h);
    int64_t nk = (int64_t)ceil(P->object_cap / h);
    double R[9];
    quat_to_matrix(s->quat, R);
    double off[3] = {(double)P->pad_lateral, (double)P->pad_lateral, (double)P->pad_bottom};
    int64_t cap_n = 0, n = 0;
    double *body = NULL;
    for (int64_t k = 0; k < nk; ++k)
        for (int64_t j = -nj; j < nj; ++j)
            for (int64_t i = -ni; i < ni; ++i) {
                double p[3] = {((double)i + 0.5) * h, ((double)j + 0.5) * h, low[2] + ((double)k + 0.5) * h};
                if (body_phi(P, p) > 0.0) continue;
                double w[3];
                int ok = 1;
                for (int a = 0; a < 3; ++a) {
                    w[a] = s->pos[a] + R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2];
                    double b = floor(w[a] / P->dx + off[a] - 0.5);
                    if (b < 1.0 || b > (double)(s->nn[a] - 4)) ok = 0;
                }
                if (!ok) continue;
                if (n == cap_n) {
                    cap_n = cap_n ? 2 * cap_n : 4096;
                    body = (double *)realloc(body, (size_t)cap_n * 3 * sizeof(double));
                }
                memcpy(body + 3 * n, p, sizeof(p));
                ++n;
            }
    s->n_obj = n;
    s->obj_body = body;
    s->obj_x = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    for (int64_t q = 0; q < n; ++q)
        for (int a = 0; a < 3; ++a)
            s->obj_x[3 * q + a] = s->pos[a] + R[3 * a] * body[3 * q] + R[3 * a + 1] * body[3 * q + 1] +
                                  R[3 * a + 2] * body[3 * q + 2];
    s->m_obj = P->object_density * s->Vp;
    /* x_o: the bottom particle of the object */
    int found = 0;
    double bz = 0.0, br2 = 0.0;
    for (int64_t q = 0; q < n; ++q) {
        const double *p = body + 3 * q;
        double r2 = p[0] * p[0] + p[1] * p[1];
        int better = !found || p[2] < bz ||
                     (p[2] == bz && (r2 > br2 ||
                                     (r2 == br2 && (p[0] < s->po_body[0] || (p[0] == s->po_body[0] && p[1] < s->po_body[1])))));
        if (better) { found = 1; bz = p[2]; br2 = r2; memcpy(s->po_body, p, 3 * sizeof(double)); }
    }
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    free(s->x); free(s->v); free(s->C); free(s->F); free(s->Xrest);
    free(s->bottom); free(s->surface); free(s->M); free(s->MG); free(s->V);
    free(s->forced); free(s->pass_log);
    free((void *)s->hf_copy);
    free(s->obj_body); free(s->obj_x);
    free(s->Mt); free(s->MGt);
    free(s->col_copy);
    free(s);
}

orc_sim *orc_create(const orc_params *P) {
    int m = cube_root_ppc(P->ppc);
    if (m < 1 || P->cells[0] < 1 || P->cells[1] < 1 || P->cells[2] < 1 || !(P->dx > 0.0)) return NULL;
    if (P->shape == 4 && (P->hf_n < 2 || !P->hf || !(P->hf_half > 0.0))) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->P = *P;
    if (P->shape == 4) {
        size_t nb = (size_t)P->hf_n * P->hf_n * sizeof(double);
        s->hf_copy = (double *)malloc(nb);
        memcpy(s->hf_copy, P->hf, nb);
        s->P.hf = s->hf_copy;
    } else {
        s->P.hf = NULL;
    }
    int Nx = P->cells[0], Ny = P->cells[1], Nz = P->cells[2];
    int64_t n_cells = (int64_t)Nx * Ny * Nz;
    s->P.columns = NULL;
    if (P->columns) {
        s->col_copy = (uint8_t *)malloc((size_t)Nx * Ny);
        memcpy(s->col_copy, P->columns, (size_t)Nx * Ny);
        s->P.columns = s->col_copy;
        n_cells = 0;
        for (int64_t q = 0; q < (int64_t)Nx * Ny; ++q) {
            if (P->columns[q] > Nz) { orc_destroy(s); return NULL; }
            n_cells += P->columns[q];
        }
    }
    s->n = n_cells * P->ppc;
    s->nn[0] = Nx + 2 * P->pad_lateral + 1;
    s->nn[1] = Ny + 2 * P->pad_lateral + 1;
    s->nn[2] = Nz + P->pad_bottom + P->pad_top + 1;
    s->n_nodes = (int64_t)s->nn[0] * s->nn[1] * s->nn[2];
    s->x = (double *)calloc(s->n * 3, sizeof(double));
    s->v = (double *)calloc(s->n * 3, sizeof(double));
    s->C = (double *)calloc(s->n * 9, sizeof(double));
    s->F = (double *)calloc(s->n * 9, sizeof(double));
    s->Xrest = (double *)calloc(s->n * 3, sizeof(double));
    s->bottom = (unsigned char *)calloc(s->n, 1);
    s->surface = (unsigned char *)calloc(s->n, 1);
    s->M = (double *)calloc(s->n_nodes, sizeof(double));
    s->MG = (double *)calloc(s->n_nodes * 3, sizeof(double));
    s->V = (double *)calloc(s->n_nodes * 3, sizeof(double));
    s->mu = P->E / (2.0 * (1.0 + P->nu));
    s->lam = P->E * P->nu / ((1.0 + P->nu) * (1.0 - 2.0 * P->nu));
    s->Vp = P->dx * P->dx * P->dx / (double)P->ppc;
    s->mp = P->rho * s->Vp;
    double H = (double)Nz * P->dx;

    /* stratified jitter: m^3 sub-cells per cell, one particle uniform in each.
     * A shaped elastomer keeps the cells k < columns[j Nx + i], numbered in the
     * same (k, j, i) order; a particle's jitter is that of the same particle of
     * the full cuboid (its draw is counted by the cuboid id), so a shaped
     * cloud is a subset of the cuboid's. */
    int64_t kept = 0;
    for (int k = 0; k < Nz; ++k)
        for (int j = 0; j < Ny; ++j)
            for (int i = 0; i < Nx; ++i) {
                if (s->P.columns && k >= s->P.columns[(int64_t)j * Nx + i]) continue;
                int top_k = s->P.columns ? s->P.columns[(int64_t)j * Nx + i] - 1 : Nz - 1;
                int64_t cell_full = ((int64_t)k * Ny + j) * Nx + i;
                int64_t cell = kept++;
                for (int sz = 0; sz < m; ++sz)
                    for (int sy = 0; sy < m; ++sy)
                        for (int sx = 0; sx < m; ++sx) {
                            int64_t sub = (sz * m + sy) * m + sx;
                            int64_t id = cell * P->ppc + sub, id_full = cell_full * P->ppc + sub;
                            int cidx[3] = {i, j, k}, sidx[3] = {sx, sy, sz};
                            for (int a = 0; a < 3; ++a) {
                                /* in-cell offset r in [0,1), rounded to FP32 so that the
                                 * start state is exactly representable on an FP32 device */
                                double u = sm64_unit(P->seed, (uint64_t)(3 * id_full + a + 1));
                                float r = (float)(((double)sidx[a] + u) / (double)m);
                                double xa = ((double)cidx[a] + (double)r) * P->dx;
                                s->x[3 * id + a] = xa;
                                s->Xrest[3 * id + a] = xa;
                            }
                            s->F[9 * id + 0] = 1.0; s->F[9 * id + 4] = 1.0; s->F[9 * id + 8] = 1.0;
                            s->bottom[id] = s->Xrest[3 * id + 2] < P->fixed_z_fraction * H;
                            s->surface[id] = (k == top_k && sz == m - 1);
                        }
            }

    memcpy(s->pos, P->pose0, 3 * sizeof(double));
    memcpy(s->quat, P->pose0 + 3, 4 * sizeof(double));
    quat_normalize(s->quat);
    memcpy(s->tpos, s->pos, sizeof(s->pos));
    memcpy(s->tquat, s->quat, sizeof(s->quat));
    s->min_margin = INFINITY;
    s->threads = 1;

    /* calibration points: x_o the body-fixed lowest point (with object particles:
     * the object's bottom particle), x_e the nearest elastomer particle */
    body_lowest_point(P, s->po_body);
    if (P->object_mode == 1 && P->shape != 0) make_object_particles(s, m);
    double Rq[9], xo[3];
    quat_to_matrix(s->quat, Rq);
    for (int a = 0; a < 3; ++a)
        xo[a] = s->pos[a] + Rq[3 * a] * s->po_body[0] + Rq[3 * a + 1] * s->po_body[1] + Rq[3 * a + 2] * s->po_body[2];
    double best = 1e300;
    s->e = 0;
    for (int64_t p = 0; p < s->n; ++p) {
        double d0 = s->x[3 * p] - xo[0], d1 = s->x[3 * p + 1] - xo[1], d2 = s->x[3 * p + 2] - xo[2];
        double d = d0 * d0 + d1 * d1 + d2 * d2;
        if (d < best) { best = d; s->e = p; }
    }
    return s;
}

/* ---------------------------------------------------------------- one exchange */

/* Particle-to-grid, Eq. (1)-(4). h is the executed step length; with_stress = 0
 * drops the elastic momentum ME_i (Eq. 4) and transfers MM_i alone. */
/* Particle-to-grid of elastomer particles [p0, p1) and object particles
 * [q0, q1) into the node arrays M, MG (added to). */
static void p2g_range(const orc_sim *s, double h, int with_stress, const step_pose *sp, int64_t p0, int64_t p1,
                      int64_t q0, int64_t q1, double *M, double *MG) {
    const double dx = s->P.dx;
    const double coef = -4.0 * h / (dx * dx);
    for (int64_t p = p0; p < p1; ++p) {
        const double *xp = s->x + 3 * p, *vp = s->v + 3 * p, *Cp = s->C + 9 * p, *Fp = s->F + 9 * p;
        int base[3];
        double w[3][3];
        stencil(s, xp, base, w);
        double tau[9], A[9];
        if (with_stress) orc_kirchhoff(Fp, s->mu, s->lam, tau);
        for (int k = 0; k < 9; ++k) A[k] = (with_stress ? coef * s->Vp * tau[k] : 0.0) + s->mp * Cp[k];
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + c;
                    double X[3];
                    node_pos(s, i, j, k, X);
                    double d[3] = {X[0] - xp[0], X[1] - xp[1], X[2] - xp[2]};
                    double wt = w[0][a] * w[1][b] * w[2][c];
                    int64_t ni = node_index(s, i, j, k);
                    M[ni] += wt * s->mp;
                    for (int r = 0; r < 3; ++r)
                        MG[3 * ni + r] += wt * (s->mp * vp[r] + (A[3 * r] * d[0] + A[3 * r + 1] * d[1] + A[3 * r + 2] * d[2]));
                }
    }
    /* Object particles (Algorithm 1: their velocities are set to the object's
     * prescribed motion before the exchange): velocity v_o + w x (x_p - c) and
     * affine matrix C = [w]x of the rigid motion, mass m_obj, no stress. */
    if (sp && q1 > q0) {
        const double *w = sp->w;
        double Cr[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
        for (int64_t q = q0; q < q1; ++q) {
            const double *xp = s->obj_x + 3 * q;
            double vq[3];
            rigid_velocity(sp, xp, vq);
            int base[3];
            double wgt[3][3];
            stencil(s, xp, base, wgt);
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) {
                        int i = base[0] + a, j = base[1] + b, k = base[2] + c;
                        double X[3];
                        node_pos(s, i, j, k, X);
                        double d[3] = {X[0] - xp[0], X[1] - xp[1], X[2] - xp[2]};
                        double wt = wgt[0][a] * wgt[1][b] * wgt[2][c];
                        int64_t ni = node_index(s, i, j, k);
                        M[ni] += wt * s->m_obj;
                        for (int r = 0; r < 3; ++r)
                            MG[3 * ni + r] += wt * (s->m_obj * vq[r] +
                                                    s->m_obj * (Cr[3 * r] * d[0] + Cr[3 * r + 1] * d[1] + Cr[3 * r + 2] * d[2]));
                    }
        }
    }
}

/* Particle-to-grid, Eq. (1)-(4). h is the executed step length; with_stress = 0
 * drops the elastic momentum ME_i (Eq. 4) and transfers MM_i alone; sp (may be
 * NULL) is the step's pose, which the object particles' velocities follow. */
static void p2g_ex(orc_sim *s, double h, int with_stress, const step_pose *sp) {
    memset(s->M, 0, s->n_nodes * sizeof(double));
    memset(s->MG, 0, s->n_nodes * 3 * sizeof(double));
    const int T = s->threads;
    if (T <= 1) {
        p2g_range(s, h, with_stress, sp, 0, s->n, 0, sp ? s->n_obj : 0, s->M, s->MG);
        return;
    }
    if (!s->Mt) {
        s->Mt = (double *)malloc((size_t)T * s->n_nodes * sizeof(double));
        s->MGt = (double *)malloc((size_t)T * s->n_nodes * 3 * sizeof(double));
    }
    const int64_t nq = sp ? s->n_obj : 0;
#pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int t = 0; t < T; ++t) {
        double *M = s->Mt + (size_t)t * s->n_nodes, *MG = s->MGt + (size_t)t * s->n_nodes * 3;
        memset(M, 0, s->n_nodes * sizeof(double));
        memset(MG, 0, s->n_nodes * 3 * sizeof(double));
        p2g_range(s, h, with_stress, sp, s->n * t / T, s->n * (t + 1) / T, nq * t / T, nq * (t + 1) / T, M, MG);
    }
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t i = 0; i < s->n_nodes; ++i)
        for (int t = 0; t < T; ++t) {
            s->M[i] += s->Mt[(size_t)t * s->n_nodes + i];
            for (int r = 0; r < 3; ++r) s->MG[3 * i + r] += s->MGt[((size_t)t * s->n_nodes + i) * 3 + r];
        }
}

void orc_p2g(orc_sim *s, double h) { p2g_ex(s, h, 1, NULL); }

/* Grid velocity, Eq. (5); relative-rest contact with the rigid indenter; zero
 * velocity on boundary nodes.  Flags let the invariant tests switch parts off. */
void orc_grid_update_ex(orc_sim *s, const step_pose *sp, int use_contact, int use_bc) {
#pragma omp parallel for num_threads(s->threads) schedule(static) if (s->threads > 1)
    for (int k = 0; k < s->nn[2]; ++k)
        for (int j = 0; j < s->nn[1]; ++j)
            for (int i = 0; i < s->nn[0]; ++i) {
                int64_t ni = node_index(s, i, j, k);
                double *V = s->V + 3 * ni;
                if (s->M[ni] > 0.0) {
                    for (int r = 0; r < 3; ++r) V[r] = s->MG[3 * ni + r] / s->M[ni];
                } else {
                    V[0] = V[1] = V[2] = 0.0;
                }
                if (use_contact && sp) {
                    double X[3];
                    node_pos(s, i, j, k, X);
                    if (node_inside(s, sp, X)) rigid_velocity(sp, X, V);
                }
                if (use_bc && is_boundary_node(s, i, j, k)) V[0] = V[1] = V[2] = 0.0;
            }
}

/* Grid-to-particle, Eq. (6)-(7), with the bottom rule of the relative-rest step. */
void orc_g2p_ex(orc_sim *s, int bottom_rule) {
    const double dx = s->P.dx;
    const double cc = 4.0 / (dx * dx);
#pragma omp parallel for num_threads(s->threads) schedule(static) if (s->threads > 1)
    for (int64_t p = 0; p < s->n; ++p) {
        const double *xp = s->x + 3 * p;
        int base[3];
        double w[3][3];
        stencil(s, xp, base, w);
        double vn[3] = {0, 0, 0}, Cn[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int i = base[0] + a, j = base[1] + b, k = base[2] + c;
                    double X[3];
                    node_pos(s, i, j, k, X);
                    double d[3] = {X[0] - xp[0], X[1] - xp[1], X[2] - xp[2]};
                    double wt = w[0][a] * w[1][b] * w[2][c];
                    const double *V = s->V + 3 * node_index(s, i, j, k);
                    for (int r = 0; r < 3; ++r) {
                        vn[r] += wt * V[r];
                        for (int q = 0; q < 3; ++q) Cn[3 * r + q] += cc * wt * V[r] * d[q];
                    }
                }
        if (bottom_rule && s->bottom[p]) vn[2] = 0.0;
        memcpy(s->v + 3 * p, vn, sizeof(vn));
        memcpy(s->C + 9 * p, Cn, sizeof(Cn));
    }
}

/* Object particles follow the rigid motion exactly: body point p at the pose
 * `sp` (its centre and rotation). */
static void place_object(orc_sim *s, const step_pose *sp) {
    for (int64_t q = 0; q < s->n_obj; ++q) {
        const double *p = s->obj_body + 3 * q;
        for (int a = 0; a < 3; ++a)
            s->obj_x[3 * q + a] = sp->c[a] + sp->R[3 * a] * p[0] + sp->R[3 * a + 1] * p[1] + sp->R[3 * a + 2] * p[2];
    }
}

/* Particle movement, Eq. (8)-(9). */
void orc_commit(orc_sim *s, double h) {
#pragma omp parallel for num_threads(s->threads) schedule(static) if (s->threads > 1)
    for (int64_t p = 0; p < s->n; ++p) {
        double *Fp = s->F + 9 * p, *Cp = s->C + 9 * p;
        double Fn[9];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                double acc = Fp[3 * r + q];
                for (int t = 0; t < 3; ++t) acc += h * Cp[3 * r + t] * Fp[3 * t + q];
                Fn[3 * r + q] = acc;
            }
        memcpy(Fp, Fn, sizeof(Fn));
        for (int a = 0; a < 3; ++a) s->x[3 * p + a] += h * s->v[3 * p + a];
    }
}

/* Velocity the grid gives the calibration particle (its G2P velocity). */
static void gather_velocity(const orc_sim *s, const double *xp, double *out) {
    int base[3];
    double w[3][3];
    stencil(s, xp, base, w);
    out[0] = out[1] = out[2] = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double *V = s->V + 3 * node_index(s, base[0] + a, base[1] + b, base[2] + c);
                double wt = w[0][a] * w[1][b] * w[2][c];
                for (int r = 0; r < 3; ++r) out[r] += wt * V[r];
            }
}

/* ---------------------------------------------------------------- Algorithm 1 */

/* Every particle's stencil inside the grid, its state finite and det F > 0. */
static int check_particle(const orc_sim *s, int64_t p, const double *off) {
    for (int a = 0; a < 3; ++a) {
        double xg = s->x[3 * p + a] / s->P.dx + off[a];
        if (!isfinite(xg) || !isfinite(s->v[3 * p + a])) return 2;
        double b = floor(xg - 0.5);
        if (b < 0.0 || b + 2.0 > (double)(s->nn[a] - 1)) return 1;
    }
    for (int k = 0; k < 9; ++k)
        if (!isfinite(s->C[9 * p + k]) || !isfinite(s->F[9 * p + k])) return 2;
    if (!(det3(s->F + 9 * p) > 0.0)) return 3;
    return 0;
}

static int check_state(orc_sim *s) {
    double off[3] = {(double)s->P.pad_lateral, (double)s->P.pad_lateral, (double)s->P.pad_bottom};
    if (s->threads > 1) {
        /* the code of the first failing particle, as the serial scan finds it */
        int64_t first = s->n;
#pragma omp parallel for num_threads(s->threads) schedule(static) reduction(min : first)
        for (int64_t p = 0; p < s->n; ++p)
            if (p < first && check_particle(s, p, off)) first = p;
        if (first < s->n) return check_particle(s, first, off);
        for (int64_t q = 0; q < s->n_obj; ++q)
            for (int a = 0; a < 3; ++a) {
                double b = floor(s->obj_x[3 * q + a] / s->P.dx + off[a] - 0.5);
                if (b < 0.0 || b + 2.0 > (double)(s->nn[a] - 1)) return 1;
            }
        return 0;
    }
    for (int64_t p = 0; p < s->n; ++p) {
        for (int a = 0; a < 3; ++a) {
            double xg = s->x[3 * p + a] / s->P.dx + off[a];
            if (!isfinite(xg) || !isfinite(s->v[3 * p + a])) return 2;
            double b = floor(xg - 0.5);
            if (b < 0.0 || b + 2.0 > (double)(s->nn[a] - 1)) return 1;
        }
        for (int k = 0; k < 9; ++k)
            if (!isfinite(s->C[9 * p + k]) || !isfinite(s->F[9 * p + k])) return 2;
        if (!(det3(s->F + 9 * p) > 0.0)) return 3;
    }
    for (int64_t q = 0; q < s->n_obj; ++q)
        for (int a = 0; a < 3; ++a) {
            double b = floor(s->obj_x[3 * q + a] / s->P.dx + off[a] - 0.5);
            if (b < 0.0 || b + 2.0 > (double)(s->nn[a] - 1)) return 1;
        }
    return 0;
}

/* One executed step (index j of N in the current orc_step call, length h). */
static void impm_step(orc_sim *s, int64_t j, int64_t N, double h) {
    step_pose sp;
    make_step_pose(s, j, N, h, &sp);
    /* object calibration point and its tangential velocity */
    double xo[3], vo_at[3];
    for (int a = 0; a < 3; ++a)
        xo[a] = sp.c[a] + sp.R[3 * a] * s->po_body[0] + sp.R[3 * a + 1] * s->po_body[1] + sp.R[3 * a + 2] * s->po_body[2];
    rigid_velocity(&sp, xo, vo_at);
    double gnorm = sqrt(vo_at[0] * vo_at[0] + vo_at[1] * vo_at[1]);

    int plain = s->P.mode == 1;
    int forced = -1;
    if (s->forced && s->forced_pos < s->n_forced) forced = s->forced[s->forced_pos++];

    int cnt = 0;
    for (;;) {
        /* The elastic impulse of the step enters the first exchange; later passes
         * only re-exchange momentum so that the velocity field relaxes towards the
         * object's (unless the literal every-pass variant is asked for). */
        p2g_ex(s, h, cnt == 0 || s->P.stress_each_pass, &sp);
        orc_grid_update_ex(s, &sp, s->P.object_mode != 1, 1);
        /* relative-rest test on the calibration particle, before its G2P */
        double ve[3];
        gather_velocity(s, s->x + 3 * s->e, ve);
        orc_g2p_ex(s, !plain);
        cnt += 1;
        int stop;
        if (forced > 0) {
            stop = cnt >= forced;
        } else if (plain) {
            stop = 1;
        } else if (gnorm <= 1e-9) {
            stop = 1;
            s->last_r = 0.0;
        } else {
            double dvx = ve[0] - vo_at[0], dvy = ve[1] - vo_at[1];
            double r = sqrt(dvx * dvx + dvy * dvy) / gnorm;
            s->last_r = r;
            if (s->P.rest_threshold > 0.0) {
                double m = fabs(r - s->P.rest_threshold) / s->P.rest_threshold;
                if (m < s->min_margin) s->min_margin = m;
            }
            stop = r <= s->P.rest_threshold;
            if (!stop && cnt >= s->P.rest_limit) { stop = 1; s->limit_hits += 1; }
        }
        if (stop) break;
    }
    s->passes += cnt;
    if (s->pass_log && s->log_len < s->log_cap) s->pass_log[s->log_len++] = cnt;
    orc_commit(s, h);
    if (s->n_obj > 0) {
        step_pose end;
        make_step_pose(s, j + 1, N, h, &end);
        place_object(s, &end);
    }
    s->steps += 1;
}

void orc_set_target_pose(orc_sim *s, const double *pos, const double *quat) {
    memcpy(s->tpos, pos, 3 * sizeof(double));
    memcpy(s->tquat, quat, 4 * sizeof(double));
    quat_normalize(s->tquat);
}

/* Advance n configured substeps (each = subcycle executed steps), moving the
 * indenter from the current pose to the target pose at constant velocity. */
int orc_step(orc_sim *s, int32_t n_substeps) {
    if (n_substeps <= 0) return -1;
    int k = s->P.subcycle > 0 ? s->P.subcycle : 1;
    int64_t N = (int64_t)n_substeps * k;
    double h = s->P.dt / (double)k;
    for (int64_t j = 0; j < N; ++j) {
        if (s->error || (s->error = check_state(s)) != 0) return -2;
        impm_step(s, j, N, h);
    }
    memcpy(s->pos, s->tpos, sizeof(s->pos));
    memcpy(s->quat, s->tquat, sizeof(s->quat));
    s->substeps += n_substeps;
    return 0;
}

/* ---------------------------------------------------------------- accessors */

int64_t orc_num_particles(const orc_sim *s) { return s->n; }
int32_t orc_error(const orc_sim *s) { return s->error; }
int64_t orc_calib_particle(const orc_sim *s) { return s->e; }
void orc_grid_dims(const orc_sim *s, int32_t *out) { out[0] = s->nn[0]; out[1] = s->nn[1]; out[2] = s->nn[2]; }

void orc_get_state(const orc_sim *s, double *x, double *v, double *C, double *F) {
    if (x) memcpy(x, s->x, s->n * 3 * sizeof(double));
    if (v) memcpy(v, s->v, s->n * 3 * sizeof(double));
    if (C) memcpy(C, s->C, s->n * 9 * sizeof(double));
    if (F) memcpy(F, s->F, s->n * 9 * sizeof(double));
}

void orc_set_state(orc_sim *s, const double *x, const double *v, const double *C, const double *F) {
    if (x) memcpy(s->x, x, s->n * 3 * sizeof(double));
    if (v) memcpy(s->v, v, s->n * 3 * sizeof(double));
    if (C) memcpy(s->C, C, s->n * 9 * sizeof(double));
    if (F) memcpy(s->F, F, s->n * 9 * sizeof(double));
}

void orc_get_rest(const orc_sim *s, double *Xrest, unsigned char *bottom, unsigned char *surface) {
    if (Xrest) memcpy(Xrest, s->Xrest, s->n * 3 * sizeof(double));
    if (bottom) memcpy(bottom, s->bottom, s->n);
    if (surface) memcpy(surface, s->surface, s->n);
}

void orc_get_grid(const orc_sim *s, double *M, double *MG, double *V) {
    if (M) memcpy(M, s->M, s->n_nodes * sizeof(double));
    if (MG) memcpy(MG, s->MG, s->n_nodes * 3 * sizeof(double));
    if (V) memcpy(V, s->V, s->n_nodes * 3 * sizeof(double));
}

/* Overwrite the grid mass and momentum (test hook: the boundary and contact
 * rules of the grid update are then exercised on a chosen grid). */
void orc_set_grid(orc_sim *s, const double *M, const double *MG) {
    if (M) memcpy(s->M, M, s->n_nodes * sizeof(double));
    if (MG) memcpy(s->MG, MG, s->n_nodes * 3 * sizeof(double));
}

void orc_get_counters(const orc_sim *s, int64_t *out4, double *last_r) {
    out4[0] = s->substeps; out4[1] = s->steps; out4[2] = s->passes; out4[3] = s->limit_hits;
    if (last_r) *last_r = s->last_r;
}

int64_t orc_num_object(const orc_sim *s) { return s->n_obj; }

/* Threads of the timing leg (1 = serial; returns the value taken). */
int32_t orc_set_threads(orc_sim *s, int32_t threads) {
    s->threads = threads > 1 ? threads : 1;
    free(s->Mt); free(s->MGt);
    s->Mt = s->MGt = NULL;
    return s->threads;
}

/* Object particles: world positions (n_obj * 3) and body-frame positions. */
void orc_get_object(const orc_sim *s, double *x, double *body) {
    if (x && s->n_obj) memcpy(x, s->obj_x, s->n_obj * 3 * sizeof(double));
    if (body && s->n_obj) memcpy(body, s->obj_body, s->n_obj * 3 * sizeof(double));
}

/* Object particle mass, and the P2G of one exchange with the object particles
 * at the start pose of a one-step move to the target (test hook). */
double orc_object_mass(const orc_sim *s) { return s->m_obj; }
void orc_phase_p2g_object(orc_sim *s, double h) {
    step_pose sp;
    make_step_pose(s, 0, 1, h, &sp);
    p2g_ex(s, h, 1, &sp);
}

/* Closest approach of the relative-rest ratio to the threshold so far, as
 * |r - threshold| / threshold (infinity before any test): near the threshold a
 * single-precision evaluation may take the other branch. */
double orc_min_margin(const orc_sim *s) { return s->min_margin; }

/* Place the indenter at a pose (current and target) without stepping: a test
 * hook that lets a state taken elsewhere continue from its pose. */
/* Set the indenter's pose (and target) without stepping; object particles,
 * which move rigidly with the object, are placed at the new pose. */
void orc_set_pose(orc_sim *s, const double *pos, const double *quat) {
    memcpy(s->pos, pos, 3 * sizeof(double));
    memcpy(s->quat, quat, 4 * sizeof(double));
    quat_normalize(s->quat);
    memcpy(s->tpos, s->pos, sizeof(s->pos));
    memcpy(s->tquat, s->quat, sizeof(s->quat));
    if (s->n_obj > 0) {
        step_pose sp;
        make_step_pose(s, 0, 1, s->P.dt, &sp);
        place_object(s, &sp);
    }
}

void orc_get_pose(const orc_sim *s, double *pose7) {
    memcpy(pose7, s->pos, 3 * sizeof(double));
    memcpy(pose7 + 3, s->quat, 4 * sizeof(double));
}

/* x_o at the current pose */
void orc_get_xo(const orc_sim *s, double *xo) {
    double R[9];
    quat_to_matrix(s->quat, R);
    for (int a = 0; a < 3; ++a)
        xo[a] = s->pos[a] + R[3 * a] * s->po_body[0] + R[3 * a + 1] * s->po_body[1] + R[3 * a + 2] * s->po_body[2];
}

void orc_force_passes(orc_sim *s, const int32_t *passes, int64_t n) {
    free(s->forced);
    s->forced = NULL; s->n_forced = 0; s->forced_pos = 0;
    if (n > 0) {
        s->forced = (int32_t *)malloc(n * sizeof(int32_t));
        memcpy(s->forced, passes, n * sizeof(int32_t));
        s->n_forced = n;
    }
}

void orc_enable_pass_log(orc_sim *s, int64_t cap) {
    free(s->pass_log);
    s->pass_log = cap > 0 ? (int32_t *)calloc(cap, sizeof(int32_t)) : NULL;
    s->log_cap = cap; s->log_len = 0;
}

int64_t orc_get_pass_log(const orc_sim *s, int32_t *out, int64_t cap) {
    int64_t n = s->log_len < cap ? s->log_len : cap;
    if (n > 0) memcpy(out, s->pass_log, n * sizeof(int32_t));
    return s->log_len;
}

/* Phase entry points for the invariant tests: one exchange with optional parts.
 * A NULL pose disables the contact rule. */
void orc_phase_p2g(orc_sim *s, double h) { orc_p2g(s, h); }
void orc_phase_p2g_momentum(orc_sim *s) { p2g_ex(s, 0.0, 0, NULL); }
void orc_phase_grid(orc_sim *s, int use_contact, int use_bc) {
    step_pose sp;
    make_step_pose(s, 0, 1, s->P.dt, &sp);
    orc_grid_update_ex(s, &sp, use_contact, use_bc);
}
void orc_phase_g2p(orc_sim *s, int bottom_rule) { orc_g2p_ex(s, bottom_rule); }
void orc_phase_commit(orc_sim *s, double h) { orc_commit(s, h); }

/* Node inside-mask at the start of a 1-step move to the target pose. */
void orc_inside_mask(const orc_sim *s, unsigned char *mask) {
    step_pose sp;
    make_step_pose(s, 0, 1, s->P.dt, &sp);
    for (int k = 0; k < s->nn[2]; ++k)
        for (int j = 0; j < s->nn[1]; ++j)
            for (int i = 0; i < s->nn[0]; ++i) {
                double X[3];
                node_pos(s, i, j, k, X);
                mask[node_index(s, i, j, k)] = (unsigned char)node_inside(s, &sp, X);
            }
}

/* Total energy: kinetic + fixed-corotated elastic. */
double orc_energy(const orc_sim *s) {
    double ek = 0.0, ee = 0.0;
    for (int64_t p = 0; p < s->n; ++p) {
        const double *v = s->v + 3 * p;
        ek += 0.5 * s->mp * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        ee += s->Vp * energy_density(s->F + 9 * p, s->mu, s->lam);
    }
    return ek + ee;
}

/* ---------------------------------------------------------------- surface maps */

static double bspline2(double t) {
    double a = fabs(t);
    if (a < 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/* Surface displacement field: at pixel centres ((u+1/2) L/W, (v+1/2) L/H) the
 * Shepard-normalised 2-D quadratic B-spline average (pitch = pixel size) of the
 * surface particles' displacement x - X_rest.  Out is H x W x 3 (row v, column u);
 * pixels without weight get 0. */
void orc_surface_displacement(const orc_sim *s, double *out, int W, int H) {
    double Lx = (double)s->P.cells[0] * s->P.dx, Ly = (double)s->P.cells[1] * s->P.dx;
    double px = Lx / (double)W, py = Ly / (double)H;
    double *acc = (double *)calloc((size_t)W * H * 4, sizeof(double));
    for (int64_t p = 0; p < s->n; ++p) {
        if (!s->surface[p]) continue;
        const double *xp = s->x + 3 * p, *X0 = s->Xrest + 3 * p;
        for (int v = 0; v < H; ++v) {
            double wy = bspline2((xp[1] - ((double)v + 0.5) * py) / py);
            if (wy == 0.0) continue;
            for (int u = 0; u < W; ++u) {
                double wx = bspline2((xp[0] - ((double)u + 0.5) * px) / px);
                if (wx == 0.0) continue;
                double wt = wx * wy;
                double *a = acc + 4 * ((size_t)v * W + u);
                a[0] += wt;
                for (int r = 0; r < 3; ++r) a[1 + r] += wt * (xp[r] - X0[r]);
            }
        }
    }
    for (size_t q = 0; q < (size_t)W * H; ++q)
        for (int r = 0; r < 3; ++r)
            out[3 * q + r] = acc[4 * q] > 0.0 ? acc[4 * q + 1 + r] / acc[4 * q] : 0.0;
    free(acc);
}

/* Height map h = H_rest + u_z (row v, column u), with H_rest the rest height
 * of the elastomer column under the pixel centre (the slab height for the
 * cuboid; 0 where a shaped elastomer has no column). */
void orc_surface_heightmap(const orc_sim *s, double *out, int W, int H) {
    double *d = (double *)calloc((size_t)W * H * 3, sizeof(double));
    orc_surface_displacement(s, d, W, H);
    int Nx = s->P.cells[0], Ny = s->P.cells[1];
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            double top = (double)s->P.cells[2] * s->P.dx;
            if (s->P.columns) {
                /* the column of the pixel centre ((u+1/2) Nx/W, (v+1/2) Ny/H) cells */
                int i = (int)floor(((double)u + 0.5) * (double)Nx / (double)W);
                int j = (int)floor(((double)v + 0.5) * (double)Ny / (double)H);
                if (i > Nx - 1) i = Nx - 1;
                if (j > Ny - 1) j = Ny - 1;
                top = (double)s->P.columns[(int64_t)j * Nx + i] * s->P.dx;
            }
            size_t q = (size_t)v * W + u;
            out[q] = top + d[3 * q + 2];
        }
    free(d);
}

/* ---------------------------------------------------------------- indenter depth map */

/* Signed inside measure (<= 0 inside) of the indenter at its current pose for
 * n world points X (n x 3): the test that node_inside applies to grid nodes. */
void orc_point_phi(const orc_sim *s, const double *X, int64_t n, double *phi) {
    double R[9];
    quat_to_matrix(s->quat, R);
    for (int64_t q = 0; q < n; ++q) {
        double d[3] = {X[3 * q] - s->pos[0], X[3 * q + 1] - s->pos[1], X[3 * q + 2] - s->pos[2]};
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
        phi[q] = s->P.shape == 0 ? 1.0 : body_phi(&s->P, p);
    }
}

/* Depth of the indenter below the slab's top face along the vertical line
 * through each pixel centre ((u+1/2) Lx/W, (v+1/2) Ly/H), times `scale`:
 * (top - z_low) scale, with z_low the lowest point of the indenter on that
 * line at the target pose (the pose the next orc_step reaches; the current
 * pose after a step); -1e9 where the line misses it.  The indenter may only be
 * rotated about z (then its body z axis is vertical); returns -1 otherwise. */
int orc_indenter_depthmap(const orc_sim *s, int W, int H, double scale, double *out) {
    const double *q = s->tquat;
    if (fabs(q[1]) > 1e-9 || fabs(q[2]) > 1e-9) return -1;
    double R[9];
    quat_to_matrix(q, R);
    const orc_params *P = &s->P;
    double Lx = (double)P->cells[0] * P->dx, Ly = (double)P->cells[1] * P->dx;
    double top = (double)P->cells[2] * P->dx;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            double dx = ((double)u + 0.5) * Lx / (double)W - s->tpos[0];
            double dy = ((double)v + 0.5) * Ly / (double)H - s->tpos[1];
            double px = R[0] * dx + R[3] * dy, py = R[1] * dx + R[4] * dy;
            int hit = 0;
            double zb = 0.0;
            if (P->shape == 1) {
                double r2 = px * px + py * py;
                if (r2 <= P->radius * P->radius) { hit = 1; zb = -sqrt(P->radius * P->radius - r2); }
            } else if (P->shape == 2) {
                double h = P->half_length;
                double t = px < -h ? -h : (px > h ? h : px);
                double d2 = (px - t) * (px - t) + py * py;
                if (d2 <= P->radius * P->radius) { hit = 1; zb = -sqrt(P->radius * P->radius - d2); }
            } else if (P->shape == 3) {
                double f = P->fillet;
                double qx = fabs(px) - (P->half_extent[0] - f), qy = fabs(py) - (P->half_extent[1] - f);
                double ox = qx > 0.0 ? qx : 0.0, oy = qy > 0.0 ? qy : 0.0;
                double o2 = ox * ox + oy * oy;
                if (o2 <= f * f) { hit = 1; zb = -(P->half_extent[2] - f) - sqrt(f * f - o2); }
            } else if (P->shape == 4) {
                if (px * px + py * py <= P->hf_half * P->hf_half) { hit = 1; zb = hf_height(P, px, py); }
            }
            out[(size_t)v * W + u] = hit ? (top - (s->tpos[2] + zb)) * scale : -1e9;
        }
    return 0;
}
