// impm_host.hip -- host runtime and C ABI (include/impm.h) of the IMPM
// elastomer simulator: particle initialisation, the per-step indenter pose
// table, the host side of the device relative-rest loop, the binned particle order
// and the surface raster (arXiv 2405.02914, Sec. III-A and Sec. IV-B).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/impm.h"
#include "impm_device.h"

namespace impm {
__global__ void k_fill(float* p, long long n, float val);
__global__ void k_scan(BatchMap m, int next, int limit_slots);
__global__ void k_scatter(BatchMap m, int cur);
__global__ void k_compact(KArgs a, int cur, float* soa_dst, uint32_t* cell_dst, uint8_t* flags_dst,
                          const uint32_t* id_src, uint32_t* id_dst, long long* e_out, int move_vc);
__global__ void k_surface_accum(KArgs a, SurfArgs s);
__global__ void k_depthmap(KArgs a, DepthArgs g, float* out);
__global__ void k_surface_finish(const unsigned long long* acc, int npix, int W, float top, float dx, int mode,
                                 float* out, const float* col_top, int Nx, int Ny);
}  // namespace impm

using namespace impm;

// Instantiated HIP graphs of step sequences, keyed by everything that is baked
// into their launches (sequence length, buffer parities, pass counts, tile
// shapes and grid sizes).  The graphs read every per-call input (poses, kernel
// records, loop flags) from device memory, so a replay equals the eager launch
// sequence.  Captured on a library-owned stream and replayed on the caller's.
struct GraphCache {
    hipStream_t cap = nullptr;
    std::map<std::vector<long long>, hipGraphExec_t> execs;
    void clear() {
        for (auto& kv : execs) (void)hipGraphExecDestroy(kv.second);
        execs.clear();
    }
    ~GraphCache() {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Capture the launches that emit(stream) enqueues as one graph the first time
// `key` is seen, then launch the graph on `st`.
template <class F>
static hipError_t graph_run(GraphCache& gc, const std::vector<long long>& key, hipStream_t st, F emit) {
    auto it = gc.execs.find(key);
    if (it == gc.execs.end()) {
        hipError_t e;
        if (!gc.cap && (e = hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking)) != hipSuccess) return e;
        if (gc.execs.size() >= 16) gc.clear();
        if ((e = hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
        emit(gc.cap);
        hipGraph_t g = nullptr;
        const hipError_t el = hipGetLastError();
        e = hipStreamEndCapture(gc.cap, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return el != hipSuccess ? el : e;
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return e;
        it = gc.execs.emplace(key, x).first;
    }
    return hipGraphLaunch(it->second, st);
}

struct sim_s {
    sim_params P;
    // Device storage order ("slots"): the particles grouped by the stencil base
    // node of the initial state, tile by tile, so that a tile's particles fill
    // whole cache lines of every plane.  The ABI addresses particles by id.
    std::vector<uint32_t> slot_of, id_of;
    uint32_t* d_id_of = nullptr;
    // Storage compaction: every `compact_every` executed steps the state moves
    // into the current binned order (the device id map moves with it), so that
    // a tile's loads stay on its own cache lines while particles migrate.  The
    // host slot maps are then refreshed from the device only when a host call
    // needs them; until then `e_slot` holds the calibration particle's slot.
    long long compact_every = 0, since_compact = 0;
    float* soa_alt = nullptr;
    uint32_t* cell_alt = nullptr;
    uint8_t* flags_alt = nullptr;
    uint32_t* id_of_alt = nullptr;
    long long* d_e_slot = nullptr;
    bool slots_stale = false;
    long long e_slot = 0;
    bool use_graph = false;       // replay step sequences as HIP graphs
    GraphCache graphs;
    std::vector<double> hf_host;  // height-field table (P.hf points here)
    double* d_hf = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    long long n = 0;             // particles in the device arrays: elastomer, then object
    long long n_el = 0;          // elastomer particles (the ones the ABI addresses)
    long long n_obj = 0;         // object particles (object_mode SIM_OBJECT_PARTICLES)
    unsigned long long* objW = nullptr;   // node accumulators of the object particles' weights
    double obj_h = 0.0, obj_z0 = 0.0;     // their body lattice: spacing, lowest layer centre
    int m = 0;
    int nn[3] = {0, 0, 0};
    long long n_nodes = 0;
    double mu = 0, lam = 0, Vp = 0, mp = 0;
    // tiles (an entry of the compiled tile-shape table)
    int tile_idx = 3;            // 8 x 4 x 4 cells, 256 threads
    int T[3] = {8, 4, 4};
    int NT[3] = {0, 0, 0};
    int n_tiles = 0;
    // device buffers
    float* soa = nullptr;
    uint32_t* cell = nullptr;
    uint8_t* flags = nullptr;
    uint32_t* order[2] = {nullptr, nullptr};
    uint32_t* bstart[2] = {nullptr, nullptr};
    int cur = 0;
    uint32_t* dirrank = nullptr;
    uint32_t* dircount = nullptr;
    uint32_t* newcnt = nullptr;
    float4* scratch = nullptr;
    size_t scratch_cap = 0;   // float4 elements
    float4* gridV = nullptr;
    float* dbgM = nullptr;
    float* dbgMG = nullptr;
    DevState* st = nullptr;
    KArgs* d_args = nullptr;     // device copy of the kernel record (single-sensor launches)
    KArgs h_args;
    bool args_valid = false;
    StepPose* poses = nullptr;
    long long pose_cap = 0;
    float4* surf_rest = nullptr;  // per surface slot: rest offsets, rest cell height
    int32_t* d_surf_of = nullptr; // surface slot of each elastomer id (-1: none)
    long long n_surf = 0;
    // shaped elastomer: column heights (empty: the cuboid), and per kept cell
    // (particle id / ppc) the index of the cuboid cell it is
    std::vector<uint8_t> cols_host;
    std::vector<long long> kept_cell;
    float* d_col_top = nullptr;   // rest height of each column (m), shaped elastomers only
    unsigned long long* surf_acc = nullptr;   // 4 per pixel
    long long surf_cap = 0;
    float* out_tmp = nullptr;
    long long out_cap = 0;
    // host state
    double pos[3], quat[4], tpos[3], tquat[4], po_body[3];
    long long e = 0;
    bool pending = false;        // scratch holds the first exchange of the next step
    int sbin = 0;                // binning under which the scratch was written
    bool keep_grid = false;
    std::vector<int> forced;
    size_t forced_pos = 0;
    long long substeps = 0;
    long long gstep = 0;
    std::string err;
    // pose upload staging: two pinned host buffers, each reused only after the
    // copy that last read it has completed
    StepPose* stage[2] = {nullptr, nullptr};
    long long stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_next = 0;
    // optional timing of the first-pass fused kernel with events on the stream
    bool prof = false;
    int prof_every = 1;            // time the launches of every prof_every-th executed step
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    long long prof_launches = 0;
};

// ------------------------------------------------------------------ helpers

static int fail(sim_t* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

#define HIPCHK(s, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((s), SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: the t-th
// output of the stream seeded with `seed`.
static uint64_t splitmix64_at(uint64_t seed, uint64_t t) {
    uint64_t z = seed + t * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static float rest_offset(uint64_t seed, long long id, int axis, int sub_a, int m) {
    const double u = (double)(splitmix64_at(seed, (uint64_t)(3 * id + axis + 1)) >> 11) *
                     (1.0 / 9007199254740992.0);
    return (float)(((double)sub_a + u) / (double)m);
}

static void quat_mul(const double* a, const double* b, double* o) {
    const double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    const double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    const double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    const double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

static void quat_matrix(const double* q, double* R) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void quat_normalise(double* q) {
    const double s = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= s;
}

// Relative rotation q0 -> q1 as a unit axis and an angle in [0, pi].
static void rel_axis_angle(const double* q0, const double* q1, double* axis, double* angle) {
    const double q0c[4] = {q0[0], -q0[1], -q0[2], -q0[3]};
    double r[4];
    quat_mul(q1, q0c, r);
    if (r[0] < 0.0) for (int k = 0; k < 4; ++k) r[k] = -r[k];
    const double s = std::sqrt(r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    if (s <= 0.0) { axis[0] = 0.0; axis[1] = 0.0; axis[2] = 1.0; *angle = 0.0; return; }
    axis[0] = r[1] / s; axis[1] = r[2] / s; axis[2] = r[3] / s;
    *angle = 2.0 * std::atan2(s, r[0]);
}

// Body-frame lowest point of the indenter (the object calibration point x_o of
// Algorithm 1); ties go to the point farthest from the body z axis, then to the
// lexicographic minimum of (x, y).
static void lowest_point(const sim_params& P, double* p) {
    p[0] = p[1] = p[2] = 0.0;
    if (P.shape == SIM_SHAPE_SPHERE) {
        p[2] = -P.radius;
    } else if (P.shape == SIM_SHAPE_CAPSULE) {
        p[0] = -P.half_length; p[2] = -P.radius;
    } else if (P.shape == SIM_SHAPE_BOX) {
        p[0] = -(P.half_extent[0] - P.fillet);
        p[1] = -(P.half_extent[1] - P.fillet);
        p[2] = -P.half_extent[2];
    } else if (P.shape == SIM_SHAPE_HEIGHTFIELD) {
        // the lowest table sample inside the footprint disc
        const int n = P.hf_n;
        const double step = 2.0 * P.hf_half / (double)(n - 1);
        double bz = 0.0, br2 = 0.0;
        bool found = false;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double x = -P.hf_half + (double)i * step, y = -P.hf_half + (double)j * step;
                const double r2 = x * x + y * y;
                if (r2 > P.hf_half * P.hf_half) continue;
                const double z = P.hf[(size_t)j * n + i];
                bool better = !found || z < bz;
                if (found && z == bz) better = r2 > br2 || (r2 == br2 && (x < p[0] || (x == p[0] && y < p[1])));
                if (better) { found = true; bz = z; br2 = r2; p[0] = x; p[1] = y; p[2] = z; }
            }
    }
}

// Inside measure of the indenter in its body frame (<= 0 inside): the same
// FP64 expressions, in the same order, as the reference's, so that both sample
// the same object particles.
static double body_phi(const sim_params& P, const double* p) {
#pragma clang fp contract(off)
    if (P.shape == SIM_SHAPE_SPHERE) {
        return p[0] * p[0] + p[1] * p[1] + p[2] * p[2] - P.radius * P.radius;
    } else if (P.shape == SIM_SHAPE_CAPSULE) {
        const double hl = P.half_length;
        const double t = p[0] < -hl ? -hl : (p[0] > hl ? hl : p[0]);
        const double qx = p[0] - t;
        return qx * qx + p[1] * p[1] + p[2] * p[2] - P.radius * P.radius;
    } else if (P.shape == SIM_SHAPE_BOX) {
        double out2 = 0.0, inmax = -1e300;
        for (int a = 0; a < 3; ++a) {
            const double q = std::fabs(p[a]) - (P.half_extent[a] - P.fillet);
            const double qp = q > 0.0 ? q : 0.0;
            out2 += qp * qp;
            if (q > inmax) inmax = q;
        }
        const double inside_part = inmax < 0.0 ? inmax : 0.0;
        return std::sqrt(out2) + inside_part - P.fillet;
    } else if (P.shape == SIM_SHAPE_HEIGHTFIELD) {
        if (p[0] * p[0] + p[1] * p[1] > P.hf_half * P.hf_half) return 1.0;
        const int n = P.hf_n;
        const double step = 2.0 * P.hf_half / (double)(n - 1);
        const double u = (p[0] + P.hf_half) / step, v = (p[1] + P.hf_half) / step;
        int i0 = (int)std::floor(u), j0 = (int)std::floor(v);
        i0 = std::min(std::max(i0, 0), n - 2);
        j0 = std::min(std::max(j0, 0), n - 2);
        const double fu = u - (double)i0, fv = v - (double)j0;
        const double* t = P.hf;
        const double z0 = (1.0 - fu) * t[j0 * n + i0] + fu * t[j0 * n + i0 + 1];
        const double z1 = (1.0 - fu) * t[(j0 + 1) * n + i0] + fu * t[(j0 + 1) * n + i0 + 1];
        return ((1.0 - fv) * z0 + fv * z1) - p[2];
    }
    return 1.0;
}

// Object particles (SIM_OBJECT_PARTICLES): the body lattice points
// ((i + 1/2) h, (j + 1/2) h, z_low + (k + 1/2) h), h = dx / m, inside the
// indenter, at most object_cap above its lowest point and with their whole
// stencil at least one node inside the grid at the initial pose (pos, R);
// ordered by k, then j, then i.  lat receives (i, j, k), world the positions.
static void sample_object(const sim_params& P, int m, const int nn[3], const double* pos, const double* R,
                          double z_low, std::vector<int32_t>& lat, std::vector<double>& world) {
#pragma clang fp contract(off)
    const double h = P.dx / (double)m;
    double hx = 0.0, hy = 0.0;
    if (P.shape == SIM_SHAPE_SPHERE) { hx = P.radius; hy = P.radius; }
    else if (P.shape == SIM_SHAPE_CAPSULE) { hx = P.half_length + P.radius; hy = P.radius; }
    else if (P.shape == SIM_SHAPE_BOX) { hx = P.half_extent[0]; hy = P.half_extent[1]; }
    else if (P.shape == SIM_SHAPE_HEIGHTFIELD) { hx = P.hf_half; hy = P.hf_half; }
    const long long ni = (long long)std::ceil(hx / h), nj = (long long)std::ceil(hy / h);
    const long long nk = (long long)std::ceil(P.object_cap / h);
    const double off[3] = {(double)P.pad_lateral, (double)P.pad_lateral, (double)P.pad_bottom};
    lat.clear();
    world.clear();
    for (long long k = 0; k < nk; ++k)
        for (long long j = -nj; j < nj; ++j)
            for (long long i = -ni; i < ni; ++i) {
                const double p[3] = {((double)i + 0.5) * h, ((double)j + 0.5) * h, z_low + ((double)k + 0.5) * h};
                if (body_phi(P, p) > 0.0) continue;
                double w[3];
                bool ok = true;
                for (int a = 0; a < 3; ++a) {
                    w[a] = pos[a] + R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2];
                    const double b = std::floor(w[a] / P.dx + off[a] - 0.5);
                    if (b < 1.0 || b > (double)(nn[a] - 4)) ok = false;
                }
                if (!ok) continue;
                lat.push_back((int32_t)i); lat.push_back((int32_t)j); lat.push_back((int32_t)k);
                world.insert(world.end(), w, w + 3);
            }
}

static void body_to_world(const double* c, const double* R, const double* pb, double* out) {
    for (int a = 0; a < 3; ++a) out[a] = c[a] + R[3 * a] * pb[0] + R[3 * a + 1] * pb[1] + R[3 * a + 2] * pb[2];
}

// Pose table of one sim_step call: N executed steps of length h moving the
// body from (pos, quat) to (tpos, tquat) at constant velocity (Sec. IV-B:
// press, slide and rotate step by step until the target pose).
static void pose_at(const sim_t* s, double frac, double* c, double* R) {
    for (int a = 0; a < 3; ++a) c[a] = s->pos[a] + (s->tpos[a] - s->pos[a]) * frac;
    double axis[3], ang;
    rel_axis_angle(s->quat, s->tquat, axis, &ang);
    const double half = 0.5 * ang * frac;
    const double qs[4] = {std::cos(half), axis[0] * std::sin(half), axis[1] * std::sin(half),
                          axis[2] * std::sin(half)};
    double qj[4];
    quat_mul(qs, s->quat, qj);
    quat_matrix(qj, R);
}

static void make_pose(const sim_t* s, long long j, long long N, double h, StepPose* sp) {
    const double frac = (double)j / (double)N;
    pose_at(s, (double)(j + 1) / (double)N, sp->c_end, sp->R_end);
    for (int a = 0; a < 3; ++a) {
        const double d = s->tpos[a] - s->pos[a];
        sp->c[a] = s->pos[a] + d * frac;
        sp->vo[a] = d / ((double)N * h);
    }
    double axis[3], ang;
    rel_axis_angle(s->quat, s->tquat, axis, &ang);
    const double half = 0.5 * ang * frac;
    const double qs[4] = {std::cos(half), axis[0] * std::sin(half), axis[1] * std::sin(half),
                          axis[2] * std::sin(half)};
    double qj[4];
    quat_mul(qs, s->quat, qj);
    quat_matrix(qj, sp->R);
    for (int a = 0; a < 3; ++a) sp->w[a] = axis[a] * ang / ((double)N * h);
    double xo[3];
    body_to_world(sp->c, sp->R, s->po_body, xo);
    const double r[3] = {xo[0] - sp->c[0], xo[1] - sp->c[1], xo[2] - sp->c[2]};
    const double vx = sp->vo[0] + (sp->w[1] * r[2] - sp->w[2] * r[1]);
    const double vy = sp->vo[1] + (sp->w[2] * r[0] - sp->w[0] * r[2]);
    sp->vot[0] = vx;
    sp->vot[1] = vy;
    sp->gnorm = std::sqrt(vx * vx + vy * vy);
    sp->forced = 0;
    sp->_pad = 0;
}

static KArgs kargs(const sim_t* s) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    const sim_params& P = s->P;
    for (int q = 0; q < 3; ++q) {
        a.nn[q] = s->nn[q];
        a.T[q] = s->T[q];
        a.NT[q] = s->NT[q];
    }
    a.n_tiles = s->n_tiles;
    a.pad_l = P.pad_lateral;
    a.pad_b = P.pad_bottom;
    a.band = P.band;
    a.mode = P.mode;
    a.bottom_rule = P.mode == SIM_MODE_IMPM ? 1 : 0;
    a.rest_limit = P.rest_limit;
    a.stress_each_pass = P.stress_each_pass;
    a.shape = P.shape;
    const double h = P.dt / (double)P.subcycle;
    a.dx = (float)P.dx;
    a.inv_dx = (float)(1.0 / P.dx);
    a.h = (float)h;
    a.h_over_dx = (float)(h / P.dx);
    a.kst = (float)(4.0 * h / (P.rho * P.dx));
    a.mu2 = (float)(2.0 * s->mu);
    a.lam = (float)s->lam;
    a.c4dx = (float)(4.0 / P.dx);
    a.dxd = P.dx;
    a.rest_threshold = P.rest_threshold;
    a.radius = P.radius;
    a.half_length = P.half_length;
    for (int q = 0; q < 3; ++q) a.he[q] = P.half_extent[q];
    a.fillet = P.fillet;
    a.hf = s->d_hf;
    a.hf_n = P.hf_n;
    a.hf_half = P.hf_half;
    a.mp = (float)s->mp;
    a.object_mode = P.object_mode;
    a.kappa = (float)(P.object_density / P.rho);
    a.obj_h = s->obj_h;
    a.obj_z0 = s->obj_z0;
    a.objW = s->objW;
    a.n = s->n;
    a.e = s->slots_stale ? s->e_slot : (long long)s->slot_of[s->e];
    a.soa = s->soa;
    a.cell = s->cell;
    a.flags = s->flags;
    a.scratch = s->scratch;
    a.gridV = s->gridV;
    a.dbgM = s->keep_grid ? s->dbgM : nullptr;
    a.dbgMG = s->keep_grid ? s->dbgMG : nullptr;
    for (int k = 0; k < 2; ++k) {
        a.order[k] = s->order[k];
        a.bstart[k] = s->bstart[k];
    }
    a.dirrank = s->dirrank;
    a.dircount = s->dircount;
    a.newcnt = s->newcnt;
    a.st = s->st;
    a.poses = s->poses;
    return a;
}

// Tile order of the particles: grouped by the tile of their stencil base node
// floor(x - 1/2) and, inside a tile, round-robin over the base nodes (the first
// particle of every base node, then the second, ...), so that the lanes of a
// wave scatter to different nodes -- particles sharing a base node add to the
// same 27 LDS addresses, and same-address LDS atomics of one instruction
// serialise.  cnt receives the tile starts (n_tiles + 1).
static void tile_order(const sim_t* s, const std::vector<uint32_t>& cells, const float* offs,
                       std::vector<uint32_t>& order, std::vector<uint32_t>& cnt) {
    const int T0 = s->T[0], T1 = s->T[1], T2 = s->T[2];
    const long long n = s->n;
    cnt.assign(s->n_tiles + 1, 0);
    std::vector<uint64_t> key(n);
    for (long long k = 0; k < n; ++k) {
        const uint32_t c = cells[k];
        int b[3] = {(int)(c & 1023) - 1, (int)((c >> 10) & 1023) - 1, (int)((c >> 20) & 1023) - 1};
        for (int q = 0; q < 3; ++q) b[q] += offs[(size_t)q * n + k] >= 0.5f ? 1 : 0;
        const int t = ((b[2] / T2) * s->NT[1] + b[1] / T1) * s->NT[0] + b[0] / T0;
        const uint64_t node = ((uint64_t)b[2] * s->nn[1] + b[1]) * s->nn[0] + b[0];   // < 2^30
        key[k] = (node << 32) | (uint64_t)k;
        cnt[t + 1]++;
    }
    std::sort(key.begin(), key.end());
    // rank among the particles of the same base node (indices ascending), then
    // sort by (tile, rank, base node in the tile), which is unique per particle
    std::vector<std::pair<uint64_t, uint32_t>> ord(n);
    uint32_t rank = 0;
    for (long long q = 0; q < n; ++q) {
        const uint64_t node = key[q] >> 32;
        rank = (q > 0 && (key[q - 1] >> 32) == node) ? rank + 1 : 0;
        const int b0 = (int)(node % s->nn[0]), b1 = (int)((node / s->nn[0]) % s->nn[1]);
        const int b2 = (int)(node / ((uint64_t)s->nn[0] * s->nn[1]));
        const uint64_t t = ((uint64_t)(b2 / T2) * s->NT[1] + b1 / T1) * s->NT[0] + b0 / T0;
        const uint64_t local = (uint64_t)tile_slot(b0 % T0, b1 % T1, b2 % T2, T0, T1, T2);   // < 512
        ord[q] = {(t << 22) | ((uint64_t)std::min<uint32_t>(rank, 4095) << 10) | local,
                  (uint32_t)(key[q] & 0xFFFFFFFFu)};
    }
    std::sort(ord.begin(), ord.end());
    for (int t = 0; t < s->n_tiles; ++t) cnt[t + 1] += cnt[t];
    order.resize(n);
    for (long long q = 0; q < n; ++q) order[q] = ord[q].second;
}

// Host-side binning of the stored particles (slots) by tile.
static int rebin_host(sim_t* s, const std::vector<uint32_t>& cells, const std::vector<float>& offs) {
    std::vector<uint32_t> order, cnt;
    tile_order(s, cells, offs.data(), order, cnt);
    HIPCHK(s, hipMemcpyAsync(s->order[s->cur], order.data(), s->n * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->bstart[s->cur], cnt.data(), (s->n_tiles + 1) * 4, hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return SIM_OK;
}

static int set_xe_snapshot(sim_t* s, uint32_t cell, const float f[3]) {
    // both parities hold x_e so that the next step reads it whichever it is
    uint32_t c2[2] = {cell, cell};
    float f2[6] = {f[0], f[1], f[2], f[0], f[1], f[2]};
    HIPCHK(s, hipMemcpyAsync(s->st->xe_cell, c2, sizeof(c2), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->st->xe_f, f2, sizeof(f2), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return SIM_OK;
}

static int alloc_tiles(sim_t* s) {
    for (int q = 0; q < 3; ++q) s->NT[q] = (s->nn[q] - 1 + s->T[q] - 1) / s->T[q];
    s->n_tiles = s->NT[0] * s->NT[1] * s->NT[2];
    const size_t need = (size_t)kTileOps[s->tile_idx].pvol * s->n_tiles;
    for (int k = 0; k < 2; ++k) {
        if (s->bstart[k]) (void)hipFree(s->bstart[k]);
        s->bstart[k] = nullptr;
        HIPCHK(s, hipMalloc(&s->bstart[k], (s->n_tiles + 1) * sizeof(uint32_t)));
    }
    if (s->dircount) (void)hipFree(s->dircount);
    if (s->newcnt) (void)hipFree(s->newcnt);
    s->dircount = s->newcnt = nullptr;
    HIPCHK(s, hipMalloc(&s->dircount, (size_t)s->n_tiles * kDirs * sizeof(uint32_t)));
    HIPCHK(s, hipMalloc(&s->newcnt, (size_t)s->n_tiles * sizeof(uint32_t)));
    HIPCHK(s, hipMemset(s->dircount, 0, (size_t)s->n_tiles * kDirs * sizeof(uint32_t)));
    HIPCHK(s, hipMemset(s->newcnt, 0, (size_t)s->n_tiles * sizeof(uint32_t)));
    if (need > s->scratch_cap) {
        if (s->scratch) (void)hipFree(s->scratch);
        s->scratch = nullptr;
        HIPCHK(s, hipMalloc(&s->scratch, need * sizeof(float4)));
        s->scratch_cap = need;
    }
    return SIM_OK;
}

static int read_cells(sim_t* s, std::vector<uint32_t>& cells, std::vector<float>& offs) {
    cells.resize(s->n);
    offs.resize((size_t)3 * s->n);
    HIPCHK(s, hipMemcpyAsync(cells.data(), s->cell, s->n * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(offs.data(), s->soa + (size_t)F0 * s->n, (size_t)3 * s->n * 4,
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return SIM_OK;
}

// Bring the host slot maps up to date after storage compactions.
static int ensure_slots(sim_t* s) {
    if (!s->slots_stale) return SIM_OK;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    HIPCHK(s, hipMemcpy(s->id_of.data(), s->d_id_of, (size_t)s->n * 4, hipMemcpyDeviceToHost));
    for (long long k = 0; k < s->n; ++k) s->slot_of[s->id_of[k]] = (uint32_t)k;
    s->slots_stale = false;
    return SIM_OK;
}

static int refresh_binning(sim_t* s) {
    if (int rc0 = ensure_slots(s)) return rc0;
    std::vector<uint32_t> cells;
    std::vector<float> offs;
    int rc = read_cells(s, cells, offs);
    if (rc) return rc;
    rc = rebin_host(s, cells, offs);
    if (rc) return rc;
    uint32_t ce;
    float fe[3];
    const size_t se = s->slot_of[s->e];
    HIPCHK(s, hipMemcpy(&ce, s->cell + se, 4, hipMemcpyDeviceToHost));
    for (int q = 0; q < 3; ++q)
        HIPCHK(s, hipMemcpy(&fe[q], s->soa + (size_t)(F0 + q) * s->n + se, 4, hipMemcpyDeviceToHost));
    s->pending = false;
    return set_xe_snapshot(s, ce, fe);
}

static int check_device_error(sim_t* s) {
    int32_t e = 0;
    HIPCHK(s, hipMemcpyAsync(&e, &s->st->error, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (e) {
        char buf[160];
        std::snprintf(buf, sizeof(buf),
                      "device error 0x%x (1: particle moved more than a cell or left the grid, "
                      "2: non-finite state, 4: det F <= 0)", e);
        return fail(s, SIM_ENUMERIC, buf);
    }
    return SIM_OK;
}

// Device copy of the handle's kernel record, refreshed when the record changes
// (buffers reallocated, grid keeping toggled).
static int sync_args(sim_t* s) {
    if (!s->d_args) HIPCHK(s, hipMalloc(&s->d_args, sizeof(KArgs)));
    const KArgs a = kargs(s);
    if (!s->args_valid || std::memcmp(&a, &s->h_args, sizeof(KArgs)) != 0) {
        HIPCHK(s, hipStreamSynchronize(s->stream));
        HIPCHK(s, hipMemcpy(s->d_args, &a, sizeof(KArgs), hipMemcpyHostToDevice));
        s->h_args = a;
        s->args_valid = true;
    }
    return SIM_OK;
}

// Pose table of the next n_substeps (host FP64, staged through pinned memory and
// uploaded on the handle's stream) and the number of exchange passes to launch
// per executed step: 1 for a pure press or PLAIN mode, the forced count when a
// schedule is replayed, LIMIT otherwise (later passes exit when the step has
// converged).
static int prepare_step(sim_t* s, int32_t n_substeps, std::vector<int>& npass) {
    const sim_params& P = s->P;
    const long long N = (long long)n_substeps * P.subcycle;
    const double h = P.dt / (double)P.subcycle;
    if (N > s->pose_cap) {
        HIPCHK(s, hipStreamSynchronize(s->stream));
        if (s->poses) (void)hipFree(s->poses);
        s->poses = nullptr;
        HIPCHK(s, hipMalloc(&s->poses, N * sizeof(StepPose)));
        s->pose_cap = N;
    }
    const int b = s->stage_next;
    s->stage_next ^= 1;
    if (!s->stage_ev[b]) HIPCHK(s, hipEventCreateWithFlags(&s->stage_ev[b], hipEventDisableTiming));
    HIPCHK(s, hipEventSynchronize(s->stage_ev[b]));   // the copy that last read this buffer
    if (N > s->stage_cap[b]) {
        if (s->stage[b]) (void)hipHostFree(s->stage[b]);
        s->stage[b] = nullptr;
        HIPCHK(s, hipHostMalloc(&s->stage[b], N * sizeof(StepPose), hipHostMallocDefault));
        s->stage_cap[b] = N;
    }
    StepPose* poses = s->stage[b];
    npass.assign(N, 1);
    for (long long j = 0; j < N; ++j) {
        StepPose& sp = poses[j];
        make_pose(s, j, N, h, &sp);
        if (s->forced_pos < s->forced.size()) sp.forced = s->forced[s->forced_pos++];
        if (sp.forced > 0) npass[j] = sp.forced;
        else if (P.mode == SIM_MODE_PLAIN || sp.gnorm <= 1e-9) npass[j] = 1;
        else npass[j] = P.rest_limit;
    }
    HIPCHK(s, hipMemcpyAsync(s->poses, poses, N * sizeof(StepPose), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipEventRecord(s->stage_ev[b], s->stream));
    return sync_args(s);
}

// The stand-alone particle-to-grid of a step's first exchange starts from
// empty object-weight accumulators (a kernel fill: no memset node in graphs).
static void clear_object_weights(sim_t* s, hipStream_t st) {
    if (!s->objW) return;
    const long long nf = s->n_nodes * 2;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<long long>((nf + 255) / 256, 4096)), dim3(256), 0, st,
                       reinterpret_cast<float*>(s->objW), nf, 0.0f);
}

static bool coop_supported() {
    static int ok = -1;
    if (ok < 0) {
        int dev = 0, coop = 0;
        ok = hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop;
    }
    return ok == 1;
}

// One group of sensors that share a tile shape, launched together.
struct LaunchSet {
    const TileOps* ops;
    BatchMap m;
    int tile_blocks, node_blocks, n;
    int limit_slots;
    hipStream_t st;
    bool coop;                 // passes after the first in one cooperative launch
};

// The kernels of one executed step: node kernel and fused exchange of the first
// pass, the passes after the first (one cooperative launch that stops when the
// relative-rest test is met, or one node + fused launch per pass slot), then
// the counting sort of the next binned order.
static hipError_t launch_step(const LaunchSet& L, int j, int npass, int cur, int sbin, int par, int store,
                              hipEvent_t e0, hipEvent_t e1) {
    L.ops->grid(L.m, L.node_blocks, sbin, j, 0, false, L.st);
    if (e0) (void)hipEventRecord(e0, L.st);
    L.ops->g2p2g(L.m, L.tile_blocks, cur, j, par, 0, store, false, L.st);
    if (e1) (void)hipEventRecord(e1, L.st);
    hipError_t err = hipSuccess;
    if (npass > 1 && L.coop) {
        err = L.ops->extra(L.m, L.tile_blocks, L.node_blocks, cur, j, par, npass, store, L.st);
    } else {
        for (int pass = 1; pass < npass; ++pass) {
            L.ops->grid(L.m, L.node_blocks, cur, j, pass, true, L.st);
            L.ops->g2p2g(L.m, L.tile_blocks, cur, j, par, pass, store, true, L.st);
        }
    }
    hipLaunchKernelGGL(k_scan, dim3(L.n), dim3(1024), 0, L.st, L.m, cur ^ 1, L.limit_slots);
    hipLaunchKernelGGL(k_scatter, dim3(L.tile_blocks), dim3(kBlock), 0, L.st, L.m, cur);
    return err;
}

static void finish_call(sim_t* s, int32_t n_substeps, long long N) {
    s->pending = true;
    std::memcpy(s->pos, s->tpos, sizeof(s->pos));
    std::memcpy(s->quat, s->tquat, sizeof(s->quat));
    s->substeps += n_substeps;
    for (long long j = 0; j < N; ++j) {
        s->sbin = s->cur;
        s->cur ^= 1;
        s->gstep += 1;
    }
}

// Move the state into binned order `cur`, the order of the next step (see
// sim_s).  The order must be a permutation, so a latched device error is
// reported first.  With move_vc false the velocity and affine planes stay
// behind (the new storage holds stale values there): only for a compaction
// inside a sim_step call, whose last step stores v and C of every elastomer
// particle before any reader, and only without object particles, whose v
// and C no step stores.
static int compact_storage(sim_t* s, int cur, bool move_vc = true) {
    const size_t n = (size_t)s->n;
    // each buffer on its own, so that a call after a failed allocation retries
    // exactly the missing ones
    if (!s->soa_alt) HIPCHK(s, hipMalloc(&s->soa_alt, (size_t)NPLANES * n * sizeof(float)));
    if (!s->cell_alt) HIPCHK(s, hipMalloc(&s->cell_alt, n * 4));
    if (!s->flags_alt) HIPCHK(s, hipMalloc(&s->flags_alt, n));
    if (!s->id_of_alt) HIPCHK(s, hipMalloc(&s->id_of_alt, n * 4));
    if (!s->d_e_slot) HIPCHK(s, hipMalloc(&s->d_e_slot, sizeof(long long)));
    if (int rc = check_device_error(s)) return rc;
    const KArgs a = kargs(s);
    long long e_new = a.e;   // kept if the kernel does not report a slot
    HIPCHK(s, hipMemcpyAsync(s->d_e_slot, &e_new, sizeof(long long), hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_compact, dim3(s->n_tiles), dim3(kBlock), 0, s->stream, a, cur, s->soa_alt, s->cell_alt,
                       s->flags_alt, s->d_id_of, s->id_of_alt, s->d_e_slot, move_vc ? 1 : 0);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(&e_new, s->d_e_slot, sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (int rc = check_device_error(s)) return rc;
    std::swap(s->soa, s->soa_alt);
    std::swap(s->cell, s->cell_alt);
    std::swap(s->flags, s->flags_alt);
    std::swap(s->d_id_of, s->id_of_alt);
    s->e_slot = e_new;
    s->slots_stale = true;
    s->since_compact = 0;
    return sync_args(s);
}

static int after_call(sim_t* s, long long N) {
    s->since_compact += N;
    if (s->compact_every > 0 && s->since_compact >= s->compact_every) return compact_storage(s, s->cur);
    return SIM_OK;
}

// Workspace of sim_surface_heightmap_noalloc: the raster's fixed-point pixel
// accumulators (4 per pixel), a fixed device array instead of the handle's
// lazily allocated buffer.  Every device the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: the kernels only ever receive the per-device
// address that hipGetSymbolAddress returns for it.
constexpr long long kNoAllocMaxPixels = 512LL * 512LL;
static __device__ __align__(256) unsigned long long scratch[kNoAllocMaxPixels * 4];   // 8 MiB

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev` (looked up once per device, with
// that device current).
static hipError_t scratch_address(int dev, unsigned long long** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

int sim_params_default(sim_params* p) {
    if (!p) return SIM_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->cells[0] = 32; p->cells[1] = 32; p->cells[2] = 8;
    p->ppc = 8;
    p->dx = 0.5e-3;
    p->seed = 2405;
    p->E = 3.0e5; p->nu = 0.45; p->rho = 1000.0;
    p->dt = 2.0e-5;
    p->subcycle = 2;
    p->pad_lateral = 4; p->pad_top = 4; p->pad_bottom = 2; p->band = 2;
    p->mode = SIM_MODE_IMPM;
    p->rest_limit = 10;
    p->rest_threshold = 0.5;
    p->fixed_z_fraction = 0.5;
    p->shape = SIM_SHAPE_SPHERE;
    p->radius = 4.0e-3;
    p->pose0[0] = 8.0e-3; p->pose0[1] = 8.0e-3; p->pose0[2] = 8.0e-3; p->pose0[3] = 1.0;
    p->object_mode = SIM_OBJECT_COLLIDER;
    p->object_density = p->rho;
    p->object_cap = 2.5e-3;
    return SIM_OK;
}

static int validate(const sim_params* p, std::string& why) {
    if (!p) { why = "null params"; return SIM_EINVAL; }
    for (int q = 0; q < 3; ++q)
        if (p->cells[q] < 1) { why = "cells must be >= 1"; return SIM_EINVAL; }
    int m = 0;
    for (int k = 1; k <= 4; ++k) if (k * k * k == p->ppc) m = k;
    if (!m) { why = "ppc must be 1, 8, 27 or 64"; return SIM_EINVAL; }
    if (!(p->dx > 0) || !(p->dt > 0) || !(p->E > 0) || !(p->rho > 0)) { why = "dx, dt, E, rho must be > 0"; return SIM_EINVAL; }
    if (!(p->nu > 0 && p->nu < 0.5)) { why = "nu must be in (0, 0.5)"; return SIM_EINVAL; }
    if (p->subcycle < 1) { why = "subcycle must be >= 1"; return SIM_EINVAL; }
    if (p->pad_lateral < 1 || p->pad_top < 1 || p->pad_bottom < 1 || p->band < 0) { why = "pads must be >= 1"; return SIM_EINVAL; }
    if (p->rest_limit < 1 || p->rest_limit > 32) { why = "rest_limit must be in [1, 32]"; return SIM_EINVAL; }
    if (!(p->rest_threshold >= 0)) { why = "rest_threshold must be >= 0"; return SIM_EINVAL; }
    if (p->mode != SIM_MODE_IMPM && p->mode != SIM_MODE_PLAIN) { why = "bad mode"; return SIM_EINVAL; }
    if (p->shape < 0 || p->shape > SIM_SHAPE_HEIGHTFIELD) { why = "bad shape"; return SIM_EINVAL; }
    if (p->shape == SIM_SHAPE_HEIGHTFIELD) {
        if (!p->hf || p->hf_n < 2 || p->hf_n > 4096 || !(p->hf_half > 0) || !std::isfinite(p->hf_half)) {
            why = "height field needs hf != NULL, 2 <= hf_n <= 4096 and hf_half > 0";
            return SIM_EINVAL;
        }
        for (long long q = 0; q < (long long)p->hf_n * p->hf_n; ++q)
            if (!std::isfinite(p->hf[q])) { why = "height field has a non-finite sample"; return SIM_EINVAL; }
    }
    const int nn[3] = {p->cells[0] + 2 * p->pad_lateral + 1, p->cells[1] + 2 * p->pad_lateral + 1,
                       p->cells[2] + p->pad_bottom + p->pad_top + 1};
    for (int q = 0; q < 3; ++q)
        if (nn[q] > 1023) { why = "grid too large (at most 1023 nodes per axis)"; return SIM_EINVAL; }
    const long long n = (long long)p->cells[0] * p->cells[1] * p->cells[2] * p->ppc;
    if (n >= (1LL << 31)) { why = "too many particles"; return SIM_EINVAL; }
    double qn = 0;
    for (int k = 3; k < 7; ++k) qn += p->pose0[k] * p->pose0[k];
    if (!(qn > 0)) { why = "pose0 quaternion is zero"; return SIM_EINVAL; }
    if (p->columns) {
        long long cells = 0;
        for (long long q = 0; q < (long long)p->cells[0] * p->cells[1]; ++q) {
            if (p->columns[q] > p->cells[2]) { why = "column heights must be <= cells[2]"; return SIM_EINVAL; }
            cells += p->columns[q];
        }
        if (cells == 0) { why = "the shaped elastomer has no cell"; return SIM_EINVAL; }
    }
    if (p->object_mode != SIM_OBJECT_COLLIDER && p->object_mode != SIM_OBJECT_PARTICLES) {
        why = "bad object_mode";
        return SIM_EINVAL;
    }
    if (p->object_mode == SIM_OBJECT_PARTICLES) {
        // the object particles' node weights (up to about 16 kappa) must stay in
        // the range of the fixed-point node sums
        if (p->shape == SIM_SHAPE_NONE || !(p->object_density > 0) || !(p->object_density <= 1e4 * p->rho) ||
            !(p->object_cap > 0) || !(p->object_cap <= 1e3 * p->dx)) {
            why = "object particles need a shape, 0 < object_density <= 1e4 rho and 0 < object_cap <= 1000 dx";
            return SIM_EINVAL;
        }
    }
    return SIM_OK;
}

int sim_create(const sim_params* p, void* hip_stream, sim_t** out) {
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    std::string why;
    if (validate(p, why) != SIM_OK) {
        std::fprintf(stderr, "sim_create: %s\n", why.c_str());
        return SIM_EINVAL;
    }
    sim_t* s = new sim_t();
    s->P = *p;
    if (p->shape == SIM_SHAPE_HEIGHTFIELD) {
        s->hf_host.assign(p->hf, p->hf + (size_t)p->hf_n * p->hf_n);
        s->P.hf = s->hf_host.data();
    } else {
        s->P.hf = nullptr;
        s->P.hf_n = 0;
    }
    if (p->columns) {
        s->cols_host.assign(p->columns, p->columns + (size_t)p->cells[0] * p->cells[1]);
        s->P.columns = s->cols_host.data();
    }
    const sim_params& P = s->P;
    for (int k = 1; k <= 4; ++k) if (k * k * k == P.ppc) s->m = k;
    const int m = s->m;
    const int Nx = P.cells[0], Ny = P.cells[1], Nz = P.cells[2];
    // the kept cells of the (shaped) elastomer in (k, j, i) order
    for (int k = 0; k < Nz; ++k)
        for (int j = 0; j < Ny; ++j)
            for (int i = 0; i < Nx; ++i)
                if (!P.columns || k < P.columns[(size_t)j * Nx + i])
                    s->kept_cell.push_back(((long long)k * Ny + j) * Nx + i);
    s->n_el = (long long)s->kept_cell.size() * P.ppc;
    s->nn[0] = Nx + 2 * P.pad_lateral + 1;
    s->nn[1] = Ny + 2 * P.pad_lateral + 1;
    s->nn[2] = Nz + P.pad_bottom + P.pad_top + 1;
    s->n_nodes = (long long)s->nn[0] * s->nn[1] * s->nn[2];
    // object particles (stored after the elastomer's ids) at the initial pose
    std::vector<int32_t> obj_lat;
    std::vector<double> obj_world;
    double body_low[3];
    lowest_point(P, body_low);
    if (P.object_mode == SIM_OBJECT_PARTICLES) {
        double q0[4] = {P.pose0[3], P.pose0[4], P.pose0[5], P.pose0[6]};
        quat_normalise(q0);
        double R0[9];
        quat_matrix(q0, R0);
        sample_object(P, m, s->nn, P.pose0, R0, body_low[2], obj_lat, obj_world);
        s->obj_h = P.dx / (double)m;
        s->obj_z0 = body_low[2];
    }
    s->n_obj = (long long)obj_world.size() / 3;
    s->n = s->n_el + s->n_obj;
    s->mu = P.E / (2.0 * (1.0 + P.nu));
    s->lam = P.E * P.nu / ((1.0 + P.nu) * (1.0 - 2.0 * P.nu));
    s->Vp = P.dx * P.dx * P.dx / (double)P.ppc;
    s->mp = P.rho * s->Vp;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return SIM_EHIP; }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) { delete s; return SIM_EHIP; }
        s->own_stream = true;
    }
    auto bail = [&](int rc) { sim_destroy(s); return rc; };
    const size_t n = (size_t)s->n;
    if (hipMalloc(&s->soa, n * NPLANES * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->cell, n * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&s->flags, n) != hipSuccess ||
        hipMalloc(&s->order[0], n * 4) != hipSuccess || hipMalloc(&s->order[1], n * 4) != hipSuccess ||
        hipMalloc(&s->dirrank, n * 4) != hipSuccess ||
        hipMalloc(&s->gridV, (size_t)s->n_nodes * sizeof(float4)) != hipSuccess ||
        hipMalloc(&s->st, sizeof(DevState)) != hipSuccess)
        return bail(SIM_ENOMEM);
    if (alloc_tiles(s) != SIM_OK) return bail(SIM_ENOMEM);
    if (P.shape == SIM_SHAPE_HEIGHTFIELD) {
        if (hipMalloc(&s->d_hf, s->hf_host.size() * sizeof(double)) != hipSuccess) return bail(SIM_ENOMEM);
        if (hipMemcpy(s->d_hf, s->hf_host.data(), s->hf_host.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(SIM_EHIP);
    }

    // stratified jittered particles: one per sub-cell of the m^3 split of each cell
    std::vector<float> host(n * NPLANES, 0.0f);
    std::vector<uint32_t> cells(n);
    std::vector<uint8_t> flags(n);
    s->n_surf = (long long)Nx * Ny * m * m;
    std::vector<float4> srest((size_t)s->n_surf, make_float4(0.f, 0.f, 0.f, 0.f));
    std::vector<int32_t> surf_of((size_t)s->n_el, -1);
    const double H = (double)Nz * P.dx;
    for (long long cell = 0; cell < (long long)s->kept_cell.size(); ++cell) {
        const long long cfull = s->kept_cell[cell];
        const int i = (int)(cfull % Nx), j = (int)((cfull / Nx) % Ny), k = (int)(cfull / ((long long)Nx * Ny));
        const int top_k = P.columns ? P.columns[(size_t)j * Nx + i] - 1 : Nz - 1;
        for (int sz = 0; sz < m; ++sz)
            for (int sy = 0; sy < m; ++sy)
                for (int sx = 0; sx < m; ++sx) {
                    const int sub = (sz * m + sy) * m + sx;
                    const long long id = cell * P.ppc + sub, id_full = cfull * P.ppc + sub;
                    const int ci[3] = {i, j, k}, si[3] = {sx, sy, sz};
                    const int gc[3] = {i + P.pad_lateral, j + P.pad_lateral, k + P.pad_bottom};
                    float r[3];
                    for (int a = 0; a < 3; ++a) {
                        // the jitter of the same particle of the full cuboid
                        r[a] = rest_offset(P.seed, id_full, a, si[a], m);
                        host[(size_t)(F0 + a) * n + id] = r[a];
                    }
                    cells[id] = pack_cell(gc);
                    const double z = ((double)ci[2] + (double)r[2]) * P.dx;
                    uint8_t fl = 0;
                    if (z < P.fixed_z_fraction * H) fl |= FLAG_BOTTOM;
                    if (k == top_k && sz == m - 1) {
                        fl |= FLAG_SURFACE;
                        const long long sidx = ((long long)j * Nx + i) * m * m + sy * m + sx;
                        srest[sidx] = make_float4(r[0], r[1], r[2], (float)k);
                        surf_of[id] = (int32_t)sidx;
                    }
                    flags[id] = fl;
                }
    }
    // object particles: cell and offset of their initial position, lattice
    // indices in G0..G2 (exact in FP32)
    for (long long q = 0; q < s->n_obj; ++q) {
        const long long id = s->n_el + q;
        const int off[3] = {P.pad_lateral, P.pad_lateral, P.pad_bottom};
        int cc[3];
        for (int a = 0; a < 3; ++a) {
            const double g = obj_world[3 * q + a] / P.dx + (double)off[a];
            double fl = std::floor(g);
            float fr = (float)(g - fl);
            if (fr >= 1.0f) { fr = 0.0f; fl += 1.0; }
            cc[a] = (int)fl;
            host[(size_t)(F0 + a) * n + id] = fr;
            host[(size_t)(G0 + a) * n + id] = (float)obj_lat[3 * q + a];
        }
        cells[id] = pack_cell(cc);
        flags[id] = FLAG_OBJECT;
    }
    // indenter pose and calibration points
    std::memcpy(s->pos, P.pose0, sizeof(s->pos));
    std::memcpy(s->quat, P.pose0 + 3, sizeof(s->quat));
    quat_normalise(s->quat);
    std::memcpy(s->tpos, s->pos, sizeof(s->pos));
    std::memcpy(s->tquat, s->quat, sizeof(s->quat));
    std::memcpy(s->po_body, body_low, sizeof(body_low));
    if (s->n_obj > 0) {
        // x_o is the object's bottom particle: the lowest, then the farthest from
        // the body z axis, then the smallest (x, y)
        bool found = false;
        double bz = 0.0, br2 = 0.0;
        for (long long q = 0; q < s->n_obj; ++q) {
#pragma clang fp contract(off)
            const double pb[3] = {((double)obj_lat[3 * q] + 0.5) * s->obj_h, ((double)obj_lat[3 * q + 1] + 0.5) * s->obj_h,
                                  s->obj_z0 + ((double)obj_lat[3 * q + 2] + 0.5) * s->obj_h};
            const double r2 = pb[0] * pb[0] + pb[1] * pb[1];
            const bool better = !found || pb[2] < bz ||
                                (pb[2] == bz && (r2 > br2 || (r2 == br2 && (pb[0] < s->po_body[0] ||
                                                                            (pb[0] == s->po_body[0] && pb[1] < s->po_body[1])))));
            if (better) { found = true; bz = pb[2]; br2 = r2; std::memcpy(s->po_body, pb, sizeof(pb)); }
        }
    }
    double R0[9], xo[3];
    quat_matrix(s->quat, R0);
    body_to_world(s->pos, R0, s->po_body, xo);
    double best = 1e300;
    s->e = 0;
    for (long long id = 0; id < s->n_el; ++id) {
        const uint32_t c = cells[id];
        const int cc[3] = {(int)(c & 1023) - P.pad_lateral, (int)((c >> 10) & 1023) - P.pad_lateral,
                           (int)((c >> 20) & 1023) - P.pad_bottom};
        double d2 = 0;
        for (int a = 0; a < 3; ++a) {
            const double xa = ((double)cc[a] + (double)host[(size_t)(F0 + a) * n + id]) * P.dx;
            const double d = xa - xo[a];
            d2 += d * d;
        }
        if (d2 < best) { best = d2; s->e = id; }
    }
    // G = 0 (F = I), v = 0, C = 0 already
    const float fe[3] = {host[(size_t)F0 * n + s->e], host[(size_t)(F0 + 1) * n + s->e],
                         host[(size_t)(F0 + 2) * n + s->e]};
    const uint32_t ce = cells[s->e];
    {
        // storage order: the tile order of the initial state, so that a wave's
        // loads and stores cover consecutive slots
        std::vector<uint32_t> cnt;
        tile_order(s, cells, host.data() + (size_t)F0 * n, s->id_of, cnt);
        s->slot_of.resize(n);
        for (size_t k = 0; k < n; ++k) s->slot_of[s->id_of[k]] = (uint32_t)k;
        std::vector<float> hp(host.size());
        std::vector<uint32_t> cp(n);
        std::vector<uint8_t> fp(n);
        for (size_t k = 0; k < n; ++k) {
            const size_t id = s->id_of[k];
            for (int q = 0; q < NPLANES; ++q) hp[(size_t)q * n + k] = host[(size_t)q * n + id];
            cp[k] = cells[id];
            fp[k] = flags[id];
        }
        host.swap(hp);
        cells.swap(cp);
        flags.swap(fp);
    }
    if (hipMemcpy(s->soa, host.data(), n * NPLANES * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->cell, cells.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->flags, flags.data(), n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->st, 0, sizeof(DevState)) != hipSuccess)
        return bail(SIM_EHIP);
    if (s->n_obj > 0) {
        if (hipMalloc(&s->objW, (size_t)s->n_nodes * sizeof(unsigned long long)) != hipSuccess) return bail(SIM_ENOMEM);
        if (hipMemset(s->objW, 0, (size_t)s->n_nodes * sizeof(unsigned long long)) != hipSuccess) return bail(SIM_EHIP);
    }
    if (hipMalloc(&s->d_id_of, n * 4) != hipSuccess) return bail(SIM_ENOMEM);
    if (hipMemcpy(s->d_id_of, s->id_of.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) return bail(SIM_EHIP);
    if (hipMalloc(&s->surf_rest, srest.size() * sizeof(float4)) != hipSuccess) return bail(SIM_ENOMEM);
    if (hipMemcpy(s->surf_rest, srest.data(), srest.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess)
        return bail(SIM_EHIP);
    if (hipMalloc(&s->d_surf_of, surf_of.size() * sizeof(int32_t)) != hipSuccess) return bail(SIM_ENOMEM);
    if (hipMemcpy(s->d_surf_of, surf_of.data(), surf_of.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
        hipSuccess)
        return bail(SIM_EHIP);
    if (P.columns) {
        std::vector<float> ct(s->cols_host.size());
        for (size_t q = 0; q < ct.size(); ++q) ct[q] = (float)((double)s->cols_host[q] * P.dx);
        if (hipMalloc(&s->d_col_top, ct.size() * sizeof(float)) != hipSuccess) return bail(SIM_ENOMEM);
        if (hipMemcpy(s->d_col_top, ct.data(), ct.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return bail(SIM_EHIP);
    }
    {
        std::vector<float> offs(host.begin() + (size_t)F0 * n, host.begin() + (size_t)(F0 + 3) * n);
        if (rebin_host(s, cells, offs) != SIM_OK) return bail(SIM_EHIP);
    }
    if (set_xe_snapshot(s, ce, fe) != SIM_OK) return bail(SIM_EHIP);
    *out = s;
    return SIM_OK;
}

void sim_destroy(sim_t* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    void* bufs[] = {s->soa, s->cell, s->flags, s->order[0], s->order[1], s->bstart[0], s->bstart[1],
                    s->dirrank, s->dircount, s->newcnt, s->scratch, s->gridV, s->dbgM, s->dbgMG,
                    s->st, s->poses, s->surf_rest, s->surf_acc, s->out_tmp, s->d_args, s->d_hf,
                    s->d_id_of, s->soa_alt, s->cell_alt, s->flags_alt, s->id_of_alt, s->d_e_slot, s->objW,
                    s->d_surf_of, s->d_col_top};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int k = 0; k < 2; ++k) {
        if (s->stage[k]) (void)hipHostFree(s->stage[k]);
        if (s->stage_ev[k]) (void)hipEventDestroy(s->stage_ev[k]);
    }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int sim_set_indenter_pose(sim_t* s, const double pos[3], const double quat_wxyz[4]) {
    if (!s || !pos || !quat_wxyz) return fail(s, SIM_EINVAL, "null argument");
    double q[4] = {quat_wxyz[0], quat_wxyz[1], quat_wxyz[2], quat_wxyz[3]};
    const double qn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(qn > 0) || !std::isfinite(qn) || !std::isfinite(pos[0] + pos[1] + pos[2]))
        return fail(s, SIM_EINVAL, "bad pose");
    quat_normalise(q);
    std::memcpy(s->tpos, pos, sizeof(s->tpos));
    std::memcpy(s->tquat, q, sizeof(s->tquat));
    return SIM_OK;
}

int sim_set_tile(sim_t* s, int32_t tx, int32_t ty, int32_t tz) {
    return sim_set_tile_threads(s, tx, ty, tz, 256);
}

int sim_set_tile_threads(sim_t* s, int32_t tx, int32_t ty, int32_t tz, int32_t threads) {
    if (!s) return SIM_EINVAL;
    int idx = -1;
    std::string avail;
    for (int k = 0; k < kNumTileOps; ++k) {
        const int* T = kTileOps[k].T;
        if (T[0] == tx && T[1] == ty && T[2] == tz && kTileOps[k].threads == threads) idx = k;
        avail += " " + std::to_string(T[0]) + "x" + std::to_string(T[1]) + "x" + std::to_string(T[2]) + "/" +
                 std::to_string(kTileOps[k].threads);
    }
    if (idx < 0) return fail(s, SIM_EINVAL, "tile shape not compiled in; available:" + avail);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->tile_idx = idx;
    for (int q = 0; q < 3; ++q) s->T[q] = kTileOps[idx].T[q];
    int rc = alloc_tiles(s);
    if (rc) return rc;
    return refresh_binning(s);
}

int sim_step(sim_t* s, int32_t n_substeps) {
    if (!s) return SIM_EINVAL;
    if (n_substeps < 1) return fail(s, SIM_EINVAL, "n_substeps must be >= 1");
    std::vector<int> npass;
    int rc = prepare_step(s, n_substeps, npass);
    if (rc) return rc;
    const long long N = (long long)npass.size();
    LaunchSet L;
    L.ops = &kTileOps[s->tile_idx];
    L.m = BatchMap{s->d_args, nullptr, nullptr, 1, s->n_obj > 0 ? 1 : 0};
    L.tile_blocks = s->n_tiles;
    L.node_blocks = (int)((s->n_nodes + kBlock - 1) / kBlock);
    L.n = 1;
    L.limit_slots = std::min(34, s->P.rest_limit + 2);
    L.st = s->stream;
    L.coop = !(s->use_graph && !s->prof) && coop_supported();   // eager launches only
    if (!s->pending) {
        clear_object_weights(s, s->stream);
        L.ops->p2g(L.m, L.tile_blocks, s->cur, s->stream);
        HIPCHK(s, hipGetLastError());
        s->sbin = s->cur;
    }
    int cur = s->cur, sbin = s->sbin;
    long long g = s->gstep;
    if (s->use_graph && !s->prof) {
        std::vector<long long> key = {N, cur, sbin, g & 1, s->tile_idx, L.tile_blocks, L.node_blocks};
        key.insert(key.end(), npass.begin(), npass.end());
        hipError_t le = hipSuccess;
        const hipError_t e = graph_run(s->graphs, key, s->stream, [&](hipStream_t cs) {
            LaunchSet Lc = L;
            Lc.st = cs;
            int c = cur, sb = sbin;
            long long gg = g;
            for (long long j = 0; j < N; ++j) {
                const hipError_t r =
                    launch_step(Lc, (int)j, npass[j], c, sb, (int)(gg & 1), j == N - 1 ? 1 : 0, nullptr, nullptr);
                if (le == hipSuccess) le = r;
                sb = c;
                c ^= 1;
                gg += 1;
            }
        });
        if (le != hipSuccess) return fail(s, SIM_EHIP, std::string("step launch: ") + hipGetErrorString(le));
        if (e != hipSuccess) return fail(s, SIM_EHIP, std::string("step graph: ") + hipGetErrorString(e));
        finish_call(s, n_substeps, N);
        return after_call(s, N);
    }
    // Eager calls compact inside the call, never at its end: a compaction that
    // fell due at the end of the previous call runs here, after the transfer
    // above (which reads v and C) and before the first step.
    const bool move_vc = s->n_obj > 0;
    if (s->compact_every > 0 && s->since_compact >= s->compact_every) {
        if (int rc2 = compact_storage(s, cur, move_vc)) return rc2;
    }
    for (long long j = 0; j < N; ++j) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (s->prof && g % s->prof_every == 0) {
            while (s->ev_pool.size() < s->ev_used + 2) {
                hipEvent_t e;
                HIPCHK(s, hipEventCreate(&e));
                s->ev_pool.push_back(e);
            }
            e0 = s->ev_pool[s->ev_used++];
            e1 = s->ev_pool[s->ev_used++];
        }
        HIPCHK(s, launch_step(L, (int)j, npass[j], cur, sbin, (int)(g & 1), j == N - 1 ? 1 : 0, e0, e1));
        HIPCHK(s, hipGetLastError());
        sbin = cur;
        cur ^= 1;
        g += 1;
        // eager calls compact between their steps as well; the launches of
        // the next step read the moved state through the refreshed record
        s->since_compact += 1;
        if (j + 1 < N && s->compact_every > 0 && s->since_compact >= s->compact_every) {
            if (int rc2 = compact_storage(s, cur, move_vc)) return rc2;
        }
    }
    finish_call(s, n_substeps, N);
    return SIM_OK;
}

int sim_synchronize(sim_t* s) {
    if (!s) return SIM_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return check_device_error(s);
}

static int surface_raster(sim_t* s, float* out, int W, int H, int on_device, int mode) {
    if (!s || !out || W < 1 || H < 1) return fail(s, SIM_EINVAL, "bad raster arguments");
    const long long npix = (long long)W * H;
    if (npix > s->surf_cap) {
        if (s->surf_acc) (void)hipFree(s->surf_acc);
        s->surf_acc = nullptr;
        HIPCHK(s, hipMalloc(&s->surf_acc, npix * 4 * sizeof(unsigned long long)));
        s->surf_cap = npix;
    }
    const long long nout = npix * (mode == 0 ? 1 : 3);
    float* dst = out;
    if (!on_device) {
        if (nout > s->out_cap) {
            if (s->out_tmp) (void)hipFree(s->out_tmp);
            s->out_tmp = nullptr;
            HIPCHK(s, hipMalloc(&s->out_tmp, nout * sizeof(float)));
            s->out_cap = nout;
        }
        dst = s->out_tmp;
    }
    KArgs a = kargs(s);
    SurfArgs sa;
    sa.W = W; sa.H = H; sa.Nx = s->P.cells[0]; sa.Ny = s->P.cells[1]; sa.m = s->m;
    sa.pad_l = s->P.pad_lateral; sa.pad_b = s->P.pad_bottom;
    sa.pitch_x = (double)s->P.cells[0] / (double)W;
    sa.pitch_y = (double)s->P.cells[1] / (double)H;
    sa.dx = (float)s->P.dx;
    sa.n = s->n;
    sa.rest_r = s->surf_rest;
    sa.surf_of = s->d_surf_of;
    sa.id_of = s->d_id_of;
    sa.acc = s->surf_acc;
    hipLaunchKernelGGL(k_fill, dim3(std::min<long long>((npix * 8 + 255) / 256, 4096)), dim3(256), 0, s->stream,
                       reinterpret_cast<float*>(s->surf_acc), npix * 8, 0.0f);
    hipLaunchKernelGGL(k_surface_accum, dim3((unsigned)((s->n + 255) / 256)), dim3(256), 0, s->stream, a, sa);
    hipLaunchKernelGGL(k_surface_finish, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s->stream,
                       s->surf_acc, (int)npix, W, (float)(s->P.cells[2] * s->P.dx), (float)s->P.dx, mode, dst,
                       s->d_col_top, s->P.cells[0], s->P.cells[1]);
    HIPCHK(s, hipGetLastError());
    if (!on_device) {
        HIPCHK(s, hipMemcpyAsync(out, dst, nout * sizeof(float), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        return check_device_error(s);
    }
    return SIM_OK;
}

int sim_indenter_depthmap(sim_t* s, float* out, int32_t W, int32_t H, double scale, int32_t out_on_device) {
    if (!s || !out || W < 1 || H < 1 || (long long)W * H > (1LL << 30) || !std::isfinite(scale))
        return fail(s, SIM_EINVAL, "bad depth map arguments");
    if (std::fabs(s->tquat[1]) > 1e-9 || std::fabs(s->tquat[2]) > 1e-9)
        return fail(s, SIM_EINVAL, "the depth map needs an indenter rotated about z only");
    const long long npix = (long long)W * H;
    float* dst = out;
    if (!out_on_device) {
        if (npix > s->out_cap) {
            if (s->out_tmp) (void)hipFree(s->out_tmp);
            s->out_tmp = nullptr;
            HIPCHK(s, hipMalloc(&s->out_tmp, npix * sizeof(float)));
            s->out_cap = npix;
        }
        dst = s->out_tmp;
    }
    DepthArgs g;
    g.W = W; g.H = H;
    g.Lx = (double)s->P.cells[0] * s->P.dx;
    g.Ly = (double)s->P.cells[1] * s->P.dx;
    g.top = (double)s->P.cells[2] * s->P.dx;
    g.scale = scale;
    std::memcpy(g.c, s->tpos, sizeof(g.c));
    quat_matrix(s->tquat, g.R);
    hipLaunchKernelGGL(k_depthmap, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s->stream, kargs(s), g, dst);
    HIPCHK(s, hipGetLastError());
    if (!out_on_device) {
        HIPCHK(s, hipMemcpyAsync(out, dst, npix * sizeof(float), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
    }
    return SIM_OK;
}

int sim_surface_heightmap(sim_t* s, float* out, int32_t W, int32_t H, int32_t out_on_device) {
    return surface_raster(s, out, W, H, out_on_device, 0);
}

// Allocation-free height map: the raster of sim_surface_heightmap with its
// accumulators in the fixed workspace `scratch` (through its per-device address).
int sim_surface_heightmap_noalloc(sim_t* s, float* out_device, int32_t W, int32_t H) {
    if (!s || !out_device || W < 1 || H < 1) return fail(s, SIM_EINVAL, "bad raster arguments");
    const long long npix = (long long)W * H;
    if (npix > kNoAllocMaxPixels)
        return fail(s, SIM_EINVAL, "sim_surface_heightmap_noalloc: W*H = " + std::to_string(npix) +
                                       " exceeds its fixed workspace of " + std::to_string(kNoAllocMaxPixels) +
                                       " pixels");
    if (s->device < 0 || s->device >= kMaxDevices) return fail(s, SIM_EINVAL, "device ordinal out of range");
    unsigned long long* acc = nullptr;
    HIPCHK(s, scratch_address(s->device, &acc));
    int prev = 0;
    HIPCHK(s, hipGetDevice(&prev));
    if (prev != s->device) HIPCHK(s, hipSetDevice(s->device));
    KArgs a = kargs(s);
    SurfArgs sa;
    sa.W = W; sa.H = H; sa.Nx = s->P.cells[0]; sa.Ny = s->P.cells[1]; sa.m = s->m;
    sa.pad_l = s->P.pad_lateral; sa.pad_b = s->P.pad_bottom;
    sa.pitch_x = (double)s->P.cells[0] / (double)W;
    sa.pitch_y = (double)s->P.cells[1] / (double)H;
    sa.dx = (float)s->P.dx;
    sa.n = s->n;
    sa.rest_r = s->surf_rest;
    sa.surf_of = s->d_surf_of;
    sa.id_of = s->d_id_of;
    sa.acc = acc;
    // the accumulators keep the previous call's sums: clear them with a kernel
    // (no memset node, so a captured graph of these launches replays correctly)
    hipLaunchKernelGGL(k_fill, dim3(std::min<long long>((npix * 8 + 255) / 256, 4096)), dim3(256), 0, s->stream,
                       reinterpret_cast<float*>(acc), npix * 8, 0.0f);
    hipLaunchKernelGGL(k_surface_accum, dim3((unsigned)((s->n + 255) / 256)), dim3(256), 0, s->stream, a, sa);
    hipLaunchKernelGGL(k_surface_finish, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s->stream, acc,
                       (int)npix, W, (float)(s->P.cells[2] * s->P.dx), (float)s->P.dx, 0, out_device,
                       s->d_col_top, s->P.cells[0], s->P.cells[1]);
    const hipError_t e = hipGetLastError();
    if (prev != s->device) (void)hipSetDevice(prev);
    HIPCHK(s, e);
    return SIM_OK;
}

int sim_surface_displacement(sim_t* s, float* out, int32_t W, int32_t H, int32_t out_on_device) {
    return surface_raster(s, out, W, H, out_on_device, 1);
}

int sim_get_stats(sim_t* s, sim_stats* out) {
    if (!s || !out) return fail(s, SIM_EINVAL, "null argument");
    DevState d;
    HIPCHK(s, hipMemcpyAsync(&d, s->st, sizeof(d), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    std::memset(out, 0, sizeof(*out));
    out->substeps = s->substeps;
    out->steps = (int64_t)d.steps;
    out->passes = (int64_t)d.passes;
    out->limit_hits = (int64_t)d.limit_hits;
    out->last_r = d.last_r;
    out->device_error = d.error;
    std::memcpy(out->pose, s->pos, sizeof(s->pos));
    std::memcpy(out->pose + 3, s->quat, sizeof(s->quat));
    double R[9];
    quat_matrix(s->quat, R);
    body_to_world(s->pos, R, s->po_body, out->xo);
    out->calib_particle = s->e;
    return d.error ? fail(s, SIM_ENUMERIC, "device error latched") : SIM_OK;
}

int sim_num_particles(const sim_t* s, int64_t* n) {
    if (!s || !n) return SIM_EINVAL;
    *n = s->n_el;
    return SIM_OK;
}

int sim_grid_dims(const sim_t* s, int32_t nodes[3]) {
    if (!s || !nodes) return SIM_EINVAL;
    for (int q = 0; q < 3; ++q) nodes[q] = s->nn[q];
    return SIM_OK;
}

int sim_read_particles(sim_t* s, double* x, float* v, float* C, float* G) {
    if (!s) return SIM_EINVAL;
    if (int rc0 = ensure_slots(s)) return rc0;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const size_t n = (size_t)s->n;          // plane pitch (object particles included)
    const size_t ne = (size_t)s->n_el;      // the particles the caller addresses
    if (x) {
        std::vector<uint32_t> cells(n);
        std::vector<float> f(3 * n);
        HIPCHK(s, hipMemcpy(cells.data(), s->cell, n * 4, hipMemcpyDeviceToHost));
        HIPCHK(s, hipMemcpy(f.data(), s->soa + (size_t)F0 * n, 3 * n * 4, hipMemcpyDeviceToHost));
        const int off[3] = {s->P.pad_lateral, s->P.pad_lateral, s->P.pad_bottom};
        for (size_t id = 0; id < ne; ++id) {
            const size_t k = s->slot_of[id];
            const uint32_t c = cells[k];
            const int cc[3] = {(int)(c & 1023), (int)((c >> 10) & 1023), (int)((c >> 20) & 1023)};
            for (int a = 0; a < 3; ++a)
                x[3 * id + a] = ((double)(cc[a] - off[a]) + (double)f[a * n + k]) * s->P.dx;
        }
    }
    auto planes = [&](float* dst, int p0, int np) -> int {
        std::vector<float> tmp((size_t)np * n);
        HIPCHK(s, hipMemcpy(tmp.data(), s->soa + (size_t)p0 * n, (size_t)np * n * 4, hipMemcpyDeviceToHost));
        for (size_t id = 0; id < ne; ++id) {
            const size_t k = s->slot_of[id];
            for (int q = 0; q < np; ++q) dst[np * id + q] = tmp[(size_t)q * n + k];
        }
        return SIM_OK;
    };
    int rc;
    if (v && (rc = planes(v, V0, 3))) return rc;
    if (C && (rc = planes(C, C0, 9))) return rc;
    if (G && (rc = planes(G, G0, 9))) return rc;
    return check_device_error(s);
}

int sim_write_particles(sim_t* s, const double* x, const float* v, const float* C, const float* G) {
    if (!s) return SIM_EINVAL;
    if (int rc0 = ensure_slots(s)) return rc0;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const size_t n = (size_t)s->n;          // plane pitch (object particles included)
    const size_t ne = (size_t)s->n_el;      // the particles the caller addresses
    if (x) {
        std::vector<uint32_t> cells(n);
        std::vector<float> f(3 * n);
        if (s->n_obj > 0) {   // the object particles' slots keep their contents
            HIPCHK(s, hipMemcpy(cells.data(), s->cell, n * 4, hipMemcpyDeviceToHost));
            HIPCHK(s, hipMemcpy(f.data(), s->soa + (size_t)F0 * n, 3 * n * 4, hipMemcpyDeviceToHost));
        }
        const int off[3] = {s->P.pad_lateral, s->P.pad_lateral, s->P.pad_bottom};
        for (size_t id = 0; id < ne; ++id) {
            int cc[3];
            for (int a = 0; a < 3; ++a) {
                const double g = x[3 * id + a] / s->P.dx;
                double fl = std::floor(g);
                float fr = (float)(g - fl);
                if (fr >= 1.0f) { fr = 0.0f; fl += 1.0; }
                cc[a] = (int)fl + off[a];
                if (!std::isfinite(g) || cc[a] < 1 || cc[a] > s->nn[a] - 3)
                    return fail(s, SIM_EINVAL, "particle position outside the grid");
                f[a * n + s->slot_of[id]] = fr;
            }
            cells[s->slot_of[id]] = pack_cell(cc);
        }
        HIPCHK(s, hipMemcpy(s->cell, cells.data(), n * 4, hipMemcpyHostToDevice));
        HIPCHK(s, hipMemcpy(s->soa + (size_t)F0 * n, f.data(), 3 * n * 4, hipMemcpyHostToDevice));
    }
    auto planes = [&](const float* src, int p0, int np) -> int {
        std::vector<float> tmp((size_t)np * n);
        if (s->n_obj > 0)
            HIPCHK(s, hipMemcpy(tmp.data(), s->soa + (size_t)p0 * n, (size_t)np * n * 4, hipMemcpyDeviceToHost));
        for (size_t id = 0; id < ne; ++id) {
            const size_t k = s->slot_of[id];
            for (int q = 0; q < np; ++q) tmp[(size_t)q * n + k] = src[np * id + q];
        }
        HIPCHK(s, hipMemcpy(s->soa + (size_t)p0 * n, tmp.data(), (size_t)np * n * 4, hipMemcpyHostToDevice));
        return SIM_OK;
    };
    int rc;
    if (v && (rc = planes(v, V0, 3))) return rc;
    if (C && (rc = planes(C, C0, 9))) return rc;
    if (G && (rc = planes(G, G0, 9))) return rc;
    return refresh_binning(s);
}

int sim_read_rest(sim_t* s, double* X, uint8_t* flags) {
    if (!s) return SIM_EINVAL;
    const sim_params& P = s->P;
    const int m = s->m;
    if (X) {
        for (long long id = 0; id < s->n_el; ++id) {
            const long long cid = s->kept_cell[id / P.ppc];     // the cuboid cell of the particle
            const int sub = (int)(id % P.ppc);
            const int ci[3] = {(int)(cid % P.cells[0]), (int)((cid / P.cells[0]) % P.cells[1]),
                               (int)(cid / ((long long)P.cells[0] * P.cells[1]))};
            const int si[3] = {sub % m, (sub / m) % m, sub / (m * m)};
            for (int a = 0; a < 3; ++a)
                X[3 * id + a] = ((double)ci[a] + (double)rest_offset(P.seed, cid * P.ppc + sub, a, si[a], m)) * P.dx;
        }
    }
    if (flags) {
        if (int rc0 = ensure_slots(s)) return rc0;
        std::vector<uint8_t> fs(s->n);
        HIPCHK(s, hipMemcpy(fs.data(), s->flags, s->n, hipMemcpyDeviceToHost));
        for (long long id = 0; id < s->n_el; ++id) flags[id] = fs[s->slot_of[id]];
    }
    return SIM_OK;
}

int sim_debug_keep_grid(sim_t* s, int32_t on) {
    if (!s) return SIM_EINVAL;
    if (on && !s->dbgM) {
        HIPCHK(s, hipMalloc(&s->dbgM, (size_t)s->n_nodes * sizeof(float)));
        HIPCHK(s, hipMalloc(&s->dbgMG, (size_t)s->n_nodes * 3 * sizeof(float)));
    }
    s->keep_grid = on != 0;
    return SIM_OK;
}

int sim_read_grid(sim_t* s, float* M, float* MG, float* V) {
    if (!s) return SIM_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if ((M || MG) && !s->dbgM) return fail(s, SIM_ESTATE, "grid keeping is off");
    const size_t nn = (size_t)s->n_nodes;
    if (M) HIPCHK(s, hipMemcpy(M, s->dbgM, nn * 4, hipMemcpyDeviceToHost));
    if (MG) HIPCHK(s, hipMemcpy(MG, s->dbgMG, nn * 12, hipMemcpyDeviceToHost));
    if (V) {
        std::vector<float4> tmp(nn);
        HIPCHK(s, hipMemcpy(tmp.data(), s->gridV, nn * sizeof(float4), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < nn; ++k) { V[3 * k] = tmp[k].x; V[3 * k + 1] = tmp[k].y; V[3 * k + 2] = tmp[k].z; }
    }
    return SIM_OK;
}

int sim_debug_force_passes(sim_t* s, const int32_t* passes, int32_t n) {
    if (!s || n < 0 || (n > 0 && !passes)) return SIM_EINVAL;
    for (int i = 0; i < n; ++i)
        if (passes[i] < 1 || passes[i] > 32) return fail(s, SIM_EINVAL, "forced passes must be in [1, 32]");
    s->forced.assign(passes, passes + n);
    s->forced_pos = 0;
    return SIM_OK;
}

int sim_set_graph(sim_t* s, int32_t on) {
    if (!s) return SIM_EINVAL;
    s->use_graph = on != 0;
    if (!s->use_graph) {
        HIPCHK(s, hipStreamSynchronize(s->stream));
        s->graphs.clear();
    }
    return SIM_OK;
}

int sim_profile(sim_t* s, int32_t on) {
    if (!s) return SIM_EINVAL;
    if (on < 0) return fail(s, SIM_EINVAL, "on must be >= 0");
    s->prof = on != 0;
    s->prof_every = on > 1 ? on : 1;
    return SIM_OK;
}

int sim_set_compaction(sim_t* s, int32_t every_steps) {
    if (!s) return SIM_EINVAL;
    if (every_steps < 0) return fail(s, SIM_EINVAL, "every_steps must be >= 0");
    s->compact_every = every_steps;
    s->since_compact = 0;
    return SIM_OK;
}

int sim_profile_read(sim_t* s, double* ms_total, int64_t* launches) {
    if (!s || !ms_total || !launches) return SIM_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (size_t k = 0; k + 1 < s->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(s, hipEventElapsedTime(&ms, s->ev_pool[k], s->ev_pool[k + 1]));
        s->prof_ms += ms;
        s->prof_launches += 1;
    }
    s->ev_used = 0;
    *ms_total = s->prof_ms;
    *launches = s->prof_launches;
    s->prof_ms = 0.0;
    s->prof_launches = 0;
    return SIM_OK;
}

const char* sim_last_error(const sim_t* s) { return s ? s->err.c_str() : "null handle"; }

// ------------------------------------------------------------------ batched sensors

}  // extern "C"

struct sim_batch_s {
    std::vector<sim_t*> sims;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    struct Group {
        int tile_idx = 0;
        std::vector<int> members;
        KArgs* d_args = nullptr;
        int* d_tile_base = nullptr;
        int* d_node_base = nullptr;
        int* d_active = nullptr;               // members' flags for the launches
        std::vector<int> h_active;             // what d_active holds
        int tile_blocks = 0, node_blocks = 0;
        std::vector<KArgs> h_args;
    };
    std::vector<int> active;                   // per sensor: stepped by sim_batch_step
    std::vector<Group> groups;
    bool use_graph = true;
    GraphCache graphs;
    std::string err;
};

static int bfail(sim_batch_t* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Group the sensors by tile shape; per group the device records of its members
// and the prefix sums that map a launch's blocks to (sensor, tile / node block).
static int batch_build_groups(sim_batch_t* b) {
    for (auto& g : b->groups) {
        (void)hipFree(g.d_args);
        (void)hipFree(g.d_tile_base);
        (void)hipFree(g.d_node_base);
        (void)hipFree(g.d_active);
    }
    b->groups.clear();
    b->active.assign(b->sims.size(), 1);
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int t = b->sims[i]->tile_idx;
        int gi = -1;
        for (int k = 0; k < (int)b->groups.size(); ++k)
            if (b->groups[k].tile_idx == t) gi = k;
        if (gi < 0) {
            b->groups.emplace_back();
            gi = (int)b->groups.size() - 1;
            b->groups[gi].tile_idx = t;
        }
        b->groups[gi].members.push_back(i);
    }
    for (auto& g : b->groups) {
        const int n = (int)g.members.size();
        std::vector<int> tb(n + 1, 0), nb(n + 1, 0);
        for (int k = 0; k < n; ++k) {
            const sim_t* s = b->sims[g.members[k]];
            tb[k + 1] = tb[k] + s->n_tiles;
            nb[k + 1] = nb[k] + (int)((s->n_nodes + kBlock - 1) / kBlock);
        }
        g.tile_blocks = tb[n];
        g.node_blocks = nb[n];
        BHIPCHK(b, hipMalloc(&g.d_args, n * sizeof(KArgs)));
        BHIPCHK(b, hipMalloc(&g.d_tile_base, (n + 1) * sizeof(int)));
        BHIPCHK(b, hipMalloc(&g.d_node_base, (n + 1) * sizeof(int)));
        BHIPCHK(b, hipMemcpy(g.d_tile_base, tb.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
        BHIPCHK(b, hipMemcpy(g.d_node_base, nb.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
        g.h_active.assign(n, 1);
        BHIPCHK(b, hipMalloc(&g.d_active, n * sizeof(int)));
        BHIPCHK(b, hipMemcpy(g.d_active, g.h_active.data(), n * sizeof(int), hipMemcpyHostToDevice));
        g.h_args.assign(n, KArgs());
    }
    return SIM_OK;
}

// Upload the members' active flags of every group whose flags changed (after
// the launches already enqueued have finished: they read the old flags).
static int batch_sync_active(sim_batch_t* b) {
    bool waited = false;
    for (auto& g : b->groups) {
        bool changed = false;
        for (int k = 0; k < (int)g.members.size(); ++k) {
            const int a = b->active[g.members[k]];
            if (a != g.h_active[k]) {
                g.h_active[k] = a;
                changed = true;
            }
        }
        if (changed) {
            if (!waited) {
                BHIPCHK(b, hipStreamSynchronize(b->stream));
                waited = true;
            }
            BHIPCHK(b, hipMemcpy(g.d_active, g.h_active.data(), g.members.size() * sizeof(int),
                                 hipMemcpyHostToDevice));
        }
    }
    return SIM_OK;
}

static int batch_sync_args(sim_batch_t* b) {
    for (auto& g : b->groups) {
        bool changed = false;
        for (int k = 0; k < (int)g.members.size(); ++k) {
            const KArgs a = kargs(b->sims[g.members[k]]);
            if (std::memcmp(&a, &g.h_args[k], sizeof(KArgs)) != 0) {
                g.h_args[k] = a;
                changed = true;
            }
        }
        if (changed) {
            BHIPCHK(b, hipStreamSynchronize(b->stream));
            BHIPCHK(b, hipMemcpy(g.d_args, g.h_args.data(), g.members.size() * sizeof(KArgs),
                                 hipMemcpyHostToDevice));
        }
    }
    return SIM_OK;
}

extern "C" {

int sim_batch_create(const sim_params* params, int32_t n, const int32_t* tiles, void* hip_stream,
                     sim_batch_t** out) {
    if (!out || !params || n < 1) return SIM_EINVAL;
    *out = nullptr;
    for (int i = 1; i < n; ++i)
        if (params[i].dt != params[0].dt || params[i].subcycle != params[0].subcycle ||
            params[i].rest_limit != params[0].rest_limit) {
            std::fprintf(stderr, "sim_batch_create: sensors of a batch share dt, subcycle and rest_limit\n");
            return SIM_EINVAL;
        }
    sim_batch_t* b = new sim_batch_t();
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) { delete b; return SIM_EHIP; }
        b->own_stream = true;
    }
    for (int i = 0; i < n; ++i) {
        sim_t* s = nullptr;
        int rc = sim_create(&params[i], b->stream, &s);
        if (rc) { sim_batch_destroy(b); return rc; }
        b->sims.push_back(s);
        if (tiles) {
            rc = sim_set_tile_threads(s, tiles[4 * i], tiles[4 * i + 1], tiles[4 * i + 2], tiles[4 * i + 3]);
            if (rc) {
                std::fprintf(stderr, "sim_batch_create: sensor %d: %s\n", i, s->err.c_str());
                sim_batch_destroy(b);
                return rc;
            }
        }
    }
    int rc = batch_build_groups(b);
    if (rc) { sim_batch_destroy(b); return rc; }
    *out = b;
    return SIM_OK;
}

void sim_batch_destroy(sim_batch_t* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& g : b->groups) {
        (void)hipFree(g.d_args);
        (void)hipFree(g.d_tile_base);
        (void)hipFree(g.d_node_base);
        (void)hipFree(g.d_active);
    }
    for (sim_t* s : b->sims) sim_destroy(s);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int sim_batch_size(const sim_batch_t* b, int32_t* n) {
    if (!b || !n) return SIM_EINVAL;
    *n = (int32_t)b->sims.size();
    return SIM_OK;
}

int sim_batch_get(sim_batch_t* b, int32_t i, sim_t** out) {
    if (!b || !out || i < 0 || i >= (int)b->sims.size()) return SIM_EINVAL;
    *out = b->sims[i];
    return SIM_OK;
}

int sim_batch_set_indenter_poses(sim_batch_t* b, const double* pos, const double* quat_wxyz) {
    if (!b || !pos || !quat_wxyz) return bfail(b, SIM_EINVAL, "null argument");
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int rc = sim_set_indenter_pose(b->sims[i], pos + 3 * i, quat_wxyz + 4 * i);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + b->sims[i]->err);
    }
    return SIM_OK;
}

int sim_batch_set_active(sim_batch_t* b, const int32_t* active) {
    if (!b || !active) return bfail(b, SIM_EINVAL, "null argument");
    for (int i = 0; i < (int)b->sims.size(); ++i) b->active[i] = active[i] ? 1 : 0;
    return SIM_OK;
}

int sim_batch_step(sim_batch_t* b, int32_t n_substeps) {
    if (!b) return SIM_EINVAL;
    if (n_substeps < 1) return bfail(b, SIM_EINVAL, "n_substeps must be >= 1");
    const int n = (int)b->sims.size();
    int first = -1;
    bool all = true;
    for (int i = 0; i < n; ++i) {
        if (b->active[i] && first < 0) first = i;
        all = all && b->active[i];
    }
    if (first < 0) return SIM_OK;                   // every member sits this call out
    if (!all) {
        // members that sit out keep their binned-order parity only over an even
        // number of executed steps, and the first call prepares every member
        if (((long long)n_substeps * b->sims[first]->P.subcycle) % 2 != 0)
            return bfail(b, SIM_EINVAL, "members can sit out only calls of an even number of executed steps");
        if (!b->sims[first]->pending)
            return bfail(b, SIM_ESTATE, "the first sim_batch_step of a batch steps every member");
    }
    std::vector<int> npass_max, npass;
    for (int i = 0; i < n; ++i) {
        if (!b->active[i]) continue;
        sim_t* s = b->sims[i];
        const int rc = prepare_step(s, n_substeps, npass);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + s->err);
        if (npass_max.empty()) npass_max = npass;
        for (size_t j = 0; j < npass.size(); ++j) npass_max[j] = std::max(npass_max[j], npass[j]);
    }
    int rc = batch_sync_args(b);
    if (rc) return rc;
    rc = batch_sync_active(b);
    if (rc) return rc;
    sim_t* s0 = b->sims[first];
    for (int i = 0; i < n; ++i) {
        const sim_t* s = b->sims[i];
        if (s->cur != s0->cur || s->sbin != s0->sbin || s->pending != s0->pending ||
            ((s->gstep ^ s0->gstep) & 1))
            return bfail(b, SIM_ESTATE, "sensors of a batch must be stepped together");
    }
    const long long N = (long long)npass_max.size();
    for (auto& g : b->groups)
        for (int k : g.members)
            if (b->sims[k]->tile_idx != g.tile_idx)
                return bfail(b, SIM_ESTATE, "sensor " + std::to_string(k) + ": tile shape changed after batch creation");
    std::vector<LaunchSet> sets;
    for (auto& g : b->groups) {
        LaunchSet L;
        L.ops = &kTileOps[g.tile_idx];
        int objects = 0;
        for (int mi : g.members) objects |= b->sims[mi]->n_obj > 0 ? 1 : 0;
        L.m = BatchMap{g.d_args, g.d_tile_base, g.d_node_base, (int)g.members.size(), objects, g.d_active};
        L.tile_blocks = g.tile_blocks;
        L.node_blocks = g.node_blocks;
        L.n = (int)g.members.size();
        L.limit_slots = std::min(34, s0->P.rest_limit + 2);
        L.st = b->stream;
        // Per-pass launches for batches: their members usually do run passes after
        // the first, and there the cooperative kernel's device-scope fences around
        // each grid barrier cost more than the launches they save (an eager batch
        // call took 2.6 times as long).
        L.coop = false;
        sets.push_back(L);
    }
    if (!s0->pending) {
        for (sim_t* s : b->sims) clear_object_weights(s, b->stream);
        for (auto& L : sets) L.ops->p2g(L.m, L.tile_blocks, s0->cur, b->stream);
        for (sim_t* s : b->sims) s->sbin = s->cur;
    }
    int cur = s0->cur, sbin = s0->sbin;
    long long g = s0->gstep;
    hipError_t le = hipSuccess;
    auto emit = [&](hipStream_t st) {
        int c = cur, sb = sbin;
        long long gg = g;
        for (long long j = 0; j < N; ++j) {
            for (auto L : sets) {
                L.st = st;
                const hipError_t r = launch_step(L, (int)j, npass_max[j], c, sb, (int)(gg & 1),
                                                 j == N - 1 ? 1 : 0, nullptr, nullptr);
                if (le == hipSuccess) le = r;
            }
            sb = c;
            c ^= 1;
            gg += 1;
        }
    };
    if (b->use_graph) {
        std::vector<long long> key = {N, cur, sbin, g & 1};
        key.insert(key.end(), npass_max.begin(), npass_max.end());
        const hipError_t e = graph_run(b->graphs, key, b->stream, emit);
        if (e != hipSuccess) return bfail(b, SIM_EHIP, std::string("batch step graph: ") + hipGetErrorString(e));
    } else {
        emit(b->stream);
    }
    if (le != hipSuccess) return bfail(b, SIM_EHIP, std::string("batch step launch: ") + hipGetErrorString(le));
    BHIPCHK(b, hipGetLastError());
    for (int i = 0; i < n; ++i)
        if (b->active[i]) finish_call(b->sims[i], n_substeps, N);
    // Members with storage compaction (sim_set_compaction on a member handle)
    // compact on their own streams once the batch's launches have completed;
    // the next call's argument sync picks up their new buffers.
    bool synced = false;
    for (int i = 0; i < n; ++i) {
        if (!b->active[i]) continue;
        sim_t* s = b->sims[i];
        s->since_compact += N;
        if (s->compact_every > 0 && s->since_compact >= s->compact_every) {
            if (!synced) {
                BHIPCHK(b, hipStreamSynchronize(b->stream));
                synced = true;
            }
            const int rc2 = compact_storage(s, s->cur);
            if (rc2) return bfail(b, rc2, "sensor " + std::to_string(i) + ": " + s->err);
        }
    }
    return SIM_OK;
}

int sim_batch_synchronize(sim_batch_t* b) {
    if (!b) return SIM_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int rc = check_device_error(b->sims[i]);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + b->sims[i]->err);
    }
    return SIM_OK;
}

int sim_batch_heightmaps(sim_batch_t* b, float* out, int32_t W, int32_t H, int32_t out_on_device) {
    if (!b || !out || W < 1 || H < 1) return bfail(b, SIM_EINVAL, "bad raster arguments");
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int rc = sim_surface_heightmap(b->sims[i], out + (size_t)i * W * H, W, H, out_on_device);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + b->sims[i]->err);
    }
    return SIM_OK;
}

int sim_batch_depthmaps(sim_batch_t* b, float* out, int32_t W, int32_t H, double scale, int32_t out_on_device) {
    if (!b || !out || W < 1 || H < 1) return bfail(b, SIM_EINVAL, "bad depth map arguments");
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int rc = sim_indenter_depthmap(b->sims[i], out + (size_t)i * W * H, W, H, scale, out_on_device);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + b->sims[i]->err);
    }
    return SIM_OK;
}

int sim_batch_displacements(sim_batch_t* b, float* out, int32_t W, int32_t H, int32_t out_on_device) {
    if (!b || !out || W < 1 || H < 1) return bfail(b, SIM_EINVAL, "bad raster arguments");
    for (int i = 0; i < (int)b->sims.size(); ++i) {
        const int rc = sim_surface_displacement(b->sims[i], out + (size_t)i * W * H * 3, W, H, out_on_device);
        if (rc) return bfail(b, rc, "sensor " + std::to_string(i) + ": " + b->sims[i]->err);
    }
    return SIM_OK;
}

int sim_batch_set_graph(sim_batch_t* b, int32_t on) {
    if (!b) return SIM_EINVAL;
    b->use_graph = on != 0;
    if (!b->use_graph) {
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        b->graphs.clear();
    }
    return SIM_OK;
}

const char* sim_batch_last_error(const sim_batch_t* b) { return b ? b->err.c_str() : "null handle"; }

// Tile-shape autotuner: time `steps` executed steps of a shallow press on a
// sensor with these parameters for every compiled tile shape (HIP events on
// the sensor's stream), three rounds, and return the fastest.
int sim_autotune_tile(const sim_params* p, int32_t steps, void* hip_stream, int32_t out[4], double* out_ms) {
    if (!p || !out || steps < 1) return SIM_EINVAL;
    sim_t* s = nullptr;
    int rc = sim_create(p, hip_stream, &s);
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { sim_destroy(s); return SIM_EHIP; }
    // every shape is timed in each of kRounds rounds (interleaved, so that a
    // slow spell of the device does not fall on one shape only) and keeps its
    // fastest round; the fastest shape wins
    constexpr int kRounds = 3;
    std::vector<double> fastest(kNumTileOps, 1e300);
    const int sub = std::max(1, steps / std::max(1, p->subcycle));
    double pos[3] = {s->pos[0], s->pos[1], s->pos[2]};
    for (int round = 0; round < kRounds && rc == SIM_OK; ++round)
        for (int k = 0; k < kNumTileOps && rc == SIM_OK; ++k) {
            const TileOps& o = kTileOps[k];
            rc = sim_set_tile_threads(s, o.T[0], o.T[1], o.T[2], o.threads);
            if (rc) break;
            pos[2] -= 1e-3 * p->dx;
            rc = sim_set_indenter_pose(s, pos, s->quat);
            if (!rc && round == 0) rc = sim_step(s, 1);          // warm-up of the shape
            if (rc) break;
            pos[2] -= 1e-3 * p->dx;
            rc = sim_set_indenter_pose(s, pos, s->quat);
            if (rc) break;
            (void)hipEventRecord(e0, s->stream);
            rc = sim_step(s, sub);
            (void)hipEventRecord(e1, s->stream);
            if (rc) break;
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            fastest[k] = std::min(fastest[k], (double)ms);
        }
    int best_k = 0;
    for (int k = 1; k < kNumTileOps; ++k)
        if (fastest[k] < fastest[best_k]) best_k = k;
    const double best = fastest[best_k];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SIM_OK) rc = check_device_error(s);
    sim_destroy(s);
    if (rc) return rc;
    for (int q = 0; q < 3; ++q) out[q] = kTileOps[best_k].T[q];
    out[3] = kTileOps[best_k].threads;
    if (out_ms) *out_ms = best / (double)(sub * p->subcycle);
    return SIM_OK;
}

}  // extern "C"
