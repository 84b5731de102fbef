// impm_device.h -- device-side data structures and math of the IMPM substep
// (arXiv 2405.02914, Sec. III-A, Eq. 1-9 and Algorithm 1) for gfx950.
//
// State layout (structure of arrays, FP32 unless noted, indexed by particle id):
//   cell   uint32  packed grid-cell coordinates ix | iy << 10 | iz << 20
//   f0..2          offset inside that cell, in [0, 1) cell units
//   v0..2          velocity (m/s)
//   C0..8          affine velocity matrix C (1/s), row-major
//   G0..8          F - I, the deformation gradient minus identity, row-major
//   flags  uint8   bit 0: lower layer (v_z = 0 under IMPM), bit 1: surface particle,
//                  bit 2: object particle (the object represented by particles)
// Holding x as cell + offset and F as I + G keeps FP32 relative precision in the
// B-spline weights and in F - R, which the stress depends on.  Object particles
// hold no v, C or G: their G0..G2 planes carry their body-fixed lattice indices
// (i, j, k), exact in FP32, from which every commit places them rigidly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace impm {

constexpr int kBlock = 256;          // threads per block of the tile kernels
constexpr int kWaves = kBlock / 64;  // wave64
constexpr int kDirs = 27;            // neighbour tiles a particle can move to in one step

enum : int { F0 = 0, V0 = 3, C0 = 6, G0 = 15, NPLANES = 24 };
enum : uint8_t { FLAG_BOTTOM = 1, FLAG_SURFACE = 2, FLAG_OBJECT = 4 };
enum : int { DEV_CFL = 1, DEV_NONFINITE = 2, DEV_DETF = 4 };

// Pose of the indenter for one executed step (host FP64 table).
struct StepPose {
    double c[3];       // body origin at the start of the step
    double R[9];       // body -> world rotation, row-major
    double vo[3];      // linear velocity over the step
    double w[3];       // angular velocity over the step
    double vot[2];     // tangential (x, y) velocity of the object point x_o
    double gnorm;      // |vot|
    double c_end[3];   // body origin and rotation at the end of the step, where
    double R_end[9];   // the commit places the object particles
    int32_t forced;    // forced pass count, 0 = decide by the relative-rest test
    int32_t _pad;
};

// Device-resident control block of the relative-rest loop.
struct DevState {
    int32_t finished[34];          // finished[k]: the step ended before pass k
    int32_t error;                 // DEV_* bits
    int32_t _pad;
    unsigned long long steps, passes, limit_hits;
    double last_r;
    uint32_t xe_cell[2];           // x_e snapshot, double-buffered by step parity
    float xe_f[2][3];
};

// Buffers reached through the argument table are generic pointers, and loads
// and stores through them compile to flat instructions, which also count on the
// LDS wait counter: every wait for an LDS read would then also wait for the
// particle loads in flight.  The kernels cast them to the global address space.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) { return (gptr<T>)p; }
// float4 is a class whose members take generic references, so its buffers are
// reached as the plain 4-float vector type instead.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ gptr<f32x4> glb4(float4* p) { return (gptr<f32x4>)p; }

struct KArgs {
    int nn[3];        // nodes per axis
    int T[3];         // tile size in cells
    int NT[3];        // tiles per axis
    int n_tiles;
    int pad_l, pad_b, band;
    int mode, bottom_rule, rest_limit, stress_each_pass;
    int shape;
    float dx, inv_dx, h, h_over_dx, kst, mu2, lam, c4dx;   // c4dx = 4 / dx
    double dxd, rest_threshold, radius, half_length, he[3], fillet;
    const double* hf;          // height-field table (hf_n x hf_n), shape 4
    int hf_n;
    double hf_half;
    float mp;         // particle mass (kg), for the debug grid copy
    // object particles (object_mode 1): mass ratio to an elastomer particle, the
    // body lattice (spacing obj_h, lowest layer centre obj_z0) and the node
    // accumulators of their fixed-point mass weights (null without them)
    int object_mode;
    float kappa;
    double obj_h, obj_z0;
    unsigned long long* objW;
    long long n;      // particles
    long long e;      // calibration particle id
    // buffers
    float* soa;                // NPLANES * n
    uint32_t* cell;
    const uint8_t* flags;
    float4* scratch;           // n_tiles * FPvol partial node sums (W, Px, Py, Pz)
    float4* gridV;             // n_nodes (Vx, Vy, Vz, W)
    float* dbgM;               // n_nodes or null
    float* dbgMG;              // 3 * n_nodes or null
    uint32_t* order[2];        // binned particle order (ids), double-buffered
    uint32_t* bstart[2];       // tile starts of each order (n_tiles + 1)
    uint32_t* dirrank;         // per binned position: rank << 5 | dir
    uint32_t* dircount;        // n_tiles * 27: particles of a tile moving in each direction
    uint32_t* newcnt;          // n_tiles: next step's tile sizes (accumulated)
    DevState* st;
    const StepPose* poses;
};

struct SurfArgs {
    int W, H, Nx, Ny, m, pad_l, pad_b;
    double pitch_x, pitch_y;     // slab cells per pixel
    float dx;
    long long n;
    const float4* rest_r;        // per surface slot (column, sub-column): in-cell rest offsets, rest cell z
    const int32_t* surf_of;      // surface slot of each elastomer particle id (-1: not a surface particle)
    const uint32_t* id_of;       // particle id of each storage slot
    unsigned long long* acc;     // H*W x 4 fixed-point sums (w, w ux, w uy, w uz), u in cells
};

// Indenter depth map: pixel grid over the slab and the indenter's current pose
// (rotation about z only, so the body z axis is vertical).
struct DepthArgs {
    int W, H;
    double Lx, Ly, top, scale;
    double c[3], R[9];        // centre and body->world rotation (row-major)
};

// One launch processes the tiles (or node blocks) of one or several sensors:
// args[s] is sensor s's record in device memory; tile_base and node_base are
// prefix sums of the sensors' tile counts and node-block counts (null for a
// single sensor).
struct BatchMap {
    const KArgs* args;
    const int* tile_base;
    const int* node_base;
    int n;
    int objects;               // some sensor of the launch has object particles
    const int* active;         // n flags: members a batch call steps (NULL: every member)
};

// A member that sits out a batch call: every kernel of the call leaves its
// state alone (its blocks exit before touching it).
__device__ __forceinline__ bool member_active(const BatchMap& m, int s) { return !m.active || m.active[s] != 0; }

__device__ __forceinline__ int batch_find(const int* base, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Launchers of the tile kernels for one compiled tile shape.
struct TileOps {
    int T[3];
    int threads;               // threads per block of the particle kernels
    int pvol;                  // nodes of a tile's particle-to-grid block (scratch record)
    size_t lds_g2p2g;
    void (*p2g)(const BatchMap& m, int tile_blocks, int cur, hipStream_t st);
    void (*grid)(const BatchMap& m, int node_blocks, int sbin, int step, int pass, bool extra,
                 hipStream_t st);
    void (*g2p2g)(const BatchMap& m, int tile_blocks, int cur, int step, int par, int pass,
                  int store_vc, bool extra, hipStream_t st);
    // passes 1..npass-1 of a step in one cooperative launch
    hipError_t (*extra)(const BatchMap& m, int tile_blocks, int node_blocks, int cur, int step, int par, int npass,
                        int store_vc, hipStream_t st);
};
// Cooperative launches are never recorded into a HIP graph: graph replays
// launch one node and one fused kernel per pass slot instead.
extern const TileOps kTileOps[];
extern const int kNumTileOps;

__host__ __device__ __forceinline__ void unpack_cell(uint32_t c, int o[3]) {
    o[0] = c & 1023; o[1] = (c >> 10) & 1023; o[2] = (c >> 20) & 1023;
}
__host__ __device__ __forceinline__ uint32_t pack_cell(const int c[3]) {
    return (uint32_t)c[0] | ((uint32_t)c[1] << 10) | ((uint32_t)c[2] << 20);
}

// Position of the base node (l0, l1, l2) of a tile in the round-robin storage
// order of its particles (a permutation of the tile's base nodes), chosen so
// that the lanes of one LDS atomic in the particle-to-grid block fall on
// distinct banks.  8-cell-wide, 4-cell-deep tiles of even height: a wave's 64
// lanes take two planes, each group of 8 lanes one row: rows 0 and 2 of the
// first plane, rows 0 and 2 of the second, then rows 1 and 3 of both; with the
// row pitch of 12 words and the plane pitch of 16 mod 32 words every 32 lanes
// address 32 distinct 8-byte bank pairs.  Other 8-cell-wide tiles: rows in the
// order 0, 2, 1, 3, 4, 6, 5, 7, ..., so that every 16 lanes do.  Otherwise
// linear.
__host__ __device__ __forceinline__ int tile_slot(int l0, int l1, int l2, int T0, int T1, int T2) {
    if (T0 == 8 && T1 == 4 && (T2 & 1) == 0)
        return (l2 >> 1) * 64 + (l1 & 1) * 32 + (l2 & 1) * 16 + (l1 >> 1) * 8 + l0;
    if (T0 == 8 && (T1 & 3) == 0) l1 = (l1 & ~3) | ((l1 & 1) << 1) | ((l1 >> 1) & 1);
    return (l2 * T1 + l1) * T0 + l0;
}

// Quadratic B-spline stencil along one axis (the 3x3x3 kernel of Eq. 1): the
// particle sits at fx in [0.5, 1.5) from its base node; weights of base, +1, +2.
__device__ __forceinline__ void bspline_axis(int cell, float f, int& base, float& fx,
                                             float w[3]) {
    const bool hi = f >= 0.5f;
    base = cell - 1 + (hi ? 1 : 0);
    fx = hi ? f : f + 1.0f;
    const float a = 1.5f - fx, b = fx - 1.0f, c = fx - 0.5f;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - b * b;
    w[2] = 0.5f * c * c;
}

// Rotation factor of the polar decomposition F = R S with F = I + G, computed
// as R = I + Q by the Newton iteration X <- (X + X^{-T}) / 2 (Higham 1986)
// written in the small quantities: X = I + Y, cof(I+Y) = (1 + tr Y) I - Y^T +
// cof(Y), det(I+Y) = 1 + d with d = tr Y + (tr^2 Y - tr Y^2) / 2 + det Y, so
// X^{-T} - I = (tr Y I - Y^T + cof(Y) - d I) / (1 + d).
__device__ __forceinline__ float det_minus_one(const float Y[9]) {
    const float tr = Y[0] + Y[4] + Y[8];
    const float m2 = (Y[0] * Y[4] - Y[1] * Y[3]) + (Y[0] * Y[8] - Y[2] * Y[6]) +
                     (Y[4] * Y[8] - Y[5] * Y[7]);
    const float d3 = Y[0] * (Y[4] * Y[8] - Y[5] * Y[7]) - Y[1] * (Y[3] * Y[8] - Y[5] * Y[6]) +
                     Y[2] * (Y[3] * Y[7] - Y[4] * Y[6]);
    return tr + m2 + d3;
}

// Each Newton step squares the error: after an update of max-norm u the
// iterate's error is at most about 4.5 u^2 (the factor covers the change of
// norms), so the loop stops after the first update with u^2 <= 2^-27 gs, which
// leaves an error below half an FP32 ulp of gs = max |G| (at most 10 steps).
__device__ __forceinline__ void polar_rotation_minus_identity(const float G[9], float Q[9]) {
    float gs = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) { Q[k] = G[k]; gs = fmaxf(gs, fabsf(G[k])); }
    const float tol2 = 7.4505806e-9f * gs;   // 2^-27 gs
    for (int it = 0; it < 10; ++it) {
        const float tr = Q[0] + Q[4] + Q[8];
        float cof[9];
        cof[0] = Q[4] * Q[8] - Q[5] * Q[7];
        cof[1] = Q[5] * Q[6] - Q[3] * Q[8];
        cof[2] = Q[3] * Q[7] - Q[4] * Q[6];
        cof[3] = Q[2] * Q[7] - Q[1] * Q[8];
        cof[4] = Q[0] * Q[8] - Q[2] * Q[6];
        cof[5] = Q[1] * Q[6] - Q[0] * Q[7];
        cof[6] = Q[1] * Q[5] - Q[2] * Q[4];
        cof[7] = Q[2] * Q[3] - Q[0] * Q[5];
        cof[8] = Q[0] * Q[4] - Q[1] * Q[3];
        const float d = tr + (cof[0] + cof[4] + cof[8]) +
                        (Q[0] * cof[0] + Q[1] * cof[1] + Q[2] * cof[2]);
        // hardware reciprocal (about 1 ulp): 1 + d stays near 1, and the
        // iteration is self-correcting, so its error does not accumulate
        const float inv = __builtin_amdgcn_rcpf(1.0f + d);
        float K[9];
        K[0] = tr - Q[0] + cof[0] - d; K[1] = -Q[3] + cof[1];      K[2] = -Q[6] + cof[2];
        K[3] = -Q[1] + cof[3];      K[4] = tr - Q[4] + cof[4] - d; K[5] = -Q[7] + cof[5];
        K[6] = -Q[2] + cof[6];      K[7] = -Q[5] + cof[7];      K[8] = tr - Q[8] + cof[8] - d;
        float diff = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float nq = 0.5f * (Q[k] + K[k] * inv);
            diff = fmaxf(diff, fabsf(nq - Q[k]));
            Q[k] = nq;
        }
        if (diff * diff <= tol2) break;
    }
}

// Fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + lambda J (J - 1) I
// (the S_p of Eq. 4), from G = F - I.
__device__ __forceinline__ void kirchhoff(const float G[9], float mu2, float lam, float tau[9]) {
    float Q[9];
    polar_rotation_minus_identity(G, Q);
    float D[9];   // F - R = G - Q
#pragma unroll
    for (int k = 0; k < 9; ++k) D[k] = G[k] - Q[k];
    const float jm1 = det_minus_one(G);
    const float vol = lam * (1.0f + jm1) * jm1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // (D (I + G)^T)_ab = D_ab + sum_c D_ac G_bc
            float s = D[3 * a + b] + (D[3 * a] * G[3 * b] + D[3 * a + 1] * G[3 * b + 1] +
                                      D[3 * a + 2] * G[3 * b + 2]);
            tau[3 * a + b] = mu2 * s + (a == b ? vol : 0.0f);
        }
}

// Inside test of the rigid indenter at a node, FP64, evaluated with the same
// expression order as the host reference so that the masks agree bitwise.
__device__ __forceinline__ int node_inside(const KArgs& a, const StepPose& sp, int i, int j, int k) {
#pragma clang fp contract(off)
    if (a.shape == 0) return 0;
    const double X0 = (double)(i - a.pad_l) * a.dxd;
    const double X1 = (double)(j - a.pad_l) * a.dxd;
    const double X2 = (double)(k - a.pad_b) * a.dxd;
    const double d0 = X0 - sp.c[0], d1 = X1 - sp.c[1], d2 = X2 - sp.c[2];
    double p[3];
    for (int q = 0; q < 3; ++q) p[q] = sp.R[q] * d0 + sp.R[3 + q] * d1 + sp.R[6 + q] * d2;
    double phi;
    if (a.shape == 1) {
        phi = p[0] * p[0] + p[1] * p[1] + p[2] * p[2] - a.radius * a.radius;
    } else if (a.shape == 2) {
        const double hl = a.half_length;
        const double t = p[0] < -hl ? -hl : (p[0] > hl ? hl : p[0]);
        const double qx = p[0] - t;
        phi = qx * qx + p[1] * p[1] + p[2] * p[2] - a.radius * a.radius;
    } else if (a.shape == 3) {
        double out2 = 0.0, inmax = -1e300;
        for (int q = 0; q < 3; ++q) {
            const double qq = fabs(p[q]) - (a.he[q] - a.fillet);
            const double qp = qq > 0.0 ? qq : 0.0;
            out2 += qp * qp;
            if (qq > inmax) inmax = qq;
        }
        const double inside_part = inmax < 0.0 ? inmax : 0.0;
        phi = sqrt(out2) + inside_part - a.fillet;
    } else if (a.shape == 4) {
        // the solid above a bilinear sampled surface over a disc footprint
        if (p[0] * p[0] + p[1] * p[1] > a.hf_half * a.hf_half) return 0;
        const int n = a.hf_n;
        const double step = 2.0 * a.hf_half / (double)(n - 1);
        const double u = (p[0] + a.hf_half) / step, v = (p[1] + a.hf_half) / step;
        const int i0 = min(max((int)floor(u), 0), n - 2), j0 = min(max((int)floor(v), 0), n - 2);
        const double fu = u - (double)i0, fv = v - (double)j0;
        const double* t = a.hf + (size_t)j0 * n + i0;
        const double z0 = (1.0 - fu) * t[0] + fu * t[1];
        const double z1 = (1.0 - fu) * t[n] + fu * t[n + 1];
        phi = ((1.0 - fv) * z0 + fv * z1) - p[2];
    } else {
        return 0;
    }
    return phi <= 0.0;
}

__device__ __forceinline__ void rigid_velocity(const KArgs& a, const StepPose& sp, int i, int j, int k,
                                               float out[3]) {
#pragma clang fp contract(off)
    const double r0 = (double)(i - a.pad_l) * a.dxd - sp.c[0];
    const double r1 = (double)(j - a.pad_l) * a.dxd - sp.c[1];
    const double r2 = (double)(k - a.pad_b) * a.dxd - sp.c[2];
    out[0] = (float)(sp.vo[0] + (sp.w[1] * r2 - sp.w[2] * r1));
    out[1] = (float)(sp.vo[1] + (sp.w[2] * r0 - sp.w[0] * r2));
    out[2] = (float)(sp.vo[2] + (sp.w[0] * r1 - sp.w[1] * r0));
}

}  // namespace impm
