// impm_kernels.hip -- gfx950 kernels of one IMPM step (arXiv 2405.02914,
// Sec. III-A): per-tile particle-to-grid into LDS (Eq. 1-4), a node kernel that
// sums the tile partials and applies Eq. 5, the sticking contact and the
// boundary rule, and a fused per-tile kernel that runs the relative-rest test of
// Algorithm 1, grid-to-particle (Eq. 6-7), the commit (Eq. 8-9) and the
// particle-to-grid transfer of the next exchange.  Particles are binned by tile
// with a counting sort every committed step.
#include <hip/hip_cooperative_groups.h>

#include "impm_device.h"

namespace impm {

// Loop flags are read at agent scope, past the compute unit's vector cache:
// inside one cooperative launch other blocks write them between grid barriers.
__device__ __forceinline__ int flag_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Each block copies its kernel record into registers before its first store:
// loads taken then are free of clobbering stores, so their uniform addresses
// go to the scalar unit once, instead of being re-fetched through vector memory
// for every particle (the particle loop's stores might alias the record).  The
// copy is only ever indexed with constants (pick() selects a buffer of a
// double-buffered pair), so it stays in registers.
__device__ __forceinline__ KArgs load_args(const BatchMap& m, int s) {
    return m.args[__builtin_amdgcn_readfirstlane(s)];
}
template <class T>
__device__ __forceinline__ T pick(const T (&pair)[2], int i) {
    return i ? pair[1] : pair[0];
}

__device__ __forceinline__ int tile_linear(const KArgs& a, const int tc[3]) {
    return (tc[2] * a.NT[1] + tc[1]) * a.NT[0] + tc[0];
}
__device__ __forceinline__ void tile_coords(const KArgs& a, int t, int tc[3]) {
    tc[0] = t % a.NT[0];
    tc[1] = (t / a.NT[0]) % a.NT[1];
    tc[2] = t / (a.NT[0] * a.NT[1]);
}

// Node sums in LDS are 64-bit fixed point with 2^-32 resolution.  A contribution
// y (already scaled by 2^32, which is exact) becomes round(y) through one FP64
// add of the constant 1.5 * 2^52, or one FMA when y is a product of two floats:
// the sum holds the rounded integer in its low mantissa bits, and the constant's
// own bits are a multiple of 2^51, so they drop out of the low 51 bits of the
// accumulated sum, which are sign-extended at the flush (valid for |sum| < 2^18).  Integer adds make the node sums exact and
// independent of order, and LDS integer atomics are several times faster than
// LDS float atomics on this chip.
constexpr float kFixScaleF = 4294967296.0f;         // 2^32
constexpr double kFixScale = 4294967296.0;
constexpr double kFixMagic = 6755399441055744.0;    // 1.5 * 2^52

__device__ __forceinline__ unsigned long long to_fixed_scaled(float y, double magic) {
    return (unsigned long long)__double_as_longlong((double)y + magic);
}
// round(w * y) for a scaled weight w already widened to FP64: the product of two
// floats is exact in FP64, so one FMA forms and rounds it.
__device__ __forceinline__ unsigned long long to_fixed_product(double w, float y, double magic) {
    return (unsigned long long)__double_as_longlong(fma(w, (double)y, magic));
}
// The low 51 bits of a sum hold the two's complement of v = round(sum * 2^32);
// xor with 2^50 turns them into v + 2^50 in [0, 2^51), which as the mantissa of
// 1.5 * 2^52 gives the double 1.5 * 2^52 + 2^50 + v exactly.  One FMA removes
// the offset and scales by 2^-32, both exact, so the float is (float)(v * 2^-32).
__device__ __forceinline__ float from_fixed(unsigned long long a) {
    const unsigned long long m = ((a & ((1ull << 51) - 1ull)) ^ (1ull << 50)) | 0x4338000000000000ull;
    return (float)fma(__longlong_as_double((long long)m), 1.0 / kFixScale,
                      -(kFixMagic + 1125899906842624.0) / kFixScale);
}

// Compile-time tile geometry.  A tile holds the particles whose stencil base
// node floor(x - 1/2) lies in its TX x TY x TZ block starting at `origin`: its
// grid-to-particle block covers nodes [origin, origin + T + 1] per axis, and
// its particle-to-grid block [origin - 1, origin + T + 2] (a particle may move
// its base by one node in the step before it is re-binned).  NB threads per
// block.
//
// Pitches of the LDS planes of the particle-to-grid block (in 64-bit words).
// When the block's row is a multiple of 8 words (4-cell-wide tiles) its rows
// would fall on the same banks, so the row pitch is made odd and the plane
// pitch 9 mod 16, which spreads the nodes one atomic instruction of a wave
// touches (a row of cells, two y and two z bases) over the 32 banks.  Rows of
// 12 words (8-cell-wide tiles) are left unpadded: measured, the padding made
// their fused kernel 0.6-1.9 % slower, while removing it from 4-cell-wide tiles
// made theirs 2 % slower.
template <int TX, int TY, int TZ, int NB>
struct Tile {
    static constexpr int T0 = TX, T1 = TY, T2 = TZ, NT = NB;
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4, PVOL = PX * PY * PZ;
    static constexpr bool PAD = PX % 8 == 0;
    static constexpr int SY = PAD ? (PX | 1) : PX;
    static constexpr bool ROWS4 = TX == 8 && TY == 4;   // planes padded to 16 mod 32 words
    static constexpr int SZ = PAD     ? SY * PY + ((9 - (SY * PY) % 16) + 16) % 16
                              : ROWS4 ? SY * PY + ((16 - (SY * PY) % 32) + 32) % 32
                                      : SY * PY;
    static constexpr int AVOL = SZ * PZ;          // words per LDS plane (>= PVOL)
    static constexpr int GX = TX + 2, GY = TY + 2, GZ = TZ + 2, GVOL = GX * GY * GZ;
    // row pitch of the G2P block in LDS (16-byte records): 12 on 8-cell-wide
    // tiles, so that the rows two apart that share 16 lanes of a gather fall
    // on different banks
    static constexpr int GXS = TX == 8 ? 12 : GX, GVOLS = GXS * GY * GZ;
    static constexpr size_t LDS_P2G = (size_t)4 * AVOL * 8;
    static constexpr int NW = NB / 64;
    static constexpr size_t LDS_G2P2G = LDS_P2G + (size_t)GVOLS * 16 + 81 * 4 + (NW * kDirs + kDirs + 4) * 4;
};

// Particle-to-grid contribution of one particle (Eq. 1-4) into the LDS node
// block `acc` whose first node is `org`: four planes (W, Px, Py, Pz) of PVOL
// fixed-point sums; the planar layout puts neighbouring nodes on different LDS
// banks.  Masses are carried as weights (every particle has the same m_p): node
// (W, P) with W = sum w, P = sum w (v + B d), d = X_i - x_p in cell units and
// B = dx C - (4 h / (rho dx)) tau, so that M_i = m_p W and MG_i = m_p P.  The
// velocity term is separable: v + B d = (v + B_.2 dz) + B_.1 dy + B_.0 dx.
// Returns 0, or DEV_CFL when the stencil leaves the block, or DEV_NONFINITE
// when the particle's terms are not finite or too large for the fixed-point
// range (the particle then contributes nothing).
template <class TL>
__device__ __forceinline__ int p2g_particle(unsigned long long* acc, const int org[3], const int cell[3],
                                            const float f[3], const float v[3], const float C[9],
                                            const float G[9], bool with_stress, const KArgs& a) {
    int base[3];
    float fx[3], w[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) bspline_axis(cell[q], f[q], base[q], fx[q], w[q]);
    const int l0 = base[0] - org[0], l1 = base[1] - org[1], l2 = base[2] - org[2];
    if (l0 < 0 || l0 + 2 >= TL::PX || l1 < 0 || l1 + 2 >= TL::PY || l2 < 0 || l2 + 2 >= TL::PZ)
        return DEV_CFL;
    float B[9];
    if (with_stress) {
        float tau[9];
        kirchhoff(G, a.mu2, a.lam, tau);
#pragma unroll
        for (int k = 0; k < 9; ++k) B[k] = a.dx * C[k] - a.kst * tau[k];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) B[k] = a.dx * C[k];
    }
    // |w (v + B d)| <= |v| + 4.5 max|B| per node; the node sums stay below the
    // fixed-point range while this bound is below 4096 m/s.  fmaxf drops NaN
    // operands, so finiteness is tested on a plain sum.
    float mag = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fabsf(v[2]));
    float bm = 0.f, sum = v[0] + v[1] + v[2];
#pragma unroll
    for (int k = 0; k < 9; ++k) { bm = fmaxf(bm, fabsf(B[k])); sum += B[k]; }
    if (!isfinite(sum) || !(mag + 4.5f * bm < 4096.0f)) return DEV_NONFINITE;

    float ax[3][3], by[3][3], cz[3][3], wx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float dxa = (float)c - fx[0], dyb = (float)c - fx[1], dzc = (float)c - fx[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            ax[c][r] = B[3 * r] * dxa;
            by[c][r] = B[3 * r + 1] * dyb;
            cz[c][r] = v[r] + B[3 * r + 2] * dzc;
        }
        wx[c] = w[0][c] * kFixScaleF;
    }
    const double magic = kFixMagic;
    unsigned long long* row0 = acc + l2 * TL::SZ + l1 * TL::SY + l0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const float wbc = w[1][b] * w[2][c];
            const float sy0 = by[b][0] + cz[c][0], sy1 = by[b][1] + cz[c][1], sy2 = by[b][2] + cz[c][2];
            unsigned long long* nd = row0 + c * TL::SZ + b * TL::SY;
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) {
                const double wt = (double)(wx[aa] * wbc);
                atomicAdd(nd + aa, (unsigned long long)__double_as_longlong(wt + magic));
                atomicAdd(nd + aa + TL::AVOL, to_fixed_product(wt, ax[aa][0] + sy0, magic));
                atomicAdd(nd + aa + 2 * TL::AVOL, to_fixed_product(wt, ax[aa][1] + sy1, magic));
                atomicAdd(nd + aa + 3 * TL::AVOL, to_fixed_product(wt, ax[aa][2] + sy2, magic));
            }
        }
    }
    return 0;
}

// Write a tile's fixed-point node sums to its scratch record as floats.
template <class TL>
__device__ __forceinline__ void flush_tile(const unsigned long long* acc, gptr<f32x4> dst) {
    for (int k = threadIdx.x; k < TL::PVOL; k += TL::NT) {
        const int x = k % TL::PX, y = (k / TL::PX) % TL::PY, z = k / (TL::PX * TL::PY);
        const int o = z * TL::SZ + y * TL::SY + x;
        dst[k] = f32x4{from_fixed(acc[o]), from_fixed(acc[TL::AVOL + o]), from_fixed(acc[2 * TL::AVOL + o]),
                       from_fixed(acc[3 * TL::AVOL + o])};
    }
}

__device__ __forceinline__ void load_particle(const KArgs& a, long long id, int cell[3],
                                              float f[3]) {
    unpack_cell(glb(a.cell)[id], cell);
#pragma unroll
    for (int q = 0; q < 3; ++q) f[q] = glb(a.soa)[(size_t)(F0 + q) * a.n + id];
}

// Object particles (the object represented by particles, Sec. III-A).  Their
// velocity is the object's prescribed rigid motion and their affine matrix that
// motion's [w]x, so their transfer to node i is m_o w_ip (v_o + w x (X_i - c)):
// the rigid velocity at the node times their mass weight.  They therefore only
// deposit kappa * w_ip (mass relative to an elastomer particle) into a
// fixed-point node array; the node kernel adds that weight and its rigid
// momentum with the step's pose.  Global 64-bit integer atomics: the sums are
// exact and independent of order.  Returns DEV_CFL if the stencil leaves the grid.
__device__ __forceinline__ int p2g_object(const KArgs& a, const int cell[3], const float f[3]) {
    int base[3];
    float fx[3], w[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) bspline_axis(cell[q], f[q], base[q], fx[q], w[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (base[q] < 0 || base[q] + 2 > a.nn[q] - 1) return DEV_CFL;
    const double scale = (double)a.kappa * kFixScale;
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b) {
            const double wbc = (double)(w[1][b] * w[2][c]) * scale;
            const long long row = ((long long)(base[2] + c) * a.nn[1] + (base[1] + b)) * a.nn[0] + base[0];
#pragma unroll
            for (int aa = 0; aa < 3; ++aa)
                atomicAdd(&a.objW[row + aa],
                          (unsigned long long)__double_as_longlong(fma((double)w[0][aa], wbc, kFixMagic)));
        }
    return 0;
}

// Rigid placement of an object particle at the end of a step: its body point
// ((i + 1/2) h, (j + 1/2) h, z0 + (k + 1/2) h) from the lattice indices in lat,
// moved by the end pose, as a grid cell plus an FP32 offset.  FP64, evaluated
// in the order of the host reference.
__device__ __forceinline__ void place_object(const KArgs& a, const StepPose& sp, const float lat[3], int cell[3],
                                             float f[3]) {
#pragma clang fp contract(off)
    const double p0 = ((double)lat[0] + 0.5) * a.obj_h, p1 = ((double)lat[1] + 0.5) * a.obj_h;
    const double p2 = a.obj_z0 + ((double)lat[2] + 0.5) * a.obj_h;
    const double off[3] = {(double)a.pad_l, (double)a.pad_l, (double)a.pad_b};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double x = sp.c_end[q] + sp.R_end[3 * q] * p0 + sp.R_end[3 * q + 1] * p1 + sp.R_end[3 * q + 2] * p2;
        const double g = x / a.dxd + off[q];
        double fl = floor(g);
        float fr = (float)(g - fl);
        if (fr >= 1.0f) { fr = 0.0f; fl += 1.0; }
        cell[q] = (int)fl;
        f[q] = fr;
    }
}

__global__ void k_fill(float* p, long long n, float val) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = val;
}

// Stand-alone particle-to-grid of the first exchange of a step (after creation or
// an external state write): one block per tile, partials to the tile's scratch.
template <class TL>
__global__ __launch_bounds__(TL::NT) void k_p2g(BatchMap m, int cur) {
    extern __shared__ unsigned long long lds_u64[];
    unsigned long long* acc = lds_u64;
    int s = 0, t = blockIdx.x;
    if (m.tile_base) {
        s = batch_find(m.tile_base, m.n, t);
        t -= m.tile_base[s];
    }
    if (!member_active(m, s)) return;
    const KArgs a = load_args(m, s);
    const gptr<const uint32_t> __restrict__ order = glb<const uint32_t>(pick(a.order, cur));
    const gptr<const uint32_t> __restrict__ bstart = glb<const uint32_t>(pick(a.bstart, cur));
    const uint32_t s0 = bstart[t], cnt = bstart[t + 1] - s0;
    if (cnt == 0) return;
    int tc[3];
    tile_coords(a, t, tc);
    const int org[3] = {tc[0] * TL::T0 - 1, tc[1] * TL::T1 - 1, tc[2] * TL::T2 - 1};
    for (int k = threadIdx.x; k < 4 * TL::AVOL; k += TL::NT) acc[k] = 0ull;
    __syncthreads();
    int err = 0;
    for (uint32_t i = threadIdx.x; i < cnt; i += TL::NT) {
        const long long id = order[s0 + i];
        int cell[3];
        float f[3], v[3], C[9], G[9];
        load_particle(a, id, cell, f);
        if (a.objW && (glb(a.flags)[id] & FLAG_OBJECT)) {
            err |= p2g_object(a, cell, f);
            continue;
        }
        for (int q = 0; q < 3; ++q) v[q] = glb(a.soa)[(size_t)(V0 + q) * a.n + id];
        for (int q = 0; q < 9; ++q) C[q] = glb(a.soa)[(size_t)(C0 + q) * a.n + id];
        for (int q = 0; q < 9; ++q) G[q] = glb(a.soa)[(size_t)(G0 + q) * a.n + id];
        err |= p2g_particle<TL>(acc, org, cell, f, v, C, G, true, a);
    }
    if (err) atomicOr(&a.st->error, err);
    __syncthreads();
    flush_tile<TL>(acc, glb4(a.scratch) + (size_t)t * TL::PVOL);
}

// Node kernel: sum the partials of the tiles whose P2G block covers the node
// (fixed order), V = MG / M (Eq. 5), nodes inside the indenter take its rigid
// velocity (relative rest with the object), boundary nodes get zero velocity.
// EXTRA: the same for the passes after the first of a step, which run only while
// the relative-rest test fails.
template <class TL, bool EXTRA>
__device__ __forceinline__ void grid_block(const BatchMap& m, int gnb, int sbin, int step, int pass) {
    int s = 0, nb = gnb;
    if (m.node_base) {
        s = batch_find(m.node_base, m.n, nb);
        nb -= m.node_base[s];
    }
    if (!member_active(m, s)) return;
    const KArgs a = load_args(m, s);
    if (flag_load(&a.st->finished[pass])) return;
    const gptr<const uint32_t> __restrict__ bstart = glb<const uint32_t>(pick(a.bstart, sbin));
    const long long nid = nb * (long long)kBlock + threadIdx.x;
    const long long n_nodes = (long long)a.nn[0] * a.nn[1] * a.nn[2];
    if (nid >= n_nodes) return;
    const int i = (int)(nid % a.nn[0]);
    const int j = (int)((nid / a.nn[0]) % a.nn[1]);
    const int k = (int)(nid / ((long long)a.nn[0] * a.nn[1]));
    const int nd[3] = {i, j, k};
    const int T[3] = {TL::T0, TL::T1, TL::T2};
    int lo[3], hi[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int m = nd[q] - T[q] - 2;
        lo[q] = m <= 0 ? 0 : (m + T[q] - 1) / T[q];
        hi[q] = min((nd[q] + 1) / T[q], a.NT[q] - 1);
    }
    // Up to K0 x K1 x K2 covering tiles (2 per axis, 3 along 2-cell axes): every
    // candidate's tile-start pair and partial is loaded before any is summed, so
    // the loads of all tiles are in flight together; the sum runs in (tz, ty, tx)
    // order.
    constexpr int K0 = (TL::T0 + 3) / TL::T0 + 1, K1 = (TL::T1 + 3) / TL::T1 + 1, K2 = (TL::T2 + 3) / TL::T2 + 1;
    constexpr int KT = K0 * K1 * K2;
    f32x4 part[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) {
        const int tx = lo[0] + q % K0, ty = lo[1] + (q / K0) % K1, tz = lo[2] + q / (K0 * K1);
        part[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (tx <= hi[0] && ty <= hi[1] && tz <= hi[2]) {
            const int t = (tz * a.NT[1] + ty) * a.NT[0] + tx;
            if (bstart[t + 1] != bstart[t]) {
                const int l0 = i - (tx * TL::T0 - 1), l1 = j - (ty * TL::T1 - 1), l2 = k - (tz * TL::T2 - 1);
                part[q] = glb4(a.scratch)[(size_t)t * TL::PVOL + (l2 * TL::PY + l1) * TL::PX + l0];
            }
        }
    }
    float W = 0.f, P0 = 0.f, P1 = 0.f, P2 = 0.f;
#pragma unroll
    for (int q = 0; q < KT; ++q) {
        W += part[q].x; P0 += part[q].y; P1 += part[q].z; P2 += part[q].w;
    }
    if (a.objW) {
        // the object particles' mass weight and its rigid momentum at this node
        // (read and cleared for the next exchange)
        const unsigned long long q = glb(a.objW)[nid];
        if (q) {
            glb(a.objW)[nid] = 0ull;
            const float Wo = from_fixed(q);
            float u[3];
            rigid_velocity(a, a.poses[step], i, j, k, u);
            W += Wo;
            P0 += Wo * u[0]; P1 += Wo * u[1]; P2 += Wo * u[2];
        }
    }
    float V[3] = {0.f, 0.f, 0.f};
    if (W > 0.f) {
        const float inv = 1.0f / W;
        V[0] = P0 * inv; V[1] = P1 * inv; V[2] = P2 * inv;
        const StepPose& sp = a.poses[step];
        if (a.object_mode == 0 && node_inside(a, sp, i, j, k)) rigid_velocity(a, sp, i, j, k, V);
        const bool bnd = i < a.band || i > a.nn[0] - 1 - a.band || j < a.band ||
                         j > a.nn[1] - 1 - a.band || k > a.nn[2] - 1 - a.band || k <= a.pad_b;
        if (bnd) V[0] = V[1] = V[2] = 0.f;
    }
    glb4(a.gridV)[nid] = f32x4{V[0], V[1], V[2], W};
    if (a.dbgM) {
        a.dbgM[nid] = a.mp * W;
        a.dbgMG[3 * nid + 0] = a.mp * P0;
        a.dbgMG[3 * nid + 1] = a.mp * P1;
        a.dbgMG[3 * nid + 2] = a.mp * P2;
    }
}

// Fused per-tile kernel of one exchange pass.
//  1. The relative-rest test of Algorithm 1 on the calibration particle x_e:
//     every block evaluates it from the same grid velocities in the same order,
//     so all blocks take the same decision without a grid-wide barrier.
//  2. Grid-to-particle (Eq. 6-7) and the bottom rule.
//  3. If the step ends here: commit F and x (Eq. 8-9), bin the particle for the
//     next step, and transfer it to the grid of the next step's first pass;
//     otherwise transfer it (same x and F, new v and C) to the next pass's grid.
// EXTRA marks the launches for passes after the first of a step.
template <class TL, bool EXTRA, bool OBJ>
__device__ __forceinline__ void g2p2g_tile(const BatchMap& m, int gt, int cur, int step, int par, int pass,
                                           int store_vc) {
    int s = 0, t = gt;
    if (m.tile_base) {
        s = batch_find(m.tile_base, m.n, t);
        t -= m.tile_base[s];
    }
    if (!member_active(m, s)) return;
    const KArgs a = load_args(m, s);
    if (flag_load(&a.st->finished[pass])) {
        // carry the flag to the next pass slot so that every later pass of the
        // step is skipped as well
        if (t == 0 && threadIdx.x == 0) a.st->finished[pass + 1] = 1;
        return;
    }
    const gptr<const uint32_t> __restrict__ order = glb<const uint32_t>(pick(a.order, cur));
    const gptr<const uint32_t> __restrict__ bstart = glb<const uint32_t>(pick(a.bstart, cur));
    extern __shared__ unsigned long long lds_u64[];
    unsigned long long* acc = lds_u64;                                   // 4 * PVOL
    f32x4* gv = reinterpret_cast<f32x4*>(lds_u64 + 4 * TL::AVOL);        // GY*GZ rows of GXS (vx, vy, vz, -)
    float* ve_part = reinterpret_cast<float*>(gv + TL::GVOLS);            // 27 * 3
    int* wc = reinterpret_cast<int*>(ve_part + 81);                      // NW * 27 wave counts
    int* running = wc + TL::NW * kDirs;                                  // 27 per-direction counts
    int* sh = running + kDirs;                                           // [0] = final

    const int tid = threadIdx.x;
    const StepPose& sp = a.poses[step];

    // ---- 1. relative-rest decision
    if (tid < 27) {
        int cell[3];
        unpack_cell(a.st->xe_cell[par], cell);
        int base[3];
        float fx[3], w[3][3];
        for (int q = 0; q < 3; ++q) bspline_axis(cell[q], a.st->xe_f[par][q], base[q], fx[q], w[q]);
        const int cx = tid % 3, cy = (tid / 3) % 3, cz = tid / 9;
        const long long nid = ((long long)(base[2] + cz) * a.nn[1] + (base[1] + cy)) * a.nn[0] +
                              (base[0] + cx);
        const f32x4 V = glb4(a.gridV)[nid];
        const float wt = w[0][cx] * w[1][cy] * w[2][cz];
        ve_part[3 * tid + 0] = wt * V.x;
        ve_part[3 * tid + 1] = wt * V.y;
        ve_part[3 * tid + 2] = wt * V.z;
    }
    if (tid < kDirs) running[tid] = 0;
    if (tid < TL::NW * kDirs) wc[tid] = 0;
    __syncthreads();
    if (tid == 0) {
        float ve0 = 0.f, ve1 = 0.f;
        for (int q = 0; q < 27; ++q) { ve0 += ve_part[3 * q]; ve1 += ve_part[3 * q + 1]; }
        int fin;
        double r = -1.0;
        bool limit = false;
        if (sp.forced > 0) {
            fin = pass + 1 >= sp.forced;
        } else if (a.mode == 1) {
            fin = 1;
        } else if (sp.gnorm <= 1e-9) {
            fin = 1;
            r = 0.0;
        } else {
            const double d0 = (double)ve0 - sp.vot[0], d1 = (double)ve1 - sp.vot[1];
            r = sqrt(d0 * d0 + d1 * d1) / sp.gnorm;
            fin = r <= a.rest_threshold;
            if (!fin && pass + 1 >= a.rest_limit) { fin = 1; limit = true; }
        }
        sh[0] = fin;
        if (t == 0) {
            a.st->finished[pass + 1] = fin;
            if (r >= 0.0) a.st->last_r = r;
            if (fin) {
                a.st->steps += 1;
                a.st->passes += (unsigned long long)(pass + 1);
                if (limit) a.st->limit_hits += 1;
            }
        }
    }
    __syncthreads();
    const bool fin = sh[0] != 0;

    const uint32_t s0 = bstart[t], cnt = bstart[t + 1] - s0;
    if (cnt == 0) {
        if (fin && tid < kDirs) glb(a.dircount)[(size_t)t * kDirs + tid] = 0;
        return;
    }
    int tc[3];
    tile_coords(a, t, tc);
    const int orgP[3] = {tc[0] * TL::T0 - 1, tc[1] * TL::T1 - 1, tc[2] * TL::T2 - 1};
    const int orgG[3] = {tc[0] * TL::T0, tc[1] * TL::T1, tc[2] * TL::T2};
    // ---- stage the grid velocities of the tile's G2P block as 16-byte records
    // (one ds_read_b128 with an immediate offset per stencil node in the
    // gather; the weight slot is unused), clear the P2G block
    for (int kk = tid; kk < TL::GVOL; kk += TL::NT) {
        const int lx = kk % TL::GX, ly = (kk / TL::GX) % TL::GY, lz = kk / (TL::GX * TL::GY);
        const int gx = orgG[0] + lx, gy = orgG[1] + ly, gz = orgG[2] + lz;
        f32x4 V = {0.f, 0.f, 0.f, 0.f};
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < a.nn[0] && gy < a.nn[1] && gz < a.nn[2])
            V = glb4(a.gridV)[((long long)gz * a.nn[1] + gy) * a.nn[0] + gx];
        gv[(lz * TL::GY + ly) * TL::GXS + lx] = V;
    }
    // (four planes of AVOL words: 2 * AVOL 16-byte stores)
    for (int kk = tid; kk < 2 * TL::AVOL; kk += TL::NT) reinterpret_cast<u32x4*>(acc)[kk] = u32x4{0u, 0u, 0u, 0u};
    __syncthreads();

    const bool with_stress = fin || a.stress_each_pass;
    const int lane = tid & 63, wid = tid >> 6;
    int err = 0;
    for (uint32_t i0 = 0; i0 < cnt; i0 += TL::NT) {
        const uint32_t i = i0 + tid;
        int dir = -1;
        if (i < cnt) {
            const long long id = order[s0 + i];
            int cell[3];
            float f[3];
            load_particle(a, id, cell, f);
            // On tiles of 128 cells or more, F and the flags are loaded before
            // the gather so that their latency overlaps it (measured: +8 % on
            // the 8x4x4 tile). Smaller tiles have LDS for more than four blocks
            // per CU, and there the registers held across the gather would cost
            // a wave per SIMD, so they load after it.
            constexpr bool kEarly = TL::T0 * TL::T1 * TL::T2 >= 128;
            float G[9];
            uint8_t fl = 0;
            if constexpr (kEarly) {
                for (int q = 0; q < 9; ++q) G[q] = glb(a.soa)[(size_t)(G0 + q) * a.n + id];
                fl = glb(a.flags)[id];
            }
            // ---- 2. grid-to-particle (Eq. 6-7), separably: column sums S_a,
            // T_b, U_c of the weighted grid velocities along each axis give
            // v = sum_a w_a S_a and C_.0 = (4/dx) sum_a w_a (a - fx) (S_a - v)
            // (the v term vanishes in exact arithmetic and removes cancellation)
            int base[3];
            float fx[3], w[3][3];
            for (int q = 0; q < 3; ++q) bspline_axis(cell[q], f[q], base[q], fx[q], w[q]);
            const int l0 = base[0] - orgG[0], l1 = base[1] - orgG[1], l2 = base[2] - orgG[2];
            float v[3] = {0.f, 0.f, 0.f}, C[9];
            for (int q = 0; q < 9; ++q) C[q] = 0.f;
            if (l0 >= 0 && l0 + 2 < TL::GX && l1 >= 0 && l1 + 2 < TL::GY && l2 >= 0 && l2 + 2 < TL::GZ) {
                float S[3][3], Tb[3][3], U[3][3];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int r = 0; r < 3; ++r) { S[q][r] = 0.f; Tb[q][r] = 0.f; U[q][r] = 0.f; }
                const f32x4* g0 = gv + ((l2 * TL::GY + l1) * TL::GXS + l0);
                // per row (b, c): R = sum_a w_a V_abc; S_a collects w_b w_c V_abc,
                // T_b collects w_c R and U_c collects w_b R
#pragma unroll
                for (int cz = 0; cz < 3; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 3; ++cy) {
                        const float wbc = w[1][cy] * w[2][cz];
                        float R[3] = {0.f, 0.f, 0.f};
#pragma unroll
                        for (int cx = 0; cx < 3; ++cx) {
                            const f32x4 V = g0[(cz * TL::GY + cy) * TL::GXS + cx];
                            S[cx][0] += wbc * V.x; S[cx][1] += wbc * V.y; S[cx][2] += wbc * V.z;
                            R[0] += w[0][cx] * V.x; R[1] += w[0][cx] * V.y; R[2] += w[0][cx] * V.z;
                        }
#pragma unroll
                        for (int r = 0; r < 3; ++r) { Tb[cy][r] += w[2][cz] * R[r]; U[cz][r] += w[1][cy] * R[r]; }
                    }
#pragma unroll
                for (int r = 0; r < 3; ++r) v[r] = w[0][0] * S[0][r] + w[0][1] * S[1][r] + w[0][2] * S[2][r];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float ea = w[0][q] * ((float)q - fx[0]);
                    const float eb = w[1][q] * ((float)q - fx[1]);
                    const float ec = w[2][q] * ((float)q - fx[2]);
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        C[3 * r + 0] += ea * (S[q][r] - v[r]);
                        C[3 * r + 1] += eb * (Tb[q][r] - v[r]);
                        C[3 * r + 2] += ec * (U[q][r] - v[r]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 9; ++q) C[q] *= a.c4dx;
            } else {
                err |= DEV_CFL;
            }
            if constexpr (!kEarly) {
                for (int q = 0; q < 9; ++q) G[q] = glb(a.soa)[(size_t)(G0 + q) * a.n + id];
                fl = glb(a.flags)[id];
            }
            if (a.bottom_rule && (fl & FLAG_BOTTOM)) v[2] = 0.f;
            // an object particle (G0..G2 hold its body lattice indices) takes no
            // part in the gather's result: its velocity is the prescribed motion
            const bool obj = OBJ && (fl & FLAG_OBJECT);
            if (fin) {
                int perr = 0;
                int moved[3];
                float nfr[3];
                if (obj) {
                    // ---- 3. the object moves rigidly to the step's end pose
                    place_object(a, sp, G, moved, nfr);
                } else {
                    // ---- 3. commit: F <- (I + h C) F, x <- x + h v
                    float Gn[9];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            Gn[3 * r + c] = G[3 * r + c] +
                                            a.h * (C[3 * r + c] + (C[3 * r] * G[c] + C[3 * r + 1] * G[3 + c] +
                                                                   C[3 * r + 2] * G[6 + c]));
                    bool finite = true;
                    for (int q = 0; q < 9; ++q) { G[q] = Gn[q]; finite = finite && isfinite(Gn[q]); }
                    for (int q = 0; q < 3; ++q) finite = finite && isfinite(v[q]);
                    if (!finite) err |= DEV_NONFINITE;
                    if (!(1.0f + det_minus_one(G) > 0.0f)) err |= DEV_DETF;
                    perr = finite ? 0 : DEV_NONFINITE;
                    for (int q = 0; q < 3; ++q) {
                        const float step_cells = a.h_over_dx * v[q];
                        if (!(fabsf(step_cells) < 1.0f)) perr |= DEV_CFL;
                        float nf = f[q] + step_cells;
                        const float fl0 = floorf(nf);
                        int c = cell[q] + (int)fl0;
                        nf -= fl0;
                        if (nf >= 1.0f) { nf -= 1.0f; c += 1; }
                        moved[q] = c;
                        nfr[q] = nf;
                    }
                }
                bool inside = true;
                for (int q = 0; q < 3; ++q) inside = inside && moved[q] >= 1 && moved[q] <= a.nn[q] - 3;
                if (!inside) perr |= DEV_CFL;
                err |= perr;
                if (perr == 0) {
                    for (int q = 0; q < 3; ++q) { cell[q] = moved[q]; f[q] = nfr[q]; }
                    glb(a.cell)[id] = pack_cell(cell);
                    for (int q = 0; q < 3; ++q) glb(a.soa)[(size_t)(F0 + q) * a.n + id] = f[q];
                    if (!obj)
                        for (int q = 0; q < 9; ++q) glb(a.soa)[(size_t)(G0 + q) * a.n + id] = G[q];
                }
                if (id == a.e) {
                    a.st->xe_cell[par ^ 1] = pack_cell(cell);
                    for (int q = 0; q < 3; ++q) a.st->xe_f[par ^ 1][q] = f[q];
                }
                // tile of the new stencil base floor(x - 1/2)
                const int nt[3] = {(cell[0] - 1 + (f[0] >= 0.5f ? 1 : 0)) / TL::T0,
                                   (cell[1] - 1 + (f[1] >= 0.5f ? 1 : 0)) / TL::T1,
                                   (cell[2] - 1 + (f[2] >= 0.5f ? 1 : 0)) / TL::T2};
                dir = 0;
                for (int q = 2; q >= 0; --q) {
                    int dd = nt[q] - tc[q];
                    dd = dd < -1 ? -1 : (dd > 1 ? 1 : dd);
                    dir = dir * 3 + (dd + 1);
                }
            }
            if (store_vc && fin && !obj) {
                for (int q = 0; q < 3; ++q) glb(a.soa)[(size_t)(V0 + q) * a.n + id] = v[q];
                for (int q = 0; q < 9; ++q) glb(a.soa)[(size_t)(C0 + q) * a.n + id] = C[q];
            }
            // ---- transfer to the grid of the next exchange
            if (obj) err |= p2g_object(a, cell, f);
            else err |= p2g_particle<TL>(acc, orgP, cell, f, v, C, G, with_stress, a);
        }
        if (fin) {
            // stable rank of this particle among the tile's particles that move to
            // the same neighbour tile (earlier positions first): the next binned
            // order keeps each tile's particles in their previous order, so the
            // loads of a wave stay on few cache lines
            int my_rank = 0;
            unsigned long long act = __ballot(dir >= 0);
            while (act) {
                const int leader = __ffsll((long long)act) - 1;
                const int d0 = __shfl(dir, leader);
                const unsigned long long m = __ballot(dir == d0);
                if (dir == d0) my_rank = __popcll(m & ((1ull << lane) - 1ull));
                if (lane == leader) wc[wid * kDirs + d0] = __popcll(m);
                act &= ~m;
            }
            __syncthreads();
            if (dir >= 0) {
                int base_r = running[dir];
                for (int w2 = 0; w2 < wid; ++w2) base_r += wc[w2 * kDirs + dir];
                glb(a.dirrank)[s0 + i] = ((uint32_t)(base_r + my_rank) << 5) | (uint32_t)dir;
            }
            __syncthreads();
            if (tid < kDirs) {
                int sum = 0;
                for (int w2 = 0; w2 < TL::NW; ++w2) { sum += wc[w2 * kDirs + tid]; wc[w2 * kDirs + tid] = 0; }
                running[tid] += sum;
            }
            __syncthreads();
        }
    }
    if (err) atomicOr(&a.st->error, err);
    __syncthreads();
    flush_tile<TL>(acc, glb4(a.scratch) + (size_t)t * TL::PVOL);
    if (fin && tid < kDirs) {
        const uint32_t c = running[tid];
        glb(a.dircount)[(size_t)t * kDirs + tid] = c;
        if (c) {
            const int dt[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
            int u[3];
            bool ok = true;
            for (int q = 0; q < 3; ++q) {
                u[q] = tc[q] + dt[q];
                ok = ok && u[q] >= 0 && u[q] < a.NT[q];
            }
            if (ok) atomicAdd(&a.newcnt[tile_linear(a, u)], c);
            else atomicOr(&a.st->error, DEV_CFL);
        }
    }
}

// The node and fused kernels stride over the launch's node blocks / tiles.  A
// first-pass launch has one block per item; the launches of later passes use a
// grid of at most kExtraBlocks blocks, so that a pass that the relative-rest
// test has already made unnecessary costs a small dispatch rather than one
// block per tile (every block exits on the step's flag).
constexpr int kExtraBlocks = 1024;

// Members of a batch whose step is still running at pass `pass`, as a bit set
// in LDS (members from kLiveMembers on count as running; their blocks test the
// flag themselves).  A pass launch of a batch then visits only the tiles and
// node blocks of running members: before, every block walked the block ranges
// of all members and looked each one up, which cost a pass launch over 64
// converged sensors as much as a third of a real pass.  With `carry`, block 0
// marks the finished members' next pass slot finished as well (what their
// tile 0 would have done).
constexpr int kLiveMembers = 2048;

__device__ __forceinline__ void running_members(const BatchMap& m, int pass, bool carry, uint32_t* live) {
    const int nm = min(m.n, kLiveMembers);
    for (int w = threadIdx.x; w < (nm + 31) / 32; w += blockDim.x) live[w] = 0u;
    __syncthreads();
    for (int s = threadIdx.x; s < nm; s += blockDim.x) {
        if (!member_active(m, s)) continue;
        if (!flag_load(&m.args[s].st->finished[pass])) atomicOr(&live[s >> 5], 1u << (s & 31));
        else if (carry && blockIdx.x == 0) m.args[s].st->finished[pass + 1] = 1;
    }
    __syncthreads();
}

__device__ __forceinline__ bool member_running(const uint32_t* live, int s) {
    return s >= kLiveMembers || ((live[s >> 5] >> (s & 31)) & 1u) != 0u;
}

// First index of this block's stride (blockIdx.x mod gridDim.x) at or after b0.
__device__ __forceinline__ int stride_start(int b0) {
    const int G = (int)gridDim.x;
    return b0 + (((int)blockIdx.x - b0) % G + G) % G;
}

template <class TL, bool EXTRA>
__global__ __launch_bounds__(kBlock) void k_grid(BatchMap m, int total, int sbin, int step, int pass) {
    if constexpr (!EXTRA) {
        grid_block<TL, EXTRA>(m, blockIdx.x, sbin, step, pass);
    } else if (!m.node_base) {
        for (int nb = blockIdx.x; nb < total; nb += gridDim.x) grid_block<TL, EXTRA>(m, nb, sbin, step, pass);
    } else {
        __shared__ uint32_t live[kLiveMembers / 32];
        running_members(m, pass, false, live);
        for (int s = 0; s < m.n; ++s) {
            if (!member_running(live, s)) continue;
            const int b1 = m.node_base[s + 1];
            for (int nb = stride_start(m.node_base[s]); nb < b1; nb += gridDim.x)
                grid_block<TL, EXTRA>(m, nb, sbin, step, pass);
        }
    }
}

// OBJ: the launch covers object particles (a separate instantiation, so that
// sensors without them run the kernel without the object branches).
template <class TL, bool EXTRA, bool OBJ>
__global__ __launch_bounds__(TL::NT) void k_g2p2g(BatchMap m, int total, int cur, int step, int par, int pass,
                                                  int store_vc) {
    if constexpr (!EXTRA) {
        g2p2g_tile<TL, EXTRA, OBJ>(m, blockIdx.x, cur, step, par, pass, store_vc);
    } else if (!m.tile_base) {
        for (int gt = blockIdx.x; gt < total; gt += gridDim.x) {
            g2p2g_tile<TL, EXTRA, OBJ>(m, gt, cur, step, par, pass, store_vc);
            __syncthreads();   // the next tile reuses the block's LDS
        }
    } else {
        __shared__ uint32_t live[kLiveMembers / 32];
        running_members(m, pass, true, live);
        for (int s = 0; s < m.n; ++s) {
            if (!member_running(live, s)) continue;
            const int b1 = m.tile_base[s + 1];
            for (int gt = stride_start(m.tile_base[s]); gt < b1; gt += gridDim.x) {
                g2p2g_tile<TL, EXTRA, OBJ>(m, gt, cur, step, par, pass, store_vc);
                __syncthreads();
            }
        }
    }
}

// Passes 2..npass of a step in one cooperative launch (every block resident):
// node phase, grid barrier, fused exchange phase, grid barrier, per pass.  The
// loop stops as soon as every sensor's relative-rest test has ended its step,
// so a step that converged at its first pass costs one short launch.  Agent-
// scope fences around each barrier publish this phase's writes (node
// velocities, tile partials, flags) and drop stale lines from the vector cache.
template <class TL, bool OBJ>
__global__ __launch_bounds__(TL::NT) void k_extra_passes(BatchMap m, int tiles, int node_blocks, int cur, int step,
                                                         int par, int npass, int store_vc) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int pass = 1; pass < npass; ++pass) {
        bool done = true;
        for (int s = 0; s < m.n; ++s)
            done = done && (!member_active(m, s) || flag_load(&m.args[s].st->finished[pass]) != 0);
        if (done) break;                      // the same decision in every block
        if (threadIdx.x < kBlock)
            for (int nb = blockIdx.x; nb < node_blocks; nb += gridDim.x) grid_block<TL, true>(m, nb, cur, step, pass);
        __threadfence();
        grid.sync();
        __threadfence();
        for (int gt = blockIdx.x; gt < tiles; gt += gridDim.x) {
            g2p2g_tile<TL, true, OBJ>(m, gt, cur, step, par, pass, store_vc);
            __syncthreads();
        }
        __threadfence();
        grid.sync();
        __threadfence();
    }
}

// Counting sort, scan part: exclusive prefix sum of the next step's tile sizes
// (accumulated by the fused kernel), one block of 16 waves per sensor; clears the
// counts and the per-step loop flags for the next step.  Each thread takes four
// consecutive counts of a 4096-entry chunk (one 16-byte load, clear and store
// where all four exist); the waves scan their thread totals with cross-lane
// shifts, so a chunk costs two block barriers.
__global__ __launch_bounds__(1024) void k_scan(BatchMap m, int next, int limit_slots) {
    if (!member_active(m, blockIdx.x)) return;
    const KArgs& a = m.args[blockIdx.x];
    const gptr<uint32_t> __restrict__ bstart_next = glb(pick(a.bstart, next));
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid < limit_slots) a.st->finished[tid] = 0;
    uint32_t carry = 0;   // the same in every thread
    for (int t0 = 0; t0 < a.n_tiles; t0 += 4096) {
        const int u0 = t0 + 4 * tid;
        uint32_t c[4];
        if (u0 + 3 < a.n_tiles) {
            // four counts in one 16-byte load, cleared with one 16-byte store
            const u32x4 v = *(gptr<const u32x4>)(glb(a.newcnt) + u0);
            *(gptr<u32x4>)(glb(a.newcnt) + u0) = u32x4{0u, 0u, 0u, 0u};
            c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = 0;
                if (u0 + q < a.n_tiles) {
                    c[q] = glb(a.newcnt)[u0 + q];
                    glb(a.newcnt)[u0 + q] = 0;
                }
            }
        }
        const uint32_t tot = c[0] + c[1] + c[2] + c[3];
        uint32_t incl = tot;   // inclusive scan of the thread totals over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        uint32_t run = carry + incl - tot, chunk = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const uint32_t ws = wsum[w];
            if (w < wid) run += ws;
            chunk += ws;
        }
        if (u0 + 3 < a.n_tiles) {
            const uint32_t r0 = run, r1 = r0 + c[0], r2 = r1 + c[1], r3 = r2 + c[2];
            *(gptr<u32x4>)(bstart_next + u0) = u32x4{r0, r1, r2, r3};
            run = r3 + c[3];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (u0 + q < a.n_tiles) bstart_next[u0 + q] = run;
                run += c[q];
            }
        }
        carry += chunk;
        __syncthreads();   // the next chunk rewrites wsum
    }
    if (tid == 0) bstart_next[a.n_tiles] = carry;
}

// Counting sort, scatter part: the particles of tile t that move in direction
// d go to next-order positions bstart_next[t + d] + (particles that entered
// t + d from the directions before d, in a fixed order) + rank.
__global__ __launch_bounds__(kBlock) void k_scatter(BatchMap m, int cur) {
    __shared__ uint32_t off[kDirs];
    int s = 0, t = blockIdx.x;
    if (m.tile_base) {
        s = batch_find(m.tile_base, m.n, t);
        t -= m.tile_base[s];
    }
    if (!member_active(m, s)) return;
    const KArgs a = load_args(m, s);
    const gptr<const uint32_t> __restrict__ order = glb<const uint32_t>(pick(a.order, cur));
    const gptr<const uint32_t> __restrict__ bstart = glb<const uint32_t>(pick(a.bstart, cur));
    const gptr<const uint32_t> __restrict__ bstart_next = glb<const uint32_t>(pick(a.bstart, cur ^ 1));
    const gptr<uint32_t> __restrict__ order_next = glb(pick(a.order, cur ^ 1));
    const uint32_t s0 = bstart[t], cnt = bstart[t + 1] - s0;
    if (cnt == 0) return;
    const int tid = threadIdx.x;
    // The first kPre rounds of (direction rank, id) pairs are loaded before the
    // destination offsets are summed, so the two memory round trips overlap.
    constexpr int kPre = 6;
    uint32_t pre_dr[kPre], pre_id[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        const uint32_t i = tid + k * kBlock;
        pre_dr[k] = i < cnt ? glb(a.dirrank)[s0 + i] : 0u;
        pre_id[k] = i < cnt ? order[s0 + i] : 0u;
    }
    if (tid < kDirs) {
        int tc[3], u[3];
        tile_coords(a, t, tc);
        const int dd[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
        bool ok = true;
        for (int q = 0; q < 3; ++q) {
            u[q] = tc[q] + dd[q];
            ok = ok && u[q] >= 0 && u[q] < a.NT[q];
        }
        uint32_t o = 0;
        if (ok) {
            o = bstart_next[tile_linear(a, u)];
            // the 26 candidate loads are independent: issue them all, then sum
            uint32_t cnts[kDirs];
#pragma unroll
            for (int d2 = 0; d2 < kDirs; ++d2) {
                const int e2[3] = {d2 % 3 - 1, (d2 / 3) % 3 - 1, d2 / 9 - 1};
                int sc[3];
                bool ok2 = d2 < tid;
                for (int q = 0; q < 3; ++q) {
                    sc[q] = u[q] - e2[q];
                    ok2 = ok2 && sc[q] >= 0 && sc[q] < a.NT[q];
                }
                cnts[d2] = ok2 ? glb(a.dircount)[(size_t)tile_linear(a, sc) * kDirs + d2] : 0u;
            }
#pragma unroll
            for (int d2 = 0; d2 < kDirs; ++d2) o += cnts[d2];
        }
        off[tid] = o;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        if (tid + k * kBlock < cnt) {
            const uint32_t dst = off[pre_dr[k] & 31u] + (pre_dr[k] >> 5);
            if (dst < (uint32_t)a.n) order_next[dst] = pre_id[k];
            else atomicOr(&a.st->error, DEV_CFL);
        }
    }
    for (uint32_t i = tid + kPre * kBlock; i < cnt; i += kBlock) {
        const uint32_t dr = glb(a.dirrank)[s0 + i];
        const uint32_t dst = off[dr & 31u] + (dr >> 5);
        if (dst < (uint32_t)a.n) order_next[dst] = order[s0 + i];
        else atomicOr(&a.st->error, DEV_CFL);
    }
}

// Storage compaction, one block per tile: the tile's particles move to the
// slots of its binned range, so that its loads fill consecutive cache lines
// again, and the order over the range becomes the identity.  Inside the range
// they go round-robin over the stencil base nodes (the first particle of every
// base node, then the second, ...), the base nodes taken in the order of
// tile_slot, so that the lanes of the next fused kernels add to different LDS
// nodes on different banks.  With r the rank of a particle among those of its
// base node, l its slot and c[.] the slot counts, the new position is
// sum_l' min(c[l'], r) + #{l' < l : c[l'] > r}, a bijection onto the range.
// Every state plane (with move_vc == 0 all but the velocity and affine planes,
// which the caller's next steps rewrite before anything reads them), the
// packed cell, the flags and the id map move together;
// the calibration particle's new slot goes to e_out.  The rank is taken with LDS
// atomics, so the storage order may differ between runs; no result depends on
// it (the node sums are exact).  dirrank, which the next fused kernel rewrites,
// holds (rank, base node) between the two passes.  Out-of-range entries latch
// DEV_CFL and are clamped, which keeps every access in bounds.
constexpr int kMaxTileNodes = 512;

__global__ __launch_bounds__(kBlock) void k_compact(KArgs a, int cur, float* __restrict__ soa_dst,
                                                    uint32_t* __restrict__ cell_dst,
                                                    uint8_t* __restrict__ flags_dst,
                                                    const uint32_t* __restrict__ id_src,
                                                    uint32_t* __restrict__ id_dst, long long* __restrict__ e_out,
                                                    int move_vc) {
    __shared__ uint32_t cnt[kMaxTileNodes];
    const int t = blockIdx.x, tid = threadIdx.x;
    const gptr<uint32_t> order = glb(pick(a.order, cur));
    const gptr<const uint32_t> bstart = glb<const uint32_t>(pick(a.bstart, cur));
    const gptr<uint32_t> keys = glb(a.dirrank);
    const gptr<const float> soa = glb<const float>(a.soa);
    const size_t n = (size_t)a.n;
    const uint32_t s0 = bstart[t], c = bstart[t + 1] - s0;
    if (c == 0) return;
    const int nl = a.T[0] * a.T[1] * a.T[2];
    for (int k = tid; k < nl; k += kBlock) cnt[k] = 0;
    __syncthreads();
    int tc[3];
    tile_coords(a, t, tc);
    int err = 0;
    for (uint32_t i = tid; i < c; i += kBlock) {
        uint32_t src = order[s0 + i];
        if (src >= n) { err |= DEV_CFL; src = 0; }
        int cell[3];
        float f[3];
        load_particle(a, src, cell, f);
        int l[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            l[q] = cell[q] - 1 + (f[q] >= 0.5f ? 1 : 0) - tc[q] * a.T[q];
            if (l[q] < 0 || l[q] >= a.T[q]) { err |= DEV_CFL; l[q] = l[q] < 0 ? 0 : a.T[q] - 1; }
        }
        const uint32_t local = (uint32_t)tile_slot(l[0], l[1], l[2], a.T[0], a.T[1], a.T[2]);
        const uint32_t r = atomicAdd(&cnt[local], 1u);
        keys[s0 + i] = (r << 9) | local;
    }
    __syncthreads();
    for (uint32_t i = tid; i < c; i += kBlock) {
        const uint32_t key = keys[s0 + i], r = key >> 9, local = key & 511u;
        uint32_t pos = 0;
        for (int k = 0; k < nl; ++k) {
            const uint32_t ck = cnt[k];
            pos += min(ck, r) + (((uint32_t)k < local && ck > r) ? 1u : 0u);
        }
        const size_t dst = s0 + min(pos, c - 1);
        uint32_t src = order[s0 + i];
        if (src >= n) src = 0;
        cell_dst[dst] = glb(a.cell)[src];
        flags_dst[dst] = glb(a.flags)[src];
        id_dst[dst] = id_src[src];
#pragma unroll
        for (int p = 0; p < NPLANES; ++p)
            if (move_vc || p < V0 || p >= G0) soa_dst[(size_t)p * n + dst] = soa[(size_t)p * n + src];
        if ((long long)src == a.e) *e_out = (long long)dst;
    }
    __syncthreads();
    for (uint32_t i = tid; i < c; i += kBlock) order[s0 + i] = s0 + i;
    if (err) atomicOr(&a.st->error, err);
}

// Surface raster: every surface particle adds its quadratic B-spline weights
// (pitch = pixel size) and weighted displacement (in cells) to a W x H
// accumulator of 64-bit fixed-point sums (2^-32), so the maps are exact and
// independent of the order of the atomics.
__global__ void k_surface_accum(KArgs a, SurfArgs s) {
    const long long slot = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (slot >= a.n) return;
    if (!(glb(a.flags)[slot] & FLAG_SURFACE)) return;
    const long long id = s.id_of[slot];
    // the particle's surface slot: column (ci, cj) and sub-column (sx, sy); the
    // record holds its rest offsets and the rest cell height of its column
    const long long sidx = s.surf_of[id];
    if (sidx < 0) return;
    const int sx = (int)(sidx % s.m), sy = (int)((sidx / s.m) % s.m);
    const long long col = sidx / ((long long)s.m * s.m);
    const int ci = (int)(col % s.Nx), cj = (int)(col / s.Nx);
    const float4 rr = s.rest_r[sidx];
    const int ck = (int)rr.w;
    int cell[3];
    float f[3];
    load_particle(a, slot, cell, f);
    const int rc[3] = {ci + s.pad_l, cj + s.pad_l, ck + s.pad_b};
    const float r3[3] = {rr.x, rr.y, rr.z};
    float u[3];
    for (int q = 0; q < 3; ++q) u[q] = (float)(cell[q] - rc[q]) + (f[q] - r3[q]);
    const double px = ((double)(cell[0] - s.pad_l) + (double)f[0]) / s.pitch_x - 0.5;
    const double py = ((double)(cell[1] - s.pad_l) + (double)f[1]) / s.pitch_y - 0.5;
    const int bx = (int)floor(px + 0.5) - 1, by = (int)floor(py + 0.5) - 1;
    const float fx = (float)(px - bx), fy = (float)(py - by);
    float wx[3], wy[3];
    {
        const float a0 = 1.5f - fx, b0 = fx - 1.0f, c0 = fx - 0.5f;
        wx[0] = 0.5f * a0 * a0; wx[1] = 0.75f - b0 * b0; wx[2] = 0.5f * c0 * c0;
        const float a1 = 1.5f - fy, b1 = fy - 1.0f, c1 = fy - 0.5f;
        wy[0] = 0.5f * a1 * a1; wy[1] = 0.75f - b1 * b1; wy[2] = 0.5f * c1 * c1;
    }
    for (int cy = 0; cy < 3; ++cy) {
        const int vy = by + cy;
        if (vy < 0 || vy >= s.H) continue;
        for (int cx = 0; cx < 3; ++cx) {
            const int ux = bx + cx;
            if (ux < 0 || ux >= s.W) continue;
            const float wt = wx[cx] * wy[cy] * kFixScaleF;
            if (wt == 0.f) continue;
            unsigned long long* d = s.acc + 4 * ((size_t)vy * s.W + ux);
            atomicAdd(d + 0, to_fixed_scaled(wt, kFixMagic));
            atomicAdd(d + 1, to_fixed_scaled(wt * u[0], kFixMagic));
            atomicAdd(d + 2, to_fixed_scaled(wt * u[1], kFixMagic));
            atomicAdd(d + 3, to_fixed_scaled(wt * u[2], kFixMagic));
        }
    }
}

// Depth of the indenter below the slab's top face along each pixel's vertical
// line: (top - z_low) * scale with z_low its lowest point on the line, -1e9
// where the line misses it.  FP64, evaluated as the body-frame formulas of the
// four shapes (the lower half of the sphere and capsule, the rounded box's
// bottom face with its fillet, the height field's bilinear surface).
__global__ __launch_bounds__(256) void k_depthmap(KArgs a, DepthArgs g, float* __restrict__ out) {
#pragma clang fp contract(off)
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= g.W * g.H) return;
    const int u = q % g.W, v = q / g.W;
    const double dx = ((double)u + 0.5) * g.Lx / (double)g.W - g.c[0];
    const double dy = ((double)v + 0.5) * g.Ly / (double)g.H - g.c[1];
    const double px = g.R[0] * dx + g.R[3] * dy, py = g.R[1] * dx + g.R[4] * dy;
    bool hit = false;
    double zb = 0.0;
    if (a.shape == 1) {
        const double r2 = px * px + py * py;
        if (r2 <= a.radius * a.radius) { hit = true; zb = -sqrt(a.radius * a.radius - r2); }
    } else if (a.shape == 2) {
        const double h = a.half_length;
        const double t = px < -h ? -h : (px > h ? h : px);
        const double d2 = (px - t) * (px - t) + py * py;
        if (d2 <= a.radius * a.radius) { hit = true; zb = -sqrt(a.radius * a.radius - d2); }
    } else if (a.shape == 3) {
        const double f = a.fillet;
        const double qx = fabs(px) - (a.he[0] - f), qy = fabs(py) - (a.he[1] - f);
        const double ox = qx > 0.0 ? qx : 0.0, oy = qy > 0.0 ? qy : 0.0;
        const double o2 = ox * ox + oy * oy;
        if (o2 <= f * f) { hit = true; zb = -(a.he[2] - f) - sqrt(f * f - o2); }
    } else if (a.shape == 4) {
        if (px * px + py * py <= a.hf_half * a.hf_half) {
            const int n = a.hf_n;
            const double step = 2.0 * a.hf_half / (double)(n - 1);
            const double fu0 = (px + a.hf_half) / step, fv0 = (py + a.hf_half) / step;
            const int i0 = min(max((int)floor(fu0), 0), n - 2), j0 = min(max((int)floor(fv0), 0), n - 2);
            const double fu = fu0 - (double)i0, fv = fv0 - (double)j0;
            const double* t = a.hf + (size_t)j0 * n + i0;
            const double z0 = (1.0 - fu) * t[0] + fu * t[1];
            const double z1 = (1.0 - fu) * t[n] + fu * t[n + 1];
            hit = true;
            zb = (1.0 - fv) * z0 + fv * z1;
        }
    }
    out[q] = hit ? (float)((g.top - (g.c[2] + zb)) * g.scale) : -1e9f;
}

// The height map's rest height under a pixel is the slab height, or with a
// shaped elastomer that of the column under the pixel centre (col_top: Nx x Ny
// rest heights in metres, null for the cuboid).
__global__ void k_surface_finish(const unsigned long long* __restrict__ acc, int npix, int W, float top,
                                 float dx, int mode, float* __restrict__ out, const float* __restrict__ col_top,
                                 int Nx, int Ny) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix) return;
    long long v[4];
    for (int k = 0; k < 4; ++k) v[k] = ((long long)(acc[4 * q + k] << 13)) >> 13;
    const double inv = v[0] > 0 ? (double)dx / (double)v[0] : 0.0;
    if (mode == 0) {
        float rest = top;
        if (col_top) {
            const int H = npix / W, u = q % W, vv = q / W;
            const int i = min((int)floor(((double)u + 0.5) * (double)Nx / (double)W), Nx - 1);
            const int j = min((int)floor(((double)vv + 0.5) * (double)Ny / (double)H), Ny - 1);
            rest = col_top[(size_t)j * Nx + i];
        }
        out[q] = rest + (float)((double)v[3] * inv);
    } else {
        out[3 * q + 0] = (float)((double)v[1] * inv);
        out[3 * q + 1] = (float)((double)v[2] * inv);
        out[3 * q + 2] = (float)((double)v[3] * inv);
    }
}

// Tile shapes compiled into the library (cells per axis): explicit kernel
// instantiations, seen by both the device and the host compilation pass.
#define IMPM_TILE_KERNELS(X, Y, Z, N)                                                             \
    template __global__ void k_p2g<Tile<X, Y, Z, N>>(BatchMap, int);                              \
    template __global__ void k_grid<Tile<X, Y, Z, N>, false>(BatchMap, int, int, int, int);       \
    template __global__ void k_grid<Tile<X, Y, Z, N>, true>(BatchMap, int, int, int, int);        \
    template __global__ void k_g2p2g<Tile<X, Y, Z, N>, false, false>(BatchMap, int, int, int, int, int, int); \
    template __global__ void k_g2p2g<Tile<X, Y, Z, N>, true, false>(BatchMap, int, int, int, int, int, int); \
    template __global__ void k_g2p2g<Tile<X, Y, Z, N>, false, true>(BatchMap, int, int, int, int, int, int); \
    template __global__ void k_g2p2g<Tile<X, Y, Z, N>, true, true>(BatchMap, int, int, int, int, int, int); \
    template __global__ void k_extra_passes<Tile<X, Y, Z, N>, false>(BatchMap, int, int, int, int, int, int, int); \
    template __global__ void k_extra_passes<Tile<X, Y, Z, N>, true>(BatchMap, int, int, int, int, int, int, int);
IMPM_TILE_KERNELS(8, 8, 2, 256)
IMPM_TILE_KERNELS(8, 8, 2, 512)
IMPM_TILE_KERNELS(4, 8, 4, 256)
IMPM_TILE_KERNELS(8, 4, 4, 256)
IMPM_TILE_KERNELS(8, 8, 4, 256)
IMPM_TILE_KERNELS(8, 8, 4, 512)
IMPM_TILE_KERNELS(4, 4, 4, 256)
IMPM_TILE_KERNELS(8, 4, 2, 256)
IMPM_TILE_KERNELS(4, 4, 2, 256)
IMPM_TILE_KERNELS(4, 8, 2, 256)
IMPM_TILE_KERNELS(8, 8, 8, 512)
#undef IMPM_TILE_KERNELS

// Host launchers and the table of the compiled tile shapes (host pass only).
#ifndef __HIP_DEVICE_COMPILE__
template <int TX, int TY, int TZ, int NB>
struct TileLaunch {
    using TL = Tile<TX, TY, TZ, NB>;
    static void p2g(const BatchMap& m, int tile_blocks, int cur, hipStream_t st) {
        hipLaunchKernelGGL(k_p2g<TL>, dim3(tile_blocks), dim3(NB), TL::LDS_P2G, st, m, cur);
    }
    static void grid(const BatchMap& m, int node_blocks, int sbin, int step, int pass, bool extra,
                     hipStream_t st) {
        if (extra)
            hipLaunchKernelGGL((k_grid<TL, true>), dim3(std::min(node_blocks, kExtraBlocks)), dim3(kBlock), 0, st,
                               m, node_blocks, sbin, step, pass);
        else
            hipLaunchKernelGGL((k_grid<TL, false>), dim3(node_blocks), dim3(kBlock), 0, st, m, node_blocks, sbin,
                               step, pass);
    }
    template <bool OBJ>
    static void g2p2g_as(const BatchMap& m, int tile_blocks, int cur, int step, int par, int pass, int store_vc,
                         bool extra, hipStream_t st) {
        if (extra)
            hipLaunchKernelGGL((k_g2p2g<TL, true, OBJ>), dim3(std::min(tile_blocks, kExtraBlocks)), dim3(NB),
                               TL::LDS_G2P2G, st, m, tile_blocks, cur, step, par, pass, store_vc);
        else
            hipLaunchKernelGGL((k_g2p2g<TL, false, OBJ>), dim3(tile_blocks), dim3(NB), TL::LDS_G2P2G, st, m,
                               tile_blocks, cur, step, par, pass, store_vc);
    }
    static void g2p2g(const BatchMap& m, int tile_blocks, int cur, int step, int par, int pass, int store_vc,
                      bool extra, hipStream_t st) {
        if (m.objects) g2p2g_as<true>(m, tile_blocks, cur, step, par, pass, store_vc, extra, st);
        else g2p2g_as<false>(m, tile_blocks, cur, step, par, pass, store_vc, extra, st);
    }
    template <bool OBJ>
    static hipError_t extra_as(const BatchMap& m, int tile_blocks, int node_blocks, int cur, int step, int par,
                               int npass, int store_vc, hipStream_t st) {
        static int max_blocks = 0;    // resident blocks of this kernel on the device
        if (max_blocks == 0) {
            int dev = 0, cus = 0, per = 0;
            hipError_t e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_extra_passes<TL, OBJ>, NB, TL::LDS_G2P2G);
            if (e != hipSuccess) return e;
            max_blocks = per * cus;
        }
        if (max_blocks < 1) return hipErrorCooperativeLaunchTooLarge;
        BatchMap mm = m;
        int a_tiles = tile_blocks, a_nodes = node_blocks, a_cur = cur, a_step = step, a_par = par, a_np = npass,
            a_st = store_vc;
        void* args[] = {&mm, &a_tiles, &a_nodes, &a_cur, &a_step, &a_par, &a_np, &a_st};
        const int grid = std::min(max_blocks, std::max(tile_blocks, node_blocks));
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_extra_passes<TL, OBJ>), dim3(grid),
                                          dim3(NB), args, (unsigned)TL::LDS_G2P2G, st);
    }
    static hipError_t extra(const BatchMap& m, int tile_blocks, int node_blocks, int cur, int step, int par,
                            int npass, int store_vc, hipStream_t st) {
        return m.objects ? extra_as<true>(m, tile_blocks, node_blocks, cur, step, par, npass, store_vc, st)
                         : extra_as<false>(m, tile_blocks, node_blocks, cur, step, par, npass, store_vc, st);
    }
    static constexpr TileOps ops() {
        return TileOps{{TX, TY, TZ}, NB, TL::PVOL, TL::LDS_G2P2G, &p2g, &grid, &g2p2g, &extra};
    }
};

const TileOps kTileOps[] = {
    TileLaunch<8, 8, 2, 256>::ops(), TileLaunch<8, 8, 2, 512>::ops(), TileLaunch<4, 8, 4, 256>::ops(),
    TileLaunch<8, 4, 4, 256>::ops(), TileLaunch<8, 8, 4, 256>::ops(), TileLaunch<8, 8, 4, 512>::ops(),
    TileLaunch<4, 4, 4, 256>::ops(), TileLaunch<8, 4, 2, 256>::ops(), TileLaunch<4, 4, 2, 256>::ops(),
    TileLaunch<4, 8, 2, 256>::ops(), TileLaunch<8, 8, 8, 512>::ops(),
};
const int kNumTileOps = sizeof(kTileOps) / sizeof(kTileOps[0]);

#endif

}  // namespace impm
