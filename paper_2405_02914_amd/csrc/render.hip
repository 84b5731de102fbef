// render.hip -- gfx950 path tracer of the tactile image (arXiv 2405.02914,
// Sec. III-B and Sec. IV-B): the elastomer surface meshed from the height map,
// textured, diffuse, lit by rectangular LEDs and seen from below.  The
// estimator, its random numbers and the scene conventions are those stated in
// include/render.h; the arithmetic is FP32.
//
// Four kernels per frame.  k_tile_range writes the height range of every
// kTile x kTile-cell tile of the mesh, k_block_range that of every block of
// kTile x kTile tiles and k_range_total that of the whole map, all into the
// caller's workspace.  k_render then takes one wave per pixel (lane l takes
// samples l, l + 64, ..., the lanes' sums combined by cross-lane shuffles) and
// four pixels per block: all lanes of a wave start their rays at the same
// surface point, so their walks stay close (measured on a 640 x 480 map with a
// 1.4 mm dent, 128 samples: 24 ms per frame, against 31 ms with 4 lanes per
// pixel and 16 pixels per wave), and the register budget is held to 4 waves
// per SIMD (128 VGPRs; 36 ms at the 141 the compiler takes unbounded, 3 waves
// per SIMD).  A ray walks the blocks it crosses in order, the tiles of
// a block, then the cells of a tile; a block or tile whose height range the
// ray's height over it does not meet is skipped whole (two triangles per cell,
// a cell skipped when the same test fails on its four corners).  The first hit found is the nearest: a triangle lies inside
// its cell's footprint, and the cells are met in order of t.  A ray heading
// down below the map's lowest point, or up above its highest, stops.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "../../include/render.h"

namespace rt {

constexpr int kTile = 8;                  // cells per tile side
constexpr int kLanes = 64;                // lanes per pixel: one pixel per wave
constexpr int kPixels = 4;                // pixels per block
constexpr int kThreads = kLanes * kPixels;
constexpr float kRayOffset = 1e-7f;       // m, off the surface along n

struct LightF {
    float c[3], e1[3], e2[3], nl[3], L[3];
    float area;
};

struct Args {
    int W, H, out_w, out_h, spp, bounces, n_lights, tex_w, tex_h;
    int TW, TH;                           // tiles per row, per column
    int BW, BH;                           // blocks (kTile x kTile tiles) per row, per column
    float Lx, Ly, px, py;
    unsigned long long seed;
    LightF lights[4];
    const float* h;
    const float* tex;
    const float2* tiles;                  // TH x TW (min, max)
    const float2* blocks;                 // BH x BW (min, max)
    const float2* total;                  // (min, max) of the map
    float* out;
};

// Work counts of one render (the counting instantiation only): rays traced,
// tiles and cells visited, triangles tested.
struct Work {
    unsigned long long rays = 0, tiles = 0, cells = 0, tris = 0;
};

__host__ __device__ inline int tiles_along(int n) { return (n - 1 + kTile - 1) / kTile; }
__host__ __device__ inline int blocks_along(int n) { return (tiles_along(n) + kTile - 1) / kTile; }

__host__ __device__ __forceinline__ float draw(const Args& a, long long pix, int s, int k) {
    const unsigned long long t =
        ((unsigned long long)pix * (unsigned long long)a.spp + (unsigned long long)s) * 32ull +
        (unsigned long long)k + 1ull;
    unsigned long long z = a.seed + t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)(z >> 40) * (1.0f / 16777216.0f);
}

__host__ __device__ __forceinline__ float hgt(const Args& a, int u, int v) { return a.h[(long long)v * a.W + u]; }

// Central-difference slope (dz/dx, dz/dy) of the map at sample (u, v),
// one-sided on the border.  Neighbouring heights are close, so their
// differences are exact in FP32.
__host__ __device__ inline void vertex_slope(const Args& a, int u, int v, float g[2]) {
    const int u0 = u > 0 ? u - 1 : u, u1 = u < a.W - 1 ? u + 1 : u;
    const int v0 = v > 0 ? v - 1 : v, v1 = v < a.H - 1 ? v + 1 : v;
    g[0] = (hgt(a, u1, v) - hgt(a, u0, v)) / ((float)(u1 - u0) * a.px);
    g[1] = (hgt(a, u, v1) - hgt(a, u, v0)) / ((float)(v1 - v0) * a.py);
}

// Height of the mesh above (x, y), clamped to it, and the shading normal
// there (visible side): the normal of the slope field that is linear on each
// triangle and equals the central-difference slope at the samples, so that it
// is continuous across the triangles' edges.
__host__ __device__ void surface_at(const Args& a, float x, float y, float p[3], float n[3]) {
    const float gx = fminf(fmaxf(x / a.px - 0.5f, 0.0f), (float)(a.W - 1));
    const float gy = fminf(fmaxf(y / a.py - 0.5f, 0.0f), (float)(a.H - 1));
    const int u = min((int)floorf(gx), a.W - 2), v = min((int)floorf(gy), a.H - 2);
    const float fx = gx - (float)u, fy = gy - (float)v;
    const float za = hgt(a, u, v), zb = hgt(a, u + 1, v), zc = hgt(a, u, v + 1), zd = hgt(a, u + 1, v + 1);
    float ga[2], gd[2], ge[2];   // slopes at (u, v), (u+1, v+1) and the third corner
    vertex_slope(a, u, v, ga);
    vertex_slope(a, u + 1, v + 1, gd);
    float z, w0, w1, w2;         // barycentric weights of (u, v), the third corner, (u+1, v+1)
    if (fx >= fy) {              // the (u, v), (u+1, v), (u+1, v+1) triangle
        z = za + fx * (zb - za) + fy * (zd - zb);
        vertex_slope(a, u + 1, v, ge);
        w0 = 1.0f - fx; w1 = fx - fy; w2 = fy;
    } else {                     // the (u, v), (u+1, v+1), (u, v+1) triangle
        z = za + fy * (zc - za) + fx * (zd - zc);
        vertex_slope(a, u, v + 1, ge);
        w0 = 1.0f - fy; w1 = fy - fx; w2 = fx;
    }
    const float sx = w0 * ga[0] + w1 * ge[0] + w2 * gd[0];
    const float sy = w0 * ga[1] + w1 * ge[1] + w2 * gd[1];
    p[0] = ((float)u + fx + 0.5f) * a.px;
    p[1] = ((float)v + fy + 0.5f) * a.py;
    p[2] = z;
    const float l = sqrtf(sx * sx + sy * sy + 1.0f);
    n[0] = sx / l;
    n[1] = sy / l;
    n[2] = -1.0f / l;
}

// Ray-triangle intersection (Moller-Trumbore); t or -1.
__host__ __device__ __forceinline__ float tri_hit(const float o[3], const float d[3], const float A[3], const float B[3],
                                         const float C[3]) {
    const float e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const float e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    const float pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const float det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (fabsf(det) < 1e-30f) return -1.0f;
    const float inv = 1.0f / det;
    const float tv[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
    const float uu = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (uu < 0.0f || uu > 1.0f) return -1.0f;
    const float qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    const float vv = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (vv < 0.0f || uu + vv > 1.0f) return -1.0f;
    return (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
}

// A ray in world space and in vertex-index space g = (x / px - 1/2, y / py - 1/2).
struct Ray {
    float o[3], d[3];
    float gx, gy;       // origin in index space
    float dgx, dgy;     // direction in index space
    float igx, igy;     // their reciprocals, 0 where the component is 0
    int su, sv;         // step directions
};

__host__ __device__ __forceinline__ Ray make_ray(const Args& a, const float o[3], const float d[3]) {
    Ray r;
    for (int k = 0; k < 3; ++k) {
        r.o[k] = o[k];
        r.d[k] = d[k];
    }
    r.gx = o[0] / a.px - 0.5f;
    r.gy = o[1] / a.py - 0.5f;
    r.dgx = d[0] / a.px;
    r.dgy = d[1] / a.py;
    r.igx = r.dgx != 0.0f ? 1.0f / r.dgx : 0.0f;
    r.igy = r.dgy != 0.0f ? 1.0f / r.dgy : 0.0f;
    r.su = r.dgx > 0.0f ? 1 : -1;
    r.sv = r.dgy > 0.0f ? 1 : -1;
    return r;
}

// t at which the ray crosses the index-space line x = bx (y = by), or FLT_MAX.
__host__ __device__ __forceinline__ float cross_x(const Ray& r, int bx) {
    return r.igx != 0.0f ? ((float)bx - r.gx) * r.igx : FLT_MAX;
}
__host__ __device__ __forceinline__ float cross_y(const Ray& r, int by) {
    return r.igy != 0.0f ? ((float)by - r.gy) * r.igy : FLT_MAX;
}

// Does the ray's height over [t0, t1] meet [lo, hi] widened by m?
__host__ __device__ __forceinline__ bool meets(const Ray& r, float t0, float t1, float lo, float hi, float m) {
    const float z0 = r.o[2] + t0 * r.d[2], z1 = r.o[2] + t1 * r.d[2];
    return fmaxf(z0, z1) >= lo - m && fminf(z0, z1) <= hi + m;
}

// Nearest hit in (0, tmax) among the cells [ulo, uhi] x [vlo, vhi] that the
// ray crosses over [ta, tb], or -1.
template <bool COUNT>
__host__ __device__ float walk_cells(const Args& a, const Ray& r, float ta, float tb, float tmax, int ulo, int uhi,
                                     int vlo, int vhi, float mz, Work& w) {
    int u = min(max((int)floorf(r.gx + ta * r.dgx), ulo), uhi);
    int v = min(max((int)floorf(r.gy + ta * r.dgy), vlo), vhi);
    float t0 = ta;
    for (int guard = 0; guard < 2 * kTile + 2; ++guard) {
        const float tx = cross_x(r, r.su > 0 ? u + 1 : u), ty = cross_y(r, r.sv > 0 ? v + 1 : v);
        const float t1 = fminf(fminf(tx, ty), tb);
        float A[3], B[3], C[3], D[3];
        A[0] = ((float)u + 0.5f) * a.px;
        A[1] = ((float)v + 0.5f) * a.py;
        A[2] = hgt(a, u, v);
        B[0] = A[0] + a.px; B[1] = A[1]; B[2] = hgt(a, u + 1, v);
        C[0] = A[0]; C[1] = A[1] + a.py; C[2] = hgt(a, u, v + 1);
        D[0] = B[0]; D[1] = C[1]; D[2] = hgt(a, u + 1, v + 1);
        if constexpr (COUNT) ++w.cells;
        const float lo = fminf(fminf(A[2], B[2]), fminf(C[2], D[2]));
        const float hi = fmaxf(fmaxf(A[2], B[2]), fmaxf(C[2], D[2]));
        if (meets(r, t0, t1, lo, hi, mz)) {
            if constexpr (COUNT) w.tris += 2;
            const float h1 = tri_hit(r.o, r.d, A, B, D), h2 = tri_hit(r.o, r.d, A, D, C);
            float best = -1.0f;
            if (h1 > 0.0f && h1 < tmax) best = h1;
            if (h2 > 0.0f && h2 < tmax && (best < 0.0f || h2 < best)) best = h2;
            if (best > 0.0f) return best;
        }
        if (t1 >= tb) break;
        if (tx < ty) {
            u += r.su;
            if (u < ulo || u > uhi) break;
        } else {
            v += r.sv;
            if (v < vlo || v > vhi) break;
        }
        t0 = t1;
    }
    return -1.0f;
}

// Nearest hit in (0, tmax) among the cells [ulo, uhi] x [vlo, vhi] that the
// ray crosses over [ta, tb], walking the blocks of level LEVEL of the height-
// range grid in order (1: kTile-cell tiles, 2: kTile^2-cell blocks) and
// skipping those whose height range the ray's height over them misses.  The
// windows passed down are aligned to the blocks below.  At the top level the
// ray also stops once it is below the map's lowest point heading down, or
// above its highest heading up.
template <int LEVEL, bool COUNT>
__host__ __device__ float walk_blocks(const Args& a, const Ray& r, float ta, float tb, float tmax, int ulo, int uhi,
                                      int vlo, int vhi, float zmin, float zmax, float mz, Work& w) {
    constexpr int S = LEVEL == 1 ? kTile : kTile * kTile;    // cells per block side
    const float2* ranges = LEVEL == 1 ? a.tiles : a.blocks;
    const int per_row = LEVEL == 1 ? a.TW : a.BW;
    const int blo = ulo / S, bhi = uhi / S, clo = vlo / S, chi = vhi / S;
    int bu = min(max((int)floorf((r.gx + ta * r.dgx) / (float)S), blo), bhi);
    int bv = min(max((int)floorf((r.gy + ta * r.dgy) / (float)S), clo), chi);
    float t0 = ta;
    for (int guard = 0; guard < (bhi - blo) + (chi - clo) + 2; ++guard) {
        if constexpr (LEVEL == 2) {
            const float z0 = r.o[2] + t0 * r.d[2];
            if ((r.d[2] < 0.0f && z0 < zmin - mz) || (r.d[2] > 0.0f && z0 > zmax + mz)) return -1.0f;
        }
        const int cu0 = max(bu * S, ulo), cu1 = min(bu * S + S - 1, uhi);
        const int cv0 = max(bv * S, vlo), cv1 = min(bv * S + S - 1, vhi);
        const float tx = cross_x(r, r.su > 0 ? cu1 + 1 : cu0), ty = cross_y(r, r.sv > 0 ? cv1 + 1 : cv0);
        const float t1 = fminf(fminf(tx, ty), tb);
        if constexpr (COUNT) ++w.tiles;
        const float2 rg = ranges[bv * per_row + bu];
        if (meets(r, t0, t1, rg.x, rg.y, mz)) {
            float t;
            if constexpr (LEVEL == 1)
                t = walk_cells<COUNT>(a, r, t0, t1, tmax, cu0, cu1, cv0, cv1, mz, w);
            else
                t = walk_blocks<LEVEL - 1, COUNT>(a, r, t0, t1, tmax, cu0, cu1, cv0, cv1, zmin, zmax, mz, w);
            if (t > 0.0f) return t;
        }
        if (t1 >= tb) break;
        if (tx < ty) {
            bu += r.su;
            if (bu < blo || bu > bhi) break;
        } else {
            bv += r.sv;
            if (bv < clo || bv > chi) break;
        }
        t0 = t1;
    }
    return -1.0f;
}

// Nearest hit in (0, tmax) of the ray o + t d with the mesh, or -1.
template <bool COUNT>
__host__ __device__ float trace(const Args& a, const float o[3], const float d[3], float tmax, float zmin, float zmax,
                                float mz, Work& w) {
    if constexpr (COUNT) ++w.rays;
    const Ray r = make_ray(a, o, d);
    return walk_blocks<2, COUNT>(a, r, 0.0f, tmax, tmax, 0, a.W - 2, 0, a.H - 2, zmin, zmax, mz, w);
}

// Texel coordinate of x along an axis of n texels over length L: the index
// of the lower texel centre and the weight of the upper one (clamped).
__host__ __device__ __forceinline__ void texel_axis(float x, float L, int n, int& i0, float& f) {
    const float s = fminf(fmaxf(x / L * (float)n - 0.5f, 0.0f), (float)(n - 1));
    i0 = max(min((int)floorf(s), n - 2), 0);
    f = n > 1 ? s - (float)i0 : 0.0f;
}

// Albedo at p: the texture interpolated bilinearly between texel centres.
__host__ __device__ __forceinline__ void albedo(const Args& a, const float p[3], float rho[3]) {
    int i, j;
    float fx, fy;
    texel_axis(p[0], a.Lx, a.tex_w, i, fx);
    texel_axis(p[1], a.Ly, a.tex_h, j, fy);
    const int i1 = a.tex_w > 1 ? i + 1 : i, j1 = a.tex_h > 1 ? j + 1 : j;
    const float* r0 = a.tex + (long long)j * a.tex_w * 3;
    const float* r1 = a.tex + (long long)j1 * a.tex_w * 3;
    for (int k = 0; k < 3; ++k) {
        const float top = (1.0f - fx) * r0[3 * i + k] + fx * r0[3 * i1 + k];
        const float bot = (1.0f - fx) * r1[3 * i + k] + fx * r1[3 * i1 + k];
        rho[k] = (1.0f - fy) * top + fy * bot;
    }
}

// Direct light at p (normal n, albedo rho), draws k0 + 2l and k0 + 2l + 1 for light l.
template <bool COUNT>
__host__ __device__ void direct(const Args& a, const float p[3], const float n[3], const float rho[3], long long pix,
                                int s, int k0, float zmin, float zmax, float mz, float out[3], Work& wk) {
    for (int l = 0; l < a.n_lights; ++l) {
        const LightF& L = a.lights[l];
        const float x1 = draw(a, pix, s, k0 + 2 * l), x2 = draw(a, pix, s, k0 + 2 * l + 1);
        float w[3];
        for (int k = 0; k < 3; ++k) w[k] = L.c[k] + (x1 - 0.5f) * L.e1[k] + (x2 - 0.5f) * L.e2[k] - p[k];
        const float d2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        const float dist = sqrtf(d2);
        for (int k = 0; k < 3; ++k) w[k] /= dist;
        const float cos_p = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
        const float cos_l = -(L.nl[0] * w[0] + L.nl[1] * w[1] + L.nl[2] * w[2]);
        if (cos_p <= 0.0f || cos_l <= 0.0f) continue;
        const float o[3] = {p[0] + kRayOffset * n[0], p[1] + kRayOffset * n[1], p[2] + kRayOffset * n[2]};
        if (trace<COUNT>(a, o, w, dist, zmin, zmax, mz, wk) >= 0.0f) continue;   // in shadow
        const float g = L.area * cos_p * cos_l / d2 * 0.318309886183791f;   // 1 / pi
        for (int k = 0; k < 3; ++k) out[k] += L.L[k] * rho[k] * g;
    }
}

__global__ __launch_bounds__(256) void k_tile_range(const float* __restrict__ h, int W, int H, int TW, int TH,
                                                    float2* __restrict__ tiles) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= TW * TH) return;
    const int ti = q % TW, tj = q / TW;
    const int u1 = min(ti * kTile + kTile, W - 1), v1 = min(tj * kTile + kTile, H - 1);
    float lo = FLT_MAX, hi = -FLT_MAX;
    for (int v = tj * kTile; v <= v1; ++v)
        for (int u = ti * kTile; u <= u1; ++u) {
            const float z = h[(long long)v * W + u];
            lo = fminf(lo, z);
            hi = fmaxf(hi, z);
        }
    tiles[q] = make_float2(lo, hi);
}

// Height range of every block of kTile x kTile tiles, from the tiles' ranges.
__global__ __launch_bounds__(256) void k_block_range(const float2* __restrict__ tiles, int TW, int TH, int BW, int BH,
                                                     float2* __restrict__ blocks) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= BW * BH) return;
    const int bi = q % BW, bj = q / BW;
    float lo = FLT_MAX, hi = -FLT_MAX;
    for (int tj = bj * kTile; tj < min(bj * kTile + kTile, TH); ++tj)
        for (int ti = bi * kTile; ti < min(bi * kTile + kTile, TW); ++ti) {
            const float2 r = tiles[tj * TW + ti];
            lo = fminf(lo, r.x);
            hi = fmaxf(hi, r.y);
        }
    blocks[q] = make_float2(lo, hi);
}

__global__ __launch_bounds__(256) void k_range_total(const float2* __restrict__ ranges, int n,
                                                     float2* __restrict__ total) {
    __shared__ float2 part[4];
    float lo = FLT_MAX, hi = -FLT_MAX;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const float2 r = ranges[q];
        lo = fminf(lo, r.x);
        hi = fmaxf(hi, r.y);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off));
        hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = make_float2(lo, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lo = fminf(lo, part[w].x);
            hi = fmaxf(hi, part[w].y);
        }
        *total = make_float2(lo, hi);
    }
}

// The samples lane, lane + lanes, ... of pixel pix, summed into acc.
template <bool COUNT>
__host__ __device__ void pixel_samples(const Args& a, long long pix, int lane, int lanes, float zmin, float zmax,
                                       float mz, float acc[3], Work& w) {
    const int u = (int)(pix % a.out_w), v = (int)(pix / a.out_w);
    float p[3], n[3], rho[3];
    surface_at(a, ((float)u + 0.5f) * a.Lx / (float)a.out_w, ((float)v + 0.5f) * a.Ly / (float)a.out_h, p, n);
    albedo(a, p, rho);
    // a frame about n for the bounce directions
    float t1[3];
    if (fabsf(n[0]) > 0.5f) {
        t1[0] = -n[1]; t1[1] = n[0]; t1[2] = 0.0f;
    } else {
        t1[0] = 0.0f; t1[1] = -n[2]; t1[2] = n[1];
    }
    const float tl = sqrtf(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int k = 0; k < 3; ++k) t1[k] /= tl;
    const float t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    const float o[3] = {p[0] + kRayOffset * n[0], p[1] + kRayOffset * n[1], p[2] + kRayOffset * n[2]};
    for (int s = lane; s < a.spp; s += lanes) {
        float c[3] = {0.0f, 0.0f, 0.0f};
        direct<COUNT>(a, p, n, rho, pix, s, 0, zmin, zmax, mz, c, w);
        if (a.bounces > 1) {
            // cosine-weighted direction about n
            const float x1 = draw(a, pix, s, 16), x2 = draw(a, pix, s, 17);
            const float rr = sqrtf(x1), phi = 6.28318530717959f * x2;
            const float lx = rr * cosf(phi), ly = rr * sinf(phi), lz = sqrtf(fmaxf(1.0f - x1, 0.0f));
            float d[3];
            for (int k = 0; k < 3; ++k) d[k] = lx * t1[k] + ly * t2[k] + lz * n[k];
            const float t = trace<COUNT>(a, o, d, FLT_MAX, zmin, zmax, mz, w);
            if (t > 0.0f) {
                float p2[3], n2[3], rho2[3];
                surface_at(a, o[0] + t * d[0], o[1] + t * d[1], p2, n2);
                if (n2[0] * d[0] + n2[1] * d[1] + n2[2] * d[2] < 0.0f) {   // met from the camera side
                    albedo(a, p2, rho2);
                    float c2[3] = {0.0f, 0.0f, 0.0f};
                    direct<COUNT>(a, p2, n2, rho2, pix, s, 18, zmin, zmax, mz, c2, w);
                    for (int k = 0; k < 3; ++k) c[k] += rho[k] * c2[k];
                }
            }
        }
        for (int k = 0; k < 3; ++k) acc[k] += c[k];
    }
}

// Slack of the height-range tests: far above FP32 rounding at these sizes.
__host__ __device__ inline float range_slack(const Args& a, float zmin, float zmax) {
    return 1e-3f * fminf(a.px, a.py) + 1e-6f * fmaxf(fabsf(zmin), fabsf(zmax));
}

// One image; the COUNT instantiation also adds its work counts to counts[4].
template <bool COUNT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_render(
    Args a, unsigned long long* counts) {
    const float2 tot = *a.total;
    const float zmin = tot.x, zmax = tot.y;
    const float mz = range_slack(a, zmin, zmax);
    const int lane = threadIdx.x % kLanes;
    const long long pix = (long long)blockIdx.x * kPixels + threadIdx.x / kLanes;
    const bool live = pix < (long long)a.out_w * a.out_h;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    Work w;
    if (live) pixel_samples<COUNT>(a, pix, lane, kLanes, zmin, zmax, mz, acc, w);
    for (int off = 1; off < kLanes; off <<= 1)
        for (int k = 0; k < 3; ++k) acc[k] += __shfl_xor(acc[k], off);
    if (live && lane == 0)
        for (int k = 0; k < 3; ++k) a.out[pix * 3 + k] = acc[k] / (float)a.spp;
    if constexpr (COUNT) {
        atomicAdd(counts + 0, w.rays);
        atomicAdd(counts + 1, w.tiles);
        atomicAdd(counts + 2, w.cells);
        atomicAdd(counts + 3, w.tris);
    }
}

__global__ void k_zero_counts(unsigned long long* counts) {
    if (threadIdx.x < 4) counts[threadIdx.x] = 0ull;
}

static bool valid(const rt_params* p) {
    return p && p->W >= 2 && p->H >= 2 && p->out_w >= 1 && p->out_h >= 1 && p->spp >= 1 && p->bounces >= 1 &&
           p->bounces <= 2 && p->n_lights >= 1 && p->n_lights <= 4 && p->tex_w >= 1 && p->tex_h >= 1 &&
           p->Lx > 0 && p->Ly > 0 && (long long)p->out_w * p->out_h <= (1LL << 30) &&
           (long long)p->W * p->H <= (1LL << 30) && (long long)p->tex_w * p->tex_h <= (1LL << 28);
}

// Kernel arguments from the caller's parameters and lights (false: a
// degenerate light).  Pointers are filled in by the caller.
static bool pack_args(const rt_params* p, const rt_light* lights, Args& a) {
    a.W = p->W; a.H = p->H; a.out_w = p->out_w; a.out_h = p->out_h;
    a.spp = p->spp; a.bounces = p->bounces; a.n_lights = p->n_lights;
    a.tex_w = p->tex_w; a.tex_h = p->tex_h;
    a.TW = tiles_along(p->W);
    a.TH = tiles_along(p->H);
    a.BW = blocks_along(p->W);
    a.BH = blocks_along(p->H);
    a.Lx = (float)p->Lx; a.Ly = (float)p->Ly;
    a.px = (float)(p->Lx / p->W); a.py = (float)(p->Ly / p->H);
    a.seed = p->seed;
    for (int l = 0; l < p->n_lights; ++l) {
        const rt_light& L = lights[l];
        LightF& F = a.lights[l];
        const double nl[3] = {L.e1[1] * L.e2[2] - L.e1[2] * L.e2[1], L.e1[2] * L.e2[0] - L.e1[0] * L.e2[2],
                              L.e1[0] * L.e2[1] - L.e1[1] * L.e2[0]};
        const double area = __builtin_sqrt(nl[0] * nl[0] + nl[1] * nl[1] + nl[2] * nl[2]);
        if (!(area > 0)) return false;
        for (int k = 0; k < 3; ++k) {
            F.c[k] = (float)L.c[k]; F.e1[k] = (float)L.e1[k]; F.e2[k] = (float)L.e2[k];
            F.nl[k] = (float)(nl[k] / area); F.L[k] = (float)L.L[k];
        }
        F.area = (float)area;
    }
    return true;
}

// The three kernels of one render on `stream`; with counts (device memory)
// the counting instantiation runs instead.
static int launch(const rt_params* p, const float* height, const float* texture, float* out, void* workspace,
                  void* stream, Args& a, unsigned long long* counts) {
    char* ws = static_cast<char*>(workspace);
    float2* total = reinterpret_cast<float2*>(ws);
    float2* tiles = reinterpret_cast<float2*>(ws + 256);
    float2* blocks = tiles + (size_t)a.TW * a.TH;
    a.h = height;
    a.tex = texture;
    a.tiles = tiles;
    a.blocks = blocks;
    a.total = total;
    a.out = out;
    const hipStream_t st = (hipStream_t)stream;
    const int nt = a.TW * a.TH, nb = a.BW * a.BH;
    hipLaunchKernelGGL(k_tile_range, dim3((nt + 255) / 256), dim3(256), 0, st, height, a.W, a.H, a.TW, a.TH, tiles);
    hipLaunchKernelGGL(k_block_range, dim3((nb + 255) / 256), dim3(256), 0, st, tiles, a.TW, a.TH, a.BW, a.BH,
                       blocks);
    hipLaunchKernelGGL(k_range_total, dim3(1), dim3(256), 0, st, blocks, nb, total);
    const long long npix = (long long)p->out_w * p->out_h;
    const unsigned grid = (unsigned)((npix + kPixels - 1) / kPixels);
    if (counts) {
        hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, st, counts);
        hipLaunchKernelGGL(k_render<true>, dim3(grid), dim3(kThreads), 0, st, a, counts);
    } else {
        hipLaunchKernelGGL(k_render<false>, dim3(grid), dim3(kThreads), 0, st, a, counts);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace rt

extern "C" uint64_t rt_workspace_bytes(const rt_params* p) {
    if (!rt::valid(p)) return 0;
    const uint64_t tiles = (uint64_t)rt::tiles_along(p->W) * (uint64_t)rt::tiles_along(p->H);
    const uint64_t blocks = (uint64_t)rt::blocks_along(p->W) * (uint64_t)rt::blocks_along(p->H);
    return 256 + (tiles + blocks) * sizeof(float2);
}

extern "C" int rt_render(const rt_params* p, const float* height_device, const rt_light* lights,
                         const float* texture_device, float* out_device, void* workspace_device,
                         uint64_t workspace_bytes, void* hip_stream) {
    if (!rt::valid(p) || !height_device || !lights || !texture_device || !out_device || !workspace_device)
        return -1;
    if ((reinterpret_cast<uintptr_t>(workspace_device) & 255) != 0 || workspace_bytes < rt_workspace_bytes(p))
        return -1;
    rt::Args a;
    if (!rt::pack_args(p, lights, a)) return -1;
    return rt::launch(p, height_device, texture_device, out_device, workspace_device, hip_stream, a, nullptr);
}

extern "C" int rt_render_work(const rt_params* p, const float* height_device, const rt_light* lights,
                              const float* texture_device, float* out_device, void* workspace_device,
                              uint64_t workspace_bytes, void* hip_stream, uint64_t work[4]) {
    if (!work || !rt::valid(p) || !height_device || !lights || !texture_device || !out_device || !workspace_device)
        return -1;
    if ((reinterpret_cast<uintptr_t>(workspace_device) & 255) != 0 || workspace_bytes < rt_workspace_bytes(p))
        return -1;
    rt::Args a;
    if (!rt::pack_args(p, lights, a)) return -1;
    // the counters sit in the workspace's first 256 bytes, after the map's range
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(static_cast<char*>(workspace_device) + 64);
    int rc = rt::launch(p, height_device, texture_device, out_device, workspace_device, hip_stream, a, counts);
    if (rc != 0) return rc;
    unsigned long long host[4];
    if (hipMemcpyAsync(host, counts, sizeof(host), hipMemcpyDeviceToHost, (hipStream_t)hip_stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess)
        return -3;
    for (int k = 0; k < 4; ++k) work[k] = host[k];
    return 0;
}
