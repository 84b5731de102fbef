/*
 * render_oracle.c -- plain, slow FP64 CPU oracle of the image renderer of the
 * tactile sensor (arXiv 2405.02914, Sec. III-B "Rendering" and Sec. IV-B: the
 * elastomer surface, meshed from the depth image, textured with the sensor's
 * base image, lit by the sensor's LEDs, diffuse at maximum roughness, and
 * path traced).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite and the benchmark's CPU baseline leg
 * load it (through ctypes).  It shares no code with the HIP path.
 *
 * What it computes, per image pixel, the mean over `spp` samples of one
 * path-traced estimate with next-event estimation:
 *   primary hit    the surface point above the pixel centre (an orthographic
 *                  camera looks up at the coated elastomer surface from below)
 *   direct light   for each rectangular light l, one uniform point y on it:
 *                  A_l L_l (rho / pi) max(0, n.w) max(0, -n_l.w) / |y - p|^2 V(p, y)
 *   one bounce     a cosine-weighted direction about n; if it meets the
 *                  surface again at p2 (from the camera side), rho(p) times
 *                  the direct light at p2
 * Shadow and bounce rays start 1e-7 m off the surface along n.  At most 4
 * lights (their draws are numbered 0..7 at p and 18..25 at p2; the bounce
 * direction takes draws 16 and 17).
 * Surface: the height map's samples at the pixel centres of the map, joined
 * into two triangles per cell along the (u, v)-(u+1, v+1) diagonal; rays meet
 * these flat triangles.  Shading normal (our reading: the paper names none):
 * the normal (sx, sy, -1) / |.| of the slope field (sx, sy) that is linear on
 * each triangle and, at each sample, the central-difference slope of the map
 * (one-sided on its border), so that it is continuous across triangle edges
 * and the same on either side of the diagonal; the visible side faces -z.
 * Texture: the base image, an RGB array over the
 * footprint, texel (i, j) centred at ((i + 1/2) Lx / tex_w, (j + 1/2) Ly / tex_h),
 * interpolated bilinearly between texel centres and held constant beyond the
 * outer centres (our reading: the paper maps the image onto the mesh by UV
 * mapping and names no filter; a continuous lookup keeps pixels that fall on
 * texel edges well defined).
 * Random numbers: the k-th draw of sample s of pixel q is the top 24 bits of
 * SplitMix64(seed, (q * spp + s) * 32 + k + 1), scaled by 2^-24 (exact in
 * FP32 and FP64, so both implementations draw the same numbers).
 * Compiled with -ffp-contract=off; pixels are independent, so they run on
 * OpenMP threads without changing any result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double c[3];      /* rectangle centre (m) */
    double e1[3];     /* edge vectors (m); the light emits on the side of e1 x e2 */
    double e2[3];
    double L[3];      /* RGB radiance */
} rt_light;

typedef struct {
    int32_t W, H;               /* height map samples (columns, rows) */
    int32_t out_w, out_h;       /* image size */
    double Lx, Ly;              /* footprint (m) */
    int32_t spp, bounces;       /* samples per pixel; 1 = direct light only, 2 = one bounce */
    uint64_t seed;
    int32_t n_lights, tex_w, tex_h, _pad;
} rt_params;

static uint64_t sm64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + t * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double draw(const rt_params *P, int64_t pix, int s, int k) {
    uint64_t t = ((uint64_t)pix * (uint64_t)P->spp + (uint64_t)s) * 32u + (uint64_t)k + 1u;
    return (double)(sm64(P->seed, t) >> 40) * (1.0 / 16777216.0);
}

typedef struct {
    const rt_params *P;
    const double *h;   /* H x W */
    double px, py;     /* sample pitch */
} surf;

static void vertex(const surf *S, int u, int v, double *out) {
    out[0] = ((double)u + 0.5) * S->px;
    out[1] = ((double)v + 0.5) * S->py;
    out[2] = S->h[(int64_t)v * S->P->W + u];
}

/* Central-difference slope (dz/dx, dz/dy) of the map at sample (u, v),
 * one-sided on the border. */
static void vertex_slope(const surf *S, int u, int v, double *g) {
    int W = S->P->W, H = S->P->H;
    int u0 = u > 0 ? u - 1 : u, u1 = u < W - 1 ? u + 1 : u;
    int v0 = v > 0 ? v - 1 : v, v1 = v < H - 1 ? v + 1 : v;
    g[0] = (S->h[(int64_t)v * W + u1] - S->h[(int64_t)v * W + u0]) / ((double)(u1 - u0) * S->px);
    g[1] = (S->h[(int64_t)v1 * W + u] - S->h[(int64_t)v0 * W + u]) / ((double)(v1 - v0) * S->py);
}

/* Height of the mesh and the shading normal (visible side, facing -z) above
 * (x, y), clamped to the mesh. */
static void surface_at(const surf *S, double x, double y, double *p, double *n) {
    int W = S->P->W, H = S->P->H;
    double gx = x / S->px - 0.5, gy = y / S->py - 0.5;
    if (gx < 0.0) gx = 0.0;
    if (gy < 0.0) gy = 0.0;
    if (gx > (double)(W - 1)) gx = (double)(W - 1);
    if (gy > (double)(H - 1)) gy = (double)(H - 1);
    int u = (int)floor(gx), v = (int)floor(gy);
    if (u > W - 2) u = W - 2;
    if (v > H - 2) v = H - 2;
    double fx = gx - (double)u, fy = gy - (double)v;
    double a[3], b[3], c[3], d[3];
    vertex(S, u, v, a);
    vertex(S, u + 1, v, b);
    vertex(S, u, v + 1, c);
    vertex(S, u + 1, v + 1, d);
    double ga[2], gb[2], gc[2], gd[2];
    vertex_slope(S, u, v, ga);
    vertex_slope(S, u + 1, v, gb);
    vertex_slope(S, u, v + 1, gc);
    vertex_slope(S, u + 1, v + 1, gd);
    double z, sl[2];
    if (fx >= fy) {      /* triangle (a, b, d): barycentric weights 1 - fx, fx - fy, fy */
        z = a[2] + fx * (b[2] - a[2]) + fy * (d[2] - b[2]);
        for (int k = 0; k < 2; ++k) sl[k] = (1.0 - fx) * ga[k] + (fx - fy) * gb[k] + fy * gd[k];
    } else {             /* triangle (a, d, c): barycentric weights 1 - fy, fx, fy - fx */
        z = a[2] + fy * (c[2] - a[2]) + fx * (d[2] - c[2]);
        for (int k = 0; k < 2; ++k) sl[k] = (1.0 - fy) * ga[k] + fx * gd[k] + (fy - fx) * gc[k];
    }
    p[0] = ((double)u + fx + 0.5) * S->px;
    p[1] = ((double)v + fy + 0.5) * S->py;
    p[2] = z;
    /* the surface z = f(x, y) has upward normal (-fx, -fy, 1); the visible side is its negative */
    double l = sqrt(sl[0] * sl[0] + sl[1] * sl[1] + 1.0);
    n[0] = sl[0] / l; n[1] = sl[1] / l; n[2] = -1.0 / l;
}

/* Ray-triangle intersection (Moller-Trumbore); returns t or -1. */
static double tri_hit(const double *o, const double *d, const double *a, const double *b, const double *c) {
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (fabs(det) < 1e-30) return -1.0;
    double inv = 1.0 / det;
    double tv[3] = {o[0] - a[0], o[1] - a[1], o[2] - a[2]};
    double uu = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (uu < 0.0 || uu > 1.0) return -1.0;
    double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    double vv = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (vv < 0.0 || uu + vv > 1.0) return -1.0;
    return (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
}

/* Nearest hit of the ray o + t d, t in (tmin, tmax), with the surface mesh: a
 * brute-force test of every triangle (the plain definition).  Returns t or -1. */
static double trace(const surf *S, const double *o, const double *d, double tmin, double tmax) {
    int W = S->P->W, H = S->P->H;
    double best = -1.0;
    for (int v = 0; v + 1 < H; ++v)
        for (int u = 0; u + 1 < W; ++u) {
            double a[3], b[3], c[3], e[3];
            vertex(S, u, v, a);
            vertex(S, u + 1, v, b);
            vertex(S, u, v + 1, c);
            vertex(S, u + 1, v + 1, e);
            double t1 = tri_hit(o, d, a, b, e), t2 = tri_hit(o, d, a, e, c);
            if (t1 > tmin && t1 < tmax && (best < 0.0 || t1 < best)) best = t1;
            if (t2 > tmin && t2 < tmax && (best < 0.0 || t2 < best)) best = t2;
        }
    return best;
}

/* Texel coordinate of x along an axis of n texels over length L: the index
 * i0 of the left centre and the weight f of the right one (clamped). */
static void texel_axis(double x, double L, int n, int *i0, double *f) {
    double s = x / L * (double)n - 0.5;
    if (s < 0.0) s = 0.0;
    if (s > (double)(n - 1)) s = (double)(n - 1);
    int i = (int)floor(s);
    if (i > n - 2) i = n - 2;
    if (i < 0) i = 0;
    *i0 = i;
    *f = n > 1 ? s - (double)i : 0.0;
}

static void albedo(const rt_params *P, const double *tex, const double *p, double *rho) {
    int i, j;
    double fx, fy;
    texel_axis(p[0], P->Lx, P->tex_w, &i, &fx);
    texel_axis(p[1], P->Ly, P->tex_h, &j, &fy);
    int i1 = P->tex_w > 1 ? i + 1 : i, j1 = P->tex_h > 1 ? j + 1 : j;
    for (int k = 0; k < 3; ++k) {
        double t00 = tex[((int64_t)j * P->tex_w + i) * 3 + k], t10 = tex[((int64_t)j * P->tex_w + i1) * 3 + k];
        double t01 = tex[((int64_t)j1 * P->tex_w + i) * 3 + k], t11 = tex[((int64_t)j1 * P->tex_w + i1) * 3 + k];
        rho[k] = (1.0 - fy) * ((1.0 - fx) * t00 + fx * t10) + fy * ((1.0 - fx) * t01 + fx * t11);
    }
}

/* Direct light at surface point p (normal n, albedo rho) with the draws
 * k0, k0 + 1 of each light (two per light). */
static void direct(const surf *S, const rt_light *Lt, const double *p, const double *n, const double *rho,
                   int64_t pix, int s, int k0, double *out) {
    const rt_params *P = S->P;
    const double eps = 1e-7;      /* ray origin offset off the surface (m) */
    for (int l = 0; l < P->n_lights; ++l) {
        const rt_light *L = Lt + l;
        double x1 = draw(P, pix, s, k0 + 2 * l), x2 = draw(P, pix, s, k0 + 2 * l + 1);
        double y[3], w[3];
        for (int k = 0; k < 3; ++k) y[k] = L->c[k] + (x1 - 0.5) * L->e1[k] + (x2 - 0.5) * L->e2[k];
        for (int k = 0; k < 3; ++k) w[k] = y[k] - p[k];
        double d2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        double dist = sqrt(d2);
        for (int k = 0; k < 3; ++k) w[k] /= dist;
        double nl[3] = {L->e1[1] * L->e2[2] - L->e1[2] * L->e2[1], L->e1[2] * L->e2[0] - L->e1[0] * L->e2[2],
                        L->e1[0] * L->e2[1] - L->e1[1] * L->e2[0]};
        double area = sqrt(nl[0] * nl[0] + nl[1] * nl[1] + nl[2] * nl[2]);
        double cos_p = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
        double cos_l = -(nl[0] * w[0] + nl[1] * w[1] + nl[2] * w[2]) / area;
        if (cos_p <= 0.0 || cos_l <= 0.0) continue;
        double o[3] = {p[0] + eps * n[0], p[1] + eps * n[1], p[2] + eps * n[2]};
        if (trace(S, o, w, 0.0, dist) >= 0.0) continue;      /* in shadow */
        double g = area * cos_p * cos_l / d2 / M_PI;
        for (int k = 0; k < 3; ++k) out[k] += L->L[k] * rho[k] * g;
    }
}

/* One pixel's mean over its samples (out: 3 doubles). */
static void render_pixel(const surf *S, const rt_light *lights, const double *tex, int64_t pix, double *out) {
    const rt_params *P = S->P;
    int u = (int)(pix % P->out_w), v = (int)(pix / P->out_w);
    double x = ((double)u + 0.5) * P->Lx / (double)P->out_w;
    double y = ((double)v + 0.5) * P->Ly / (double)P->out_h;
    double p[3], n[3], rho[3];
    surface_at(S, x, y, p, n);
    albedo(P, tex, p, rho);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < P->spp; ++s) {
        double c[3] = {0.0, 0.0, 0.0};
        direct(S, lights, p, n, rho, pix, s, 0, c);
        if (P->bounces > 1) {
            /* cosine-weighted direction about n (a frame built from n) */
            double x1 = draw(P, pix, s, 16), x2 = draw(P, pix, s, 17);
            double r = sqrt(x1), phi = 2.0 * M_PI * x2;
            double lx = r * cos(phi), ly = r * sin(phi), lz = sqrt(1.0 - x1 > 0.0 ? 1.0 - x1 : 0.0);
            double t1[3];
            if (fabs(n[0]) > 0.5) { t1[0] = -n[1]; t1[1] = n[0]; t1[2] = 0.0; }
            else { t1[0] = 0.0; t1[1] = -n[2]; t1[2] = n[1]; }
            double tl = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
            for (int k = 0; k < 3; ++k) t1[k] /= tl;
            double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = lx * t1[k] + ly * t2[k] + lz * n[k];
            double o[3] = {p[0] + 1e-7 * n[0], p[1] + 1e-7 * n[1], p[2] + 1e-7 * n[2]};
            double t = trace(S, o, d, 0.0, 1e30);
            if (t > 0.0) {
                double q[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                double p2[3], n2[3], rho2[3];
                surface_at(S, q[0], q[1], p2, n2);
                /* only the camera side reflects back */
                if (n2[0] * d[0] + n2[1] * d[1] + n2[2] * d[2] < 0.0) {
                    albedo(P, tex, p2, rho2);
                    double c2[3] = {0.0, 0.0, 0.0};
                    direct(S, lights, p2, n2, rho2, pix, s, 18, c2);
                    for (int k = 0; k < 3; ++k) c[k] += rho[k] * c2[k];
                }
            }
        }
        for (int k = 0; k < 3; ++k) acc[k] += c[k];
    }
    for (int k = 0; k < 3; ++k) out[k] = acc[k] / (double)P->spp;
}

/* Render out (out_h x out_w x 3) from the height map h (H x W, metres). */
void rt_render_oracle(const rt_params *P, const double *h, const rt_light *lights, const double *tex, double *out) {
    surf S = {P, h, P->Lx / (double)P->W, P->Ly / (double)P->H};
    int64_t npix = (int64_t)P->out_w * P->out_h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t pix = 0; pix < npix; ++pix) render_pixel(&S, lights, tex, pix, out + 3 * pix);
}

/* The pixels pix[0..n) of the same image only (out: n x 3), for images too
 * large to render whole by brute force. */
void rt_render_oracle_pixels(const rt_params *P, const double *h, const rt_light *lights, const double *tex,
                             const int64_t *pix, int64_t n, double *out) {
    surf S = {P, h, P->Lx / (double)P->W, P->Ly / (double)P->H};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n; ++q) render_pixel(&S, lights, tex, pix[q], out + 3 * q);
}
