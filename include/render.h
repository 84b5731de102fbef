/*
 * render.h -- C ABI of the tactile image renderer in libimpm.so.
 *
 * The second stage of the simulator of arXiv 2405.02914 (Sec. III-B, Fig. 2(C)
 * and (D); Sec. IV-B): the elastomer surface, meshed from the depth image the
 * elastomer simulation produces (sim_surface_heightmap), carries the sensor's
 * base texture, is diffuse (the coating's roughness at its maximum), is lit by
 * the sensor's LEDs and is path traced.  Here the surface is seen from below
 * by an orthographic camera (the sensor's camera looks at the coating through
 * the gel); each pixel is the mean over spp samples of a path-traced estimate
 * with next-event estimation: the direct light of every rectangular light
 * (one uniform point on each, shadowed by the surface itself) at the primary
 * hit and, with bounces = 2, at the point a cosine-weighted bounce ray meets
 * the surface again (one interreflection; rays that leave the surface are
 * black).
 *
 * Surface: the H x W height map (row v, column u) sampled at the pixel
 * centres ((u+1/2) Lx/W, (v+1/2) Ly/H), two triangles per cell along the
 * (u, v)-(u+1, v+1) diagonal; the visible side faces -z.  Shading normal: the
 * normal of the slope field that is linear on each triangle and equals the
 * central-difference slope of the map at its samples (one-sided on the
 * border), continuous across triangle edges.  Texture: an RGB array over the
 * footprint, texel (i, j) centred at ((i+1/2) Lx/tex_w, (j+1/2) Ly/tex_h),
 * interpolated bilinearly between centres and constant beyond the outer ones.
 * Random numbers: draw k of sample s of pixel q is the top 24 bits of
 * SplitMix64(seed, (q * spp + s) * 32 + k + 1) times 2^-24 (draws 0..7: the
 * lights at the primary hit, 16..17: the bounce direction, 18..25: the lights
 * at the bounce hit).  Shadow and bounce rays start 1e-7 m off the surface.
 */
#ifndef RENDER_H
#define RENDER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double c[3];      /* rectangle centre (m) */
    double e1[3];     /* edge vectors (m); emits on the side of e1 x e2 */
    double e2[3];
    double L[3];      /* RGB radiance */
} rt_light;

typedef struct {
    int32_t W, H;               /* height map samples (columns, rows), each >= 2 */
    int32_t out_w, out_h;       /* image size, >= 1 */
    double Lx, Ly;              /* footprint of the map (m), > 0 */
    int32_t spp;                /* samples per pixel, >= 1 */
    int32_t bounces;            /* 1: direct light only; 2: plus one interreflection */
    uint64_t seed;
    int32_t n_lights;           /* 1..4 */
    int32_t tex_w, tex_h;       /* texture size, >= 1 */
    int32_t _pad;
} rt_params;

/* Bytes of device workspace rt_render needs for these parameters (the height
 * range of every 8 x 8-cell tile, every 64 x 64-cell block and the whole map),
 * or 0 when the parameters are invalid.  Depends on W and H only. */
uint64_t rt_workspace_bytes(const rt_params* p);

/* Render out_h x out_w x 3 floats (row-major, RGB) into out_device from the
 * height map height_device (H * W floats, metres), the lights (host memory,
 * n_lights records, read during the call) and the texture texture_device
 * (tex_h * tex_w * 3 floats).  workspace_device holds at least
 * rt_workspace_bytes(p) bytes, 256-byte aligned; its contents on entry do not
 * matter and it must not be used by other work until the render has finished
 * on the stream.  All device pointers are on the current HIP device and
 * caller-owned; nothing is allocated.  The work is enqueued on hip_stream
 * (NULL: the null stream) and the call returns without waiting.  Returns 0,
 * -1 (invalid arguments, or workspace_bytes too small: nothing is enqueued) or
 * -3 (a HIP launch error). */
int rt_render(const rt_params* p, const float* height_device, const rt_light* lights,
              const float* texture_device, float* out_device, void* workspace_device,
              uint64_t workspace_bytes, void* hip_stream);

/* rt_render, then a wait for it, returning the work it did: work[0] rays
 * traced (shadow and bounce rays), work[1] blocks of the height-range grid
 * (8 x 8-cell tiles and 64 x 64-cell blocks) and work[2] cells of the mesh
 * the rays visited, work[3] ray-triangle tests.  The same image is written to
 * out_device (the traversal is unchanged; only counting is added).  Used to
 * price a frame's arithmetic; blocks the calling thread until the stream has
 * finished the render.  Returns as rt_render. */
int rt_render_work(const rt_params* p, const float* height_device, const rt_light* lights,
                   const float* texture_device, float* out_device, void* workspace_device,
                   uint64_t workspace_bytes, void* hip_stream, uint64_t work[4]);

#ifdef __cplusplus
}
#endif

#endif /* RENDER_H */
