/* A plain C99 client of the library's C ABI: no Python, no torch.  It reads a
 * scene and a camera from a binary file, renders one frame with msgs_render
 * (the scene copied from host arrays), runs msgs_render_backward with dL/dRGB
 * = 1, and writes the image, the statistics and the opacity gradient to a
 * binary file.  The GPU test compares its output with the Python binding's.
 *
 * Input (little-endian): int64 n, int32 sh_degree, int32 n_levels,
 *   int32 downscale, int32 selective, msgs_camera, then the planar float
 *   arrays means[3n], scales[3n], quats[4n], opacity[n], sh[(D+1)^2*3*n],
 *   uint8 level[n], float s_max[n], float s_min[n].
 * Output: int32 W_d, int32 H_d, float rgb[H_d*W_d*3], int64 n_selected,
 *   int64 n_instances, int64 n_blends, float d_opacity[n].
 * Exit status 0 on success; otherwise the failing call and msgs_last_error()
 * go to stderr. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "msgs.h"

static int fail(const char* what, int rc) {
  fprintf(stderr, "%s failed: %d (%s)\n", what, rc, msgs_last_error());
  return 1;
}

static void* read_n(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (p && bytes && fread(p, 1, bytes, f) != bytes) {
    free(p);
    return NULL;
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return fail("fopen input", -1);
  int64_t n;
  int32_t hdr[4];
  msgs_camera cam;
  if (fread(&n, sizeof n, 1, in) != 1 || fread(hdr, sizeof hdr, 1, in) != 1 ||
      fread(&cam, sizeof cam, 1, in) != 1)
    return fail("read header", -1);
  const int D = hdr[0], L = hdr[1], ds = hdr[2], selective = hdr[3];
  const size_t K3 = (size_t)(D + 1) * (D + 1) * 3, un = (size_t)n;
  float* means = (float*)read_n(in, 3 * un * sizeof(float));
  float* scales = (float*)read_n(in, 3 * un * sizeof(float));
  float* quats = (float*)read_n(in, 4 * un * sizeof(float));
  float* opacity = (float*)read_n(in, un * sizeof(float));
  float* sh = (float*)read_n(in, K3 * un * sizeof(float));
  uint8_t* level = (uint8_t*)read_n(in, un);
  float* s_max = (float*)read_n(in, un * sizeof(float));
  float* s_min = (float*)read_n(in, un * sizeof(float));
  fclose(in);
  if (!means || !scales || !quats || !opacity || !sh || !level || !s_max || !s_min)
    return fail("read arrays", -1);

  msgs_context* ctx = NULL;
  int rc = msgs_context_create(0, 0, &ctx);
  if (rc != MSGS_OK) return fail("msgs_context_create", rc);
  msgs_scene_desc d = {n, D, L, means, scales, quats, opacity, sh, level, s_max, s_min, 0};
  msgs_scene* scene = NULL;
  rc = msgs_scene_create(ctx, &d, 1, &scene);
  if (rc != MSGS_OK) return fail("msgs_scene_create", rc);

  msgs_render_opts o;
  msgs_default_opts(&o);
  o.downscale = ds;
  o.selective = selective;
  const int W = cam.width / ds, H = cam.height / ds;
  const size_t npix = (size_t)W * (size_t)H;
  float *rgb_d = NULL, *dl_d = NULL, *g_d = NULL;
  if (hipMalloc((void**)&rgb_d, npix * 3 * sizeof(float) + 4) != hipSuccess ||
      hipMalloc((void**)&dl_d, npix * 3 * sizeof(float) + 4) != hipSuccess)
    return fail("hipMalloc image", -1);
  msgs_frame* fr = NULL;
  rc = msgs_render(ctx, scene, &cam, &o, rgb_d, &fr, NULL);
  if (rc != MSGS_OK) return fail("msgs_render", rc);
  msgs_stats st;
  rc = msgs_frame_stats(fr, &st);
  if (rc != MSGS_OK) return fail("msgs_frame_stats", rc);

  /* gradient planes: means 3n, scales 3n, quats 4n, opacity n, sh K3 n */
  const size_t gsz = (3 + 3 + 4 + 1 + K3) * un;
  if (hipMalloc((void**)&g_d, gsz * sizeof(float) + 4) != hipSuccess)
    return fail("hipMalloc gradients", -1);
  float* ones = (float*)malloc(npix * 3 * sizeof(float) + 4);
  if (!ones) return fail("malloc", -1);
  for (size_t i = 0; i < npix * 3; ++i) ones[i] = 1.0f;
  if (hipMemcpy(dl_d, ones, npix * 3 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return fail("hipMemcpy dL", -1);
  msgs_grads g;
  g.means = g_d;
  g.scales = g_d + 3 * un;
  g.quats = g_d + 6 * un;
  g.opacity = g_d + 10 * un;
  g.sh = g_d + 11 * un;
  g.accumulate = 0;
  rc = msgs_render_backward(ctx, fr, dl_d, &g, NULL);
  if (rc != MSGS_OK) return fail("msgs_render_backward", rc);

  float* rgb = (float*)malloc(npix * 3 * sizeof(float) + 4);
  float* dop = (float*)malloc(un * sizeof(float) + 4);
  if (!rgb || !dop) return fail("malloc", -1);
  if (hipMemcpy(rgb, rgb_d, npix * 3 * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(dop, g.opacity, un * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return fail("hipMemcpy results", -1);

  FILE* out = fopen(argv[2], "wb");
  if (!out) return fail("fopen output", -1);
  const int32_t wh[2] = {W, H};
  const int64_t cnt[3] = {st.n_selected, st.n_instances, st.n_blends};
  fwrite(wh, sizeof wh, 1, out);
  fwrite(rgb, sizeof(float), npix * 3, out);
  fwrite(cnt, sizeof cnt, 1, out);
  fwrite(dop, sizeof(float), un, out);
  fclose(out);

  msgs_frame_release(fr);
  msgs_scene_destroy(scene);
  (void)hipFree(rgb_d);
  (void)hipFree(dl_d);
  (void)hipFree(g_d);
  msgs_context_destroy(ctx);
  free(means); free(scales); free(quats); free(opacity); free(sh); free(level);
  free(s_max); free(s_min); free(ones); free(rgb); free(dop);
  return 0;
}
