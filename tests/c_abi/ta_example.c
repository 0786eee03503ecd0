/*
 * ta_example.c -- uses libta.so from plain C (no C++, no torch): device
 * buffers from hipMalloc, one ta_sincos (sin, cos and tan of n floats) and
 * one ta_sin_fwdbwd call on a stream the program creates, and the
 * validation paths of the ABI.
 *
 * usage: ta_example IN OUT
 *   IN : n little-endian FP32 values; OUT receives 5n FP32 values:
 *        sin, cos, tan (ta_sincos), sin and g*d sin/dx with g = 1
 *        (ta_sin_fwdbwd).
 * Exit status 0 on success; messages on stderr otherwise.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "ta.h"

#define HIP_OK(call)                                                      \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));   \
      return 1;                                                           \
    }                                                                     \
  } while (0)

#define TA_OK_OR_FAIL(call)                                               \
  do {                                                                    \
    ta_status s_ = (call);                                                \
    if (s_ != TA_OK) {                                                    \
      fprintf(stderr, "%s: %s\n", #call, ta_status_str(s_));              \
      return 1;                                                           \
    }                                                                     \
  } while (0)

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) {
    perror(argv[1]);
    return 1;
  }
  fseek(f, 0, SEEK_END);
  long bytes = ftell(f);
  fseek(f, 0, SEEK_SET);
  size_t n = (size_t)bytes / sizeof(float);
  float *h = (float *)malloc(n * sizeof(float) * 5);
  if (!h || fread(h, sizeof(float), n, f) != n) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 1;
  }
  fclose(f);

  /* validation happens before any HIP call */
  if (ta_sin(NULL, NULL, -1, TA_F32, NULL) != TA_EINVAL ||
      ta_sin(h, h, 4, (ta_dtype)9, NULL) != TA_EDTYPE ||
      ta_taylor_sin(h, h + 4, 4, 6, TA_F32, NULL) != TA_EINVAL ||
      ta_sin(NULL, NULL, 0, TA_F32, NULL) != TA_OK) {
    fprintf(stderr, "validation results differ from the header\n");
    return 1;
  }

  void *x, *ys, *yc, *yt, *g, *gx;
  HIP_OK(hipMalloc(&x, n * sizeof(float)));
  HIP_OK(hipMalloc(&ys, n * sizeof(float)));
  HIP_OK(hipMalloc(&yc, n * sizeof(float)));
  HIP_OK(hipMalloc(&yt, n * sizeof(float)));
  HIP_OK(hipMalloc(&g, n * sizeof(float)));
  HIP_OK(hipMalloc(&gx, n * sizeof(float)));
  hipStream_t stream;
  HIP_OK(hipStreamCreate(&stream));
  HIP_OK(hipMemcpy(x, h, n * sizeof(float), hipMemcpyHostToDevice));
  float *ones = h + n;
  for (size_t i = 0; i < n; ++i) ones[i] = 1.0f;
  HIP_OK(hipMemcpy(g, ones, n * sizeof(float), hipMemcpyHostToDevice));

  TA_OK_OR_FAIL(ta_sincos(x, ys, yc, yt, (int64_t)n, TA_F32, stream));
  HIP_OK(hipStreamSynchronize(stream));
  HIP_OK(hipMemcpy(h + n, ys, n * sizeof(float), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(h + 2 * n, yc, n * sizeof(float), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(h + 3 * n, yt, n * sizeof(float), hipMemcpyDeviceToHost));
  /* the fused forward+backward reuses ys (value) and gx (gradient) */
  TA_OK_OR_FAIL(ta_sin_fwdbwd(x, g, ys, gx, (int64_t)n, TA_F32, stream));
  HIP_OK(hipStreamSynchronize(stream));
  float *outv = (float *)malloc(n * sizeof(float) * 2);
  if (!outv) return 1;
  HIP_OK(hipMemcpy(outv, ys, n * sizeof(float), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(outv + n, gx, n * sizeof(float), hipMemcpyDeviceToHost));

  FILE *o = fopen(argv[2], "wb");
  if (!o) {
    perror(argv[2]);
    return 1;
  }
  if (fwrite(h + n, sizeof(float), 3 * n, o) != 3 * n ||
      fwrite(outv, sizeof(float), 2 * n, o) != 2 * n) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    return 1;
  }
  fclose(o);
  HIP_OK(hipStreamDestroy(stream));
  hipFree(x); hipFree(ys); hipFree(yc); hipFree(yt); hipFree(g); hipFree(gx);
  free(h);
  free(outv);
  printf("%s: %zu elements\n", ta_version(), n);
  return 0;
}
