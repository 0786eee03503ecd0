/*
 * Every entry point of include/ta.h with arguments that the library must
 * reject (or accept with n = 0) before any HIP call; built against a
 * host-only build of the library with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  The fake device
 * addresses are never dereferenced.  Exit status 0 when every call returned
 * the expected status.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "ta.h"

static int failures = 0;

static void expect(const char *what, ta_status got, ta_status want) {
  if (got != want) {
    fprintf(stderr, "%s: status %d, expected %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

int main(void) {
  void *a = (void *)(uintptr_t)0x100000, *b = (void *)(uintptr_t)0x200000;
  char *bc = (char *)b;
  const ta_dtype bad = (ta_dtype)7;
  expect("sin dtype", ta_sin(a, b, 16, bad, NULL), TA_EDTYPE);
  expect("cos n<0", ta_cos(a, b, -1, TA_F32, NULL), TA_EINVAL);
  expect("tan null", ta_tan(NULL, b, 16, TA_F32, NULL), TA_EINVAL);
  expect("sin overlap", ta_sin(a, (char *)a + 4, 16, TA_F32, NULL), TA_EOVERLAP);
  expect("sin n=0", ta_sin(NULL, NULL, 0, TA_BF16, NULL), TA_OK);
  expect("sin_ex flags", ta_sin_ex(a, b, 16, TA_F32, NULL, 16u), TA_EINVAL);
  expect("cos_ex f64+fp32", ta_cos_ex(a, b, 16, TA_F64, NULL, 4u), TA_EINVAL);
  expect("tan_ex both", ta_tan_ex(a, b, 16, TA_F32, NULL, 6u), TA_EINVAL);
  expect("sincos yc", ta_sincos(a, b, NULL, NULL, 16, TA_F32, NULL), TA_EINVAL);
  expect("sincos_ex overlap",
         ta_sincos_ex(a, b, bc + 32, bc + 16, 16, TA_F32, NULL, 0u), TA_EOVERLAP);
  expect("taylor terms", ta_taylor_sin(a, b, 16, 6, TA_F32, NULL), TA_EINVAL);
  expect("taylor dtype", ta_taylor_cos(a, b, 16, 5, bad, NULL), TA_EDTYPE);
  expect("taylor n=0", ta_taylor_tan(a, b, 0, 9, TA_F32, NULL), TA_OK);
  expect("bwd gy", ta_sin_bwd(a, NULL, b, 16, TA_F32, NULL), TA_EINVAL);
  expect("bwd overlap", ta_cos_bwd(a, b, bc + 4, 16, TA_F32, NULL), TA_EOVERLAP);
  expect("bwd f64", ta_tan_bwd(a, b, bc + 64, 16, TA_F64, NULL), TA_EOVERLAP);
  expect("sincos_bwd none", ta_sincos_bwd(a, NULL, NULL, b, 16, TA_F32, NULL),
         TA_EINVAL);
  expect("fwdbwd y", ta_sin_fwdbwd(a, b, NULL, bc + 512, 16, TA_F32, NULL),
         TA_EINVAL);
  expect("fwdbwd overlap",
         ta_cos_fwdbwd(a, b, bc + 512, bc + 520, 16, TA_F32, NULL), TA_EOVERLAP);
  expect("fwdbwd dtype",
         ta_tan_fwdbwd(a, b, bc + 512, bc + 1024, 16, bad, NULL), TA_EDTYPE);
  expect("paper flags", ta_paper_sincos(a, b, NULL, NULL, 16, TA_F32, NULL, 4u),
         TA_EINVAL);
  expect("paper none", ta_paper_sincos(a, NULL, NULL, NULL, 16, TA_F32, NULL, 0u),
         TA_EINVAL);
  expect("encode nfreq", ta_sincos_encode(a, b, 16, 17, TA_F32, NULL), TA_EINVAL);
  expect("encode overlap", ta_sincos_encode(a, (char *)a + 32, 16, 4, TA_F32, NULL),
         TA_EOVERLAP);
  expect("builtin kind", ta_builtin_sincos(a, b, bc + 256, NULL, 16, 3, TA_F32, NULL),
         TA_EINVAL);
  expect("builtin outputs", ta_builtin_sincos(a, b, NULL, bc + 256, 16, 0, TA_F16, NULL),
         TA_EINVAL);
  expect("builtin f64 kind", ta_builtin_sincos(a, b, NULL, NULL, 16, 1, TA_F64, NULL),
         TA_EDTYPE);
  expect("builtin fwdbwd kind",
         ta_builtin_sin_fwdbwd(a, b, bc + 256, bc + 512, 16, 2, TA_F32, NULL), TA_EINVAL);
  expect("builtin fwdbwd overlap",
         ta_builtin_sin_fwdbwd(a, b, bc + 256, bc + 260, 16, 0, TA_BF16, NULL), TA_EOVERLAP);
  {
    const void *ins[1] = {a};
    void *outs[4] = {b, bc + 256, bc + 512, bc + 768};
    expect("copy n_in", ta_copy(ins, 0, outs, 1, 16, TA_F32, NULL), TA_EINVAL);
    expect("copy dtype", ta_copy(ins, 1, outs, 1, 16, (ta_dtype)9, NULL), TA_EDTYPE);
    void *far[3] = {b, bc + 0x10000, bc + 0x20000};
    expect("probe kind", ta_stream_probe(3, a, far, 1, 16, 0u, NULL), TA_EINVAL);
    expect("probe flags", ta_stream_probe(1, NULL, far, 3, 16, 8u, NULL), TA_EINVAL);
    expect("probe align", ta_stream_probe(2, (char *)a + 4, far, 1, 16, 0u, NULL),
           TA_EINVAL);
    expect("probe n%4", ta_stream_probe(2, a, far, 2, 18, 0u, NULL), TA_EINVAL);
    expect("probe overlap", ta_stream_probe(2, bc + 16, far, 1, 16, 0u, NULL),
           TA_EOVERLAP);
    expect("probe n=0", ta_stream_probe(0, a, far, 1, 0, 7u, NULL), TA_OK);
  }
  for (int s = 0; s < 5; ++s)
    if (strncmp(ta_status_str((ta_status)s), "TA_", 3) != 0) {
      fprintf(stderr, "status string %d\n", s);
      ++failures;
    }
  if (ta_status_str((ta_status)42) == NULL || ta_version() == NULL ||
      ta_last_hip_error() != 0)
    ++failures;
  if (failures) return 1;
  puts("abi driver ok");
  return 0;
}
