/* A plain C99 caller of the library, built and run by test_abi.py: it includes
 * include/ffpat.h, links libffpat.so and makes only the calls that need no device
 * (version, workspace size, argument validation).  Prints one line per check;
 * exit status 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "ffpat.h"

static int failures = 0;

static void check(int ok, const char *what)
{
  printf("%s %s\n", ok ? "ok" : "FAIL", what);
  if (!ok) ++failures;
}

int main(void)
{
  double angles[16];
  ffpat_geom g;
  size_t bytes = 0;
  int32_t v = 0;
  ffpat_plan *plan = NULL;
  int i;

  for (i = 0; i < 16; ++i) angles[i] = 3.141592653589793 * i / 16.0;
  memset(&g, 0, sizeof g);
  g.nx = 64;
  g.ny = 64;
  g.nz = 64;
  g.ndim = 3;
  g.dx = 0.05;
  g.T = 0.5;
  g.cfl = 0.3;
  g.n_angles = 16;
  g.angles = angles;
  g.dtype = FFPAT_F32;

  check(strstr(ffpat_version(), "gfx950") != NULL, "version names gfx950");
  check(ffpat_workspace_bytes(&g, &bytes) == FFPAT_OK && bytes >= (size_t)7 * 64 * 64 * 64 * 4,
        "workspace of a 64^3 FP32 plan holds seven volumes");

  g.cfl = 0.9;
  check(ffpat_workspace_bytes(&g, &bytes) == FFPAT_ECFL && ffpat_last_error()[0] != '\0',
        "cfl 0.9 rejected with a message");
  g.cfl = 0.3;
  g.dtype = 7;
  check(ffpat_workspace_bytes(&g, &bytes) == FFPAT_EDTYPE, "unknown dtype rejected");
  g.dtype = FFPAT_F64;
  check(ffpat_workspace_bytes(&g, NULL) == FFPAT_EINVAL, "null output pointer rejected");

  check(ffpat_plan_create(&g, NULL, NULL, &plan) == FFPAT_EINVAL && plan == NULL,
        "plan without a sound-speed field rejected");
  check(ffpat_plan_steps_per_pass(NULL, &v) == FFPAT_EINVAL, "null plan rejected");
  check(ffpat_forward(NULL, NULL, NULL, NULL) == FFPAT_EINVAL, "forward on a null plan rejected");
  check(ffpat_plan_destroy(NULL) == FFPAT_OK, "destroying a null plan is a no-op");
  return failures == 0 ? 0 : 1;
}
