/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitize.py)
 * and run without a GPU: every rejection path of gempic_create and
 * gempic_dn_create, the NULL-argument paths of the other entry points, the
 * error strings, and a valid configuration whose device allocation fails
 * (the clean-up of a partly built handle).  Prints "host checks ok" and
 * returns 0 when every call returned what the header promises. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "gempic.h"
#include "gempic_denoise.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAILED: %s\n", what);
    failures += 1;
  }
}

/* a small valid 3-D configuration (FP64, 32 x 32 x 64 cells, 8 x 8 x 8 tiles) */
static void base(gempic_config* c) {
  memset(c, 0, sizeof *c);
  c->abi_version = GEMPIC_ABI_VERSION;
  c->dims = 3;
  c->n[0] = 32; c->n[1] = 32; c->n[2] = 64;
  c->d[0] = 0.4; c->d[1] = 0.4; c->d[2] = 0.05;
  c->length_unit = 6.283185307179586;
  c->dtau = 0.0;
  c->precision = GEMPIC_FP64;
  c->tile[0] = 8; c->tile[1] = 8; c->tile[2] = 8;
  c->n_e = 0.01;
  c->ppc[0] = 1; c->ppc[1] = 1; c->ppc[2] = 2;
  c->a0 = 0.5; c->waist = 3.0; c->fwhm = 1.5;
  c->zeta_c = NAN;
  c->filter_passes = 1;
  c->beam_zc = NAN;
  c->beam_gamma = 1.0;
  c->stream = NULL;
}

static void rejected(const gempic_config* c, int want, const char* what) {
  gempic_t* g = (gempic_t*)&failures;   /* must be reset to NULL */
  int rc = gempic_create(c, &g);
  char msg[256];
  snprintf(msg, sizeof msg, "%s: status %d, want %d", what, rc, want);
  expect(rc == want, msg);
  expect(g == NULL, what);
  const char* why = gempic_last_error(NULL);
  expect(why != NULL && why[0] != '\0', what);
}

int main(void) {
  gempic_config c;

  /* arguments */
  base(&c);
  expect(gempic_create(&c, NULL) == GEMPIC_EINVAL, "create without out");
  {
    gempic_t* g = NULL;
    expect(gempic_create(NULL, &g) == GEMPIC_EINVAL && g == NULL, "create without config");
  }

  /* configurations */
  base(&c); c.abi_version = GEMPIC_ABI_VERSION + 1; rejected(&c, GEMPIC_EABI, "abi version");
  base(&c); c.dims = 4; rejected(&c, GEMPIC_EINVAL, "dims 4");
  base(&c); c.n[0] = 48; rejected(&c, GEMPIC_EINVAL, "Nx not a power of two");
  base(&c); c.n[2] = 1; rejected(&c, GEMPIC_EINVAL, "Nzeta below 2");
  base(&c); c.tile[0] = 16; c.tile[1] = 16; rejected(&c, GEMPIC_EINVAL, "tile 16");
  base(&c); c.tile[1] = 4; rejected(&c, GEMPIC_EINVAL, "tile 8 x 4 x 8");
  base(&c); c.d[0] = 0.0; rejected(&c, GEMPIC_EINVAL, "zero grid step");
  base(&c); c.n_e = -1.0; rejected(&c, GEMPIC_EINVAL, "negative density");
  base(&c); c.dtau = 1.0; rejected(&c, GEMPIC_ECFL, "slow step beyond h / 2");
  base(&c); c.precision = 7; rejected(&c, GEMPIC_EINVAL, "unknown precision");
  base(&c); c.ppc[0] = 0; rejected(&c, GEMPIC_EINVAL, "zero particles per cell");
  base(&c); c.fwhm = 0.0; rejected(&c, GEMPIC_EINVAL, "laser without duration");
  base(&c); c.filter_passes = 3; rejected(&c, GEMPIC_EINVAL, "three filter passes");
  base(&c); c.scheme = 3; rejected(&c, GEMPIC_EINVAL, "unknown slow-step scheme");
  base(&c); c.scheme = 1; c.delta = 0.0; rejected(&c, GEMPIC_EINVAL, "zeta march without Delta");
  {
    double nodes[65];
    for (int i = 0; i <= 64; ++i) nodes[i] = 0.05 * i;
    nodes[10] = nodes[9];
    base(&c); c.scheme = 1; c.delta = 1.0; c.zeta_nodes = nodes;
    rejected(&c, GEMPIC_EINVAL, "zeta nodes not increasing");
  }
  base(&c); c.n[0] = 8192; c.n[1] = 8192; c.n[2] = 1024; c.ppc[0] = 2; c.ppc[1] = 2;
  rejected(&c, GEMPIC_EINVAL, "particle capacity beyond 2^31 - 1");

  /* a valid configuration: without a GPU the device allocation (or the
   * first HIP call) fails, and the partly built handle is released */
  base(&c);
  {
    gempic_t* g = (gempic_t*)&failures;
    int rc = gempic_create(&c, &g);
    expect(rc == GEMPIC_ENOMEM || rc == GEMPIC_EDEVICE || rc == GEMPIC_OK, "valid configuration");
    if (rc == GEMPIC_OK) gempic_destroy(g);
    else expect(g == NULL, "failed creation leaves no handle");
  }

  /* NULL handles */
  expect(gempic_step(NULL, 1, NULL) == GEMPIC_EINVAL, "step without handle");
  expect(gempic_fields_bytes(NULL, ~0u) == 0, "fields_bytes without handle");
  expect(gempic_timing(NULL, 1) == GEMPIC_EINVAL, "timing without handle");
  expect(gempic_set_deterministic(NULL, 1) == GEMPIC_EINVAL, "deterministic deposit without handle");
  {
    double axis[4];
    expect(gempic_axis_field(NULL, 2, axis, 4) == GEMPIC_EINVAL, "axis field without handle");
  }
  {
    double ms[5];
    expect(gempic_get_timing(NULL, ms, NULL) == GEMPIC_EINVAL, "get_timing without handle");
  }
  gempic_destroy(NULL);
  for (int code = -10; code <= 2; ++code) {
    const char* s = gempic_strerror(code);
    expect(s != NULL && s[0] != '\0', "strerror");
  }

  /* denoiser */
  {
    gempic_dn_t* d = (gempic_dn_t*)&failures;
    expect(gempic_dn_create(NULL, 0, NULL, &d) == GEMPIC_EINVAL, "dn_create without parameters");
    float theta[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    d = (gempic_dn_t*)&failures;
    int rc = gempic_dn_create(theta, 4, NULL, &d);
    expect(rc == GEMPIC_EINVAL, "dn_create with the wrong parameter count");
    gempic_dn_destroy(NULL);
  }

  if (failures == 0) printf("host checks ok\n");
  return failures == 0 ? 0 : 1;
}
