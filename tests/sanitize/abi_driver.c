/* Sanitizer driver for the host code of libswe (C ABI): built, like the
 * library, with the host half under -fsanitize=address,undefined by
 * tests/test_sanitizers.py.  It exercises what runs without a GPU: defaults,
 * validation of bad configurations, NULL handles and the error messages.
 * Every call must return its documented error code. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "swe.h"

static int fails = 0;
#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "abi driver: failed: %s (line %d)\n", #cond, __LINE__); \
            fails++;                                                     \
        }                                                                \
    } while (0)

int main(void) {
    EXPECT(swe_abi_version() == SWE_ABI_VERSION);
    swe_config c;
    swe_config_init(&c);
    swe_config_init(NULL);
    EXPECT(c.g == 9.81 && c.h_film == 0.0 && c.dtype == SWE_F64);
    static double fake[16];
    c.nx = 16; c.ny = 12; c.pitch = 16; c.dx = c.dy = 1.0;
    c.z = c.n = fake; c.eta = c.qx = c.qy = fake;
    double ht[2] = {0.0, 1.0}, hq[2] = {0.0, 2.0};
    c.hydro_len = 2; c.hydro_t = ht; c.hydro_q = hq;
    swe_handle* h = (swe_handle*)&c;
    /* invalid configurations: SWE_EINVAL before any device call */
    swe_config bad;
    bad = c; bad.nx = 4;           EXPECT(swe_create(&bad, &h) == SWE_EINVAL && h == NULL);
    bad = c; bad.pitch = 8;        EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    bad = c; bad.cfl = 1.5;        EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    bad = c; bad.h_film = -1.0;  EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    bad = c; bad.h_film = NAN;   EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    bad = c; bad.hydro_t = NULL;   EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    ht[1] = 0.0;                   EXPECT(swe_create(&c, &h) == SWE_EINVAL);
    ht[1] = 1.0;
    bad = c; bad.dry_skip = 1; bad.path = SWE_PATH_UNFUSED;
    EXPECT(swe_create(&bad, &h) == SWE_EINVAL);
    EXPECT(swe_create(NULL, &h) == SWE_EINVAL);
    EXPECT(swe_create(&c, NULL) == SWE_EINVAL);
    EXPECT(strlen(swe_last_error(NULL)) > 0);
    /* the allocation-free run validates before touching a device */
    bad = c; bad.nx = 2000; bad.ny = 1000; bad.pitch = 2000;
    EXPECT(swe_run_noalloc(&bad, 1, INFINITY, NULL) == SWE_EINVAL);
    bad = c; bad.path = SWE_PATH_UNFUSED;
    EXPECT(swe_run_noalloc(&bad, 1, INFINITY, NULL) == SWE_EINVAL);
    EXPECT(swe_run_noalloc(&c, -1, INFINITY, NULL) == SWE_EINVAL);
    /* NULL handles */
    swe_stats st;
    double dt = 0.0, J = 0.0;
    swe_gauges g;
    memset(&g, 0, sizeof g);
    EXPECT(swe_step(NULL, &dt) == SWE_EINVAL);
    EXPECT(swe_run(NULL, 1, INFINITY, &st) == SWE_EINVAL);
    EXPECT(swe_run_dt(NULL, 1, &dt, &st) == SWE_EINVAL);
    EXPECT(swe_get_stats(NULL, &st) == SWE_EINVAL);
    EXPECT(swe_grad(NULL, 1, &g, 0, &J, fake, fake) == SWE_EINVAL);
    EXPECT(swe_loss(NULL, 1, &g, &J) == SWE_EINVAL);
    EXPECT(swe_save(NULL, NULL) == SWE_EINVAL);
    EXPECT(swe_load(NULL, NULL) == SWE_EINVAL);
    swe_destroy(NULL);
    EXPECT(strlen(swe_last_error(NULL)) > 0);
    printf(fails ? "abi driver: %d failures\n" : "abi driver: ok\n", fails);
    return fails != 0;
}
