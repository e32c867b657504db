/* sanitize_check.c -- drives the host-side entry points of the library that
 * need no device, for a build of the host code with AddressSanitizer and
 * UndefinedBehaviorSanitizer (build.py, build_sanitized): the tuning cache
 * file, the RKB small-component arithmetic (two-spinor and quaternion forms,
 * which must describe the same spinors), the ABI version, and the argument
 * checks that every entry point makes before any device call.  Exit status 0
 * when every check holds; the sanitizers report memory and undefined-behaviour
 * errors on stderr. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "qdcb.h"

static int fails = 0;
#define CHECK(cond)                                              \
    do {                                                         \
        if (!(cond)) {                                           \
            printf("FAIL line %d: %s\n", __LINE__, #cond);      \
            ++fails;                                             \
        }                                                        \
    } while (0)

int main(int argc, char **argv)
{
    const char *path = argc > 1 ? argv[1] : "sanitize_tune.jsonl";
    remove(path);
    CHECK(qdcb_abi_version() == QDCB_ABI_VERSION);

    /* tuning cache: missing file, store, last line wins, other keys */
    qdcb_tune t = {1, 0, 128, 0}, r;
    int32_t found = 1;
    CHECK(qdcb_tune_cache_lookup(path, "absent", &r, &found) == QDCB_OK && found == 0);
    CHECK(qdcb_tune_cache_store(path, "k1", &t) == QDCB_OK);
    t.sq_tile = 64;
    CHECK(qdcb_tune_cache_store(path, "k1", &t) == QDCB_OK);
    t.eri_sched = 0;
    CHECK(qdcb_tune_cache_store(path, "k2 with spaces", &t) == QDCB_OK);
    CHECK(qdcb_tune_cache_lookup(path, "k1", &r, &found) == QDCB_OK && found == 1);
    CHECK(r.eri_sched == 1 && r.sq_tile == 64);
    CHECK(qdcb_tune_cache_lookup(path, "k2 with spaces", &r, &found) == QDCB_OK && found);
    CHECK(r.eri_sched == 0);
    CHECK(qdcb_tune_cache_lookup(path, "k", &r, &found) == QDCB_OK && found == 0);
    remove(path);

    /* RKB small components: the quaternion form's Kramers-pair spinors are the
     * two-spinor form's small components */
    enum { N = 4, n = 3 };
    double CS[4 * N * n], norms[3 * N], Cq[4 * 3 * N * n];
    double PS[4 * N * 2 * n], Pq[4 * 3 * N * 2 * n], Pref[4 * 3 * N * 2 * n];
    unsigned s = 12345u;
    for (int i = 0; i < 4 * N * n; ++i) {
        s = s * 1103515245u + 12345u;
        CS[i] = ((s >> 8) & 0xffff) / 65536.0 - 0.5;
    }
    for (int i = 0; i < 3 * N; ++i) norms[i] = 0.5 + 0.1 * i;
    CHECK(qdcb_rkb_small_quat(N, n, CS, norms, 2.5, Cq) == QDCB_OK);
    /* spinor planes of quaternion coefficients C[4][M][n] -> P[4][M][2n]:
     * spinor 2p = (C0 + i C1, -C2 + i C3), spinor 2p + 1 = (C2 + i C3, C0 - i C1) */
#define SPINORS(C, P, M)                                                        \
    for (int mu = 0; mu < (M); ++mu)                                            \
        for (int p = 0; p < n; ++p) {                                           \
            double c0 = C[(0 * (M) + mu) * n + p], c1 = C[(1 * (M) + mu) * n + p]; \
            double c2 = C[(2 * (M) + mu) * n + p], c3 = C[(3 * (M) + mu) * n + p]; \
            double *q = P + (size_t)mu * 2 * n + 2 * p;                         \
            size_t pl = (size_t)(M) * 2 * n;                                    \
            q[0] = c0; q[pl] = c1; q[2 * pl] = -c2; q[3 * pl] = c3;             \
            q[1] = c2; q[pl + 1] = c3; q[2 * pl + 1] = c0; q[3 * pl + 1] = -c1; \
        }
    SPINORS(CS, PS, N)
    SPINORS(Cq, Pq, 3 * N)
    CHECK(qdcb_rkb_small_planes(N, 2 * n, PS, norms, 2.5, Pref) == QDCB_OK);
    double d = 0.0;
    for (int i = 0; i < 4 * 3 * N * 2 * n; ++i)
        if (fabs(Pq[i] - Pref[i]) > d) d = fabs(Pq[i] - Pref[i]);
    CHECK(d <= 1e-15);
    CHECK(qdcb_rkb_small_quat(N, n, CS, norms, 0.0, Cq) == QDCB_E_INVALID);
    CHECK(qdcb_rkb_small_planes(0, n, PS, norms, 1.0, Pref) == QDCB_E_INVALID);

    /* argument checks before any device call */
    qdcb_ctx *ctx = NULL;
    CHECK(qdcb_ctx_create(0, 0, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_basis_create(NULL, 1, NULL, NULL, NULL, NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_basis_schwarz(NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_plan_footprint(NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_plan_create(ctx, NULL, NULL, NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_transform(NULL, NULL, NULL, NULL, 0, NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_eri_quartets(NULL, NULL, 1, NULL, NULL) == QDCB_E_INVALID);
    CHECK(qdcb_plan_set_tune(NULL, &t) == QDCB_E_INVALID);
    CHECK(qdcb_tune_cache_lookup(NULL, "k", &r, &found) == QDCB_E_INVALID);
    CHECK(strlen(qdcb_last_error()) > 0);

    printf("%s\n", fails ? "FAILED" : "all checks passed");
    return fails ? 1 : 0;
}
