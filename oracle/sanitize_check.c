/* sanitize_check.c -- drives every entry point of the oracle on a tiny
 * seeded system, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure; see oracle/__init__.py,
 * build_sanitized).  Exit status 0 when the routes agree; the sanitizers
 * report any out-of-bounds access, use after free, leak or undefined
 * operation on stderr and make the run fail.
 *
 * System: 3 atoms, an L basis of s, p and d functions (contraction depths 1
 * to 3) and an s-only L' basis with an s-only S basis for the Breit routes;
 * n = 2 quaternion MOs (4 spinors).  Checks: the definition route equals the
 * direct route at tau = 0 (LL with s/p/d; DC, DCG and DCB with s), the
 * column-subset first-half rows equal the full rows, the general-spinor
 * definition and direct routes agree on random spinors, and the direct route
 * with the all-pairs density bound given equals the direct route. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static unsigned long long g_state = 88172645463325252ULL;
static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

static double maxabs_diff(const double *a, const double *b, size_t n, double *amax)
{
    double d = 0.0, m = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (fabs(a[i] - b[i]) > d) d = fabs(a[i] - b[i]);
        if (fabs(b[i]) > m) m = fabs(b[i]);
    }
    if (amax) *amax = m;
    return d;
}

typedef struct {
    int nfunc, nprim_tot;
    double *centers, *exps, *coefs;
    int32_t *nprim, *cart;
} owned_basis;

static owned_basis make_basis(const double atoms[3][3], int nfunc, const int32_t *codes,
                              double scale)
{
    owned_basis b;
    b.nfunc = nfunc;
    b.centers = malloc(sizeof(double) * 3 * nfunc);
    b.nprim = malloc(sizeof(int32_t) * nfunc);
    b.cart = codes ? malloc(sizeof(int32_t) * nfunc) : NULL;
    b.nprim_tot = 0;
    for (int f = 0; f < nfunc; ++f) {
        b.nprim[f] = 1 + f % 3;
        b.nprim_tot += b.nprim[f];
        for (int k = 0; k < 3; ++k) b.centers[3 * f + k] = atoms[f % 3][k];
        if (codes) b.cart[f] = codes[f];
    }
    b.exps = malloc(sizeof(double) * b.nprim_tot);
    b.coefs = malloc(sizeof(double) * b.nprim_tot);
    for (int i = 0; i < b.nprim_tot; ++i) {
        b.exps[i] = scale * pow(10.0, -0.7 + 1.4 * urand());
        b.coefs[i] = 0.1 + 0.9 * urand();
    }
    return b;
}

static orc_basis view(const owned_basis *b)
{
    orc_basis v = {b->nfunc, b->centers, b->nprim, b->exps, b->coefs, b->cart};
    return v;
}

static void free_basis(owned_basis *b)
{
    free(b->centers);
    free(b->nprim);
    free(b->exps);
    free(b->coefs);
    free(b->cart);
}

static int check(const char *what, double err, double scale, double tol)
{
    int ok = err <= tol * scale;
    printf("%-40s max|d| %.3e  scale %.3e  %s\n", what, err, scale, ok ? "ok" : "FAIL");
    return ok ? 0 : 1;
}

/* max|a - b| against tol * max|b| */
static int compare(const char *what, const double *a, const double *b, size_t n, double tol)
{
    double amax = 0.0;
    double err = maxabs_diff(a, b, n, &amax);
    if (!(amax > 0.0)) {
        printf("%-40s reference is zero  FAIL\n", what);
        return 1;
    }
    return check(what, err, amax, tol);
}

int main(void)
{
    const double atoms[3][3] = {{0.0, 0.0, 0.0}, {1.4, 0.3, -0.2}, {-0.5, 1.1, 0.9}};
    const int32_t codes[9] = {0, 1, 2, 3, 0, 4, 7, 9, 0};
    owned_basis Lspd = make_basis(atoms, 9, codes, 1.0);
    owned_basis L = make_basis(atoms, 5, NULL, 1.0);
    owned_basis S = make_basis(atoms, 6, NULL, 4.0);
    orc_basis vspd = view(&Lspd), vL = view(&L), vS = view(&S);
    const int n = 2, m = 2 * n;
    int fails = 0;

    /* Boys, primitive and contracted integrals, Schwarz factors, bounds */
    double f = orc_boys0(0.0) + orc_boys0(1e-10) + orc_boys0(50.0) + orc_boys(3, 2.5);
    double A[3] = {0, 0, 0}, B[3] = {0.5, 0, 0};
    f += orc_prim_eri_cart(1.0, A, 4, 0.7, B, 2, 0.3, A, 0, 1.2, B, 8);
    double t9[9];
    orc_eri3(&vL, 0, &vS, 1, &vL, 2, &vS, 3, t9);
    f += orc_eri(&vspd, 1, 5, &vspd, 7, 8) + t9[4];
    double *T = malloc(sizeof(double) * 5 * 5 * 6 * 6);
    orc_eri_tensor(&vL, &vL, &vS, &vS, T);
    double *Q = malloc(sizeof(double) * 9 * 9);
    orc_schwarz(&vspd, &vspd, Q);
    double *nc = malloc(sizeof(double) * Lspd.nprim_tot);
    orc_norm_coefs(&vspd, nc);
    if (!isfinite(f) || !isfinite(T[17]) || !isfinite(Q[10]) || !isfinite(nc[3])) ++fails;

    /* coefficients: seeded, planar [4][N][n] */
    double *CP = malloc(sizeof(double) * 4 * 9 * n), *CL = malloc(sizeof(double) * 4 * 5 * n);
    double *CS = malloc(sizeof(double) * 4 * 6 * n);
    for (int i = 0; i < 4 * 9 * n; ++i) CP[i] = urand() - 0.5;
    for (int i = 0; i < 4 * 5 * n; ++i) CL[i] = urand() - 0.5;
    for (int i = 0; i < 4 * 6 * n; ++i) CS[i] = urand() - 0.5;
    double *D1 = malloc(sizeof(double) * 6 * 6), *D2 = malloc(sizeof(double) * 5 * 6);
    orc_dmax_coulomb(6, CS, n, D1);
    orc_dmax_gaunt(5, CL, 6, CS, n, D2);

    const size_t gsz = (size_t)n * n * n * n * 16;
    double *G1 = malloc(sizeof(double) * gsz), *G2 = malloc(sizeof(double) * gsz);
    double *sp = malloc(sizeof(double) * 2 * (size_t)m * m * m * m);
    double im = 0.0;
    orc_stats st;

    /* LL with s, p and d functions: definition = direct route at tau = 0 */
    if (orc_transform_def(&vspd, NULL, CP, NULL, n, 0, G1, sp, &im)) return 2;
    if (orc_transform_direct(&vspd, NULL, CP, NULL, n, 0, 0.0, NULL, 0, 1, G2, &st)) return 2;
    fails += compare("LL s/p/d: def vs direct", G1, G2, gsz, 1e-12);

    /* DC, DCG, DCB over s functions */
    for (int ham = 1; ham <= 5; ++ham) {
        char what[64];
        if (orc_transform_def(&vL, &vS, CL, CS, n, ham, G1, NULL, &im)) return 2;
        if (orc_transform_direct(&vL, &vS, CL, CS, n, ham, 0.0, NULL, 0, 1, G2, &st)) return 2;
        snprintf(what, sizeof what, "ham %d: def vs direct", ham);
        fails += compare(what, G1, G2, gsz, 1e-12);
        /* and screened */
        if (orc_transform_direct(&vL, &vS, CL, CS, n, ham, 1e-3, NULL, 0, 1, G1, &st)) return 2;
    }

    /* first-half rows: full and column subset (DCG: Coulomb and L-S rows) */
    int64_t np = orc_num_bra_pairs(&vL, &vS, 2);
    int64_t rows[4] = {0, 7, np / 2, np - 1};
    const int64_t npair = n * (n + 1) / 2;
    double *V = malloc(sizeof(double) * 4 * 3 * 4 * npair);
    if (orc_first_half_rows(&vL, &vS, CL, CS, n, 2, 1e-6, rows, 4, V)) return 2;
    int64_t cols[2] = {2, 0};
    double *Vc = malloc(sizeof(double) * 4 * 3 * 4 * 2);
    if (orc_first_half_rows_cols(&vL, &vS, CL, CS, n, 2, 1e-6, rows, 4, cols, 2, NULL, Vc))
        return 2;
    double d = 0.0;
    for (int r = 0; r < 4; ++r)
        for (int K = 0; K < 3; ++K)
            for (int j = 0; j < 2; ++j)
                for (int y = 0; y < 4; ++y) {
                    double a = V[(size_t)r * 12 * npair + K * 4 * npair + 4 * cols[j] + y];
                    double b = Vc[(size_t)r * 24 + K * 8 + 4 * j + y];
                    if (fabs(a - b) > d) d = fabs(a - b);
                }
    fails += check("first-half rows: column subset", d, 1.0, 0.0);

    /* general two-spinor routes on random spinors (DCG) */
    double *PL = malloc(sizeof(double) * 4 * 5 * m), *PS = malloc(sizeof(double) * 4 * 6 * m);
    for (int i = 0; i < 4 * 5 * m; ++i) PL[i] = urand() - 0.5;
    for (int i = 0; i < 4 * 6 * m; ++i) PS[i] = urand() - 0.5;
    double *s1 = malloc(sizeof(double) * 2 * (size_t)m * m * m * m);
    double *s2 = malloc(sizeof(double) * 2 * (size_t)m * m * m * m);
    if (orc_transform_spinor_def(&vL, &vS, PL, PS, m, 2, s1)) return 2;
    if (orc_transform_spinor_direct(&vL, &vS, PL, PS, m, 2, 0.0, s2, &st)) return 2;
    fails += compare("spinor DCG: def vs direct", s1, s2, 2 * (size_t)m * m * m * m, 1e-12);

    /* MO-driven bound route: the all-pairs bound reproduces the direct route */
    double *dm = malloc(sizeof(double) * np);
    int64_t k = 0;
    double *DL = malloc(sizeof(double) * 5 * 5);
    orc_dmax_coulomb(5, CL, n, DL);
    for (int nu = 0; nu < 5; ++nu)
        for (int mu = 0; mu <= nu; ++mu) dm[k++] = DL[mu * 5 + nu];
    for (int nu = 0; nu < 6; ++nu)
        for (int mu = 0; mu <= nu; ++mu) dm[k++] = D1[mu * 6 + nu];
    for (int i = 0; i < 5 * 6; ++i) dm[k++] = D2[i];
    if (orc_transform_direct_dmax(&vL, &vS, CL, CS, n, 2, 1e-4, dm, G1, &st)) return 2;
    if (orc_transform_direct(&vL, &vS, CL, CS, n, 2, 1e-4, NULL, 0, 1, G2, &st)) return 2;
    fails += compare("given all-pairs bound vs direct", G1, G2, gsz, 0.0);

    /* invalid arguments are refused */
    if (orc_transform_direct(&vL, NULL, CL, NULL, n, 1, 0.0, NULL, 0, 1, G1, &st) != -1) ++fails;
    if (orc_first_half_rows_cols(&vL, &vS, CL, CS, n, 2, 0.0, rows, 4, cols, 0, NULL, Vc) != -1)
        ++fails;

    free(T); free(Q); free(nc); free(CP); free(CL); free(CS); free(D1); free(D2);
    free(G1); free(G2); free(sp); free(V); free(Vc); free(PL); free(PS); free(s1); free(s2);
    free(dm); free(DL);
    free_basis(&Lspd); free_basis(&L); free_basis(&S);
    printf("%s\n", fails ? "FAILED" : "all checks passed");
    return fails ? 1 : 0;
}
