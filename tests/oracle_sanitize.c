/* The C oracle under the host sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer): a small
 * random model of every descriptor kind on a small periodic cell (L < 2 r_c, so several images of
 * each atom), both neighbour searches, the table, an open cluster and a ghost domain. Every call
 * must return ORC_OK with finite outputs, and the brute-force and cell-list searches must agree.
 * Built and run by tests/test_oracle_sanitize.py (gcc, no OpenMP). */
#include <stdio.h>

#include "../oracle/dp_oracle.c"

static unsigned long long lcg = 88172645463325252ULL;
static double urand(void)   /* uniform in [-1, 1) */
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int finite_all(const double *x, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

int main(void)
{
    enum { N = 24 };
    const double L = 7.0, box[9] = {L, 0, 0, 0, L, 0, 0, 0, L};
    double coord[3 * N];
    int type[N];
    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) coord[3 * i + k] = 0.5 * L * (1.0 + urand());
        type[i] = i % 3 == 0 ? 0 : 1;
    }
    int bad = 0;
    for (int desc = 0; desc < 3; ++desc) {
        for (int tos = 0; tos < 2; ++tos) {
            orc_model m;
            memset(&m, 0, sizeof(m));
            m.ntypes = 2;
            m.sel[0] = desc == 2 ? 6 : 12;
            m.sel[1] = desc == 2 ? 10 : 24;
            m.rcut = 4.0;
            m.rcut_smth = 0.8;
            m.emb[0] = 4; m.emb[1] = 8; m.emb[2] = 16;
            m.axis = 4;
            m.fit[0] = 8; m.fit[1] = 8; m.fit[2] = 8;
            m.type_one_side = desc == 2 ? 0 : tos;
            m.descriptor = desc;
            const long np = orc_param_count(&m);
            double *p = malloc(sizeof(double) * (size_t)np);
            for (long i = 0; i < np; ++i) p[i] = 0.3 * urand();
            m.params = p;
            double e[2], f[2][3 * N], v[2][9], ei[N];
            long nd = 0, oor = 0;
            for (int method = 0; method < 2; ++method) {
                const int rc = orc_compute(&m, N, coord, type, box, method, NULL, 0.0, 0, &e[method], f[method],
                                           v[method], ei, &nd, &oor, NULL, NULL, NULL);
                if (rc != ORC_OK || !finite_all(f[method], 3 * N) || !finite_all(v[method], 9) || !isfinite(e[method])) {
                    printf("descriptor %d tos %d method %d: rc %d\n", desc, tos, method, rc);
                    bad = 1;
                }
            }
            double df = fabs(e[0] - e[1]);
            for (int i = 0; i < 3 * N; ++i) df = fmax(df, fabs(f[0][i] - f[1][i]));
            if (df > 1e-10) {
                printf("descriptor %d tos %d: brute force and cell list differ by %g\n", desc, tos, df);
                bad = 1;
            }
            if (desc != 2) {
                /* the table of the two-body nets over s in [0, 1/r_min] */
                const int nint = 300;
                const double dx = 0.01;
                const int nets = m.type_one_side ? m.ntypes : m.ntypes * m.ntypes;
                double *coef = malloc(sizeof(double) * (size_t)nets * nint * m.emb[2] * 6);
                double et, ft[3 * N], vt[9];
                if (orc_table_build(&m, dx, nint, coef) != ORC_OK ||
                    orc_compute(&m, N, coord, type, box, 1, coef, dx, nint, &et, ft, vt, NULL, &nd, &oor, NULL, NULL,
                                NULL) != ORC_OK ||
                    !finite_all(ft, 3 * N) || !isfinite(et)) {
                    printf("descriptor %d tos %d: table evaluation failed\n", desc, tos);
                    bad = 1;
                }
                free(coef);
            }
            /* an open cluster (no box), and the first half owned with the rest as ghosts */
            double eo, fo[3 * N], vo[9], eg, fg[3 * N], vg[9];
            if (orc_compute(&m, N, coord, type, NULL, 0, NULL, 0.0, 0, &eo, fo, vo, NULL, &nd, &oor, NULL, NULL, NULL) != ORC_OK ||
                orc_compute_ghost(&m, N / 2, N - N / 2, coord, type, &eg, fg, vg, NULL) != ORC_OK ||
                !finite_all(fo, 3 * N) || !finite_all(fg, 3 * N)) {
                printf("descriptor %d tos %d: open or ghost evaluation failed\n", desc, tos);
                bad = 1;
            }
            free(p);
        }
    }
    if (!bad) printf("oracle sanitizer run ok\n");
    return bad;
}
