/*
 * dp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU evaluation of the smooth two-body-embedding Deep Potential (se_e2_a)
 * with energy, forces and virial, written from the DeePMD-kit v2 paper (arXiv 2304.09409).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this library;
 * the product path (HIP kernels behind the C ABI) shares no code with it and never calls it.
 *
 * Sections followed (paper numbering):
 *   Sec. II.A          model form y_i = F(D(x_i, {x_j})) and E = sum_i E_i; N_c padding.
 *   Sec. II.A.1        se_e2_a descriptor D = N_c^-2 G^T R R^T G_<, the environment-matrix row
 *                      (s, s x/r, s y/r, s z/r) with r_ij = r_j - r_i, the switching function
 *                      s(r) (eq. switch), the embedding G_j = N(s(r_ij)) (eq. G2), and the
 *                      per-species nets N^{alpha_i, alpha_j} (or N^{alpha_j}).
 *   Sec. II.A.2        E_i = F_0(D^i) (eq. fitting_energy); F = -dE/dr; virial
 *                      Xi_ab = -sum_g dE/dh_ga h_gb.
 *   Sec. II.A.6        layer y = w_hat * phi(x W + b) (+ x, or + {x,x}) (eq. NN); tabulated
 *                      inference with quintic pieces (eq. compress) and its coefficient formulas.
 *   Sec. III.B.1       neighbour formatting order: type, then distance, then index.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - N_c is the sum of the per-type capacities sel[]; each type block is padded separately.
 *   - Neighbours are ordered by (type, squared distance, index j, image shift n0, n1, n2); more
 *     than sel[t] neighbours of type t keep the nearest sel[t] and the rest are counted as dropped.
 *   - The fitting output layer is linear (identity activation), without a skip connection.
 *   - Skip connections follow the sizes: +x when n_out == n_in, +{x,x} when n_out == 2 n_in.
 *   - The tabulated variable is the embedding input x = s(r); node l sits at x_l = l * dx and
 *     pieces are evaluated in the local variable t = x - x_l.
 *   - Periodic images: coordinates are wrapped into the cell, and every image shift n with
 *     |r_j + n h - r_i| < r_c is a candidate (small cells give several images of one atom).
 *
 * Parity status: every function here is pinned by the CPU tests (closed forms, finite
 * differences, invariances, the dimer special case, brute force vs cell list, table node
 * identities). Absolute energy values of a random model have no printed value in the paper.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXT 8

typedef struct {
    int ntypes;
    int sel[ORC_MAXT];
    double rcut, rcut_smth;
    int emb[3];          /* embedding net widths, e.g. 25, 50, 100          */
    int axis;            /* M_<                                              */
    int fit[3];          /* fitting hidden widths, e.g. 240, 240, 240        */
    int type_one_side;   /* 0: one net per (type_i, type_j); 1: one per type_j */
    int descriptor;      /* 0: se_e2_a (full), 1: se_e2_r (radial-only), 2: se_e3 (three-body) */
    const double *params;
} orc_model;

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_TYPE = -2, ORC_E_BOX = -3, ORC_E_MEM = -4 };

/* ------------------------------------------------------------------------------------------
 * Switching function, Sec. II.A.1 (eq. switch):
 *   s = 1/r for r < r_s;  s = u(x)/r for r_s <= r < r_c with x = (r - r_s)/(r_c - r_s) and
 *   u(x) = x^3 (-6 x^2 + 15 x - 10) + 1;  s = 0 for r >= r_c.
 *   u is evaluated as (1 - x)^3 (1 + 3 x + 6 x^2), the same polynomial factored: no cancellation
 *   near x = 1, so s >= 0 holds in floating point too.
 *   ds/dr by the quotient rule, with u'(x) = -30 x^2 (x - 1)^2.
 * ---------------------------------------------------------------------------------------- */
void orc_switch(double r, double rs, double rc, double *s, double *ds)
{
    if (r < rs) {
        *s = 1.0 / r;
        *ds = -1.0 / (r * r);
    } else if (r < rc) {
        double x = (r - rs) / (rc - rs);
        double y = 1.0 - x;
        double u = y * y * y * (1.0 + 3.0 * x + 6.0 * x * x);
        double du = -30.0 * x * x * (x - 1.0) * (x - 1.0);
        *s = u / r;
        *ds = du / ((rc - rs) * r) - u / (r * r);
    } else {
        *s = 0.0;
        *ds = 0.0;
    }
}

/* ------------------------------------------------------------------------------------------
 * Parameter layout: embedding nets first (index ti*ntypes+tj, or tj with type_one_side), each
 * with layers 1->emb0->emb1->emb2; then one fitting net per type with layers
 * (emb2*axis)->fit0->fit1->fit2->1. Every layer stores W [n_in][n_out] row-major, b [n_out],
 * w_hat [n_out].
 * ---------------------------------------------------------------------------------------- */
typedef struct { int nin, nout; const double *W, *b, *wh; } orc_layer;

/* se_e3 always has a net per ordered pair of neighbour types (a_j, a_k), Sec. II.A.1 */
static int n_emb_nets(const orc_model *m)
{
    return (m->type_one_side && m->descriptor != 2) ? m->ntypes : m->ntypes * m->ntypes;
}

/* Width of the descriptor: M x M_< for se_e2_a, M for se_e2_r and se_e3 */
static int fit_in(const orc_model *m) { return m->descriptor == 0 ? m->emb[2] * m->axis : m->emb[2]; }

long orc_param_count(const orc_model *m)
{
    long c = 0;
    int e[4] = {1, m->emb[0], m->emb[1], m->emb[2]};
    int f[5] = {fit_in(m), m->fit[0], m->fit[1], m->fit[2], 1};
    for (int k = 0; k < 3; ++k) c += (long)n_emb_nets(m) * (e[k] * e[k + 1] + 2 * e[k + 1]);
    for (int k = 0; k < 4; ++k) c += (long)m->ntypes * (f[k] * f[k + 1] + 2 * f[k + 1]);
    return c;
}

static const double *take_layer(const double *p, int nin, int nout, orc_layer *L)
{
    L->nin = nin; L->nout = nout;
    L->W = p; p += (long)nin * nout;
    L->b = p; p += nout;
    L->wh = p; p += nout;
    return p;
}

static void emb_layers(const orc_model *m, int net, orc_layer L[3])
{
    int e[4] = {1, m->emb[0], m->emb[1], m->emb[2]};
    const double *p = m->params;
    for (int n = 0; n < net; ++n)
        for (int k = 0; k < 3; ++k) p += (long)e[k] * e[k + 1] + 2 * e[k + 1];
    for (int k = 0; k < 3; ++k) p = take_layer(p, e[k], e[k + 1], &L[k]);
}

static void fit_layers(const orc_model *m, int t, orc_layer L[4])
{
    int e[4] = {1, m->emb[0], m->emb[1], m->emb[2]};
    int f[5] = {fit_in(m), m->fit[0], m->fit[1], m->fit[2], 1};
    const double *p = m->params;
    for (int n = 0; n < n_emb_nets(m); ++n)
        for (int k = 0; k < 3; ++k) p += (long)e[k] * e[k + 1] + 2 * e[k + 1];
    for (int n = 0; n < t; ++n)
        for (int k = 0; k < 4; ++k) p += (long)f[k] * f[k + 1] + 2 * f[k + 1];
    for (int k = 0; k < 4; ++k) p = take_layer(p, f[k], f[k + 1], &L[k]);
}

/* Skip connection of eq. NN, chosen by the layer sizes. */
static double skip_of(const double *x, int nin, int nout, int o)
{
    if (nout == nin) return x[o];
    if (nout == 2 * nin) return x[o % nin];
    return 0.0;
}

/* ------------------------------------------------------------------------------------------
 * Embedding net N_e (eq. G2 with the layers of eq. NN, tanh activation) at the scalar input x,
 * with the first and second derivatives d/dx carried forward through every layer:
 *   a = z W + b, a' = z' W, a'' = z'' W; t = tanh a, t' = (1 - t^2) a',
 *   t'' = (1 - t^2) a'' - 2 t (1 - t^2) a'^2; y = w_hat t + skip(z) (same for y', y'').
 * dy and d2y may be NULL.
 * ---------------------------------------------------------------------------------------- */
#define ORC_MAXW 512
void orc_embed_eval(const orc_model *m, int net, double x, double *y, double *dy, double *d2y)
{
    orc_layer L[3];
    emb_layers(m, net, L);
    double z[ORC_MAXW], z1[ORC_MAXW], z2[ORC_MAXW];
    double nz[ORC_MAXW], nz1[ORC_MAXW], nz2[ORC_MAXW];
    z[0] = x; z1[0] = 1.0; z2[0] = 0.0;
    for (int k = 0; k < 3; ++k) {
        const orc_layer *l = &L[k];
        for (int o = 0; o < l->nout; ++o) {
            double a = l->b[o], a1 = 0.0, a2 = 0.0;
            for (int i = 0; i < l->nin; ++i) {
                double w = l->W[(long)i * l->nout + o];
                a += z[i] * w;
                a1 += z1[i] * w;
                a2 += z2[i] * w;
            }
            double t = tanh(a);
            double g = 1.0 - t * t;
            double t1 = g * a1;
            double t2 = g * a2 - 2.0 * t * g * a1 * a1;
            nz[o] = l->wh[o] * t + skip_of(z, l->nin, l->nout, o);
            nz1[o] = l->wh[o] * t1 + skip_of(z1, l->nin, l->nout, o);
            nz2[o] = l->wh[o] * t2 + skip_of(z2, l->nin, l->nout, o);
        }
        memcpy(z, nz, sizeof(double) * l->nout);
        memcpy(z1, nz1, sizeof(double) * l->nout);
        memcpy(z2, nz2, sizeof(double) * l->nout);
    }
    int M = m->emb[2];
    memcpy(y, z, sizeof(double) * M);
    if (dy) memcpy(dy, z1, sizeof(double) * M);
    if (d2y) memcpy(d2y, z2, sizeof(double) * M);
}

/* ------------------------------------------------------------------------------------------
 * Fitting net F_0 of type t (eq. fitting_energy, layers of eq. NN: three tanh layers and a linear
 * output layer). Returns E_i; if grad != NULL writes dE_i/dd (reverse pass through the layers).
 * ---------------------------------------------------------------------------------------- */
#define ORC_MAXF 2048
double orc_fit_eval(const orc_model *m, int t, const double *d, double *grad)
{
    orc_layer L[4];
    fit_layers(m, t, L);
    double h[5][ORC_MAXF];     /* h[0] = d, h[k+1] = output of layer k */
    double act[4][ORC_MAXF];   /* phi(a) of layer k                      */
    memcpy(h[0], d, sizeof(double) * L[0].nin);
    for (int k = 0; k < 4; ++k) {
        const orc_layer *l = &L[k];
        int linear = (k == 3);
        for (int o = 0; o < l->nout; ++o) {
            double a = l->b[o];
            for (int i = 0; i < l->nin; ++i) a += h[k][i] * l->W[(long)i * l->nout + o];
            act[k][o] = linear ? a : tanh(a);
            h[k + 1][o] = l->wh[o] * act[k][o] + (linear ? 0.0 : skip_of(h[k], l->nin, l->nout, o));
        }
    }
    double e = h[4][0];
    if (grad) {
        double gh[ORC_MAXF], gprev[ORC_MAXF];
        gh[0] = 1.0;
        for (int k = 3; k >= 0; --k) {
            const orc_layer *l = &L[k];
            int linear = (k == 3);
            double ga[ORC_MAXF];
            for (int o = 0; o < l->nout; ++o) {
                double dphi = linear ? 1.0 : 1.0 - act[k][o] * act[k][o];
                ga[o] = gh[o] * l->wh[o] * dphi;
            }
            for (int i = 0; i < l->nin; ++i) {
                double s = 0.0;
                for (int o = 0; o < l->nout; ++o) s += l->W[(long)i * l->nout + o] * ga[o];
                gprev[i] = s;
            }
            if (!linear) {
                if (l->nout == l->nin)
                    for (int i = 0; i < l->nin; ++i) gprev[i] += gh[i];
                else if (l->nout == 2 * l->nin)
                    for (int i = 0; i < l->nin; ++i) gprev[i] += gh[i] + gh[i + l->nin];
            }
            memcpy(gh, gprev, sizeof(double) * l->nin);
        }
        memcpy(grad, gh, sizeof(double) * L[0].nin);
    }
    return e;
}

/* ------------------------------------------------------------------------------------------
 * Tabulated embedding (Sec. II.A.6, eq. compress). Nodes x_l = l*dx, l = 0..nint. On interval l
 * the m-th output is the quintic  a t^5 + b t^4 + c t^3 + d t^2 + e t + f  in t = x - x_l, with
 * the paper's coefficients from y, y', y'' at both ends of the interval (h = y_{l+1} - y_l):
 *   a = [12h - 6(y'_{l+1} + y'_l)dx + (y''_{l+1} - y''_l)dx^2] / (2 dx^5)
 *   b = [-30h + (14y'_{l+1} + 16y'_l)dx + (-2y''_{l+1} + 3y''_l)dx^2] / (2 dx^4)
 *   c = [20h - (8y'_{l+1} + 12y'_l)dx + (y''_{l+1} - 3y''_l)dx^2] / (2 dx^3)
 *   d = y''_l / 2,  e = y'_l,  f = y_l.
 * coef layout: [net][interval][m][6] = (a, b, c, d, e, f).
 * ---------------------------------------------------------------------------------------- */
int orc_table_build(const orc_model *m, double dx, int nint, double *coef)
{
    int M = m->emb[2];
    int nn = n_emb_nets(m);
    double *y = malloc(sizeof(double) * (size_t)(nint + 1) * M * 3);
    if (!y) return ORC_E_MEM;
    for (int net = 0; net < nn; ++net) {
        for (int l = 0; l <= nint; ++l) {
            double *row = y + (size_t)l * M * 3;
            orc_embed_eval(m, net, l * dx, row, row + M, row + 2 * M);
        }
        for (int l = 0; l < nint; ++l) {
            const double *p0 = y + (size_t)l * M * 3, *p1 = y + (size_t)(l + 1) * M * 3;
            for (int o = 0; o < M; ++o) {
                double y0 = p0[o], d0 = p0[M + o], s0 = p0[2 * M + o];
                double y1 = p1[o], d1 = p1[M + o], s1 = p1[2 * M + o];
                double h = y1 - y0;
                double *c = coef + (((size_t)net * nint + l) * M + o) * 6;
                c[0] = (12.0 * h - 6.0 * (d1 + d0) * dx + (s1 - s0) * dx * dx) / (2.0 * pow(dx, 5));
                c[1] = (-30.0 * h + (14.0 * d1 + 16.0 * d0) * dx + (-2.0 * s1 + 3.0 * s0) * dx * dx) / (2.0 * pow(dx, 4));
                c[2] = (20.0 * h - (8.0 * d1 + 12.0 * d0) * dx + (s1 - 3.0 * s0) * dx * dx) / (2.0 * pow(dx, 3));
                c[3] = 0.5 * s0;
                c[4] = d0;
                c[5] = y0;
            }
        }
    }
    free(y);
    return ORC_OK;
}

/* Evaluate the tabulated net at x: value and d/dx. Returns 1 if x lies outside [0, nint*dx]. */
int orc_table_eval(const orc_model *m, const double *coef, double dx, int nint, int net, double x,
                   double *y, double *dy)
{
    int M = m->emb[2];
    int l = (int)floor(x / dx);
    int oor = (x < 0.0 || x > nint * dx);
    if (l < 0) l = 0;
    if (l > nint - 1) l = nint - 1;
    double t = x - l * dx;
    for (int o = 0; o < M; ++o) {
        const double *c = coef + (((size_t)net * nint + l) * M + o) * 6;
        y[o] = ((((c[0] * t + c[1]) * t + c[2]) * t + c[3]) * t + c[4]) * t + c[5];
        dy[o] = (((5.0 * c[0] * t + 4.0 * c[1]) * t + 3.0 * c[2]) * t + 2.0 * c[3]) * t + c[4];
    }
    return oor;
}

/* ------------------------------------------------------------------------------------------
 * Cell geometry. Rows of h are the lattice vectors a_0, a_1, a_2; fractional s = r h^-1.
 * Perpendicular width along a_k: d_k = |det h| / |a_l x a_m|.
 * ---------------------------------------------------------------------------------------- */
static int box_geometry(const double *h, double hinv[9], double width[3])
{
    double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                 h[2] * (h[3] * h[7] - h[4] * h[6]);
    if (!(det > 0.0)) return ORC_E_BOX;
    hinv[0] = (h[4] * h[8] - h[5] * h[7]) / det;
    hinv[1] = (h[2] * h[7] - h[1] * h[8]) / det;
    hinv[2] = (h[1] * h[5] - h[2] * h[4]) / det;
    hinv[3] = (h[5] * h[6] - h[3] * h[8]) / det;
    hinv[4] = (h[0] * h[8] - h[2] * h[6]) / det;
    hinv[5] = (h[2] * h[3] - h[0] * h[5]) / det;
    hinv[6] = (h[3] * h[7] - h[4] * h[6]) / det;
    hinv[7] = (h[1] * h[6] - h[0] * h[7]) / det;
    hinv[8] = (h[0] * h[4] - h[1] * h[3]) / det;
    for (int k = 0; k < 3; ++k) {
        const double *a = h + 3 * ((k + 1) % 3), *b = h + 3 * ((k + 2) % 3);
        double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
        width[k] = det / sqrt(cx * cx + cy * cy + cz * cz);
    }
    return ORC_OK;
}

/* A candidate neighbour: squared distance, owner index, image shift, and r_ij = r_j + n h - r_i. */
typedef struct { double r2; int j; int n[3]; double rij[3]; int type; } orc_cand;

static int cand_cmp(const void *pa, const void *pb)
{
    const orc_cand *a = pa, *b = pb;
    if (a->type != b->type) return a->type < b->type ? -1 : 1;
    if (a->r2 != b->r2) return a->r2 < b->r2 ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    for (int k = 0; k < 3; ++k)
        if (a->n[k] != b->n[k]) return a->n[k] < b->n[k] ? -1 : 1;
    return 0;
}

static void add_cand(orc_cand **buf, int *cnt, int *cap, const double *ri, const double *rj, const double *h,
                     const int n[3], int j, int type, double rc2)
{
    double d[3];
    for (int c = 0; c < 3; ++c) {
        double shift = h ? (n[0] * h[c] + n[1] * h[3 + c]) + n[2] * h[6 + c] : 0.0;
        d[c] = (rj[c] + shift) - ri[c];
    }
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < rc2)) return;
    if (*cnt == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *buf = realloc(*buf, sizeof(orc_cand) * (size_t)*cap);
    }
    orc_cand *c = *buf + (*cnt)++;
    c->r2 = r2; c->j = j; c->type = type;
    for (int k = 0; k < 3; ++k) { c->n[k] = n[k]; c->rij[k] = d[k]; }
}

static int floordiv(int a, int b) { int q = a / b; if ((a % b != 0) && ((a < 0) != (b < 0))) --q; return q; }

/* ------------------------------------------------------------------------------------------
 * Neighbour list (Sec. II.A n(i) and N_c padding; Sec. II.A.1 per-species blocks; Sec. III.B.1
 * ordering). method 0: brute force over all atoms and image shifts; method 1: cell list.
 * Outputs (caller order): nlist [n][N_c] owner index or -1, rij [n][N_c][3] (0 for padding).
 * ndrop receives the number of neighbours cut by the per-type capacities.
 * ---------------------------------------------------------------------------------------- */
int orc_nlist(const orc_model *m, long n, const double *coord, const int *type, const double *box,
              int method, int *nlist, double *rij, long *ndrop)
{
    if (n < 1 || !coord || !type || !nlist) return ORC_E_ARG;
    for (long i = 0; i < n; ++i)
        if (type[i] < 0 || type[i] >= m->ntypes) return ORC_E_TYPE;
    int Nc = 0, off[ORC_MAXT + 1];
    for (int t = 0; t < m->ntypes; ++t) { off[t] = Nc; Nc += m->sel[t]; }
    off[m->ntypes] = Nc;
    double rc = m->rcut, rc2 = rc * rc;
    double hinv[9], width[3];
    double *pos = malloc(sizeof(double) * 3 * (size_t)n);
    int nb[3] = {1, 1, 1}, K[3] = {0, 0, 0};
    if (box) {
        int rcode = box_geometry(box, hinv, width);
        if (rcode) { free(pos); return rcode; }
        for (long i = 0; i < n; ++i) {
            double s[3];
            for (int c = 0; c < 3; ++c) {
                s[c] = (coord[3 * i] * hinv[c] + coord[3 * i + 1] * hinv[3 + c]) + coord[3 * i + 2] * hinv[6 + c];
                s[c] -= floor(s[c]);
                if (s[c] >= 1.0) s[c] = 0.0;
            }
            for (int c = 0; c < 3; ++c)
                pos[3 * i + c] = (s[0] * box[c] + s[1] * box[3 + c]) + s[2] * box[6 + c];
        }
        for (int k = 0; k < 3; ++k) {
            if (method == 1) {
                nb[k] = (int)floor(width[k] / rc);
                if (nb[k] < 1) nb[k] = 1;
            }
            K[k] = (int)ceil(rc / (width[k] / nb[k]));
        }
    } else {
        memcpy(pos, coord, sizeof(double) * 3 * (size_t)n);
        method = 0;   /* open boundary: brute force, no images */
    }

    /* cell list over fractional coordinates */
    int ncell = nb[0] * nb[1] * nb[2];
    int *cell_of = NULL, *cstart = NULL, *catoms = NULL;
    if (method == 1) {
        cell_of = malloc(sizeof(int) * (size_t)n);
        cstart = calloc((size_t)ncell + 1, sizeof(int));
        catoms = malloc(sizeof(int) * (size_t)n);
        for (long i = 0; i < n; ++i) {
            int b[3];
            for (int c = 0; c < 3; ++c) {
                double s = (pos[3 * i] * hinv[c] + pos[3 * i + 1] * hinv[3 + c]) + pos[3 * i + 2] * hinv[6 + c];
                b[c] = (int)floor(s * nb[c]);
                if (b[c] < 0) b[c] = 0;
                if (b[c] >= nb[c]) b[c] = nb[c] - 1;
            }
            cell_of[i] = (b[2] * nb[1] + b[1]) * nb[0] + b[0];
            cstart[cell_of[i] + 1]++;
        }
        for (int c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
        int *fill = malloc(sizeof(int) * (size_t)ncell);
        memcpy(fill, cstart, sizeof(int) * (size_t)ncell);
        for (long i = 0; i < n; ++i) catoms[fill[cell_of[i]]++] = (int)i;
        free(fill);
    }

    long drops = 0;
#pragma omp parallel reduction(+ : drops)
    {
        orc_cand *buf = NULL;
        int cap = 0;
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < n; ++i) {
            int cnt = 0;
            const double *ri = pos + 3 * i;
            if (method == 0) {
                for (long j = 0; j < n; ++j)
                    for (int a = -K[0]; a <= K[0]; ++a)
                        for (int b = -K[1]; b <= K[1]; ++b)
                            for (int c = -K[2]; c <= K[2]; ++c) {
                                if (j == i && a == 0 && b == 0 && c == 0) continue;
                                int sh[3] = {a, b, c};
                                add_cand(&buf, &cnt, &cap, ri, pos + 3 * j, box, sh, (int)j, type[j], rc2);
                            }
            } else {
                int ci = cell_of[i];
                int bi[3] = {ci % nb[0], (ci / nb[0]) % nb[1], ci / (nb[0] * nb[1])};
                for (int a = -K[0]; a <= K[0]; ++a)
                    for (int b = -K[1]; b <= K[1]; ++b)
                        for (int c = -K[2]; c <= K[2]; ++c) {
                            int tg[3] = {bi[0] + a, bi[1] + b, bi[2] + c}, sh[3], bb[3];
                            for (int k = 0; k < 3; ++k) {
                                sh[k] = floordiv(tg[k], nb[k]);
                                bb[k] = tg[k] - sh[k] * nb[k];
                            }
                            int cell = (bb[2] * nb[1] + bb[1]) * nb[0] + bb[0];
                            for (int q = cstart[cell]; q < cstart[cell + 1]; ++q) {
                                int j = catoms[q];
                                if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
                                add_cand(&buf, &cnt, &cap, ri, pos + 3 * j, box, sh, j, type[j], rc2);
                            }
                        }
            }
            qsort(buf, (size_t)cnt, sizeof(orc_cand), cand_cmp);
            int *row = nlist + i * Nc;
            double *rrow = rij ? rij + i * Nc * 3 : NULL;
            for (int s = 0; s < Nc; ++s) row[s] = -1;
            if (rrow) for (int s = 0; s < 3 * Nc; ++s) rrow[s] = 0.0;
            int fillc[ORC_MAXT] = {0};
            for (int q = 0; q < cnt; ++q) {
                int t = buf[q].type;
                if (fillc[t] < m->sel[t]) {
                    int slot = off[t] + fillc[t];
                    row[slot] = buf[q].j;
                    if (rrow) for (int k = 0; k < 3; ++k) rrow[3 * slot + k] = buf[q].rij[k];
                    fillc[t]++;
                } else {
                    drops++;
                }
            }
        }
        free(buf);
    }
    if (ndrop) *ndrop = drops;
    free(pos); free(cell_of); free(cstart); free(catoms);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------
 * Full evaluation of E, F, Xi (and per-atom E_i). Per centre atom i:
 *   R_j = (s, s x/r, s y/r, s z/r) for each kept slot (Sec. II.A.1, eq. rij);
 *   G_j = N^{a_i,a_j}(s) and dG_j/ds (or the quintic table, eq. compress);
 *   T = N_c^-1 G^T R  (M x 4);  D = T T_<^T (M x M_<), d[m*M_< + n] = D_mn;
 *   E_i = F_0(d) and dE_i/dd by the reverse pass (eq. fitting_energy);
 *   dT_pk = sum_n dD_pn T_nk + [p < M_<] sum_m dD_mp T_mk;
 *   per slot: dG_m = N_c^-1 sum_k dT_mk R_k,  dR_k = N_c^-1 sum_m G_m dT_mk,
 *             dE/ds (through G) = sum_m dG_m dG_m/ds;
 *   g_ij = dE/dr_ij = [(dR_0 + dE/ds) s' + q (s' - s/r)] r^ + (s/r) dR_{1:3}, q = sum_a dR_a r^_a;
 *   F_i += g_ij, F_j -= g_ij (F = -dE/dr, Sec. II.A.2);
 *   Xi_ab -= g_ij,a r_ij,b, which is -sum_g dE/dh_ga h_gb for r_ij = (s_j + n - s_i) h.
 * table == NULL selects the network; otherwise table holds orc_table_build() coefficients.
 * Optional dumps: nlist_out [n][N_c], T_out [n][M][4], dT_out [n][M][4].
 * Centre atoms are 0.. ncentre - 1 (all atoms in orc_compute; the owned atoms of a domain with
 * ghost atoms in orc_compute_ghost): only they have E_i and contribute pairs; the neighbours of a
 * centre are taken from all n atoms.
 * ---------------------------------------------------------------------------------------- */
static int compute_impl(const orc_model *m, long n, long ncentre, const double *coord, const int *type,
                        const double *box, int method, const double *table, double tab_dx, int tab_nint,
                        double *energy, double *force, double *virial, double *atom_energy,
                        long *ndrop, long *ntab_oor, int *nlist_out, double *T_out, double *dT_out)
{
    int Nc = 0, M = m->emb[2], A = m->axis, nt = m->ntypes;
    int slot_type[4096];
    for (int t = 0; t < nt; ++t)
        for (int s = 0; s < m->sel[t]; ++s) slot_type[Nc++] = t;
    int *nlist = malloc(sizeof(int) * (size_t)n * Nc);
    double *rij = malloc(sizeof(double) * (size_t)n * Nc * 3);
    double *g = malloc(sizeof(double) * (size_t)n * Nc * 3);
    double *ei = malloc(sizeof(double) * (size_t)n);
    if (!nlist || !rij || !g || !ei) { free(nlist); free(rij); free(g); free(ei); return ORC_E_MEM; }
    int rcode = orc_nlist(m, n, coord, type, box, method, nlist, rij, ndrop);
    if (rcode) { free(nlist); free(rij); free(g); free(ei); return rcode; }
    const double inv_nc = 1.0 / Nc;
    long oor_total = 0;

#pragma omp parallel reduction(+ : oor_total)
    {
        double *G = malloc(sizeof(double) * (size_t)Nc * M);
        double *dGds = malloc(sizeof(double) * (size_t)Nc * M);
        double *R = malloc(sizeof(double) * (size_t)Nc * 4);
        double *dRs = malloc(sizeof(double) * (size_t)Nc * 4);   /* se_e3: dE/dR per slot */
        double *S = malloc(sizeof(double) * (size_t)Nc * 3);   /* s, s', r per slot */
        double *T = malloc(sizeof(double) * (size_t)M * 4);
        double *dT = malloc(sizeof(double) * (size_t)M * 4);
        double *d = malloc(sizeof(double) * (size_t)M * A);
        double *dd = malloc(sizeof(double) * (size_t)M * A);
        double *Gp = malloc(sizeof(double) * (size_t)M), *Gpd = malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(dynamic, 8)
        for (long i = 0; i < ncentre; ++i) {
            int ti = type[i];
            /* environment rows (eq. rij, eq. switch) of the kept slots */
            for (int sl = 0; sl < Nc; ++sl) {
                if (nlist[i * Nc + sl] < 0) continue;
                const double *v = rij + (i * Nc + sl) * 3;
                double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double s, ds;
                orc_switch(r, m->rcut_smth, m->rcut, &s, &ds);
                S[3 * sl] = s; S[3 * sl + 1] = ds; S[3 * sl + 2] = r;
                R[4 * sl] = s;
                for (int k = 0; k < 3; ++k) R[4 * sl + 1 + k] = s * v[k] / r;
            }
            if (m->descriptor == 2) {
                /* se_e3 (eq. descrpt-e3, eq. nn-descrpt-e3): theta_ab = R_a . R_b over every ordered
                 * pair of kept slots (a = b included), G_ab = N^{a_a, a_b}(theta_ab),
                 * D_m = N_c^-2 sum_ab theta_ab G_ab,m */
                const double inv2 = inv_nc * inv_nc;
                for (int mm = 0; mm < M; ++mm) d[mm] = 0.0;
                for (int a = 0; a < Nc; ++a) {
                    if (nlist[i * Nc + a] < 0) continue;
                    for (int b = 0; b < Nc; ++b) {
                        if (nlist[i * Nc + b] < 0) continue;
                        double th = 0.0;
                        for (int k = 0; k < 4; ++k) th += R[4 * a + k] * R[4 * b + k];
                        int net = slot_type[a] * nt + slot_type[b];
                        if (table) oor_total += orc_table_eval(m, table, tab_dx, tab_nint, net, th, Gp, Gpd);
                        else orc_embed_eval(m, net, th, Gp, NULL, NULL);
                        for (int mm = 0; mm < M; ++mm) d[mm] += th * Gp[mm];
                    }
                }
                for (int mm = 0; mm < M; ++mm) d[mm] *= inv2;
                ei[i] = orc_fit_eval(m, ti, d, dd);
                /* dE/dtheta_ab = N_c^-2 sum_m dd_m (G_m + theta G'_m); theta_ab = R_a . R_b gives
                 * dE/dR_a += dE/dtheta_ab R_b and dE/dR_b += dE/dtheta_ab R_a */
                for (int q = 0; q < 4 * Nc; ++q) dRs[q] = 0.0;
                for (int a = 0; a < Nc; ++a) {
                    if (nlist[i * Nc + a] < 0) continue;
                    for (int b = 0; b < Nc; ++b) {
                        if (nlist[i * Nc + b] < 0) continue;
                        double th = 0.0;
                        for (int k = 0; k < 4; ++k) th += R[4 * a + k] * R[4 * b + k];
                        int net = slot_type[a] * nt + slot_type[b];
                        if (table) orc_table_eval(m, table, tab_dx, tab_nint, net, th, Gp, Gpd);
                        else orc_embed_eval(m, net, th, Gp, Gpd, NULL);
                        double de = 0.0;
                        for (int mm = 0; mm < M; ++mm) de += dd[mm] * (Gp[mm] + th * Gpd[mm]);
                        de *= inv2;
                        for (int k = 0; k < 4; ++k) {
                            dRs[4 * a + k] += de * R[4 * b + k];
                            dRs[4 * b + k] += de * R[4 * a + k];
                        }
                    }
                }
                if (T_out) {
                    for (int q = 0; q < 4 * M; ++q) T_out[i * 4 * M + q] = 0.0;
                    for (int mm = 0; mm < M; ++mm) T_out[i * 4 * M + 4 * mm] = d[mm];
                }
                if (dT_out) {
                    for (int q = 0; q < 4 * M; ++q) dT_out[i * 4 * M + q] = 0.0;
                    for (int mm = 0; mm < M; ++mm) dT_out[i * 4 * M + 4 * mm] = dd[mm];
                }
                for (int sl = 0; sl < Nc; ++sl) {
                    double *gv = g + (i * Nc + sl) * 3;
                    gv[0] = gv[1] = gv[2] = 0.0;
                    if (nlist[i * Nc + sl] < 0) continue;
                    const double *dR = dRs + 4 * sl, *v = rij + (i * Nc + sl) * 3;
                    double s = S[3 * sl], ds = S[3 * sl + 1], r = S[3 * sl + 2];
                    double u[3] = {v[0] / r, v[1] / r, v[2] / r};
                    double q = dR[1] * u[0] + dR[2] * u[1] + dR[3] * u[2];
                    double radial = dR[0] * ds + q * (ds - s / r);
                    for (int k = 0; k < 3; ++k) gv[k] = radial * u[k] + (s / r) * dR[1 + k];
                }
                continue;
            }
            /* se_e2_a / se_e2_r: G_j = N(s_j) and T = N_c^-1 G^T R */
            for (int q = 0; q < 4 * M; ++q) T[q] = 0.0;
            for (int sl = 0; sl < Nc; ++sl) {
                if (nlist[i * Nc + sl] < 0) continue;
                double s = S[3 * sl];
                int net = m->type_one_side ? slot_type[sl] : ti * nt + slot_type[sl];
                if (table)
                    oor_total += orc_table_eval(m, table, tab_dx, tab_nint, net, s, G + (size_t)sl * M, dGds + (size_t)sl * M);
                else
                    orc_embed_eval(m, net, s, G + (size_t)sl * M, dGds + (size_t)sl * M, NULL);
                for (int mm = 0; mm < M; ++mm)
                    for (int k = 0; k < 4; ++k) T[4 * mm + k] += G[(size_t)sl * M + mm] * R[4 * sl + k];
            }
            for (int q = 0; q < 4 * M; ++q) T[q] *= inv_nc;
            if (m->descriptor == 1) {
                /* se_e2_r (radial-only, reading: the environment matrix is the one column s):
                 * D_m = N_c^-1 sum_j s_j G_j,m = T[m][0]; dE/dT[m][0] = dE/dD_m, other columns 0 */
                for (int mm = 0; mm < M; ++mm) d[mm] = T[4 * mm];
                ei[i] = orc_fit_eval(m, ti, d, dd);
                for (int p = 0; p < M; ++p) {
                    dT[4 * p] = dd[p];
                    dT[4 * p + 1] = dT[4 * p + 2] = dT[4 * p + 3] = 0.0;
                }
            } else {
                for (int mm = 0; mm < M; ++mm)
                    for (int nn = 0; nn < A; ++nn) {
                        double acc = 0.0;
                        for (int k = 0; k < 4; ++k) acc += T[4 * mm + k] * T[4 * nn + k];
                        d[mm * A + nn] = acc;
                    }
                ei[i] = orc_fit_eval(m, ti, d, dd);
                for (int p = 0; p < M; ++p)
                    for (int k = 0; k < 4; ++k) {
                        double acc = 0.0;
                        for (int nn = 0; nn < A; ++nn) acc += dd[p * A + nn] * T[4 * nn + k];
                        if (p < A)
                            for (int mm = 0; mm < M; ++mm) acc += dd[mm * A + p] * T[4 * mm + k];
                        dT[4 * p + k] = acc;
                    }
            }
            if (T_out) memcpy(T_out + i * 4 * M, T, sizeof(double) * 4 * M);
            if (dT_out) memcpy(dT_out + i * 4 * M, dT, sizeof(double) * 4 * M);
            for (int sl = 0; sl < Nc; ++sl) {
                double *gv = g + (i * Nc + sl) * 3;
                gv[0] = gv[1] = gv[2] = 0.0;
                if (nlist[i * Nc + sl] < 0) continue;
                const double *Gs = G + (size_t)sl * M, *Gd = dGds + (size_t)sl * M;
                double dR[4] = {0, 0, 0, 0}, dEds = 0.0;
                for (int mm = 0; mm < M; ++mm) {
                    double dGm = 0.0;
                    for (int k = 0; k < 4; ++k) {
                        dGm += dT[4 * mm + k] * R[4 * sl + k];
                        dR[k] += Gs[mm] * dT[4 * mm + k];
                    }
                    dEds += inv_nc * dGm * Gd[mm];
                }
                for (int k = 0; k < 4; ++k) dR[k] *= inv_nc;
                const double *v = rij + (i * Nc + sl) * 3;
                double s = S[3 * sl], ds = S[3 * sl + 1], r = S[3 * sl + 2];
                double u[3] = {v[0] / r, v[1] / r, v[2] / r};
                double q = dR[1] * u[0] + dR[2] * u[1] + dR[3] * u[2];
                double radial = (dR[0] + dEds) * ds + q * (ds - s / r);
                for (int k = 0; k < 3; ++k) gv[k] = radial * u[k] + (s / r) * dR[1 + k];
            }
        }
        free(G); free(dGds); free(R); free(dRs); free(S); free(T); free(dT); free(d); free(dd); free(Gp); free(Gpd);
    }

    /* serial accumulation in a fixed order */
    double e = 0.0, xi[9] = {0};
    if (force) for (long q = 0; q < 3 * n; ++q) force[q] = 0.0;
    for (long i = 0; i < ncentre; ++i) {
        e += ei[i];
        for (int sl = 0; sl < Nc; ++sl) {
            int j = nlist[i * Nc + sl];
            if (j < 0) continue;
            const double *gv = g + (i * Nc + sl) * 3, *v = rij + (i * Nc + sl) * 3;
            if (force)
                for (int k = 0; k < 3; ++k) { force[3 * i + k] += gv[k]; force[3 * (long)j + k] -= gv[k]; }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) xi[3 * a + b] -= gv[a] * v[b];
        }
    }
    if (energy) *energy = e;
    if (virial) memcpy(virial, xi, sizeof(xi));
    if (atom_energy) memcpy(atom_energy, ei, sizeof(double) * (size_t)ncentre);
    if (nlist_out) memcpy(nlist_out, nlist, sizeof(int) * (size_t)n * Nc);
    if (ntab_oor) *ntab_oor = oor_total;
    free(nlist); free(rij); free(g); free(ei);
    return ORC_OK;
}

int orc_compute(const orc_model *m, long n, const double *coord, const int *type, const double *box,
                int method, const double *table, double tab_dx, int tab_nint,
                double *energy, double *force, double *virial, double *atom_energy,
                long *ndrop, long *ntab_oor, int *nlist_out, double *T_out, double *dT_out)
{
    return compute_impl(m, n, n, coord, type, box, method, table, tab_dx, tab_nint, energy, force, virial,
                        atom_energy, ndrop, ntab_oor, nlist_out, T_out, dT_out);
}

/* ------------------------------------------------------------------------------------------
 * One domain of a spatially decomposed frame (Sec. III.B.2): atoms 0.. nlocal - 1 are owned, the
 * rest are ghost copies at the positions the neighbouring domains sent; no cell (every atom within
 * r_c of an owned atom is present). E sums E_i over owned atoms (atom_energy: nlocal values), the
 * forces cover owned and ghost atoms (a ghost's force belongs to its owner), and the virial sums
 * the pairs whose centre is owned. ndrop counts the cuts by sel of all atoms' lists (ghosts'
 * included, as orc_nlist builds every list).
 * ---------------------------------------------------------------------------------------- */
int orc_compute_ghost(const orc_model *m, long nlocal, long nghost, const double *coord, const int *type,
                      double *energy, double *force, double *virial, double *atom_energy)
{
    long nd = 0;
    return compute_impl(m, nlocal + nghost, nlocal, coord, type, NULL, 0, NULL, 0.0, 0, energy, force, virial,
                        atom_energy, &nd, NULL, NULL, NULL, NULL);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following evaluations (for timing the oracle single-threaded). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
