// trainer.cpp -- the training path (Sec. II.B): per frame, the model's E, F and virial with the
// current parameters, the loss of eq. loss, and its parameter gradient from the forward-mode
// tangent along the loss's force/virial direction followed by reverse mode (kernels_train.hip);
// Adam steps and the learning-rate and prefactor schedules.
//
// Per frame, on the trainer's stream:
//   1. geometry (the inference path's partition, bins and neighbour search);
//   2. the pair list grouped by embedding net (host, from the per-atom kept counts);
//   3. inference: environment rows, embedding nets with their unit tangents d/ds, T and D, fitting
//      nets, the input adjoint down to dE/dT, pair forces and the virial;
//   4. host: E, the loss, cE = 2 p_E (E - E*)/N, the direction vdir = -2 p_F q (F - F*)/(3N) and
//      CV = -2 p_Xi (Xi - Xi*)/(9N) (times the frame weight);
//   5. training: pair tangents, T and D with tangents, fitting nets with tangents, the reverse pass
//      through fitting and embedding nets with every weight gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dpk.h"
#include "dpk_launch.h"
#include "dpk_train.h"

using namespace dpk;

namespace {

#define TRCHK(expr)                                                                                 \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return set_error(DPK_E_DEVICE, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

struct LayerOff {
    int64_t W, b, wh;
    int nin, nout;
};

// Device buffer that grows to the largest request (contents not kept).
struct DBuf {
    double* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t need) {
        if (need <= n && p) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(need, 1) * sizeof(double));
        if (e == hipSuccess) n = need;
        return e;
    }
    ~DBuf() { if (p) hipFree(p); }
};
struct IBuf {
    int* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t need) {
        if (need <= n && p) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(need, 1) * sizeof(int));
        if (e == hipSuccess) n = need;
        return e;
    }
    ~IBuf() { if (p) hipFree(p); }
};

}  // namespace

struct dpk_trainer {
    dpk_model* model = nullptr;   // private copy (geometry context)
    dpk_ctx* geo = nullptr;
    dpk_model_desc desc;
    int device = 0, nets = 0, nt = 0, nc = 0;
    int64_t np = 0;
    int64_t step = 0;
    std::vector<LayerOff> emb, fit;   // [nets][3], [nt][4]
    DBuf theta, grad, mom1, mom2;
    // frame workspace
    IBuf pa, ps, apo;
    DBuf R, X0, ones, sigma, Rd;
    DBuf eA[3], eZd[3], eY[3], eYd[3];   // embedding layers (eY[2] = G, eYd[2] = dG/ds)
    DBuf yb[2], xb[2], zb, zdb, hb;      // pair-level reverse buffers
    DBuf T, Td, Tb, Tdb, D, Dd, Db, Ddb;
    DBuf fA[3], fZd[3], fY[3], fYd[3], fyb[2], fydb[2], fzb, fzdb, fhb;
    DBuf Ei, F, vir, vdir, sums, csum;
    ~dpk_trainer() {
        if (geo) dpk_ctx_free(geo);
        if (model) dpk_model_free(model);
    }
};

namespace {

void layer_offsets(dpk_trainer* t)
{
    const dpk_model_desc& d = t->desc;
    const int e[4] = {1, d.emb[0], d.emb[1], d.emb[2]};
    const int f[5] = {d.emb[2] * d.axis, d.fit[0], d.fit[1], d.fit[2], 1};
    int64_t off = 0;
    auto take = [&](int nin, int nout) {
        LayerOff L{off, off + (int64_t)nin * nout, off + (int64_t)nin * nout + nout, nin, nout};
        off += (int64_t)nin * nout + 2 * nout;
        return L;
    };
    t->emb.clear();
    t->fit.clear();
    for (int n = 0; n < t->nets; ++n)
        for (int k = 0; k < 3; ++k) t->emb.push_back(take(e[k], e[k + 1]));
    for (int ty = 0; ty < d.ntypes; ++ty)
        for (int k = 0; k < 4; ++k) t->fit.push_back(take(f[k], f[k + 1]));
}

// Forward pass of one hidden layer over rows [0, M) (dual: with tangents).
void layer_fwd(const dpk_trainer* t, const LayerOff& L, int M, const double* X, const double* Xd, double* A,
               double* Y, double* Zd, double* Yd, hipStream_t s)
{
    TrGemm g;
    std::memset(&g, 0, sizeof(g));
    g.M = M;
    g.N = L.nout;
    g.K = L.nin;
    g.mode = TR_FWD;
    g.A = X;
    g.A2 = Xd;
    g.W = t->theta.p + L.W;
    g.bias = t->theta.p + L.b;
    g.wh = t->theta.p + L.wh;
    g.C = A;
    g.Y = Y;
    g.Zd = Zd;
    g.Yd = Yd;
    tr_gemm(g, s);
}

// Reverse pass of one hidden layer over rows [0, M): adjoints (Yb, Ydb) of (y, ydot) in; weight
// gradients added; input adjoints (Xb, Xdb) out if Xb is set. X, Xd: the layer's inputs and their
// (unit) tangents; Zd: the stored (unit) pre-activation tangents; sigma: per-row tangent scale.
void layer_bwd(dpk_trainer* t, const LayerOff& L, int M, const double* X, const double* Xd, const double* A,
               const double* Zd, const double* sigma, const double* Yb, const double* Ydb, double* Zb, double* Zdb,
               double* H, double* Xb, double* Xdb, bool wgrad, hipStream_t s)
{
    const bool tan = Ydb != nullptr;
    if (wgrad) {
        // pre-activation adjoints with the bias and w_hat gradients, then the weight gradient
        tr_adj_sum(M, L.nout, A, tan ? Zd : nullptr, sigma, Yb, Ydb, t->theta.p + L.wh, Zb, tan ? Zdb : nullptr,
                   t->grad.p + L.b, t->grad.p + L.wh, s);
        tr_wgrad(M, L.nout, L.nin, X, Zb, tan ? Xd : nullptr, tan ? Zdb : nullptr, sigma, t->grad.p + L.W, s);
    } else {
        tr_adj_elem(M, L.nout, A, tan ? Zd : nullptr, sigma, Yb, Ydb, t->theta.p + L.wh, Zb, tan ? Zdb : nullptr, H, s);
    }
    if (Xb) {
        TrGemm g;
        std::memset(&g, 0, sizeof(g));
        g.M = M;
        g.N = L.nin;
        g.K = L.nout;
        g.transB = 1;
        g.mode = TR_BWD;
        g.NS = L.nout;
        g.A = Zb;
        g.A2 = tan ? Zdb : nullptr;
        g.W = t->theta.p + L.W;
        g.S = Yb;
        g.S2 = Ydb;
        g.C = Xb;
        g.C2 = Xdb;
        tr_gemm(g, s);
    }
}

int frame(dpk_trainer* t, int64_t natoms, const double* coord, const int32_t* atype, const double* box,
          const dpk_loss_spec* spec, double weight, double* loss, double* energy, double* force, double* virial)
{
    FrameGeom fg;
    int rc = frame_geometry(t->geo, natoms, coord, atype, box, &fg);
    if (rc) return rc;
    hipStream_t s = fg.stream;
    const int n = fg.n, nt = t->nt, nc = t->nc;
    // pair list grouped by net, then atom, then slot
    std::vector<int> nnei((size_t)n * nt), itype(n), toff(nt + 1, 0);
    TRCHK(hipMemcpyAsync(nnei.data(), fg.nnei, sizeof(int) * nnei.size(), hipMemcpyDeviceToHost, s));
    TRCHK(hipMemcpyAsync(itype.data(), fg.itype, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    TRCHK(hipStreamSynchronize(s));
    for (int a = 0; a < n; ++a) toff[itype[a] + 1]++;
    for (int ty = 0; ty < nt; ++ty) toff[ty + 1] += toff[ty];
    std::vector<int> pa, ps, apo((size_t)n * nt, 0), q0(t->nets), q1(t->nets);
    const bool tos = t->desc.type_one_side != 0;
    for (int e = 0; e < t->nets; ++e) {
        q0[e] = (int)pa.size();
        for (int a = 0; a < n; ++a)
            for (int tj = 0; tj < nt; ++tj) {
                const int net = tos ? tj : itype[a] * nt + tj;
                if (net != e) continue;
                apo[(size_t)a * nt + tj] = (int)pa.size();
                for (int k = 0; k < nnei[(size_t)a * nt + tj]; ++k) {
                    pa.push_back(a);
                    ps.push_back(fg.off[tj] + k);
                }
            }
        q1[e] = (int)pa.size();
    }
    const int P = (int)pa.size();
    const size_t Pz = std::max(P, 1), Nz = n;
    // workspace
    TRCHK(t->pa.ensure(Pz));
    TRCHK(t->ps.ensure(Pz));
    TRCHK(t->apo.ensure((size_t)n * nt));
    for (DBuf* b : {&t->R, &t->Rd}) TRCHK(b->ensure(4 * Pz));
    for (DBuf* b : {&t->X0, &t->ones, &t->sigma}) TRCHK(b->ensure(Pz));
    const int ew[3] = {E0, E1, E2};
    for (int l = 0; l < 3; ++l)
        for (DBuf* b : {&t->eA[l], &t->eZd[l], &t->eY[l], &t->eYd[l]}) TRCHK(b->ensure(ew[l] * Pz));
    for (DBuf* b : {&t->yb[0], &t->yb[1], &t->xb[0], &t->xb[1], &t->zb, &t->zdb, &t->hb}) TRCHK(b->ensure(E2 * Pz));
    for (DBuf* b : {&t->T, &t->Td, &t->Tb, &t->Tdb}) TRCHK(b->ensure(E2 * 4 * Nz));
    for (DBuf* b : {&t->D, &t->Dd, &t->Db, &t->Ddb}) TRCHK(b->ensure((size_t)DD * Nz));
    for (int l = 0; l < 3; ++l)
        for (DBuf* b : {&t->fA[l], &t->fZd[l], &t->fY[l], &t->fYd[l]}) TRCHK(b->ensure((size_t)FW * Nz));
    for (DBuf* b : {&t->fyb[0], &t->fyb[1], &t->fydb[0], &t->fydb[1], &t->fzb, &t->fzdb, &t->fhb})
        TRCHK(b->ensure((size_t)FW * Nz));
    TRCHK(t->Ei.ensure(Nz));
    TRCHK(t->F.ensure(3 * Nz));
    TRCHK(t->vdir.ensure(3 * Nz));
    TRCHK(t->vir.ensure(9));
    TRCHK(t->sums.ensure(2 * MAXT));
    TRCHK(t->csum.ensure(2 * FW));
    if (P > 0) {
        TRCHK(hipMemcpyAsync(t->pa.p, pa.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
        TRCHK(hipMemcpyAsync(t->ps.p, ps.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
    }
    TRCHK(hipMemcpyAsync(t->apo.p, apo.data(), sizeof(int) * apo.size(), hipMemcpyHostToDevice, s));

    const double inv_nc = 1.0 / nc;
    TrEnv env;
    std::memset(&env, 0, sizeof(env));
    env.P = P;
    env.nc = nc;
    env.pa = t->pa.p;
    env.ps = t->ps.p;
    env.nl_j = fg.nl_j;
    env.perm = fg.perm;
    env.nl_r = fg.nl_r;
    env.rs = t->desc.rcut_smth;
    env.rc = t->desc.rcut;
    env.R = t->R.p;
    env.X0 = t->X0.p;
    env.ones = t->ones.p;
    env.sigma = t->sigma.p;
    env.Rd = t->Rd.p;

    // ------------------------------------------------------------------ 3. inference
    tr_env(env, s);
    for (int e = 0; e < t->nets; ++e) {
        const int M = q1[e] - q0[e];
        if (M == 0) continue;
        const int64_t r0 = q0[e];
        const double* X = t->X0.p + r0;
        const double* Xd = t->ones.p + r0;
        for (int l = 0; l < 3; ++l) {
            const int w = ew[l];
            layer_fwd(t, t->emb[(size_t)e * 3 + l], M, X, Xd, t->eA[l].p + r0 * w, t->eY[l].p + r0 * w,
                      t->eZd[l].p + r0 * w, t->eYd[l].p + r0 * w, s);
            X = t->eY[l].p + r0 * w;
            Xd = t->eYd[l].p + r0 * w;
        }
    }
    TrContract con;
    std::memset(&con, 0, sizeof(con));
    con.n = n;
    con.nt = nt;
    con.inv_nc = inv_nc;
    con.apo = t->apo.p;
    con.nnei = fg.nnei;
    con.G = t->eY[2].p;
    con.Gd = t->eYd[2].p;
    con.R = t->R.p;
    con.Rd = t->Rd.p;
    con.sigma = t->sigma.p;
    con.T = t->T.p;
    con.D = t->D.p;
    tr_contract(con, s);
    TRCHK(hipMemsetAsync(t->sums.p, 0, sizeof(double) * 2 * MAXT, s));
    for (int ty = 0; ty < nt; ++ty) {
        const int M = toff[ty + 1] - toff[ty];
        if (M == 0) continue;
        const int64_t r0 = toff[ty];
        const double* X = t->D.p + r0 * DD;
        for (int l = 0; l < 3; ++l) {
            layer_fwd(t, t->fit[(size_t)ty * 4 + l], M, X, nullptr, t->fA[l].p + r0 * FW, t->fY[l].p + r0 * FW,
                      nullptr, nullptr, s);
            X = t->fY[l].p + r0 * FW;
        }
        const LayerOff& Lo = t->fit[(size_t)ty * 4 + 3];
        tr_fit_out(M, X, nullptr, t->theta.p + Lo.W, t->theta.p + Lo.b, t->theta.p + Lo.wh, 1.0, t->Ei.p + r0,
                   t->sums.p + 2 * ty, t->fyb[0].p + r0 * FW, nullptr, s);
        // input adjoint dE/dD (no tangent, no weight gradient)
        const double* Yb = t->fyb[0].p + r0 * FW;
        for (int l = 2; l >= 0; --l) {
            const LayerOff& L = t->fit[(size_t)ty * 4 + l];
            double* Xb = l == 0 ? t->Db.p + r0 * DD : t->fyb[(3 - l) & 1].p + r0 * FW;
            layer_bwd(t, L, M, nullptr, nullptr, t->fA[l].p + r0 * FW, nullptr, nullptr, Yb, nullptr,
                      t->fzb.p + r0 * FW, nullptr, t->fhb.p + r0 * FW, Xb, nullptr, false, s);
            Yb = Xb;
        }
    }
    tr_dT(n, t->T.p, nullptr, t->Db.p, nullptr, t->Tb.p, nullptr, s);
    TRCHK(hipMemsetAsync(t->F.p, 0, sizeof(double) * 3 * n, s));
    TRCHK(hipMemsetAsync(t->vir.p, 0, sizeof(double) * 9, s));
    TrPairForce pf;
    std::memset(&pf, 0, sizeof(pf));
    pf.P = P;
    pf.nc = nc;
    pf.inv_nc = inv_nc;
    pf.rs = t->desc.rcut_smth;
    pf.rc = t->desc.rcut;
    pf.pa = t->pa.p;
    pf.ps = t->ps.p;
    pf.nl_j = fg.nl_j;
    pf.perm = fg.perm;
    pf.nl_r = fg.nl_r;
    pf.R = t->R.p;
    pf.G = t->eY[2].p;
    pf.Gd = t->eYd[2].p;
    pf.dT = t->Tb.p;
    pf.F = t->F.p;
    pf.vir = t->vir.p;
    tr_pair_force(pf, s);
    std::vector<double> hEi(n), hF(3 * (size_t)n), hV(9);
    TRCHK(hipMemcpyAsync(hEi.data(), t->Ei.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    TRCHK(hipMemcpyAsync(hF.data(), t->F.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
    TRCHK(hipMemcpyAsync(hV.data(), t->vir.p, sizeof(double) * 9, hipMemcpyDeviceToHost, s));
    TRCHK(hipStreamSynchronize(s));
    double E = 0.0;
    for (int a = 0; a < n; ++a) E += hEi[a];
    if (energy) *energy = E;
    if (force) std::memcpy(force, hF.data(), sizeof(double) * 3 * n);
    if (virial) std::memcpy(virial, hV.data(), sizeof(double) * 9);

    // ------------------------------------------------------------------ 4. loss and direction
    const double N = (double)n;
    double LE = 0.0, LF = 0.0, LV = 0.0, cE = 0.0, CV[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<double> vd(3 * (size_t)n, 0.0);
    if (spec->energy) {
        const double dE = E - *spec->energy;
        LE = dE * dE / N;
        cE = 2.0 * spec->pe * dE / N * weight;
    }
    if (spec->force) {
        for (int64_t k = 0; k < n; ++k) {
            const double q = spec->atom_pref ? spec->atom_pref[k] : 1.0;
            for (int c = 0; c < 3; ++c) {
                const double d = hF[3 * k + c] - spec->force[3 * k + c];
                LF += q * d * d;
                vd[3 * k + c] = -2.0 * spec->pf * q * d / (3.0 * N) * weight;
            }
        }
        LF /= 3.0 * N;
    }
    if (spec->virial) {
        for (int k = 0; k < 9; ++k) {
            const double d = hV[k] - spec->virial[k];
            LV += d * d;
            CV[k] = -2.0 * spec->pv * d / (9.0 * N) * weight;
        }
        LV /= 9.0 * N;
    }
    if (loss) {
        loss[0] = spec->pe * LE + spec->pf * LF + spec->pv * LV;
        loss[1] = LE;
        loss[2] = LF;
        loss[3] = LV;
    }

    // ------------------------------------------------------------------ 5. training pass
    TRCHK(hipMemcpyAsync(t->vdir.p, vd.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    env.vdir = t->vdir.p;
    std::memcpy(env.CV, CV, sizeof(CV));
    tr_env(env, s);
    con.Td = t->Td.p;
    con.Dd = t->Dd.p;
    tr_contract(con, s);
    TRCHK(hipMemsetAsync(t->sums.p, 0, sizeof(double) * 2 * MAXT, s));
    for (int ty = 0; ty < nt; ++ty) {
        const int M = toff[ty + 1] - toff[ty];
        if (M == 0) continue;
        const int64_t r0 = toff[ty];
        const double* X = t->D.p + r0 * DD;
        const double* Xd = t->Dd.p + r0 * DD;
        for (int l = 0; l < 3; ++l) {
            layer_fwd(t, t->fit[(size_t)ty * 4 + l], M, X, Xd, t->fA[l].p + r0 * FW, t->fY[l].p + r0 * FW,
                      t->fZd[l].p + r0 * FW, t->fYd[l].p + r0 * FW, s);
            X = t->fY[l].p + r0 * FW;
            Xd = t->fYd[l].p + r0 * FW;
        }
        const LayerOff& Lo = t->fit[(size_t)ty * 4 + 3];
        tr_fit_out(M, X, Xd, t->theta.p + Lo.W, t->theta.p + Lo.b, t->theta.p + Lo.wh, cE, t->Ei.p + r0,
                   t->sums.p + 2 * ty, t->fyb[0].p + r0 * FW, t->fydb[0].p + r0 * FW, s);
        TRCHK(hipMemsetAsync(t->csum.p, 0, sizeof(double) * 2 * FW, s));
        tr_colsum(M, FW, X, t->csum.p, Xd, t->csum.p + FW, s);
        tr_out_grad(M, t->csum.p, t->csum.p + FW, t->sums.p + 2 * ty, t->theta.p + Lo.wh, cE, t->grad.p + Lo.W,
                    t->grad.p + Lo.b, t->grad.p + Lo.wh, s);
        const double* Yb = t->fyb[0].p + r0 * FW;
        const double* Ydb = t->fydb[0].p + r0 * FW;
        for (int l = 2; l >= 0; --l) {
            const LayerOff& L = t->fit[(size_t)ty * 4 + l];
            const double* Xl = l == 0 ? t->D.p + r0 * DD : t->fY[l - 1].p + r0 * FW;
            const double* Xdl = l == 0 ? t->Dd.p + r0 * DD : t->fYd[l - 1].p + r0 * FW;
            double* Xb = l == 0 ? t->Db.p + r0 * DD : t->fyb[(3 - l) & 1].p + r0 * FW;
            double* Xdb = l == 0 ? t->Ddb.p + r0 * DD : t->fydb[(3 - l) & 1].p + r0 * FW;
            layer_bwd(t, L, M, Xl, Xdl, t->fA[l].p + r0 * FW, t->fZd[l].p + r0 * FW, nullptr, Yb, Ydb,
                      t->fzb.p + r0 * FW, t->fzdb.p + r0 * FW, t->fhb.p + r0 * FW, Xb, Xdb, true, s);
            Yb = Xb;
            Ydb = Xdb;
        }
    }
    tr_dT(n, t->T.p, t->Td.p, t->Db.p, t->Ddb.p, t->Tb.p, t->Tdb.p, s);
    tr_pair_adj(P, inv_nc, t->pa.p, t->Tb.p, t->Tdb.p, t->R.p, t->Rd.p, t->yb[0].p, t->yb[1].p, s);
    for (int e = 0; e < t->nets; ++e) {
        const int M = q1[e] - q0[e];
        if (M == 0) continue;
        const int64_t r0 = q0[e];
        // adjoints of layer l's output: layer 3 from the pair adjoint (yb), then alternating
        const double* Yb = t->yb[0].p + r0 * E2;
        const double* Ydb = t->yb[1].p + r0 * E2;
        for (int l = 2; l >= 0; --l) {
            const LayerOff& L = t->emb[(size_t)e * 3 + l];
            const int w = ew[l];
            const double* Xl = l == 0 ? t->X0.p + r0 : t->eY[l - 1].p + r0 * ew[l - 1];
            const double* Xdl = l == 0 ? t->ones.p + r0 : t->eYd[l - 1].p + r0 * ew[l - 1];
            // (each net's rows keep to their own slab of E2 values per row in every buffer, so the
            // adjoints of the later nets, written before this loop, are never overwritten)
            double* Xb = l == 0 ? nullptr : (l == 2 ? t->xb[0].p : t->yb[0].p) + r0 * E2;
            double* Xdb = l == 0 ? nullptr : (l == 2 ? t->xb[1].p : t->yb[1].p) + r0 * E2;
            layer_bwd(t, L, M, Xl, Xdl, t->eA[l].p + r0 * w, t->eZd[l].p + r0 * w, t->sigma.p + r0, Yb, Ydb,
                      t->zb.p + r0 * w, t->zdb.p + r0 * w, t->hb.p + r0 * w, Xb, Xdb, true, s);
            Yb = Xb;
            Ydb = Xdb;
        }
    }
    TRCHK(hipGetLastError());
    TRCHK(hipStreamSynchronize(s));
    return DPK_OK;
}

}  // namespace

extern "C" {

int dpk_trainer_create(const dpk_model* m, int device, dpk_trainer** out)
{
    if (!m || !out) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    dpk_model_desc d;
    int rc = dpk_model_describe(m, &d, nullptr, nullptr, nullptr);
    if (rc) return rc;
    if (d.descriptor != DPK_SE_E2_A) return set_error(DPK_E_UNIMPLEMENTED, "training covers se_e2_a models");
    const int64_t np = dpk_model_param_count(&d);
    std::vector<double> p(np);
    if ((rc = dpk_model_describe(m, nullptr, p.data(), nullptr, nullptr))) return rc;
    auto* t = new dpk_trainer;
    t->desc = d;
    t->device = device;
    t->nt = d.ntypes;
    t->nets = d.type_one_side ? d.ntypes : d.ntypes * d.ntypes;
    t->nc = 0;
    for (int ty = 0; ty < d.ntypes; ++ty) t->nc += d.sel[ty];
    t->np = np;
    layer_offsets(t);
    if ((rc = dpk_model_create(&d, p.data(), np, &t->model)) ||
        (rc = dpk_ctx_create(t->model, device, DPK_FP64, 0, 0, &t->geo))) {
        delete t;
        return rc;
    }
    if (t->theta.ensure(np) != hipSuccess || t->grad.ensure(np) != hipSuccess || t->mom1.ensure(np) != hipSuccess ||
        t->mom2.ensure(np) != hipSuccess) {
        hipGetLastError();
        delete t;
        return set_error(DPK_E_OOM, "hipMalloc of the trainer's parameter buffers failed");
    }
    if (hipMemcpy(t->theta.p, p.data(), sizeof(double) * np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(t->grad.p, 0, sizeof(double) * np) != hipSuccess ||
        hipMemset(t->mom1.p, 0, sizeof(double) * np) != hipSuccess ||
        hipMemset(t->mom2.p, 0, sizeof(double) * np) != hipSuccess) {
        delete t;
        return set_error(DPK_E_DEVICE, "copy of the parameters to the device failed");
    }
    *out = t;
    return DPK_OK;
}

void dpk_trainer_free(dpk_trainer* t)
{
    if (!t) return;
    hipSetDevice(t->device);
    hipDeviceSynchronize();
    delete t;
}

int dpk_trainer_accumulate(dpk_trainer* t, int64_t natoms, const double* coord, const int32_t* atype,
                           const double* box, const dpk_loss_spec* spec, double weight, double* loss,
                           double* energy, double* force, double* virial)
{
    if (!t || !coord || !atype || !spec) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    TRCHK(hipSetDevice(t->device));
    return frame(t, natoms, coord, atype, box, spec, weight, loss, energy, force, virial);
}

int dpk_trainer_gradient(dpk_trainer* t, double* grad)
{
    if (!t || !grad) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    TRCHK(hipSetDevice(t->device));
    TRCHK(hipDeviceSynchronize());
    TRCHK(hipMemcpy(grad, t->grad.p, sizeof(double) * t->np, hipMemcpyDeviceToHost));
    return DPK_OK;
}

int dpk_trainer_zero_grad(dpk_trainer* t)
{
    if (!t) return set_error(DPK_E_INVALID_ARG, "NULL trainer");
    TRCHK(hipSetDevice(t->device));
    TRCHK(hipDeviceSynchronize());
    TRCHK(hipMemset(t->grad.p, 0, sizeof(double) * t->np));
    return DPK_OK;
}

int dpk_trainer_adam_step(dpk_trainer* t, double lr, double beta1, double beta2, double eps)
{
    if (!t) return set_error(DPK_E_INVALID_ARG, "NULL trainer");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return set_error(DPK_E_INVALID_ARG, "need 0 <= beta1, beta2 < 1 and eps > 0");
    TRCHK(hipSetDevice(t->device));
    t->step += 1;
    const double c1 = 1.0 - std::pow(beta1, (double)t->step), c2 = 1.0 - std::pow(beta2, (double)t->step);
    tr_adam(t->np, t->theta.p, t->grad.p, t->mom1.p, t->mom2.p, lr, beta1, beta2, eps, c1, c2, nullptr);
    TRCHK(hipGetLastError());
    TRCHK(hipDeviceSynchronize());
    return DPK_OK;
}

int dpk_trainer_params(dpk_trainer* t, double* params)
{
    if (!t || !params) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    TRCHK(hipSetDevice(t->device));
    TRCHK(hipDeviceSynchronize());
    TRCHK(hipMemcpy(params, t->theta.p, sizeof(double) * t->np, hipMemcpyDeviceToHost));
    return DPK_OK;
}

int dpk_trainer_set_params(dpk_trainer* t, const double* params)
{
    if (!t || !params) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    TRCHK(hipSetDevice(t->device));
    TRCHK(hipDeviceSynchronize());
    TRCHK(hipMemcpy(t->theta.p, params, sizeof(double) * t->np, hipMemcpyHostToDevice));
    return DPK_OK;
}

double dpk_learning_rate(double lr0, double lr_stop, int64_t step, int64_t stop_steps, int64_t decay_steps)
{
    if (stop_steps <= 0 || decay_steps <= 0 || step < 0) return lr0;
    const double r = std::pow(lr_stop / lr0, (double)decay_steps / (double)stop_steps);
    return lr0 * std::pow(r, (double)(step / decay_steps));
}

double dpk_loss_prefactor(double p_start, double p_limit, double lr, double lr0)
{
    return p_limit * (1.0 - lr / lr0) + p_start * lr / lr0;
}

}  // extern "C"
