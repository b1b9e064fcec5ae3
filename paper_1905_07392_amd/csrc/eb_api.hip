// eb_api.hip -- host orchestration and the C ABI declared in include/eb.h.
//
// The caller's device workspace is carved into every array the step needs; the library never
// allocates device memory.  Solvers keep their vectors on the device and read back one or two
// scalars per Krylov iteration (dot products and max-norms) for the stopping test and the
// Krylov coefficients.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "eb_internal.hpp"

namespace {

thread_local std::string g_err;

int set_err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

thread_local hipError_t g_hip_first = hipSuccess;
thread_local const char* g_hip_first_what = "";

// reports (and clears) the first failed runtime call noted since the last check, else the
// last kernel-launch error
int hip_check(const char* where) {
    hipError_t e = hipGetLastError();
    if (g_hip_first != hipSuccess) {
        hipError_t f = g_hip_first;
        g_hip_first = hipSuccess;
        return set_err(EB_EHIP, "%s: %s in %s", where, hipGetErrorString(f), g_hip_first_what);
    }
    if (e != hipSuccess) return set_err(EB_EHIP, "%s: %s", where, hipGetErrorString(e));
    return EB_OK;
}

struct Carver {
    char* base;
    size_t used;
    bool dry;
    template <typename T>
    T* take(size_t count) {
        size_t bytes = count * sizeof(T);
        size_t off = (used + 255) & ~size_t(255);
        used = off + bytes;
        return dry ? nullptr : reinterpret_cast<T*>(base + off);
    }
};

// rejects an unknown law, or parameters its formula cannot use (Table rheology)
int check_rheology(const eb_rheology& r) {
    if (r.law < EB_LAW_NEWTONIAN || r.law > EB_LAW_SOUZA_MENDES_DUTRA)
        return set_err(EB_EINVAL, "unknown viscosity law %d", r.law);
    bool pl = r.law >= EB_LAW_POWER;
    if (pl && !(r.kappa > 0.0 && r.n > 0.0))
        return set_err(EB_EINVAL, "the power-law laws need kappa > 0 and n > 0");
    bool uses_eps = r.law == EB_LAW_BINGHAM_REG || r.law == EB_LAW_PAPANASTASIOU ||
                    r.law == EB_LAW_HERSCHEL_BULKLEY || (pl && r.n < 1.0);
    if (uses_eps && !(r.eps > 0.0)) return set_err(EB_EINVAL, "this viscosity law needs eps > 0");
    if (r.law == EB_LAW_SOUZA_MENDES_DUTRA && !(r.eta0 > 0.0))
        return set_err(EB_EINVAL, "the Souza Mendes-Dutra law needs eta0 > 0");
    return EB_OK;
}

}  // namespace

void hip_note(hipError_t e, const char* what) {
    if (e != hipSuccess && g_hip_first == hipSuccess) {
        g_hip_first = e;
        g_hip_first_what = what;
    }
}

bool hip_failed() { return g_hip_first != hipSuccess; }

namespace {
constexpr int NSLOT = 8;
}

// one read-back of a solve's progress: its (state, count) slot
struct PollWord {
    int st[2];
};

struct eb_ctx {
    eb_box box;
    eb_body body;
    GridV grid;
    BodyV bodyv;
    long N;
    int ncut, ncut_max, nlev, nfallback;
    GeomV g;
    Level lev[EB_MAXLEV];
    hipStream_t s;
    // geometry
    uint8_t* flag;
    double* alpha;
    double* ap[3];
    int *cutid, *cut, *sidx, *nfb, *blockcount, *errdev;
    uint8_t* near;
    double *nrm, *aeb, *bc, *delta, *dd, *sw, *psi_nodes;
    // reductions
    double *part, *red;
    // work arrays
    double *G9, *gw, *eta0, *eta1, *eb0, *eb1, *C0, *V0, *C1, *V1, *DC, *DH, *rS, *rdD, *psi,
        *gp, *u1, *p1, *div, *phi, *pb;
    double* f[3];
    double* kv[10];
    double* pk[5];
    int built_sys;    // operator currently held by the levels (-1 none)
    bool built_mixed;
    // device Krylov scalars, per-solve (state, count) slots, per-solve divergence norms
    double* ks;
    int* kst;
    double* divs;
    // pinned host words for the lagged convergence poll (two buffers), and their events
    struct PollWord* pin;
    hipEvent_t ev[2];
    // the library's own stream (fenced to the caller's with two events) and the captured
    // Krylov iterations replayed on it
    hipStream_t own;
    hipEvent_t fence_in, fence_out;
    int graphs_on;
    struct GraphCache* graphs;
    // adjoint: transposed wall stencil and reverse-sweep arrays
    int *wt_map, *wt_ptr, *wt_ent;
    WallT wt;
    double *Gb, *ubm, *lam, *ehb, *ebhb, *rX, *rY, *gwb;
    double* tbs;  // the per-cell yield-stress adjoint of one reverse call, before it is handed out
    // nodal projection: boundary flux, diagonal of L and mask of the unknowns (per geometry),
    // the step's nodal pressure, the wall pressures of the drag
    double *nd_bflux, *nd_dg, *pn1, *peb;
    uint8_t* nd_mask;
    double* ufb[3];
    LRV lr;
    // mixed precision: iterations a solve ran with the FP32 V-cycle before it continued with
    // the FP64 one (per slot, in the slot's count units), and such switches since the last
    // reset (host side)
    int slot_off[NSLOT];
    int fp64_fallbacks;
    // branch record/replay of the derived quantities (eb_ctx_set_switches): mode, the caller's
    // buffer and the offset of the next evaluation's record in it
    int sw_mode;
    uint8_t* sw_buf;
    size_t sw_bytes, sw_cur;
};

namespace {

int level_count(const int n[3]) {
    int nl = 1;
    int m[3] = {n[0], n[1], n[2]};
    while (nl < EB_MAXLEV && m[0] % 4 == 0 && m[1] % 4 == 0 && m[2] % 4 == 0) {
        for (int d = 0; d < 3; d++) m[d] /= 2;
        nl++;
    }
    return nl;
}

long ncut_bound(const int n[3]) {
    long N = (long)n[0] * n[1] * n[2];
    long b = 24L * ((long)n[0] * n[1] + (long)n[1] * n[2] + (long)n[0] * n[2]);
    return b < N ? b : N;
}

// assigns every device array of the context; returns the bytes used
size_t carve(eb_ctx* c, char* base, bool dry) {
    Carver cv{base, 0, dry};
    GridV g = c->grid;
    long N = c->N;
    long M = c->ncut_max > 0 ? c->ncut_max : 1;
    long nn = (long)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1);
    c->psi_nodes = cv.take<double>(nn);
    c->flag = cv.take<uint8_t>(N);
    c->alpha = cv.take<double>(N);
    for (int d = 0; d < 3; d++) c->ap[d] = cv.take<double>(face_count(g, d));
    c->cutid = cv.take<int>(N);
    c->near = cv.take<uint8_t>(N);
    c->cut = cv.take<int>(M);
    c->nrm = cv.take<double>(3 * M);
    c->aeb = cv.take<double>(M);
    c->bc = cv.take<double>(3 * M);
    c->delta = cv.take<double>(M);
    c->dd = cv.take<double>(2 * M);
    c->sidx = cv.take<int>(18 * M);
    c->sw = cv.take<double>(18 * M);
    c->nfb = cv.take<int>(M);
    c->blockcount = cv.take<int>(grid_for(N) + 1);
    c->errdev = cv.take<int>(1);
    c->part = cv.take<double>(4 * 1024);
    c->red = cv.take<double>(64);
    c->ks = cv.take<double>(KS_COUNT);
    c->kst = cv.take<int>(3 * NSLOT);  // (state, count) per slot, then the iteration counters
    c->divs = cv.take<double>(NSLOT);
    char* pack = cv.take<char>(MG_PACK_BYTES);
    // levels
    int m[3] = {g.n[0], g.n[1], g.n[2]};
    double h = g.h;
    for (int l = 0; l < c->nlev; l++) {
        Level& L = c->lev[l];
        for (int d = 0; d < 3; d++) {
            L.grid.n[d] = m[d];
            L.grid.per[d] = g.per[d];
        }
        L.grid.h = h;
        L.N = (long)m[0] * m[1] * m[2];
        if (l == 0) {
            L.alpha = c->alpha;
            for (int d = 0; d < 3; d++) L.ap[d] = c->ap[d];
        } else {
            L.alpha = cv.take<double>(L.N);
            for (int d = 0; d < 3; d++) L.ap[d] = cv.take<double>(face_count(L.grid, d));
        }
        L.pack = pack;
        L.mask = cv.take<uint8_t>(L.N);
        for (int d = 0; d < 3; d++) L.K[d] = cv.take<double>(face_count(L.grid, d));
        L.S = cv.take<double>(L.N);
        L.D = cv.take<double>(L.N);
        for (int d = 0; d < 3; d++) L.Kf[d] = cv.take<float>(face_count(L.grid, d));
        L.Df = cv.take<float>(L.N);
        L.x = cv.take<double>(3 * L.N);
        L.b = cv.take<double>(3 * L.N);
        L.xf = cv.take<float>(3 * L.N);
        L.bf = cv.take<float>(3 * L.N);
        if (l == 0) {
            L.etaf = cv.take<float>(L.N);
            L.etacs = cv.take<double>(L.N);
            L.etafcs = cv.take<float>(L.N);
            L.flagcs = cv.take<uint8_t>(L.N);
        }
        for (int d = 0; d < 3; d++) m[d] /= 2;
        h *= 2.0;
    }
    c->G9 = cv.take<double>(9 * N);
    c->gw = cv.take<double>(3 * M);
    c->eta0 = cv.take<double>(N);
    c->eta1 = cv.take<double>(N);
    c->eb0 = cv.take<double>(M);
    c->eb1 = cv.take<double>(M);
    c->C0 = cv.take<double>(3 * N);
    c->V0 = cv.take<double>(3 * N);
    c->C1 = cv.take<double>(3 * N);
    c->V1 = cv.take<double>(3 * N);
    c->DC = cv.take<double>(3 * N);
    c->DH = cv.take<double>(3 * M);
    c->rS = cv.take<double>(M);
    c->rdD = cv.take<double>(3 * M);
    c->psi = cv.take<double>(3 * N);
    c->gp = cv.take<double>(3 * N);
    c->u1 = cv.take<double>(3 * N);
    c->p1 = cv.take<double>(N);
    c->div = cv.take<double>(N);
    c->phi = cv.take<double>(N);
    c->pb = cv.take<double>(N);
    for (int d = 0; d < 3; d++) c->f[d] = cv.take<double>(face_count(g, d));
    for (int t = 0; t < 10; t++) c->kv[t] = cv.take<double>(3 * N);
    for (int t = 0; t < 5; t++) c->pk[t] = cv.take<double>(N);
    c->wt_map = cv.take<int>(N);
    c->wt_ptr = cv.take<int>(18 * M + 1);
    c->wt_ent = cv.take<int>(18 * M);
    c->Gb = cv.take<double>(9 * N);
    c->ubm = cv.take<double>(3 * N);
    c->lam = cv.take<double>(3 * N);
    c->ehb = cv.take<double>(N);
    c->ebhb = cv.take<double>(M);
    c->rX = cv.take<double>(3 * M);
    c->rY = cv.take<double>(3 * M);
    c->gwb = cv.take<double>(3 * M);
    c->tbs = cv.take<double>(N);
    long NM = (long)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1);
    c->nd_bflux = cv.take<double>(NM);
    c->nd_dg = cv.take<double>(NM);
    c->pn1 = cv.take<double>(NM);
    c->nd_mask = cv.take<uint8_t>(NM);
    c->peb = cv.take<double>(M);
    for (int d = 0; d < 3; d++) {
        c->ufb[d] = cv.take<double>(face_count(g, d));
        c->lr.L[d] = cv.take<double>(3 * face_count(g, d));
        c->lr.R[d] = cv.take<double>(3 * face_count(g, d));
    }
    return cv.used + 256;
}

// Intermediate fields of one step kept for the reverse sweep (a caller-owned device buffer).
struct TapeV {
    double* ufm[3];  // projected face velocities of the predictor
    double* uf1[3];  // and of the corrector
    double *em, *ea;   // viscosity of the predictor and averaged (corrector) operators
    double *ebm, *eba; // their wall viscosities
    double *us1, *u1, *us2;  // predictor solve, projected u*, corrector solve
};

size_t tape_carve(const eb_ctx* c, char* base, TapeV* t) {
    Carver cv{base, 0, base == nullptr};
    long N = c->N;
    long M = c->ncut > 0 ? c->ncut : 1;
    for (int d = 0; d < 3; d++) t->ufm[d] = cv.take<double>(face_count(c->grid, d));
    for (int d = 0; d < 3; d++) t->uf1[d] = cv.take<double>(face_count(c->grid, d));
    t->em = cv.take<double>(N);
    t->ea = cv.take<double>(N);
    t->ebm = cv.take<double>(M);
    t->eba = cv.take<double>(M);
    t->us1 = cv.take<double>(3 * N);
    t->u1 = cv.take<double>(3 * N);
    t->us2 = cv.take<double>(3 * N);
    return cv.used;
}

// transposed wall stencil, built on the host from the device stencil (once per geometry):
// entries sorted by (cell, flat position) so every gather sums in a fixed order
int build_wall_transpose(eb_ctx* c) {
    int nc = c->ncut;
    long N = c->N;
    std::vector<int> sidx((size_t)18 * nc);
    std::vector<int> map(N, -1);
    std::vector<int> ptr(1, 0), ent;
    if (nc > 0) {
        HIPN(hipMemcpy(sidx.data(), c->sidx, sidx.size() * sizeof(int), hipMemcpyDeviceToHost));
        std::vector<std::pair<int, int>> pairs;
        pairs.reserve(sidx.size());
        for (size_t e = 0; e < sidx.size(); e++)
            if (sidx[e] >= 0) pairs.emplace_back(sidx[e], (int)e);
        std::sort(pairs.begin(), pairs.end());
        ent.reserve(pairs.size());
        for (size_t t = 0; t < pairs.size(); t++) {
            if (t == 0 || pairs[t].first != pairs[t - 1].first) {
                if (t > 0) ptr.push_back((int)t);
                map[pairs[t].first] = (int)ptr.size() - 1;
            }
            ent.push_back(pairs[t].second);
        }
        ptr.push_back((int)pairs.size());
        if (pairs.empty()) ptr.assign(1, 0);
    }
    HIPN(hipMemcpy(c->wt_map, map.data(), N * sizeof(int), hipMemcpyHostToDevice));
    HIPN(hipMemcpy(c->wt_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!ent.empty())
        HIPN(hipMemcpy(c->wt_ent, ent.data(), ent.size() * sizeof(int), hipMemcpyHostToDevice));
    c->wt.map = c->wt_map;
    c->wt.ptr = c->wt_ptr;
    c->wt.ent = c->wt_ent;
    return hip_check("wall stencil transpose");
}

void rotation_zyx(const double e[3], double R[3][3]) {
    double ca = cos(e[0]), sa = sin(e[0]), cb = cos(e[1]), sb = sin(e[1]);
    double cc = cos(e[2]), sc = sin(e[2]);
    double Rz[3][3] = {{ca, -sa, 0}, {sa, ca, 0}, {0, 0, 1}};
    double Ry[3][3] = {{cb, 0, sb}, {0, 1, 0}, {-sb, 0, cb}};
    double Rx[3][3] = {{1, 0, 0}, {0, cc, -sc}, {0, sc, cc}};
    double T[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            T[a][b] = 0;
            for (int k = 0; k < 3; k++) T[a][b] += Rz[a][k] * Ry[k][b];
        }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            R[a][b] = 0;
            for (int k = 0; k < 3; k++) R[a][b] += T[a][k] * Rx[k][b];
        }
}

int init_ctx(eb_ctx* c, const eb_box* box, const eb_body* body) {
    if (!box || !body) return set_err(EB_EINVAL, "null box or body");
    for (int d = 0; d < 3; d++)
        if (box->n[d] < 2 || box->n[d] % 2)
            return set_err(EB_EINVAL, "n[%d]=%d must be an even number >= 2", d, box->n[d]);
    if (!(box->h > 0.0)) return set_err(EB_EINVAL, "h must be positive");
    // cell indices are taken apart with 32-bit arithmetic (multiply-high divisions of indices
    // below 2^31): far beyond what one GPU's memory holds anyway
    if ((long long)box->n[0] * box->n[1] * box->n[2] >= (1LL << 31))
        return set_err(EB_EINVAL, "a box holds fewer than 2^31 cells");
    if (body->kind < EB_BODY_NONE || body->kind > EB_BODY_CAVITY)
        return set_err(EB_EINVAL, "unknown body kind %d", body->kind);
    memset(c, 0, sizeof(*c));
    c->built_sys = -1;
    c->box = *box;
    c->body = *body;
    for (int d = 0; d < 3; d++) {
        c->grid.n[d] = box->n[d];
        c->grid.per[d] = box->periodic[d] ? 1 : 0;
    }
    c->grid.h = box->h;
    c->N = (long)box->n[0] * box->n[1] * box->n[2];
    c->ncut_max = (int)ncut_bound(box->n);
    c->nlev = level_count(box->n);
    BodyV& b = c->bodyv;
    b.kind = body->kind;
    for (int d = 0; d < 3; d++) {
        b.lo[d] = box->lo[d];
        b.c[d] = body->center[d];
        b.r[d] = (body->kind == EB_BODY_SPHERE || body->kind == EB_BODY_CYLINDER ||
                  body->kind == EB_BODY_CAVITY)
                     ? body->radii[0] : body->radii[d];
        b.pn[d] = body->plane_n[d];
    }
    b.zlo = body->zlo;
    b.zhi = body->zhi;
    b.pd = body->plane_d;
    if (body->kind == EB_BODY_ELLIPSOID) rotation_zyx(body->euler_zyx, b.R);
    else
        for (int a = 0; a < 3; a++)
            for (int e = 0; e < 3; e++) b.R[a][e] = a == e ? 1.0 : 0.0;
    return EB_OK;
}

void fill_geomv(eb_ctx* c) {
    GeomV& g = c->g;
    g.grid = c->grid;
    g.N = c->N;
    g.ncut = c->ncut;
    for (int f = 0; f < 6; f++)
        for (int m = 0; m < 3; m++) g.wall[f][m] = c->box.wall_u[f][m];
    for (int m = 0; m < 3; m++) g.ueb[m] = c->body.u_eb[m];
    g.flag = c->flag;
    g.alpha = c->alpha;
    for (int d = 0; d < 3; d++) g.ap[d] = c->ap[d];
    g.cutid = c->cutid;
    g.cut = c->cut;
    g.nrm = c->nrm;
    g.aeb = c->aeb;
    g.bc = c->bc;
    g.delta = c->delta;
    g.dd = c->dd;
    g.sidx = c->sidx;
    g.sw = c->sw;
    g.near = c->near;
}

// host copy of `n` reduced values
int fetch(eb_ctx* c, double* host, int n) {
    HIPN(hipMemcpyAsync(host, c->red, n * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPN(hipStreamSynchronize(c->s));
    return hip_check("read-back");
}

// Hands out the yield-stress adjoint tbs of one reverse call (tau0_c = tau0 theta_c):
// tau0b += tbs per cell, thetab += tau0 tbs (d loss / d theta_c), and *tau0bar (host) +=
// sum_c theta_c tbs_c (d loss / d tau0; theta null = 1), a fixed-order reduction.
int yield_adjoint_out(eb_ctx* c, double tau0, const double* theta, double* tau0b,
                      double* thetab, double* tau0bar) {
    long N = c->N;
    if (tau0b) vec_axpby(N, 1.0, c->tbs, 1.0, tau0b, c->s);
    if (thetab) vec_axpby(N, tau0, c->tbs, 1.0, thetab, c->s);
    if (tau0bar) {
        if (theta) {
            const double* a[4] = {theta, nullptr, nullptr, nullptr};
            const double* b[4] = {c->tbs, nullptr, nullptr, nullptr};
            red_dots(N, 1, a, b, c->part, c->red, c->s);
        } else {
            red_sum(N, 1, c->tbs, c->part, c->red, c->s);
        }
        double v = 0.0;
        if (int e = fetch(c, &v, 1)) return e;
        *tau0bar += v;
    }
    return EB_OK;
}

// ------------------------------------------------------------------------------------------
// solvers.  Krylov scalars and the convergence state live on the device (eb_krylov.hip): the
// host enqueues whole iterations and polls the state of the previous iteration while the
// current one runs, so the GPU never waits for the host.  Each solve reports into a state
// slot (state, count) that callers read once at the end.
// ------------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------------
// Krylov iterations as captured graphs.  An iteration launches a fixed sequence of kernels
// whose arguments depend only on the solve's configuration (buffers, coefficients, slot), so it
// is captured once per configuration and replayed with one launch.  The key holds every value
// baked into the captured kernels' arguments.
// ------------------------------------------------------------------------------------------
}  // namespace

struct GraphKey {
    int kind, slot, nc, mixed, nu1, nu2, nbottom, transposed;
    const void* p[6];
    double v[4];
};

struct GraphCache {
    std::vector<std::pair<GraphKey, hipGraphExec_t>> entries;
    ~GraphCache() {
        for (auto& e : entries)
            if (e.second) (void)hipGraphExecDestroy(e.second);
    }
};

namespace {

GraphKey make_key() {
    GraphKey k;
    memset(&k, 0, sizeof(k));  // padding too, so keys compare bytewise
    return k;
}

// runs one iteration body: replayed from the cache when graphs are on, captured on first use;
// if capture or instantiation fails the body runs eagerly from then on for that key
template <typename F>
void run_iteration(eb_ctx* c, const GraphKey& key, F&& body) {
    if (!c->graphs_on || !c->graphs) {
        body();
        return;
    }
    for (auto& e : c->graphs->entries)
        if (memcmp(&e.first, &key, sizeof(GraphKey)) == 0) {
            if (e.second) HIPN(hipGraphLaunch(e.second, c->s));
            else body();
            return;
        }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        body();
        if (hipStreamEndCapture(c->s, &graph) == hipSuccess && graph) {
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                exec = nullptr;
            (void)hipGraphDestroy(graph);
        }
    }
    (void)hipGetLastError();  // a failed capture leaves no sticky error; run eagerly instead
    c->graphs->entries.emplace_back(key, exec);
    if (exec) HIPN(hipGraphLaunch(exec, c->s));
    else body();
}

// work of a public call runs on the library's stream, ordered after the caller's prior work
// and before the caller's later work
struct StreamScope {
    eb_ctx* c;
    hipStream_t user;
    StreamScope(eb_ctx* ctx, void* stream) : c(ctx), user((hipStream_t)stream) {
        HIPN(hipEventRecord(c->fence_in, user));
        HIPN(hipStreamWaitEvent(c->own, c->fence_in, 0));
        c->s = c->own;
    }
    ~StreamScope() {
        HIPN(hipEventRecord(c->fence_out, c->own));
        HIPN(hipStreamWaitEvent(user, c->fence_out, 0));
        c->s = user;
    }
};

struct SolveCfg {
    bool mixed;
    int nu1, nu2, nbottom, max_iter;
};

SolveCfg cfg_of(const eb_step_opts* o) {
    SolveCfg k;
    k.mixed = o && o->precision == EB_MIXED;
    k.nu1 = o && o->nu1 >= 0 ? o->nu1 : 2;
    k.nu2 = o && o->nu2 >= 0 ? o->nu2 : 2;
    k.nbottom = o && o->nbottom > 0 ? o->nbottom : 16;
    k.max_iter = o && o->max_iter > 0 ? o->max_iter : 400;
    return k;
}

void vcyc(eb_ctx* c, int ncomp, const SolveCfg& k, const double* b, double* x, const int* gate) {
    mg_vcycle(c->lev, c->nlev, ncomp, k.mixed, b, x, k.nu1, k.nu2, k.nbottom, c->s, gate);
}

// lagged convergence test: enqueue the read-back of the slot's state after iteration it and
// wait for the one of iteration it-1 (already executed or about to be)
// (the state word: 0 while running)
int poll_done(eb_ctx* c, int slot, int it) {
    int b = it & 1;
    HIPN(hipMemcpyAsync(c->pin[b].st, c->kst + 2 * slot, 2 * sizeof(int), hipMemcpyDeviceToHost,
                   c->s));
    HIPN(hipEventRecord(c->ev[b], c->s));
    if (it < 2) return 0;
    int pb = (it - 1) & 1;
    HIPN(hipEventSynchronize(c->ev[pb]));
    if (hip_failed()) return 3;  // the runtime failed: stop; the entry point reports EB_EHIP
    return c->pin[pb].st[0];
}

// state word of `slot` once the stream has drained
int slot_state(eb_ctx* c, int slot) {
    int sl[2] = {0, 0};
    HIPN(hipMemcpyAsync(sl, c->kst + 2 * slot, 2 * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPN(hipStreamSynchronize(c->s));
    return sl[0];
}

// preconditioner applications made so far by the solve in `slot` (its device iteration
// counter: CG iterations; BiCGSTAB iterations, two applications each), stream drained
int slot_count_now(eb_ctx* c, int slot) {
    int n = 0;
    HIPN(hipMemcpyAsync(&n, c->kst + 2 * NSLOT + slot, sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPN(hipStreamSynchronize(c->s));
    return n;
}

// Mixed precision keeps the FP32 V-cycle as long as it works as a preconditioner, i.e. while
// the conditioning of the level operators times the FP32 unit roundoff stays well below one
// (high viscosity contrast, as in a nearly rigid plug next to a sheared layer, breaks this).
// A mixed solve is given up when its residual max-norm has not fallen tenfold within
// KS_STALL_W iterations (the device's stall test, which ends the solve with state 4), or when
// it has not converged within mixed_budget iterations; the caller then solves again from the
// same starting iterate with the FP64 V-cycle, so the result is the FP64 solve's.  The step's
// stats count such switches.

int mixed_budget(const SolveCfg& k) {
    int b = k.max_iter / 10 > 20 ? k.max_iter / 10 : 20;
    return b < k.max_iter ? b : k.max_iter;
}

// up to max_iter iterations of a solve whose state lives in `slot`; returns the final state
// (2 converged, 3 non-finite, 4 stalled (a watched solve), 0 iterations exhausted)
template <class Body>
int iterate(eb_ctx* c, const GraphKey& key, int slot, int max_iter, Body& body) {
    for (int it = 1; it <= max_iter; it++) {
        run_iteration(c, key, body);
        if (int s = poll_done(c, slot, it)) return s == 1 ? 2 : s;
    }
    return slot_state(c, slot);
}

// The preconditioned residual z minus its mean over open cells.  The Poisson system is singular
// (constants on the fluid are its null space) and the V-cycle's output carries a constant
// component, which in exact arithmetic only shifts the iterate by a constant (removed by the
// final normalisation) and changes no CG coefficient; in floating point, near the tolerance it
// dominates the search direction, whose A-product is then rounding noise times a huge step, and
// CG breaks down.  (KS_SUM, KS_CNT are free during the iterations.)
void cg_mean_free(eb_ctx* c, double* z, const int* gate) {
    red_sum_open(c->g, z, c->part, c->ks + KS_SUM, c->s, gate);
    op_shift_open(c->g, z, c->ks + KS_SUM, c->s, gate);
}

// preconditioned CG for M x = b on level 0 (operator already built), state in `slot`, from
// the iterate in x; ks[KS_RTOL] and ks[KS_SCALE] must be set.  Returns the final state.
int pcg(eb_ctx* c, const double* b, double* x, const SolveCfg& k, int slot) {
    long N = c->N;
    double *r = c->pk[0], *z = c->pk[1], *pd = c->pk[2], *q = c->pk[3];
    double* ks = c->ks;
    int* st = c->kst + 2 * slot;
    int* itc = c->kst + 2 * NSLOT + slot;
    const double* A1[4] = {nullptr, nullptr, nullptr, nullptr};
    const double* B1[4] = {nullptr, nullptr, nullptr, nullptr};
    mg_apply_level0(c->lev[0], 1, x, q, c->s);
    vec_sub_scaled(N, b, 1.0, q, r, c->s);
    red_maxabs(N, 1, b, c->part, ks + KS_BN, c->s);
    red_maxabs(N, 1, r, c->part, ks + KS_RN, c->s);
    ks_op(k.mixed ? KS_INIT_WATCH : KS_INIT, ks, st, itc, c->s);
    vcyc(c, 1, k, r, z, st);
    cg_mean_free(c, z, st);
    vec_copy(N, z, pd, c->s);
    A1[0] = r;
    B1[0] = z;
    red_dots(N, 1, A1, B1, c->part, ks + KS_RZ, c->s, st);
    GraphKey key = make_key();
    key.kind = 1;
    key.slot = slot;
    key.nc = 1;
    key.mixed = k.mixed;
    key.nu1 = k.nu1;
    key.nu2 = k.nu2;
    key.nbottom = k.nbottom;
    key.p[0] = x;
    key.v[0] = c->lev[0].beta;
    auto body = [&]() {
        const double* A[4] = {pd, nullptr, nullptr, nullptr};
        const double* B[4] = {q, nullptr, nullptr, nullptr};
        mg_apply_level0(c->lev[0], 1, pd, q, c->s, st);
        red_dots_op(N, 1, A, B, c->part, KS_PQ, KS_CG_ALPHA, ks, st, itc, c->s);
        ks_cg_xr_op(N, x, r, pd, q, c->part, ks, st, itc, c->s);
        vcyc(c, 1, k, r, z, st);
        cg_mean_free(c, z, st);
        A[0] = r;
        B[0] = z;
        red_dots_op(N, 1, A, B, c->part, KS_RZN, KS_CG_BETA, ks, st, itc, c->s);
        ks_cg_p(N, pd, z, ks, st, c->s);
    };
    return iterate(c, key, slot, k.max_iter, body);
}

// Poisson solve for the projections: M p = -(D w - mean), then p normalised to zero mean
void poisson_solve(eb_ctx* c, double beta, const double* div, double* p, const SolveCfg& k,
                   int slot) {
    mg_build_poisson(c->lev, c->nlev, c->g, beta, k.mixed, c->s);
    c->built_sys = EB_SYS_POISSON;
    c->built_mixed = k.mixed;
    red_sum_open(c->g, div, c->part, c->ks + KS_SUM, c->s);
    op_poisson_rhs(c->g, div, c->ks + KS_SUM, c->pb, c->s);
    c->slot_off[slot] = 0;
    SolveCfg kk = k;
    if (k.mixed) {
        kk.max_iter = mixed_budget(k);
        vec_copy(c->N, p, c->pk[4], c->s);  // the starting iterate, for a switch to FP64
    }
    int state = pcg(c, c->pb, p, kk, slot);
    if (state != 2 && k.mixed) {
        vec_copy(c->N, c->pk[4], p, c->s);
        c->slot_off[slot] = slot_count_now(c, slot);
        c->fp64_fallbacks++;
        kk.mixed = false;
        kk.max_iter = k.max_iter;
        mg_build_poisson(c->lev, c->nlev, c->g, beta, false, c->s);
        c->built_mixed = false;
        pcg(c, c->pb, p, kk, slot);
    }
    red_sum_open(c->g, p, c->part, c->ks + KS_SUM, c->s);
    op_shift_open(c->g, p, c->ks + KS_SUM, c->s);
}

// stop rule: max|r| <= rtol * max(max|b|, max_f |A_f w_f|/h)
void mac_project(eb_ctx* c, double beta, double* f[3], double* phi, double rtol,
                 const SolveCfg& k, int slot, bool want_div) {
    op_divergence(c->g, f, c->div, c->s);
    op_face_flux_max(c->g, f, c->part, c->ks + KS_SCALE, c->s);
    ks_set(c->ks, KS_RTOL, rtol, c->s);
    poisson_solve(c, beta, c->div, phi, k, slot);
    op_face_correct(c->g, beta, phi, f, c->s);
    if (want_div) {
        op_divergence(c->g, f, c->div, c->s);
        red_maxabs(c->N, 1, c->div, c->part, c->divs + slot, c->s);
    }
}

void cc_project(eb_ctx* c, double beta, double* u, double* p, double rtol, const SolveCfg& k,
                int slot, bool want_div) {
    op_gcc(c->g, p, c->gp, c->s);
    op_axpy_open(c->g, beta, c->gp, u, 3, c->s);
    op_cell_to_face(c->g, u, c->f, c->s);
    mac_project(c, beta, c->f, p, rtol, k, slot, want_div);
    op_gcc(c->g, p, c->gp, c->s);
    op_axpy_open(c->g, -beta, c->gp, u, 3, c->s);
}

// the iteration cap of a nodal solve: max_iter, or ten times the largest cell count along an
// axis if that is more (the diagonally preconditioned CG needs a number of iterations that grows
// with the grid)
int nodal_max_iter(const eb_ctx* c, const SolveCfg& k) {
    int nmax = std::max(c->grid.n[0], std::max(c->grid.n[1], c->grid.n[2]));
    return std::max(k.max_iter, 10 * nmax);
}

// CG for L x = b on the nodal unknowns, the diagonal as preconditioner and the preconditioned
// residual mean-free over the unknowns (L is singular: constants); state in `slot`; KS_RTOL and
// KS_SCALE must be set.  Vectors: the Krylov scratch (idle during a projection).
int nodal_pcg(eb_ctx* c, const double* b, double* x, const SolveCfg& k, int slot) {
    long M = nd_count(c->grid);
    double *r = c->kv[0], *z = c->kv[1], *pd = c->kv[2], *q = c->kv[3];
    double* ks = c->ks;
    int* st = c->kst + 2 * slot;
    int* itc = c->kst + 2 * NSLOT + slot;
    const uint8_t* mk = c->nd_mask;
    nd_apply(c->g, x, mk, q, c->s);
    vec_sub_scaled(M, b, 1.0, q, r, c->s);  // zero off the unknowns: b and q are
    red_maxabs(M, 1, b, c->part, ks + KS_BN, c->s);
    red_maxabs(M, 1, r, c->part, ks + KS_RN, c->s);
    ks_op(KS_INIT, ks, st, itc, c->s);
    nd_jacobi(M, r, c->nd_dg, mk, z, c->s, st);
    nd_mean_free(M, z, mk, c->part, ks + KS_SUM, c->s, st);
    vec_copy(M, z, pd, c->s);
    const double* A1[4] = {r, nullptr, nullptr, nullptr};
    const double* B1[4] = {z, nullptr, nullptr, nullptr};
    red_dots(M, 1, A1, B1, c->part, ks + KS_RZ, c->s, st);
    GraphKey key = make_key();
    key.kind = 3;
    key.slot = slot;
    key.nc = 1;
    key.p[0] = x;
    key.p[1] = b;
    auto body = [&]() {
        const double* A[4] = {pd, nullptr, nullptr, nullptr};
        const double* B[4] = {q, nullptr, nullptr, nullptr};
        nd_apply(c->g, pd, mk, q, c->s, st);
        red_dots_op(M, 1, A, B, c->part, KS_PQ, KS_CG_ALPHA, ks, st, itc, c->s);
        ks_cg_xr_op(M, x, r, pd, q, c->part, ks, st, itc, c->s);
        nd_jacobi(M, r, c->nd_dg, mk, z, c->s, st);
        nd_mean_free(M, z, mk, c->part, ks + KS_SUM, c->s, st);
        A[0] = r;
        B[0] = z;
        red_dots_op(M, 1, A, B, c->part, KS_RZN, KS_CG_BETA, ks, st, itc, c->s);
        ks_cg_p(M, pd, z, ks, st, c->s);
    };
    return iterate(c, key, slot, nodal_max_iter(c, k), body);
}

// The nodal end-of-stage projection (Sec. III.A.4): u += beta G(pn_old); solve
// L phi = D(u) - B (the right-hand side made mean-free over the unknowns), from phi = beta pn_old;
// phi normalised to zero mean; u -= G(phi) on open cells; pn = phi / beta.  want_div: the
// largest |D(u) - B| left over the unknowns into divs[slot] (not zero: the projection is
// approximate).
void nodal_project(eb_ctx* c, double beta, double* u, double* pn, double rtol, const SolveCfg& k,
                   int slot, bool want_div) {
    long M = nd_count(c->grid);
    double *phi = c->kv[4], *rhs = c->kv[5], *tsum = c->kv[6];
    const uint8_t* mk = c->nd_mask;
    nd_grad(c->g, pn, c->gp, c->s);
    op_axpy_open(c->g, beta, c->gp, u, 3, c->s);
    nd_div(c->g, u, c->nd_bflux, mk, rhs, tsum, c->s);
    red_maxabs(M, 1, tsum, c->part, c->ks + KS_SCALE, c->s);
    ks_set(c->ks, KS_RTOL, rtol, c->s);
    nd_mean_free(M, rhs, mk, c->part, c->ks + KS_SUM, c->s);
    nd_scale_masked(M, beta, pn, mk, phi, c->s);
    c->slot_off[slot] = 0;
    nodal_pcg(c, rhs, phi, k, slot);
    nd_mean_free(M, phi, mk, c->part, c->ks + KS_SUM, c->s);
    nd_sync(c->grid, phi, c->s);
    nd_grad(c->g, phi, c->gp, c->s);
    op_axpy_open(c->g, -1.0, c->gp, u, 3, c->s);
    vec_axpby(M, 1.0 / beta, phi, 0.0, pn, c->s);
    if (want_div) {
        nd_div(c->g, u, c->nd_bflux, mk, rhs, nullptr, c->s);
        red_maxabs(M, 1, rhs, c->part, c->divs + slot, c->s);
    }
}

// BiCGSTAB on the three-component system, right-preconditioned by the viscous V-cycle; the
// slot's count holds half-iterations (= V-cycles)
//
// transposed: solve A^T x = psi instead (psi is then the right-hand side itself, already zero
// on covered cells; x starts from zero).  The V-cycle preconditioner is symmetric, so the same
// hierarchy serves both systems.
int bicgstab(eb_ctx* c, double rho, double dt, const double* eta, const double* eta_eb,
             double* x, const SolveCfg& k, int slot, bool transposed);

void visc_solve(eb_ctx* c, double rho, double dt, const double* eta, const double* eta_eb,
                const double* psi, double* x, double rtol, const SolveCfg& k, int slot,
                bool transposed = false) {
    long N3 = 3 * c->N;
    double *t = c->kv[7], *b = c->kv[8], *a0 = c->kv[9];
    double* ks = c->ks;
    mg_build_visc(c->lev, c->nlev, c->g, rho, dt, eta, eta_eb, k.mixed, c->s);
    c->built_sys = EB_SYS_VISC;
    c->built_mixed = k.mixed;
    if (transposed) {
        vec_copy(N3, psi, b, c->s);
        vec_fill(N3, 0.0, x, c->s);
    } else {
        // effective right-hand side: alpha psi minus the boundary part A(0)
        vec_fill(N3, 0.0, t, c->s);
        op_visc_apply(c->g, rho, dt, eta, eta_eb, t, a0, 0, c->s);
        vec_mask_rhs(c->g, psi, a0, b, c->s);
    }
    red_maxabs(N3, 1, b, c->part, ks + KS_BN, c->s);
    ks_set(ks, KS_SCALE, 0.0, c->s);
    ks_set(ks, KS_RTOL, rtol, c->s);
    c->slot_off[slot] = 0;
    SolveCfg kk = k;
    if (k.mixed) {
        kk.max_iter = mixed_budget(k);
        vec_copy(N3, x, a0, c->s);  // the starting iterate, for a switch to FP64
    }
    int state = bicgstab(c, rho, dt, eta, eta_eb, x, kk, slot, transposed);
    if (state != 2 && k.mixed) {
        vec_copy(N3, a0, x, c->s);
        c->slot_off[slot] = 2 * slot_count_now(c, slot);
        c->fp64_fallbacks++;
        kk.mixed = false;
        kk.max_iter = k.max_iter;
        mg_build_visc(c->lev, c->nlev, c->g, rho, dt, eta, eta_eb, false, c->s);
        c->built_mixed = false;
        bicgstab(c, rho, dt, eta, eta_eb, x, kk, slot, transposed);
    }
}

// the BiCGSTAB iterations of visc_solve from the iterate in x (right-hand side in kv[8], tol
// scalars set); returns the final state
int bicgstab(eb_ctx* c, double rho, double dt, const double* eta, const double* eta_eb,
             double* x, const SolveCfg& k, int slot, bool transposed) {
    long N3 = 3 * c->N;
    double *r = c->kv[0], *rh = c->kv[1], *p = c->kv[2], *v = c->kv[3], *ph = c->kv[4],
           *sv = c->kv[5], *sh = c->kv[6], *t = c->kv[7], *b = c->kv[8];
    double* ks = c->ks;
    int* st = c->kst + 2 * slot;
    int* itc = c->kst + 2 * NSLOT + slot;
    auto apply = [&](const double* in, double* out, const int* gate) {
        if (transposed) adj_visc_apply_T(c->g, rho, dt, eta, eta_eb, c->wt, in, out, c->s, gate);
        else op_visc_apply(c->g, rho, dt, eta, eta_eb, in, out, 1, c->s, gate);
    };
    // r = b - A_lin(x)
    apply(x, t, nullptr);
    vec_sub_scaled(N3, b, 1.0, t, r, c->s);
    red_maxabs(N3, 1, r, c->part, ks + KS_RN, c->s);
    ks_op(k.mixed ? KS_INIT_WATCH : KS_INIT, ks, st, itc, c->s);
    vec_copy(N3, r, rh, c->s);
    vec_fill(N3, 0.0, p, c->s);
    vec_fill(N3, 0.0, v, c->s);
    const double* A1[4] = {rh, nullptr, nullptr, nullptr};
    const double* B1[4] = {r, nullptr, nullptr, nullptr};
    red_dots(N3, 1, A1, B1, c->part, ks + KS_RR, c->s, st);
    GraphKey key = make_key();
    key.kind = 2;
    key.slot = slot;
    key.nc = 3;
    key.mixed = k.mixed;
    key.nu1 = k.nu1;
    key.nu2 = k.nu2;
    key.nbottom = k.nbottom;
    key.transposed = transposed;
    key.p[0] = x;
    key.p[1] = eta;
    key.p[2] = eta_eb;
    key.v[0] = rho;
    key.v[1] = dt;
    // With an FP32 finest level the preconditioner's results are FP32 values, so ph and sh are
    // kept in FP32 storage (the first half of their FP64 buffers) and widened where they are
    // read (the operator, the x update): the same numbers, half the bytes.
    bool f32 = k.mixed && !transposed &&
               mg_vcycle_f32_out(c->lev, c->nlev, 3, true, k.nu1, k.nu2);
    float* phf = reinterpret_cast<float*>(ph);
    float* shf = reinterpret_cast<float*>(sh);
    auto precond = [&](const double* in, double* out, float* out32) {
        if (f32)
            mg_vcycle(c->lev, c->nlev, 3, true, in, out32, k.nu1, k.nu2, k.nbottom, c->s, st);
        else
            vcyc(c, 3, k, in, out, st);
    };
    auto body = [&]() {
        ks_bi_p(N3, p, r, v, ks, st, c->s);
        precond(p, ph, phf);
        if (f32) op_visc_apply(c->g, rho, dt, eta, eta_eb, phf, v, 1, c->s, st);
        else apply(ph, v, st);
        const double* Av[4] = {rh, nullptr, nullptr, nullptr};
        const double* Bv[4] = {v, nullptr, nullptr, nullptr};
        red_dots_op(N3, 1, Av, Bv, c->part, KS_RV, KS_BI_ALPHA, ks, st, itc, c->s);
        ks_bi_s_op(N3, sv, r, v, c->part, ks, st, itc, c->s);
        if (f32) ks_bi_xs(N3, x, phf, ks, st, c->s);
        else ks_bi_xs(N3, x, ph, ks, st, c->s);
        precond(sv, sh, shf);
        if (f32) op_visc_apply(c->g, rho, dt, eta, eta_eb, shf, t, 1, c->s, st);
        else apply(sh, t, st);
        const double* A2[4] = {t, t, nullptr, nullptr};
        const double* B2[4] = {sv, t, nullptr, nullptr};
        red_dots_op(N3, 2, A2, B2, c->part, KS_TS, KS_BI_OMEGA, ks, st, itc, c->s);
        if (f32) ks_bi_xr_op(N3, x, r, phf, shf, sv, t, rh, c->part, ks, st, itc, c->s);
        else ks_bi_xr_op(N3, x, r, ph, sh, sv, t, rh, c->part, ks, st, itc, c->s);
    };
    return iterate(c, key, slot, k.max_iter, body);
}

// reads `n` solve slots (state, count) after the stream drains
int read_slots(eb_ctx* c, int n, int* host) {
    HIPN(hipMemcpyAsync(host, c->kst, 2 * n * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPN(hipStreamSynchronize(c->s));
    if (int h = hip_check("solver state read-back")) return h;
    for (int q = 0; q < n; q++)  // counts include the FP32 phase of a solve that switched
        if (host[2 * q] == 2) host[2 * q + 1] += c->slot_off[q];
    return EB_OK;
}

// return code of one solve from its slot
int slot_code(const int* sl, const char* what, int max_iter) {
    if (sl[0] == 2) return EB_OK;
    if (sl[0] == 3) return set_err(EB_ENAN, "%s: non-finite residual", what);
    return set_err(EB_ENOCONV, "%s: no convergence in %d iterations", what, max_iter);
}

// bytes of one evaluation's branch record: slopes [3][3][N], then the normal and the
// transverse upwind sides per face of each direction
size_t switch_bytes(const eb_ctx* c) {
    size_t nf = 0;
    for (int d = 0; d < 3; d++) nf += (size_t)face_count(c->grid, d);
    return 9 * (size_t)c->N + 2 * nf;
}

// the branch record of the next derived-quantities evaluation (mode 0: none)
int next_switches(eb_ctx* c, SwitchV* sw) {
    *sw = SwitchV{};
    if (c->sw_mode == 0) return EB_OK;
    size_t blk = switch_bytes(c);
    if (c->sw_cur + blk > c->sw_bytes)
        return set_err(EB_EINVAL, "branch record buffer of %zu bytes holds no evaluation at "
                                  "offset %zu (%zu bytes each)", c->sw_bytes, c->sw_cur, blk);
    uint8_t* b = c->sw_buf + c->sw_cur;
    sw->mode = c->sw_mode;
    sw->slope = b;
    b += 9 * (size_t)c->N;
    for (int d = 0; d < 3; d++) {
        sw->norm[d] = b;
        b += face_count(c->grid, d);
    }
    for (int d = 0; d < 3; d++) {
        sw->tr[d] = b;
        b += face_count(c->grid, d);
    }
    c->sw_cur += blk;
    return EB_OK;
}

// DerivedQuantities; the MAC projection reports into `slot` and starts from phi = 0, or, with
// warm, from the phi its previous call left (the corrector starts from the predictor's: the
// converged phi is the same to the solve's tolerance, in fewer iterations)
int derived(eb_ctx* c, const eb_rheology& rh, const double* theta, const double* u,
            const eb_step_opts* o, double* C, double* eta, double* eta_eb, double* V,
            int slot, bool warm = false) {
    SolveCfg k = cfg_of(o);
    double rtol = o && o->rtol_mac > 0 ? o->rtol_mac : 1e-12;
    SwitchV sw;
    if (int h = next_switches(c, &sw)) return h;
    op_face_extrap(c->g, u, c->f, sw, c->s);
    if (!warm) vec_fill(c->N, 0.0, c->phi, c->s);
    mac_project(c, 1.0, c->f, c->phi, rtol, k, slot, false);
    op_conv_dc(c->g, u, c->f, c->DC, sw, c->s);
    op_redistribute(c->g, c->DC, c->DH, c->rS, c->rdD, C, c->s);
    op_wall_grad(c->g, u, c->gw, c->s);
    op_grad_eta(c->g, rh, u, c->gw, theta, c->G9, eta, nullptr, c->s);
    op_eta_eb(c->g, rh, c->gw, theta, eta_eb, c->s);
    op_transpose_dc(c->g, u, c->G9, eta, eta_eb, c->gw, c->DC, c->s);
    op_redistribute(c->g, c->DC, c->DH, c->rS, c->rdD, V, c->s);
    return hip_check("derived");
}

// ------------------------------------------------------------------------------------------
// reverse sweep.  Each helper is the adjoint of the forward helper of the same name; solves
// are transposed (the Poisson matrix is symmetric, the viscous one is not), never
// differentiated through their iterations.
// ------------------------------------------------------------------------------------------
// MAC projection: fb += beta D^T L^+ G_f^T fb   (fb in place)
void mac_project_adj(eb_ctx* c, double beta, double* fb[3], double rtol, const SolveCfg& k,
                     int slot) {
    adj_face_grad_T_neg(c->g, fb, c->div, c->s);
    red_maxabs(c->N, 1, c->div, c->part, c->ks + KS_SCALE, c->s);
    ks_set(c->ks, KS_RTOL, rtol, c->s);
    vec_fill(c->N, 0.0, c->phi, c->s);
    poisson_solve(c, beta, c->div, c->phi, k, slot);
    adj_div_T_add(c->g, beta, c->phi, fb, c->s);
}

// end-of-stage projection: (ub, pb) of (u_new, p_new) in, of (u, p_old) out
void cc_project_adj(eb_ctx* c, double beta, double* ub, double* pb, double rtol,
                    const SolveCfg& k, int slot) {
    // phib = pb - beta Gcc^T ub, stored negated for the Poisson solve (which returns L^+ phib)
    adj_gcc_T(c->g, -beta, ub, pb, c->div, c->s);
    adj_scale(c->N, -1.0, c->div, c->s);
    red_maxabs(c->N, 1, c->div, c->part, c->ks + KS_SCALE, c->s);
    ks_set(c->ks, KS_RTOL, rtol, c->s);
    vec_fill(c->N, 0.0, c->phi, c->s);
    poisson_solve(c, beta, c->div, c->phi, k, slot);
    adj_cc_cell(c->g, c->phi, ub, c->s);
    adj_gcc_T(c->g, beta, ub, nullptr, pb, c->s);
}

// implicit viscous solve: lam = A^-T xb (in c->lam); etab, etaebb (acc)
void visc_solve_adj(eb_ctx* c, double rho, double dt, const double* eta, const double* eta_eb,
                    const double* x, const double* xb, double rtol, const SolveCfg& k, int slot,
                    double* etab, double* etaebb) {
    adj_mask_open(c->g, 3, xb, c->gp, c->s);
    visc_solve(c, rho, dt, eta, eta_eb, c->gp, c->lam, rtol, k, slot, true);
    adj_visc_coef(c->g, dt, x, c->lam, etab, etaebb, c->s);
}

// derived quantities at u; uf: the projected face velocities of the forward pass
void derived_adj(eb_ctx* c, const eb_rheology& rh, const double* theta, const double* u,
                 double* const uf[3], const double* Cb, const double* etab,
                 const double* etaebb, const double* Vb, double* ub, double* tau0b, double rtol,
                 const SolveCfg& k, int slot) {
    const GeomV& g = c->g;
    op_wall_grad(g, u, c->gw, c->s);
    op_grad_eta(g, rh, u, c->gw, theta, c->G9, c->eta0, nullptr, c->s);
    op_eta_eb(g, rh, c->gw, theta, c->eb0, c->s);
    adj_redistribute(g, Vb, c->rX, c->rY, c->DC, c->s);
    adj_visc_terms(g, rh, theta, u, c->G9, c->eta0, c->eb0, c->gw, c->DC, etab, etaebb, ub, c->Gb,
                   c->gwb, tau0b, c->s);
    adj_grad_gather(g, c->wt, c->Gb, c->gwb, ub, c->s);
    adj_redistribute(g, Cb, c->rX, c->rY, c->DC, c->s);
    adj_conv_face_w(g, u, uf, c->DC, c->ufb, c->s);
    mac_project_adj(c, 1.0, c->ufb, rtol, k, slot);
    adj_conv_lr(g, u, uf, c->DC, c->ufb, c->lr, ub, c->s);
}

// psi = rho u + dt (rho C + V - Gcc p + f): from lam = A^-T xb
void psi_adj(eb_ctx* c, double rho, double dt, double* ub, double* Cb, double* Vb, double* pb) {
    adj_psi(c->g, rho, dt, c->lam, c->psi, ub, Cb, Vb, c->s);
    adj_gcc_T(c->g, -dt, c->psi, pb, pb, c->s);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------
// Device scratch of eb_drag_noalloc: a file-scope device array (each GPU the library runs on
// holds its own copy until the process ends), so that entry point needs no allocation and writes
// nothing into the caller's workspace.  Layout (doubles): wall gradients [3][NOALLOC_NCUT], drag
// terms [3][NOALLOC_NCUT], reduction partials [4096], reduced forces [8].  Host code uses only
// the address hipGetSymbolAddress returns for the current device, taken once per device at
// set-up (eb_geometry_build), never the array's name.
// ------------------------------------------------------------------------------------------
namespace {
constexpr long NOALLOC_NCUT = 65536;
constexpr long NOALLOC_DOUBLES = 6 * NOALLOC_NCUT + 4096 + 8;
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEV] = {nullptr};

// the current device's scratch address (looked up on its first use on that device)
int noalloc_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_err(EB_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV)
        return set_err(EB_EINVAL, "device %d beyond the %d the library tracks", dev,
                       NOALLOC_MAX_DEV);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_err(EB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_noalloc_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_noalloc_ptr[dev];
    return EB_OK;
}
}  // namespace

// ------------------------------------------------------------------------------------------
extern "C" {

const char* eb_last_error(void) { return g_err.c_str(); }

size_t eb_workspace_bytes(const eb_box* box, const eb_body* body) {
    eb_ctx c;
    if (init_ctx(&c, box, body) != EB_OK) return 0;
    return carve(&c, nullptr, true);
}

int eb_geometry_build(const eb_box* box, const eb_body* body, void* ws, size_t ws_bytes,
                      eb_ctx** out, void* stream) {
    if (!out || !ws) return set_err(EB_EINVAL, "null workspace or context pointer");
    eb_ctx* c = new eb_ctx;
    int e = init_ctx(c, box, body);
    if (e) {
        delete c;
        return e;
    }
    size_t need = carve(c, nullptr, true);
    if (ws_bytes < need) {
        delete c;
        return set_err(EB_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    }
    carve(c, (char*)ws, false);
    c->s = (hipStream_t)stream;
    double* scr = nullptr;  // eb_drag_noalloc's scratch address on this device, looked up once
    if ((e = noalloc_scratch(&scr))) {
        delete c;
        return e;
    }
    int ncut = 0;
    geom_build_device(c->grid, c->bodyv, c->psi_nodes, c->flag, c->alpha, c->ap, c->cutid,
                      c->cut, c->blockcount, c->ncut_max, &ncut, c->errdev, c->s);
    if ((e = hip_check("geometry"))) {
        delete c;
        return e;
    }
    if (ncut > c->ncut_max) {
        delete c;
        return set_err(EB_EGEOM, "%d cut cells exceed the bound %d", ncut, c->ncut_max);
    }
    c->ncut = ncut;
    const double* apc[3] = {c->ap[0], c->ap[1], c->ap[2]};
    geom_cut_fill(c->grid, c->bodyv, c->psi_nodes, apc, c->cut, ncut, c->cutid, c->nrm, c->aeb,
                  c->bc, c->delta, c->s);
    // per-cut arrays are [component][ncut]: rebase the strided views on the real count
    fill_geomv(c);
    geom_wall_stencil(c->g, c->dd, c->sidx, c->sw, c->nfb, c->errdev, c->s);
    geom_mark_near(c->grid, c->cut, ncut, c->near, c->s);
    nd_setup(c->g, c->nd_bflux, c->nd_dg, c->nd_mask, c->s);
    for (int l = 1; l < c->nlev; l++) level_coarsen_geometry(c->lev[l - 1], c->lev[l], c->s);
    for (int l = 0; l < c->nlev; l++) level_mask(c->lev[l], c->s);
    int err = 0;
    HIPN(hipMemcpyAsync(&err, c->errdev, sizeof(int), hipMemcpyDeviceToHost, c->s));
    hipError_t he = hipStreamSynchronize(c->s);
    if (he != hipSuccess) {
        delete c;
        return set_err(EB_EHIP, "geometry sync: %s", hipGetErrorString(he));
    }
    if ((e = hip_check("geometry"))) {
        delete c;
        return e;
    }
    if (err) {
        delete c;
        return set_err(EB_EGEOM, "geometry error flags 0x%x (1 ambiguous face, 2 degenerate cut "
                                 "cell, 4 wall stencil outside the box)", err);
    }
    // fallback count
    c->nfallback = 0;
    if (ncut > 0) {
        int* tmp = new int[ncut];
        HIPN(hipMemcpyAsync(tmp, c->nfb, ncut * sizeof(int), hipMemcpyDeviceToHost, c->s));
        HIPN(hipStreamSynchronize(c->s));
        for (int q = 0; q < ncut; q++) c->nfallback += tmp[q];
        delete[] tmp;
    }
    if (hipHostMalloc((void**)&c->pin, 2 * sizeof(PollWord), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
        eb_ctx_destroy(c);
        return set_err(EB_EHIP, "pinned polling buffer or events: %s",
                       hipGetErrorString(hipGetLastError()));
    }
    HIPN(hipMemsetAsync(c->kst, 0, 3 * NSLOT * sizeof(int), c->s));
    HIPN(hipStreamSynchronize(c->s));
    if ((e = hip_check("geometry"))) {
        eb_ctx_destroy(c);
        return e;
    }
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fence_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fence_out, hipEventDisableTiming) != hipSuccess) {
        eb_ctx_destroy(c);
        return set_err(EB_EHIP, "library stream or events: %s",
                       hipGetErrorString(hipGetLastError()));
    }
    c->graphs = new GraphCache;
    const char* env = getenv("EB_GRAPHS");
    c->graphs_on = env ? atoi(env) != 0 : 1;
    if ((e = build_wall_transpose(c))) {
        eb_ctx_destroy(c);
        return e;
    }
    *out = c;
    return EB_OK;
}

void eb_ctx_destroy(eb_ctx* ctx) {
    if (!ctx) return;
    // teardown has no caller to report to: failures here are dropped on purpose
    if (ctx->own) (void)hipStreamSynchronize(ctx->own);
    delete ctx->graphs;
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    if (ctx->fence_in) (void)hipEventDestroy(ctx->fence_in);
    if (ctx->fence_out) (void)hipEventDestroy(ctx->fence_out);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    for (int b = 0; b < 2; b++)
        if (ctx->ev[b]) (void)hipEventDestroy(ctx->ev[b]);
    delete ctx;
}

int eb_ctx_set_graphs(eb_ctx* c, int enable) {
    if (!c) return set_err(EB_EINVAL, "null context");
    c->graphs_on = enable ? 1 : 0;
    return EB_OK;
}

size_t eb_switch_bytes(const eb_ctx* c) { return c ? switch_bytes(c) : 0; }

int eb_ctx_set_switches(eb_ctx* c, int mode, void* buf, size_t bytes) {
    if (!c) return set_err(EB_EINVAL, "null context");
    if (mode != EB_SWITCH_OFF && mode != EB_SWITCH_RECORD && mode != EB_SWITCH_REPLAY)
        return set_err(EB_EINVAL, "unknown branch record mode %d", mode);
    if (mode != EB_SWITCH_OFF && (!buf || bytes < switch_bytes(c)))
        return set_err(EB_EINVAL, "branch record buffer of %zu bytes < %zu", bytes,
                       switch_bytes(c));
    c->sw_mode = mode;
    c->sw_buf = mode == EB_SWITCH_OFF ? nullptr : (uint8_t*)buf;
    c->sw_bytes = mode == EB_SWITCH_OFF ? 0 : bytes;
    c->sw_cur = 0;
    return EB_OK;
}

int eb_ctx_info(const eb_ctx* c, int* ncut, int* nlevels, int* nfallback) {
    if (!c) return set_err(EB_EINVAL, "null context");
    if (ncut) *ncut = c->ncut;
    if (nlevels) *nlevels = c->nlev;
    if (nfallback) *nfallback = c->nfallback;
    return EB_OK;
}

}  // extern "C"

namespace {
__global__ void k_export_cut(GeomV g, const int* __restrict__ nfb, int64_t* __restrict__ cell,
                             double* __restrict__ data) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    if (cell) cell[q] = g.cut[q];
    if (data) {
        double* row = data + 9L * q;
        for (int e = 0; e < 3; e++) row[e] = g.nrm[(long)e * nc + q];
        row[3] = g.aeb[q];
        for (int e = 0; e < 3; e++) row[4 + e] = g.bc[(long)e * nc + q];
        row[7] = g.delta[q];
        row[8] = nfb[q];
    }
}
}  // namespace

extern "C" {

int eb_geometry_export(const eb_ctx* c, uint8_t* flag, double* alpha, double* ax, double* ay,
                       double* az, int64_t* cut_cell, double* cut_data, void* stream) {
    if (!c) return set_err(EB_EINVAL, "null context");
    hipStream_t s = (hipStream_t)stream;
    if (flag) HIPN(hipMemcpyAsync(flag, c->flag, c->N, hipMemcpyDeviceToDevice, s));
    if (alpha) HIPN(hipMemcpyAsync(alpha, c->alpha, c->N * 8, hipMemcpyDeviceToDevice, s));
    double* dst[3] = {ax, ay, az};
    for (int d = 0; d < 3; d++)
        if (dst[d])
            HIPN(hipMemcpyAsync(dst[d], c->ap[d], face_count(c->grid, d) * 8, hipMemcpyDeviceToDevice,
                           s));
    if (c->ncut > 0 && (cut_cell || cut_data))
        k_export_cut<<<grid_for(c->ncut), EB_BLOCK, 0, s>>>(c->g, c->nfb, cut_cell, cut_data);
    return hip_check("eb_geometry_export");
}

int eb_apparent_viscosity(const eb_ctx* cc, const eb_rheology* rheo, const double* u,
                          const double* theta, double* eta, double* eta_eb, double* sr,
                          void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !rheo || !u || !eta || (!eta_eb && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    hipStream_t s = (hipStream_t)stream;
    op_wall_grad(c->g, u, c->gw, s);
    op_grad_eta(c->g, *rheo, u, c->gw, theta, c->G9, eta, sr, s);
    op_eta_eb(c->g, *rheo, c->gw, theta, eta_eb, s);
    return hip_check("eb_apparent_viscosity");
}

int eb_viscous_apply(const eb_ctx* cc, int mode, double rho, double dt, const double* eta,
                     const double* eta_eb, const double* u, double* out, void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !eta || !u || !out || (!eta_eb && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    if (mode == EB_OP_HELMHOLTZ || mode == EB_OP_HELMHOLTZ_H) {
        op_visc_apply(c->g, rho, dt, eta, eta_eb, u, out, mode == EB_OP_HELMHOLTZ_H, s);
    } else if (mode == EB_OP_TRANSPOSE) {
        eb_rheology nw{EB_LAW_NEWTONIAN, 1.0, 0.0, 1.0, 1.0};
        op_wall_grad(c->g, u, c->gw, s);
        op_grad_eta(c->g, nw, u, c->gw, nullptr, c->G9, c->eta1, nullptr, s);
        op_transpose_dc(c->g, u, c->G9, eta, eta_eb, c->gw, c->DC, s);
        op_redistribute(c->g, c->DC, c->DH, c->rS, c->rdD, out, s);
    } else {
        return set_err(EB_EINVAL, "unknown mode %d", mode);
    }
    return hip_check("eb_viscous_apply");
}

int eb_mg_vcycle(eb_ctx* c, int system, int precision, double beta, double rho, double dt,
                 const double* eta, const double* eta_eb, const double* r, double* e,
                 const eb_step_opts* opts, void* stream) {
    if (!c || !r || !e) return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    k.mixed = precision == EB_MIXED;
    if (system == EB_SYS_POISSON) {
        mg_build_poisson(c->lev, c->nlev, c->g, beta, k.mixed, c->s);
        c->built_sys = EB_SYS_POISSON;
        c->built_mixed = k.mixed;
        vcyc(c, 1, k, r, e, nullptr);
    } else if (system == EB_SYS_VISC) {
        if (!eta || (!eta_eb && c->ncut > 0)) return set_err(EB_EINVAL, "null viscosity");
        mg_build_visc(c->lev, c->nlev, c->g, rho, dt, eta, eta_eb, k.mixed, c->s);
        c->built_sys = EB_SYS_VISC;
        c->built_mixed = k.mixed;
        vcyc(c, 3, k, r, e, nullptr);
    } else {
        return set_err(EB_EINVAL, "unknown system %d", system);
    }
    return hip_check("eb_mg_vcycle");
}

int eb_mg_sweep(eb_ctx* c, int system, int precision, int colour, const void* b, void* x,
                void* stream) {
    if (!c || !b || !x) return set_err(EB_EINVAL, "null argument");
    bool f32 = precision == EB_MIXED;
    if (c->built_sys != system || c->built_mixed != f32)
        return set_err(EB_EINVAL, "no operator for system %d precision %d is built", system,
                       precision);
    if (f32 && !mg_level0_f32(c->lev, c->nlev))
        return set_err(EB_EINVAL, "the finest level of this hierarchy runs in FP64");
    mg_sweep_level0(c->lev[0], system == EB_SYS_VISC ? 3 : 1, f32, b, x, colour & 1,
                    (hipStream_t)stream);
    return hip_check("eb_mg_sweep");
}

int eb_visc_solve(eb_ctx* c, double rho, double dt, const double* eta, const double* eta_eb,
                  const double* psi, double* x, double rtol, const eb_step_opts* opts,
                  int* iters, void* stream) {
    if (!c || !eta || !psi || !x || (!eta_eb && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    visc_solve(c, rho, dt, eta, eta_eb, psi, x, rtol, k, 0);
    int h = hip_check("eb_visc_solve");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = (sl[1] + 1) / 2;
    return slot_code(sl, "viscous solve", k.max_iter);
}

int eb_mac_project(eb_ctx* c, double beta, double* fx, double* fy, double* fz, double* phi,
                   double rtol, const eb_step_opts* opts, double* div_inf, int* iters,
                   void* stream) {
    if (!c || !fx || !fy || !fz || !phi) return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    double* f[3] = {fx, fy, fz};
    SolveCfg k = cfg_of(opts);
    mac_project(c, beta, f, phi, rtol, k, 0, true);
    int h = hip_check("eb_mac_project");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    if (div_inf) HIPN(hipMemcpy(div_inf, c->divs, sizeof(double), hipMemcpyDeviceToHost));
    if ((h = hip_check("divergence read-back"))) return h;
    return slot_code(sl, "MAC projection", k.max_iter);
}

int eb_cc_project(eb_ctx* c, double beta, double* u, double* p, double rtol,
                  const eb_step_opts* opts, double* div_inf, int* iters, void* stream) {
    if (!c || !u || !p) return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    cc_project(c, beta, u, p, rtol, k, 0, true);
    int h = hip_check("eb_cc_project");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    if (div_inf) HIPN(hipMemcpy(div_inf, c->divs, sizeof(double), hipMemcpyDeviceToHost));
    if ((h = hip_check("divergence read-back"))) return h;
    return slot_code(sl, "projection", k.max_iter);
}

int eb_nodal_project(eb_ctx* c, double beta, double* u, double* pn, double rtol,
                     const eb_step_opts* opts, double* div_inf, int* iters, void* stream) {
    if (!c || !u || !pn) return set_err(EB_EINVAL, "null argument");
    if (!(beta > 0.0)) return set_err(EB_EINVAL, "beta must be > 0");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    nodal_project(c, beta, u, pn, rtol, k, 0, true);
    int h = hip_check("eb_nodal_project");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    if (div_inf) HIPN(hipMemcpy(div_inf, c->divs, sizeof(double), hipMemcpyDeviceToHost));
    if ((h = hip_check("divergence read-back"))) return h;
    return slot_code(sl, "nodal projection", nodal_max_iter(c, k));
}

int eb_derived(eb_ctx* c, const eb_rheology* rheo, const double* theta, const double* u,
               const eb_step_opts* opts, double* C, double* eta, double* eta_eb, double* V,
               int* iters, void* stream) {
    if (!c || !rheo || !u || !C || !eta || !V || (!eta_eb && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    StreamScope scope_(c, stream);
    int h = derived(c, *rheo, theta, u, opts, C, eta, eta_eb, V, 0);
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    return slot_code(sl, "MAC projection", cfg_of(opts).max_iter);
}

}  // extern "C"

namespace {

// the time step of the stability rule (Sec. II.C.1: Eqs. cfl:convective, cfl:forcing,
// cfl:viscous:new combined by Eq. cfl:dt) from umax = max over open cells of |u|+|v|+|w| and
// tmax = the largest yield-stress multiplier there
double stable_dt_of(const eb_ctx* c, const eb_rheology& r, double umax, double tmax,
                    const double force[3], double c_cfl) {
    double h = c->box.h;
    double cc = umax / h;
    if (r.law >= EB_LAW_POWER) return 0.0;  // the rule covers the first three laws only
    double bi = r.law == EB_LAW_NEWTONIAN ? 0.0 : r.tau0 * tmax;
    if (bi < 0.0) bi = 0.0;
    double cf = sqrt((fabs(force[0]) + fabs(force[1]) + fabs(force[2])) / h);
    double cv = 2.0 * r.mu / r.rho * (bi + 1.0) * (3.0 / (h * h));
    double a = cc + cv;
    return c_cfl / (0.5 * (a + sqrt(a * a + 4.0 * cf * cf)));
}

// stats and return code of a step (forward or reverse) from its six solve slots; a forward
// step also reports the stability-rule time step of its input state (reduced into divs[6..7])
int step_status(eb_ctx* c, const SolveCfg& k, eb_step_stats* stats, bool adjoint,
                const eb_rheology* rheo = nullptr, const eb_step_opts* o = nullptr) {
    int sl[12];
    double dv[8];
    int h;
    if ((h = read_slots(c, 6, sl))) return h;
    HIPN(hipMemcpy(dv, c->divs, 8 * sizeof(double), hipMemcpyDeviceToHost));
    if ((h = hip_check("step statistics"))) return h;
    eb_step_stats st;
    memset(&st, 0, sizeof(st));
    int status = EB_OK;
    const char* names[2][3] = {{"MAC projection", "viscous solve", "projection"},
                               {"adjoint MAC projection", "transposed viscous solve",
                                "adjoint projection"}};
    for (int q = 0; q < 6; q++) {
        int cnt = sl[2 * q + 1];
        int stage = q / 3, kind = q % 3;
        if (kind == 0) st.it_mac[stage] = cnt;
        if (kind == 1) st.it_visc[stage] = (cnt + 1) / 2;
        if (kind == 2) {
            st.it_proj[stage] = cnt;
            st.div_proj[stage] = adjoint ? 0.0 : dv[q];
        }
        st.vcycles += cnt;
        if (status == EB_OK && sl[2 * q] != 2)
            status = slot_code(&sl[2 * q], names[adjoint][kind], k.max_iter);
    }
    st.status = status;
    st.fp64_fallbacks = c->fp64_fallbacks;
    st.dt_stable = (!adjoint && rheo && o) ? stable_dt_of(c, *rheo, dv[6], dv[7], o->force, 0.5)
                                           : 0.0;
    if (stats) *stats = st;
    return status;
}

int rk2_impl(eb_ctx* c, const eb_rheology* rheo, const double* theta, double dt,
             const eb_step_opts* o, double* u, double* p, eb_step_stats* stats, TapeV* tp) {
    if (!c || !rheo || !o || !u || !p) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    if (!(rheo->rho > 0.0) || !(dt > 0.0)) return set_err(EB_EINVAL, "rho and dt must be > 0");
    SolveCfg k = cfg_of(o);
    long N = c->N, N3 = 3 * N;
    int nc = c->ncut;
    double rho = rheo->rho, beta = dt / rho;
    int h;
    c->fp64_fallbacks = 0;
    red_cfl(c->g, u, theta, c->part, c->divs + 6, c->s);  // for the stats' stable time step
    // slots: 0/3 MAC projection, 1/4 viscous solve, 2/5 end-of-stage projection
    // predictor: derived quantities at u^m
    bool nodal = o->projection == EB_PROJ_NODAL;
    if (nodal && tp) return set_err(EB_EINVAL, "the adjoint covers the cell-centred projection only");
    long NP = nodal ? nd_count(c->grid) : N;  // the pressure's storage: nodes or cells
    double* pw = nodal ? c->pn1 : c->p1;
    auto grad_p = [&](const double* q) {
        if (nodal) nd_grad(c->g, q, c->gp, c->s);
        else op_gcc(c->g, q, c->gp, c->s);
    };
    auto project = [&](int slot) {
        if (nodal) nodal_project(c, beta, c->u1, pw, o->rtol_proj, k, slot, true);
        else cc_project(c, beta, c->u1, pw, o->rtol_proj, k, slot, true);
    };
    if ((h = derived(c, *rheo, theta, u, o, c->C0, c->eta0, c->eb0, c->V0, 0))) return h;
    if (tp) {
        for (int d = 0; d < 3; d++) vec_copy(face_count(c->grid, d), c->f[d], tp->ufm[d], c->s);
        vec_copy(N, c->eta0, tp->em, c->s);
        if (nc > 0) vec_copy(nc, c->eb0, tp->ebm, c->s);
    }
    grad_p(p);
    op_psi(c->g, rho, dt, u, c->C0, c->V0, c->gp, o->force, c->psi, c->s);
    vec_copy(N3, u, c->u1, c->s);
    visc_solve(c, rho, dt, c->eta0, c->eb0, c->psi, c->u1, o->rtol_visc, k, 1);
    if (tp) vec_copy(N3, c->u1, tp->us1, c->s);
    vec_copy(NP, p, pw, c->s);
    project(2);
    if (tp) vec_copy(N3, c->u1, tp->u1, c->s);
    // corrector: derived quantities at u*, averaged with the predictor's
    if ((h = derived(c, *rheo, theta, c->u1, o, c->C1, c->eta1, c->eb1, c->V1, 3, true)))
        return h;
    if (tp)
        for (int d = 0; d < 3; d++) vec_copy(face_count(c->grid, d), c->f[d], tp->uf1[d], c->s);
    op_average(N3, c->C1, c->C0, c->s);
    op_average(N3, c->V1, c->V0, c->s);
    op_average(N, c->eta1, c->eta0, c->s);
    op_average(nc, c->eb1, c->eb0, c->s);
    if (tp) {
        vec_copy(N, c->eta0, tp->ea, c->s);
        if (nc > 0) vec_copy(nc, c->eb0, tp->eba, c->s);
    }
    grad_p(pw);
    op_psi(c->g, rho, dt, u, c->C0, c->V0, c->gp, o->force, c->psi, c->s);
    visc_solve(c, rho, dt, c->eta0, c->eb0, c->psi, c->u1, o->rtol_visc, k, 4);
    if (tp) vec_copy(N3, c->u1, tp->us2, c->s);
    project(5);
    vec_copy(N3, c->u1, u, c->s);
    vec_copy(NP, pw, p, c->s);
    op_finalize_state(c->g, u, nodal ? nullptr : p, c->s);
    if ((h = hip_check("eb_rk2_step"))) return h;
    // one read-back for the whole step
    return step_status(c, k, stats, false, rheo, o);
}

}  // namespace

extern "C" {

int eb_rk2_step(eb_ctx* c, const eb_rheology* rheo, const double* theta, double dt,
                const eb_step_opts* o, double* u, double* p, eb_step_stats* stats,
                void* stream) {
    if (!c) return set_err(EB_EINVAL, "null context");
    StreamScope scope_(c, stream);
    return rk2_impl(c, rheo, theta, dt, o, u, p, stats, nullptr);
}

size_t eb_tape_bytes(const eb_ctx* c) {
    if (!c) return 0;
    TapeV t;
    return tape_carve(c, nullptr, &t);
}

int eb_rk2_step_taped(eb_ctx* c, const eb_rheology* rheo, const double* theta, double dt,
                      const eb_step_opts* o, double* u, double* p, void* tape,
                      eb_step_stats* stats, void* stream) {
    if (!c || !tape) return set_err(EB_EINVAL, "null context or tape");
    StreamScope scope_(c, stream);
    TapeV t;
    tape_carve(c, (char*)tape, &t);
    return rk2_impl(c, rheo, theta, dt, o, u, p, stats, &t);
}

int eb_rk2_step_adjoint(eb_ctx* c, const eb_rheology* rheo, const double* theta, double dt,
                        const eb_step_opts* o, const double* u0, const void* tape, double* ub,
                        double* pb, double* tau0b, double* thetab, double* tau0bar,
                        eb_step_stats* stats, void* stream) {
    if (!c || !rheo || !o || !u0 || !tape || !ub || !pb)
        return set_err(EB_EINVAL, "null argument");
    if (o->projection == EB_PROJ_NODAL)
        return set_err(EB_EINVAL, "the adjoint covers the cell-centred projection only");
    if (int e_ = check_rheology(*rheo)) return e_;
    if (!(rheo->rho > 0.0) || !(dt > 0.0)) return set_err(EB_EINVAL, "rho and dt must be > 0");
    StreamScope scope_(c, stream);
    TapeV t;
    tape_carve(c, (char*)const_cast<void*>(tape), &t);
    SolveCfg k = cfg_of(o);
    c->fp64_fallbacks = 0;
    const GeomV& g = c->g;
    long N = c->N, N3 = 3 * N;
    int nc = c->ncut;
    double rho = rheo->rho, beta = dt / rho;
    double rt_mac = o->rtol_mac > 0 ? o->rtol_mac : 1e-12;
    double *x = c->u1, *pbs = c->p1, *Cb = c->C0, *Vb = c->V0;
    vec_fill(N3, 0.0, c->ubm, c->s);
    vec_fill(N3, 0.0, Cb, c->s);
    vec_fill(N3, 0.0, Vb, c->s);
    vec_fill(N, 0.0, c->ehb, c->s);
    vec_fill(N, 0.0, c->tbs, c->s);
    if (nc > 0) vec_fill(nc, 0.0, c->ebhb, c->s);
    adj_mask_open(g, 3, ub, x, c->s);
    adj_mask_open(g, 1, pb, pbs, c->s);
    // corrector: projection, viscous solve, psi
    cc_project_adj(c, beta, x, pbs, o->rtol_proj, k, 5);
    visc_solve_adj(c, rho, dt, t.ea, t.eba, t.us2, x, o->rtol_visc, k, 4, c->ehb, c->ebhb);
    psi_adj(c, rho, dt, c->ubm, Cb, Vb, pbs);
    // the averaged operator and explicit terms: half to each stage
    adj_scale(N3, 0.5, Cb, c->s);
    adj_scale(N3, 0.5, Vb, c->s);
    adj_scale(N, 0.5, c->ehb, c->s);
    adj_scale(nc, 0.5, c->ebhb, c->s);
    vec_fill(N3, 0.0, x, c->s);
    derived_adj(c, *rheo, theta, t.u1, t.uf1, Cb, c->ehb, c->ebhb, Vb, x, c->tbs, rt_mac, k, 3);
    // predictor
    cc_project_adj(c, beta, x, pbs, o->rtol_proj, k, 2);
    visc_solve_adj(c, rho, dt, t.em, t.ebm, t.us1, x, o->rtol_visc, k, 1, c->ehb, c->ebhb);
    psi_adj(c, rho, dt, c->ubm, Cb, Vb, pbs);
    derived_adj(c, *rheo, theta, u0, t.ufm, Cb, c->ehb, c->ebhb, Vb, c->ubm, c->tbs, rt_mac, k,
                0);
    adj_mask_open(g, 3, c->ubm, ub, c->s);
    adj_mask_open(g, 1, pbs, pb, c->s);
    int h;
    if ((h = hip_check("eb_rk2_step_adjoint"))) return h;
    if ((h = yield_adjoint_out(c, rheo->tau0, theta, tau0b, thetab, tau0bar))) return h;
    return step_status(c, k, stats, true);
}

int eb_drag(const eb_ctx* cc, const eb_rheology* rheo, const double* theta, const double* u,
            const double* p, double F[3], void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !rheo || !u || !p || !F) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    StreamScope scope_(c, stream);
    F[0] = F[1] = F[2] = 0.0;
    if (c->ncut == 0) return EB_OK;
    op_wall_grad(c->g, u, c->gw, c->s);
    op_gcc(c->g, p, c->gp, c->s);
    op_drag_terms(c->g, *rheo, theta, c->gw, p, c->gp, c->DC, c->s);
    red_sum(c->ncut, 3, c->DC, c->part, c->red, c->s);
    int e = fetch(c, F, 3);
    if (e) return e;
    return hip_check("eb_drag");
}

int eb_drag_nodal(const eb_ctx* cc, const eb_rheology* rheo, const double* theta,
                  const double* u, const double* pn, double F[3], void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !rheo || !u || !pn || !F) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    StreamScope scope_(c, stream);
    F[0] = F[1] = F[2] = 0.0;
    if (c->ncut == 0) return EB_OK;
    op_wall_grad(c->g, u, c->gw, c->s);
    nd_peb(c->g, pn, c->peb, c->s);
    op_drag_terms(c->g, *rheo, theta, c->gw, nullptr, nullptr, c->DC, c->s, c->peb);
    red_sum(c->ncut, 3, c->DC, c->part, c->red, c->s);
    int e = fetch(c, F, 3);
    if (e) return e;
    return hip_check("eb_drag_nodal");
}

int eb_drag_noalloc(const eb_ctx* c, const eb_rheology* rheo, const double* theta,
                    const double* u, const double* p, double F[3], void* stream) {
    if (!c || !rheo || !u || !p || !F) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    if (c->ncut > NOALLOC_NCUT)
        return set_err(EB_EINVAL, "eb_drag_noalloc: %d cut cells exceed its scratch limit of %ld",
                       c->ncut, NOALLOC_NCUT);
    F[0] = F[1] = F[2] = 0.0;
    if (c->ncut == 0) return EB_OK;
    double* scr = nullptr;
    if (int e = noalloc_scratch(&scr)) return e;
    hipStream_t s = (hipStream_t)stream;
    // views of the scratch for this geometry: per-cut arrays are [component][ncut]
    double* gw = scr;
    double* terms = scr + 3 * NOALLOC_NCUT;
    double* part = scr + 6 * NOALLOC_NCUT;
    double* out = part + 4096;
    op_wall_grad(c->g, u, gw, s);
    op_drag_terms(c->g, *rheo, theta, gw, p, nullptr, terms, s);
    red_sum(c->ncut, 3, terms, part, out, s);
    HIPN(hipMemcpyAsync(F, out, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPN(hipStreamSynchronize(s));
    return hip_check("eb_drag_noalloc");
}

int eb_drag_adjoint(const eb_ctx* cc, const eb_rheology* rheo, const double* theta,
                    const double* u, const double fbar[3], double* ub, double* pb,
                    double* tau0b, double* thetab, double* tau0bar, void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !rheo || !u || !fbar || !ub || !pb) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    StreamScope scope_(c, stream);
    if (c->ncut == 0) return EB_OK;
    op_wall_grad(c->g, u, c->gw, c->s);
    vec_fill(3 * c->N, 0.0, c->gp, c->s);
    vec_fill(c->N, 0.0, c->tbs, c->s);
    adj_drag(c->g, *rheo, theta, c->gw, fbar, c->gwb, c->tbs, pb, c->gp, c->s);
    adj_grad_gather(c->g, c->wt, nullptr, c->gwb, ub, c->s);
    adj_gcc_T(c->g, 1.0, c->gp, pb, pb, c->s);
    if (int h = hip_check("eb_drag_adjoint")) return h;
    return yield_adjoint_out(c, rheo->tau0, theta, tau0b, thetab, tau0bar);
}

int eb_mac_project_adjoint(eb_ctx* c, double beta, double* fbx, double* fby, double* fbz,
                           double rtol, const eb_step_opts* opts, int* iters, void* stream) {
    if (!c || !fbx || !fby || !fbz) return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    double* fb[3] = {fbx, fby, fbz};
    mac_project_adj(c, beta, fb, rtol, k, 0);
    int h = hip_check("eb_mac_project_adjoint");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    return slot_code(sl, "adjoint MAC projection", k.max_iter);
}

int eb_cc_project_adjoint(eb_ctx* c, double beta, double* ub, double* pb, double rtol,
                          const eb_step_opts* opts, int* iters, void* stream) {
    if (!c || !ub || !pb) return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    adj_mask_open(c->g, 3, ub, c->u1, c->s);
    adj_mask_open(c->g, 1, pb, c->p1, c->s);
    cc_project_adj(c, beta, c->u1, c->p1, rtol, k, 0);
    vec_copy(3 * c->N, c->u1, ub, c->s);
    vec_copy(c->N, c->p1, pb, c->s);
    int h = hip_check("eb_cc_project_adjoint");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = sl[1];
    return slot_code(sl, "adjoint projection", k.max_iter);
}

int eb_visc_solve_adjoint(eb_ctx* c, double rho, double dt, const double* eta,
                          const double* eta_eb, const double* x, const double* xb, double rtol,
                          const eb_step_opts* opts, double* psib, double* etab, double* etaebb,
                          int* iters, void* stream) {
    if (!c || !eta || !x || !xb || !psib || !etab || ((!eta_eb || !etaebb) && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    visc_solve_adj(c, rho, dt, eta, eta_eb, x, xb, rtol, k, 0, etab, etaebb);
    adj_psi(c->g, 0.0, 0.0, c->lam, psib, c->ubm, c->C0, c->V0, c->s);
    int h = hip_check("eb_visc_solve_adjoint");
    if (h) return h;
    int sl[2];
    if ((h = read_slots(c, 1, sl))) return h;
    if (iters) *iters = (sl[1] + 1) / 2;
    return slot_code(sl, "transposed viscous solve", k.max_iter);
}

int eb_derived_adjoint(eb_ctx* c, const eb_rheology* rheo, const double* theta, const double* u,
                       const double* Cb, const double* etab, const double* etaebb,
                       const double* Vb, double* ub, double* tau0b, const eb_step_opts* opts,
                       int* iters, void* stream) {
    if (!c || !rheo || !u || !Cb || !etab || !Vb || !ub || !tau0b ||
        (!etaebb && c->ncut > 0))
        return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    StreamScope scope_(c, stream);
    SolveCfg k = cfg_of(opts);
    double rtol = opts && opts->rtol_mac > 0 ? opts->rtol_mac : 1e-12;
    // the forward face velocities: extrapolate and project (slot 1), keep a copy
    op_face_extrap(c->g, u, c->f, SwitchV{}, c->s);
    vec_fill(c->N, 0.0, c->phi, c->s);
    mac_project(c, 1.0, c->f, c->phi, rtol, k, 1, false);
    double* uf[3];
    for (int d = 0; d < 3; d++) {
        uf[d] = c->kv[d];  // Krylov scratch, idle here
        vec_copy(face_count(c->grid, d), c->f[d], uf[d], c->s);
    }
    derived_adj(c, *rheo, theta, u, uf, Cb, etab, etaebb, Vb, ub, tau0b, rtol, k, 0);
    int h = hip_check("eb_derived_adjoint");
    if (h) return h;
    int sl[4];
    if ((h = read_slots(c, 2, sl))) return h;
    if (iters) *iters = sl[1];
    if (sl[2] != 2) return slot_code(sl + 2, "MAC projection", k.max_iter);
    return slot_code(sl, "adjoint MAC projection", k.max_iter);
}

int eb_stable_dt(const eb_ctx* cc, const eb_rheology* rheo, const double* theta,
                 const double* u, const double force[3], double c_cfl, double* dt,
                 void* stream) {
    if (!cc || !rheo || !u || !force || !dt) return set_err(EB_EINVAL, "null argument");
    if (int e_ = check_rheology(*rheo)) return e_;
    if (!(c_cfl > 0.0) || !(rheo->rho > 0.0)) return set_err(EB_EINVAL, "c_cfl and rho must be > 0");
    if (rheo->law >= EB_LAW_POWER)
        return set_err(EB_EINVAL, "the time-step rule is stated for the Newtonian and Bingham laws");
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    hipStream_t s = (hipStream_t)stream;
    double m[2];
    red_cfl(c->g, u, theta, c->part, c->red, s);
    HIPN(hipMemcpyAsync(m, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPN(hipStreamSynchronize(s));
    if (int h = hip_check("eb_stable_dt")) return h;
    *dt = stable_dt_of(c, *rheo, m[0], m[1], force, c_cfl);
    return EB_OK;
}

int eb_pressure_gradient(const eb_ctx* cc, const double* p, double* gp, void* stream) {
    eb_ctx* c = const_cast<eb_ctx*>(cc);
    if (!c || !p || !gp) return set_err(EB_EINVAL, "null argument");
    op_gcc(c->g, p, gp, (hipStream_t)stream);
    return hip_check("eb_pressure_gradient");
}

}  // extern "C"
