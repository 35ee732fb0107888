// Host side of the elmddm C ABI: problem validation, point layout, index maps
// for the interface system, device workspace, and the solve pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/elmddm.h"
#include "internal.h"

using namespace elmddm;

namespace {

// The batched kernels index the subdomains of a batch (and the instances)
// by a grid dimension other than x, which holds at most 65535 blocks.
constexpr int64_t kMaxSubdomains = 65535;

thread_local std::string g_last_error;
}

namespace elmddm {
int record_error(int status, const char* msg)
{
    g_last_error = msg;
    return status;
}
}  // namespace elmddm

namespace {

elmddm_status fail(elmddm_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// tanh feature blocks grow worse conditioned with the neuron count (at the
// configured scales: column-scaled kappa ~1e9 at n = 400, 1e12..1e13 at
// n = 800, ~1e15 at n = 1000); each shifted pass divides kappa by ~1e4 and
// the unshifted passes need it below ~1e8
int default_passes(int n) { return n >= 900 ? 5 : (n >= 600 ? 4 : 3); }

long long interface_count(const elmddm_problem& p)
{
    return ((long long)(p.nsub_x - 1) * p.nsub_y + (long long)p.nsub_x * (p.nsub_y - 1)) * p.m_ifc_edge;
}

struct EdgeOwner {
    int s;     // subdomain
    int slot;  // local interface slot of the edge's first point
};

}  // namespace

struct elmddm_plan {
    elmddm_problem p{};
    int B = 1;    // problem instances per solve (same geometry)
    int gram_code = -2;   // kernel for the Gram products (see gram_product)
    float tune_ms[2][9] = {};   // last autotune: Gram / triangular-solve time per candidate
    int trsm_code = -2;   // kernel for the triangular-solve products
    bool env_fused = true;
    int mode = ELMDDM_MODE_FP64;
    int NT = 0;   // subdomains over all instances, B * N
    int N = 0, n = 0, nx = 0, ny = 0, q2 = 0, mg = 0, mb = 0;
    int maxb = 0, maxk = 0, max_rows = 0;
    int mI = 0, kpad = 0, hrow = 0, dbase = 0, ldx = 0, gram_rows = 0, ldg = 0, ldp = 0;
    int nG = 0, nE = 0, nblk = 0, nblkS = 0, lds = 0;
    int64_t nB = 0;
    long long sX = 0, sG = 0, sL = 0, sD = 0, sP = 0;
    double hx = 0, hy = 0;

    // host layout
    std::vector<double> int_pts, bnd_pts, ifc_pts;  // interleaved (x, y)
    std::vector<double> cx, cy;

    // device memory
    std::vector<void*> allocs;
    uint64_t bytes = 0;
    double *X0 = nullptr, *X1 = nullptr, *G = nullptr, *Linv[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // CholeskyQR passes (3 to 5): passes 1 .. npass - 2 are shifted, the last
    // one also factors the rhs row.  After a solve, Qprev holds Q of pass
    // npass - 1 (all rows) and Xfin the last pass's interface rows, h row and
    // flux rows.
    int npass = 3;
    double *Qprev = nullptr, *Xfin = nullptr;
    double *Dinv = nullptr, *Tbuf = nullptr, *P = nullptr, *Mbuf = nullptr, *abuf = nullptr;
    double *Sx = nullptr, *Skeep = nullptr, *DinvS = nullptr, *yvec = nullptr, *dsave = nullptr;
    double *uperm = nullptr, *bs1 = nullptr, *bs2 = nullptr, *SL = nullptr;
    int32_t* d_perm = nullptr;
    std::vector<int> rend;   // per 64-panel of S: one past the last row of the envelope
    std::vector<int> kbeg;   // per 64-block row of S: first column reaching it
    double *d_rx = nullptr, *d_ry = nullptr, *d_rnx = nullptr, *d_rny = nullptr;
    double *d_cx = nullptr, *d_cy = nullptr;
    int32_t *d_kind = nullptr, *d_src = nullptr, *d_cmap = nullptr, *d_gidx = nullptr;
    int32_t *d_mdesc = nullptr, *d_adesc = nullptr, *d_tptr = nullptr, *d_tdesc = nullptr;
    int32_t *d_mptr = nullptr, *d_mlist = nullptr, *d_qdesc = nullptr, *d_gptr = nullptr;
    int32_t *d_nzb = nullptr, *d_zb = nullptr;   // S blocks with / without contributions
    int32_t* d_zb_env = nullptr;                 // the zero blocks the envelope factorisation reads
    int n_nzb = 0, n_zb = 0, n_zb_env = 0;
    int32_t *d_gdesc = nullptr;
    int n_mblocks = 0;
    DevInfo* d_info = nullptr;
    bool keep_schur = false;
    bool schur_valid = false;
    hipStream_t last_stream = nullptr;
    bool solved = false;
    // side stream and fork / join events of the envelope Cholesky's lookahead
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // interface system without a dense S: CG on the matrix-free operator
    bool mfree = false;
    double cg_tol = 1e-12;
    int cg_maxit = 100000;
    std::vector<int32_t> cg_iters;
    std::vector<double> cg_relres;
    bool cg_failed = false;
    double *MbT = nullptr;   // transposed M blocks (matrix-free operator)
    int cg_precond = 1;      // 0: plain CG (the paper's), 1: block-Jacobi on the edge blocks
    double *DE = nullptr, *DEinv = nullptr;   // edge blocks of S and their inverse factors
    double *tbuf = nullptr, *wbuf = nullptr, *mfX = nullptr, *mfR = nullptr, *mfP = nullptr, *mfQ = nullptr,
           *mfS = nullptr;
    int32_t *d_mstart = nullptr, *d_mE = nullptr, *d_ident = nullptr;
    bool factors_valid = false;   // the workspace holds the factors of the last solve
    // further right-hand sides (elmddm_plan_reserve_rhs / elmddm_solve_rhs)
    int rhs_cap = 0;
    double *Fr = nullptr, *Tm = nullptr, *Hm = nullptr, *Ph = nullptr, *abufR = nullptr;
    double *yR = nullptr, *uR = nullptr, *Vm = nullptr;
    double *cgX = nullptr, *cgR = nullptr, *cgP = nullptr, *cgQ = nullptr, *cgS = nullptr;
    double *tbufR = nullptr, *wbufR = nullptr;   // matrix-free operator scratch for R right-hand sides
    int32_t *d_rb = nullptr, *d_re = nullptr;   // row band of each 64-column block of S
    // stage timing
    bool timing = false;
    hipEvent_t ev[ELMDDM_NUM_STAGES + 1] = {};
    hipEvent_t pev[16] = {};  // per-pass Gram / Cholesky / triangular-solve boundaries
    bool ev_ready = false;
    bool ev_pending = false;
    double stage_ms[ELMDDM_NUM_STAGES] = {};
    double pass_ms[15] = {};  // per CholeskyQR pass: Gram, Cholesky + inverses, triangular solve
    int timed_solves = 0;

    bool dry = false;   // size query only: count bytes, allocate nothing

    template <class T>
    elmddm_status dalloc(T** ptr, size_t count)
    {
        *ptr = nullptr;
        if (count == 0) count = 1;
        if (dry) {
            bytes += count * sizeof(T);
            return ELMDDM_OK;
        }
        void* q = nullptr;
        if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ELMDDM_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
        allocs.push_back(q);
        bytes += count * sizeof(T);
        *ptr = static_cast<T*>(q);
        return ELMDDM_OK;
    }

    template <class T>
    elmddm_status upload(T** ptr, const std::vector<T>& v)
    {
        elmddm_status st = dalloc(ptr, v.size());
        if (st != ELMDDM_OK || dry) return st;
        if (!v.empty() && hipMemcpy(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return fail(ELMDDM_HIP_ERROR, "hipMemcpy failed during plan creation");
        return ELMDDM_OK;
    }

    void mark(int i, hipStream_t st)
    {
        if (timing) (void)hipEventRecord(ev[i], st);
    }

    // Fold the events of the previous timed solve into the totals.
    void harvest()
    {
        if (!ev_pending) return;
        (void)hipEventSynchronize(ev[ELMDDM_NUM_STAGES]);
        auto el = [](hipEvent_t a, hipEvent_t b) {
            float ms = 0.f;
            return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
        };
        stage_ms[0] += el(ev[0], ev[1]);
        for (int p = 0; p < npass; ++p) {
            const double tg = el(pev[3 * p], pev[3 * p + 1]);
            const double tc = el(pev[3 * p + 1], pev[3 * p + 2]);
            const double tt = el(pev[3 * p + 2], pev[3 * p + 3]);
            stage_ms[1] += tg;
            stage_ms[2] += tc;
            stage_ms[3] += tt;
            pass_ms[3 * p] += tg;
            pass_ms[3 * p + 1] += tc;
            pass_ms[3 * p + 2] += tt;
        }
        stage_ms[3] += el(pev[3 * npass], ev[4]);
        for (int i = 4; i < ELMDDM_NUM_STAGES; ++i) stage_ms[i] += el(ev[i], ev[i + 1]);
        ++timed_solves;
        ev_pending = false;
    }

    ~elmddm_plan()
    {
        if (ev_ready)
            {
            for (auto& e : ev) (void)hipEventDestroy(e);
            for (auto& e : pev) (void)hipEventDestroy(e);
        }
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        for (void* q : allocs) (void)hipFree(q);
    }
};

namespace {

elmddm_status validate(const elmddm_problem* p)
{
    if (!p) return fail(ELMDDM_INVALID_ARG, "problem is NULL");
    if (!(p->x1 > p->x0) || !(p->y1 > p->y0) || !std::isfinite(p->x0) || !std::isfinite(p->x1) ||
        !std::isfinite(p->y0) || !std::isfinite(p->y1))
        return fail(ELMDDM_INVALID_ARG, "domain must be a finite rectangle with x1 > x0, y1 > y0");
    if (p->nsub_x < 1 || p->nsub_y < 1 || p->nsub_x > 4096 || p->nsub_y > 4096)
        return fail(ELMDDM_INVALID_ARG, "nsub_x, nsub_y must be in [1, 4096]");
    if (p->neurons < 1 || p->neurons > 1024)
        return fail(ELMDDM_INVALID_ARG, "neurons must be in [1, 1024]");
    if (p->q_x < 1 || p->q_y < 1 || p->m_bdry_edge < 1 || p->m_ifc_edge < 1)
        return fail(ELMDDM_INVALID_ARG, "point counts must be positive");
    if (p->m_ifc_edge > 64) return fail(ELMDDM_UNSUPPORTED, "m_ifc_edge > 64 is not supported");
    if ((int64_t)p->q_x * p->q_y < p->neurons)
        return fail(ELMDDM_INVALID_ARG,
                    "q_x*q_y must be >= neurons (full column rank needs m_i >= n_N, Section 3)");
    if ((int64_t)p->q_x * p->q_y > (1 << 22)) return fail(ELMDDM_INVALID_ARG, "too many interior points");
    if (p->op != ELMDDM_OP_POISSON && p->op != ELMDDM_OP_VARCOEF)
        return fail(ELMDDM_INVALID_ARG, "unknown operator");
    return ELMDDM_OK;
}

void edge_points(double p0x, double p0y, double p1x, double p1y, int m, std::vector<double>& out)
{
    for (int k = 0; k < m; ++k) {
        const double t = ((double)k + 0.5) / (double)m;
        out.push_back(p0x + t * (p1x - p0x));
        out.push_back(p0y + t * (p1y - p0y));
    }
}

elmddm_status build(elmddm_plan* P)
{
    const elmddm_problem& p = P->p;
    const int nx = p.nsub_x, ny = p.nsub_y;
    P->nx = nx;
    P->ny = ny;
    P->N = nx * ny;
    P->NT = P->B * P->N;
    P->n = p.neurons;
    P->q2 = p.q_x * p.q_y;
    P->mg = p.m_ifc_edge;
    P->mb = p.m_bdry_edge;
    P->hx = (p.x1 - p.x0) / nx;
    P->hy = (p.y1 - p.y0) / ny;
    const double hx = P->hx, hy = P->hy;
    auto xline = [&](int i) { return p.x0 + i * hx; };
    auto yline = [&](int j) { return p.y0 + j * hy; };
    const int mg = P->mg, mb = P->mb, N = P->N, n = P->n;

    // interface edges: vertical (edge row outer, x inner), then horizontal
    const int nV = (nx - 1) * ny, nH = nx * (ny - 1);
    P->nE = nV + nH;
    P->nG = P->nE * mg;
    auto vid = [&](int i, int j) { return j * (nx - 1) + (i - 1); };
    auto hid = [&](int i, int j) { return nV + (j - 1) * nx + i; };
    P->ifc_pts.clear();
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) edge_points(xline(i), yline(j), xline(i), yline(j + 1), mg, P->ifc_pts);
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) edge_points(xline(i), yline(j), xline(i + 1), yline(j), mg, P->ifc_pts);

    // per-subdomain edges
    static const double NRM[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
    std::vector<std::vector<std::pair<int, int>>> sub_edges(N);  // (edge, slot)
    std::vector<std::vector<EdgeOwner>> owners(P->nE);
    std::vector<int> nbnd(N, 0), nifc(N, 0);
    P->cx.assign(N, 0.0);
    P->cy.assign(N, 0.0);
    struct SubPts {
        std::vector<double> bnd, ifc, nrm;
        std::vector<int> gidx;
    };
    std::vector<SubPts> sp(N);
    P->int_pts.clear();
    P->bnd_pts.clear();
    for (int sy = 0; sy < ny; ++sy)
        for (int sx = 0; sx < nx; ++sx) {
            const int s = sy * nx + sx;
            const double xa = xline(sx), ya = yline(sy), xb = xline(sx + 1), yb = yline(sy + 1);
            P->cx[s] = xa + 0.5 * hx;
            P->cy[s] = ya + 0.5 * hy;
            for (int iy = 0; iy < p.q_y; ++iy)
                for (int ix = 0; ix < p.q_x; ++ix) {
                    const double tx = ((double)ix + 0.5) / (double)p.q_x;
                    const double ty = ((double)iy + 0.5) / (double)p.q_y;
                    P->int_pts.push_back(xa + tx * hx);
                    P->int_pts.push_back(ya + ty * hy);
                }
            struct E {
                double p0x, p0y, p1x, p1y;
                bool ext;
                int id;
            } edges[4] = {
                {xa, ya, xb, ya, sy == 0, sy == 0 ? -1 : hid(sx, sy)},
                {xb, ya, xb, yb, sx == nx - 1, sx == nx - 1 ? -1 : vid(sx + 1, sy)},
                {xa, yb, xb, yb, sy == ny - 1, sy == ny - 1 ? -1 : hid(sx, sy + 1)},
                {xa, ya, xa, yb, sx == 0, sx == 0 ? -1 : vid(sx, sy)},
            };
            for (int e = 0; e < 4; ++e) {
                if (edges[e].ext) {
                    edge_points(edges[e].p0x, edges[e].p0y, edges[e].p1x, edges[e].p1y, mb, sp[s].bnd);
                } else {
                    const int id = edges[e].id;
                    const int slot = (int)sp[s].gidx.size();
                    sub_edges[s].push_back({id, slot});
                    owners[id].push_back({s, slot});
                    for (int k = 0; k < mg; ++k) {
                        const int gi = id * mg + k;
                        sp[s].gidx.push_back(gi);
                        sp[s].ifc.push_back(P->ifc_pts[2 * gi]);
                        sp[s].ifc.push_back(P->ifc_pts[2 * gi + 1]);
                        sp[s].nrm.push_back(NRM[e][0]);
                        sp[s].nrm.push_back(NRM[e][1]);
                    }
                }
            }
            nbnd[s] = (int)sp[s].bnd.size() / 2;
            nifc[s] = (int)sp[s].gidx.size();
            P->bnd_pts.insert(P->bnd_pts.end(), sp[s].bnd.begin(), sp[s].bnd.end());
        }
    P->nB = (int64_t)P->bnd_pts.size() / 2;
    P->maxb = *std::max_element(nbnd.begin(), nbnd.end());
    P->maxk = *std::max_element(nifc.begin(), nifc.end());
    P->max_rows = 0;
    for (int s = 0; s < N; ++s) P->max_rows = std::max(P->max_rows, P->q2 + nbnd[s] + nifc[s]);

    // X row layout per subdomain:
    // [0, mI) interior + boundary (+ zero pad) | [mI, mI+kpad) interface values |
    // [hrow, hrow+16) h row + pad | [dbase, dbase+kpad) flux rows
    P->mI = round_up(P->q2 + P->maxb, 16);
    P->kpad = round_up(P->maxk, 16);
    P->hrow = P->mI + P->kpad;
    P->dbase = P->hrow + 16;
    P->ldx = P->dbase + P->kpad;
    P->gram_rows = P->mI + P->kpad;
    P->ldg = round_up(n + 1, 16);
    P->ldp = 2 * P->kpad + 16;
    P->nblk = (n + NB - 1) / NB;
    P->nblkS = (P->nG + NB - 1) / NB;
    P->lds = P->nG + 1;
    P->sX = (long long)P->ldx * (n + 1);
    P->sG = (long long)P->ldg * (n + 1);
    P->sL = (long long)P->ldg * n;
    P->sD = (long long)P->nblk * NB * NB;
    P->sP = (long long)P->ldp * (P->kpad + 1);

    const int ldx = P->ldx;
    std::vector<double> rx((size_t)N * ldx, 0.0), ry((size_t)N * ldx, 0.0), rnx((size_t)N * ldx, 0.0),
        rny((size_t)N * ldx, 0.0);
    std::vector<int32_t> kind((size_t)N * ldx, ROW_ZERO), src((size_t)N * ldx, 0),
        cmap((size_t)N * ldx, -1), gidx((size_t)N * std::max(P->kpad, 1), -1);
    int64_t bcount = 0;
    for (int s = 0; s < N; ++s) {
        const size_t base = (size_t)s * ldx;
        for (int i = 0; i < P->q2; ++i) {
            rx[base + i] = P->int_pts[2 * ((size_t)s * P->q2 + i)];
            ry[base + i] = P->int_pts[2 * ((size_t)s * P->q2 + i) + 1];
            kind[base + i] = ROW_INTERIOR;
            src[base + i] = s * P->q2 + i;
            cmap[base + i] = i;
        }
        for (int i = 0; i < nbnd[s]; ++i) {
            const size_t r = base + P->q2 + i;
            rx[r] = sp[s].bnd[2 * i];
            ry[r] = sp[s].bnd[2 * i + 1];
            kind[r] = ROW_BOUNDARY;
            src[r] = (int32_t)(bcount + i);
            cmap[r] = P->q2 + i;
        }
        bcount += nbnd[s];
        for (int i = 0; i < nifc[s]; ++i) {
            size_t r = base + P->mI + i;
            rx[r] = sp[s].ifc[2 * i];
            ry[r] = sp[s].ifc[2 * i + 1];
            kind[r] = ROW_IFC_VALUE;
            cmap[r] = P->q2 + nbnd[s] + i;
            r = base + P->dbase + i;
            rx[r] = sp[s].ifc[2 * i];
            ry[r] = sp[s].ifc[2 * i + 1];
            rnx[r] = sp[s].nrm[2 * i];
            rny[r] = sp[s].nrm[2 * i + 1];
            kind[r] = ROW_FLUX;
            cmap[r] = -2 - i;
            gidx[(size_t)s * P->kpad + i] = sp[s].gidx[i];
        }
    }

    // Interface system index structures.
    // adjacency of a flux edge g: all interface edges of its two owners
    std::vector<std::vector<int>> adj(P->nE);
    for (int g = 0; g < P->nE; ++g) {
        for (const EdgeOwner& o : owners[g])
            for (auto& es : sub_edges[o.s]) adj[g].push_back(es.first);
        std::sort(adj[g].begin(), adj[g].end());
        adj[g].erase(std::unique(adj[g].begin(), adj[g].end()), adj[g].end());
    }
    auto slot_of = [&](int s, int e) {
        for (auto& es : sub_edges[s])
            if (es.first == e) return es.second;
        return -1;
    };
    std::vector<int32_t> mdesc, adesc, qdesc;
    std::map<std::pair<int, int>, int> mid;
    for (int g = 0; g < P->nE; ++g) {
        for (int E : adj[g]) {
            int32_t d[8] = {-1, 0, 0, -1, 0, 0, 0, 0};
            int t = 0;
            for (const EdgeOwner& o : owners[g]) {
                const int se = slot_of(o.s, E);
                if (se < 0) continue;
                d[3 * t] = o.s;
                d[3 * t + 1] = o.slot;
                d[3 * t + 2] = se;
                ++t;
            }
            mid[{g, E}] = (int)(mdesc.size() / 8);
            mdesc.insert(mdesc.end(), d, d + 8);
        }
        int32_t a[4] = {-1, 0, -1, 0};
        for (size_t t = 0; t < owners[g].size() && t < 2; ++t) {
            a[2 * t] = owners[g][t].s;
            a[2 * t + 1] = owners[g][t].slot;
        }
        adesc.insert(adesc.end(), a, a + 4);
        qdesc.insert(qdesc.end(), a, a + 4);
    }
    P->n_mblocks = (int)(mdesc.size() / 8);
    // matrix-free operator: the value edge of every M block, blocks grouped by flux edge
    std::vector<int32_t> mstart(P->nE + 1, 0), mE;
    for (int g = 0; g < P->nE; ++g) {
        mstart[g + 1] = mstart[g] + (int32_t)adj[g].size();
        for (int E : adj[g]) mE.push_back(E);
    }
    std::vector<int32_t> ident(std::max(P->nE, 1));
    for (int e = 0; e < P->nE; ++e) ident[e] = e;
    const size_t nEE = P->mfree ? 0 : (size_t)P->nE * P->nE;
    if (nEE > (size_t)INT32_MAX)
        return fail(ELMDDM_UNSUPPORTED, "too many interface edges for a dense interface system (use MATRIX_FREE)");
    std::vector<std::vector<int32_t>> tl(nEE), ml(nEE);
    for (int s = 0; s < N && !P->mfree; ++s)
        for (auto& e1 : sub_edges[s])
            for (auto& e2 : sub_edges[s]) {
                const size_t blk = (size_t)e1.first + (size_t)e2.first * P->nE;
                tl[blk].insert(tl[blk].end(), {s, e1.second, e2.second, e1.first == e2.first ? 1 : 0});
            }
    std::vector<std::vector<int32_t>> gl(P->nE);
    for (int g = 0; g < P->nE; ++g)
        for (int E1 : adj[g]) {
            gl[E1].push_back(mid[{g, E1}]);
            gl[E1].push_back(g);
            for (int E2 : adj[g]) {
                if (P->mfree) break;
                const size_t blk = (size_t)E1 + (size_t)E2 * P->nE;
                ml[blk].push_back(mid[{g, E1}]);
                ml[blk].push_back(mid[{g, E2}]);
            }
        }
    std::vector<int32_t> tptr(nEE + 1, 0), mptr(nEE + 1, 0), tdesc, mlist, gptr(P->nE + 1, 0), gdesc;
    std::vector<int32_t> nzb, zb, zb_env;
    for (size_t b = 0; b < nEE; ++b) {
        tptr[b + 1] = tptr[b] + (int32_t)(tl[b].size() / 4);
        mptr[b + 1] = mptr[b] + (int32_t)(ml[b].size() / 2);
        tdesc.insert(tdesc.end(), tl[b].begin(), tl[b].end());
        mlist.insert(mlist.end(), ml[b].begin(), ml[b].end());
        (tl[b].empty() && ml[b].empty() ? zb : nzb).push_back((int32_t)b);
    }
    P->n_nzb = (int)nzb.size();
    P->n_zb = (int)zb.size();
    for (int e = 0; e < P->nE; ++e) {
        gptr[e + 1] = gptr[e] + (int32_t)(gl[e].size() / 2);
        gdesc.insert(gdesc.end(), gl[e].begin(), gl[e].end());
    }

    // Edge order for the interface system: by edge midpoint (y, then x).  With
    // this order S is confined to a narrow envelope around its diagonal.
    std::vector<int32_t> perm(P->nE, 0);
    {
        std::vector<std::pair<std::pair<double, double>, int>> key(P->nE);
        for (int e = 0; e < P->nE; ++e) {
            double mx, my;
            if (e < nV) {
                const int i = e % (nx - 1) + 1, j = e / (nx - 1);
                mx = p.x0 + i * hx;
                my = p.y0 + (j + 0.5) * hy;
            } else {
                const int e2 = e - nV, i = e2 % nx, j = e2 / nx + 1;
                mx = p.x0 + (i + 0.5) * hx;
                my = p.y0 + j * hy;
            }
            key[e] = {{my, mx}, e};
        }
        std::sort(key.begin(), key.end());
        for (int r = 0; r < P->nE; ++r) perm[key[r].second] = r;
        std::vector<int> lastb(P->nE, 0);
        for (int e2 = 0; e2 < P->nE; ++e2) lastb[perm[e2]] = perm[e2];
        for (int e1 = 0; e1 < P->nE && !P->mfree; ++e1)
            for (int e2 = 0; e2 < P->nE; ++e2) {
                const size_t blk = (size_t)e1 + (size_t)e2 * P->nE;
                if (tl[blk].empty() && ml[blk].empty()) continue;
                const int p1 = perm[e1], p2 = perm[e2];
                if (p1 > p2) lastb[p2] = std::max(lastb[p2], p1);
            }
        std::vector<int> env(P->nG, 0);
        int run = 0;
        for (int c = 0; c < P->nG; ++c) {
            run = std::max(run, (lastb[c / mg] + 1) * mg - 1);
            env[c] = run;
        }
        P->rend.assign(P->nblkS, 0);
        P->kbeg.assign(P->nblkS, 0);
        for (int pb = 0; pb < P->nblkS; ++pb) {
            const int j0 = pb * NB;
            P->rend[pb] = std::min(P->nG, env[std::min(j0 + NB - 1, P->nG - 1)] + 1);
            int c = 0;
            while (c < j0 && env[c] < j0) ++c;
            P->kbeg[pb] = c;
        }
        // Zero blocks that the envelope factorisation reads: some (row, col)
        // of the block with col <= row < rend[col / NB].  The others are never
        // read unless the caller keeps S (then every block is written).
        for (int32_t b : zb) {
            const int pr = perm[b % P->nE] * mg, pc = perm[b / P->nE] * mg;
            bool need = false;
            for (int col = pc; col < pc + mg && !need; ++col)
                need = std::max(pr, col) < std::min(pr + mg, P->rend[col / NB]);
            if (need) zb_env.push_back(b);
        }
        P->n_zb_env = (int)zb_env.size();
    }

    // ---- device allocations ----
    elmddm_status st;
#define TRY(x)                       \
    do {                             \
        st = (x);                    \
        if (st != ELMDDM_OK) return st; \
    } while (0)
    TRY(P->upload(&P->d_rx, rx));
    TRY(P->upload(&P->d_ry, ry));
    TRY(P->upload(&P->d_rnx, rnx));
    TRY(P->upload(&P->d_rny, rny));
    TRY(P->upload(&P->d_kind, kind));
    TRY(P->upload(&P->d_src, src));
    TRY(P->upload(&P->d_cmap, cmap));
    TRY(P->upload(&P->d_gidx, gidx));
    TRY(P->upload(&P->d_cx, P->cx));
    TRY(P->upload(&P->d_cy, P->cy));
    TRY(P->upload(&P->d_mdesc, mdesc));
    TRY(P->upload(&P->d_adesc, adesc));
    TRY(P->upload(&P->d_qdesc, qdesc));
    TRY(P->upload(&P->d_tptr, tptr));
    TRY(P->upload(&P->d_tdesc, tdesc));
    TRY(P->upload(&P->d_mptr, mptr));
    TRY(P->upload(&P->d_mlist, mlist));
    TRY(P->upload(&P->d_nzb, nzb));
    TRY(P->upload(&P->d_zb, zb));
    TRY(P->upload(&P->d_zb_env, zb_env));
    TRY(P->upload(&P->d_gptr, gptr));
    TRY(P->upload(&P->d_gdesc, gdesc));
    TRY(P->upload(&P->d_perm, perm));
    const size_t NT = (size_t)P->NT, Bn = (size_t)P->B;
    const size_t nGm = (size_t)std::max(P->nG, 1);
    TRY(P->dalloc(&P->X0, NT * P->sX));
    TRY(P->dalloc(&P->X1, NT * P->sX));
    TRY(P->dalloc(&P->G, NT * P->sG));
    for (int i = 0; i < P->npass; ++i) TRY(P->dalloc(&P->Linv[i], NT * P->sL));
    TRY(P->dalloc(&P->Dinv, NT * P->sD));
    TRY(P->dalloc(&P->Tbuf, NT * NB * n));
    TRY(P->dalloc(&P->P, NT * P->sP));
    TRY(P->dalloc(&P->Mbuf, Bn * std::max(P->n_mblocks, 1) * mg * mg));
    TRY(P->dalloc(&P->abuf, Bn * std::max(P->nE, 1) * mg));
    if (!P->mfree) {
        TRY(P->dalloc(&P->Sx, Bn * P->lds * nGm));
        TRY(P->dalloc(&P->DinvS, Bn * std::max(P->nblkS, 1) * NB * NB));
        TRY(P->dalloc(&P->SL, Bn * P->lds * nGm));
    } else {
        TRY(P->upload(&P->d_mstart, mstart));
        TRY(P->upload(&P->d_mE, mE));
        TRY(P->upload(&P->d_ident, ident));
        TRY(P->dalloc(&P->tbuf, NT * std::max(P->kpad, 1)));
        TRY(P->dalloc(&P->MbT, Bn * std::max(P->n_mblocks, 1) * mg * mg));
        TRY(P->dalloc(&P->wbuf, Bn * std::max(P->nE, 1) * mg));
        for (double** q : {&P->mfX, &P->mfR, &P->mfP, &P->mfQ}) TRY(P->dalloc(q, Bn * nGm));
        TRY(P->dalloc(&P->mfS, 8 * Bn));
        TRY(P->dalloc(&P->DE, Bn * std::max(P->nE, 1) * 4096));
        TRY(P->dalloc(&P->DEinv, Bn * std::max(P->nE, 1) * 4096));
    }
    TRY(P->dalloc(&P->yvec, Bn * nGm));
    TRY(P->dalloc(&P->dsave, std::max(NT * n, Bn * nGm)));
    TRY(P->dalloc(&P->uperm, Bn * nGm));
    TRY(P->dalloc(&P->bs1, NT * n));
    TRY(P->dalloc(&P->bs2, NT * n));
    TRY(P->dalloc(&P->d_info, 1));
    if (P->dry) return ELMDDM_OK;
    // The strictly upper parts of the inverse factors are never written by the
    // solve and must read as zero.
    for (int i = 0; i < P->npass; ++i)
        if (hipMemset(P->Linv[i], 0, NT * P->sL * sizeof(double)) != hipSuccess)
            return fail(ELMDDM_HIP_ERROR, "hipMemset failed during plan creation");
    // Entries of the interface factor outside the envelope are never written and read as zero.
    if (P->SL && hipMemset(P->SL, 0, Bn * P->lds * nGm * sizeof(double)) != hipSuccess)
        return fail(ELMDDM_HIP_ERROR, "hipMemset failed during plan creation");
    if (hipMemset(P->X1, 0, NT * P->sX * sizeof(double)) != hipSuccess)
        return fail(ELMDDM_HIP_ERROR, "hipMemset failed during plan creation");
#undef TRY
    return ELMDDM_OK;
}

RowTable row_table(const elmddm_plan* P)
{
    RowTable t;
    t.x = P->d_rx;
    t.y = P->d_ry;
    t.nx = P->d_rnx;
    t.ny = P->d_rny;
    t.kind = P->d_kind;
    t.src = P->d_src;
    t.cmap = P->d_cmap;
    return t;
}

SubGeom sub_geom(const elmddm_plan* P)
{
    SubGeom g;
    g.cx = P->d_cx;
    g.cy = P->d_cy;
    g.sx = 2.0 / P->hx;
    g.sy = 2.0 / P->hy;
    return g;
}

elmddm_status check_launch(const char* where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ELMDDM_HIP_ERROR, std::string(where) + ": " + hipGetErrorString(e));
    return ELMDDM_OK;
}

}  // namespace

extern "C" {

elmddm_status elmddm_plan_create(const elmddm_problem* problem, elmddm_plan** plan)
{
    return elmddm_plan_create_batch(problem, 1, plan);
}

elmddm_status elmddm_plan_create_ex(const elmddm_problem* problem, int32_t batch, uint32_t flags,
                                    elmddm_plan** plan)
{
    if (!plan) return fail(ELMDDM_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    elmddm_status st = validate(problem);
    if (st != ELMDDM_OK) return st;
    if (batch < 1 || (int64_t)batch * problem->nsub_x * problem->nsub_y > kMaxSubdomains)
        return fail(ELMDDM_INVALID_ARG, "batch must be >= 1 and batch * nsub <= 65535");
    if ((flags & ELMDDM_PLAN_MATRIX_FREE) && (flags & ELMDDM_PLAN_DENSE))
        return fail(ELMDDM_INVALID_ARG, "MATRIX_FREE and DENSE are exclusive");
    elmddm_plan* P = new (std::nothrow) elmddm_plan();
    if (!P) return fail(ELMDDM_OOM, "host allocation failed");
    P->p = *problem;
    P->B = batch;
    // one fused launch per envelope step is latency-optimal for few systems;
    // a separate panel + trailing GEMM wins once several systems share the launches
    P->env_fused = batch < 4;
    P->npass = default_passes(problem->neurons);
    // dense interface factorisation unless its three nG x nG arrays would
    // exceed 64 GB (or the caller chooses)
    const double nGd = (double)interface_count(*problem);
    P->mfree = (flags & ELMDDM_PLAN_MATRIX_FREE) ||
               (!(flags & ELMDDM_PLAN_DENSE) && 3.0 * batch * nGd * nGd * 8.0 > 64e9);
    try {
        st = build(P);
    } catch (const std::bad_alloc&) {
        st = fail(ELMDDM_OOM, "host allocation failed while building the layout");
    }
    if (st == ELMDDM_OK && !P->mfree && !P->env_fused && P->nG > 0) {
        if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess)
            st = check_launch("side stream");
    }
    if (st != ELMDDM_OK) {
        delete P;
        return st;
    }
    *plan = P;
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_create_batch(const elmddm_problem* problem, int32_t batch, elmddm_plan** plan)
{
    return elmddm_plan_create_ex(problem, batch, 0, plan);
}

elmddm_status elmddm_plan_query(const elmddm_problem* problem, int32_t batch, elmddm_sizes* sizes)
{
    if (!sizes) return fail(ELMDDM_INVALID_ARG, "sizes is NULL");
    elmddm_status st = validate(problem);
    if (st != ELMDDM_OK) return st;
    if (batch < 1 || (int64_t)batch * problem->nsub_x * problem->nsub_y > kMaxSubdomains)
        return fail(ELMDDM_INVALID_ARG, "batch must be >= 1 and batch * nsub <= 65535");
    elmddm_plan Q;
    Q.p = *problem;
    Q.B = batch;
    Q.npass = default_passes(problem->neurons);
    const double nGd = (double)interface_count(*problem);
    Q.mfree = 3.0 * batch * nGd * nGd * 8.0 > 64e9;
    Q.dry = true;
    try {
        st = build(&Q);
    } catch (const std::bad_alloc&) {
        st = fail(ELMDDM_OOM, "host allocation failed while building the layout");
    }
    if (st != ELMDDM_OK) return st;
    return elmddm_plan_sizes(&Q, sizes);
}

elmddm_status elmddm_plan_destroy(elmddm_plan* plan)
{
    if (plan) {
        if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
        delete plan;
    }
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_sizes(const elmddm_plan* P, elmddm_sizes* s)
{
    if (!P || !s) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    s->nsub = P->N;
    s->batch = P->B;
    s->neurons = P->n;
    s->n_interior = P->q2;
    s->n_interface = P->nG;
    s->n_boundary = P->nB;
    s->max_rows = P->max_rows;
    s->max_ifc = P->maxk;
    s->device_bytes = P->bytes;
    return ELMDDM_OK;
}

elmddm_status elmddm_points(const elmddm_plan* P, int32_t kind, double* xy, int64_t capacity)
{
    if (!P || !xy) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    const std::vector<double>* v = nullptr;
    if (kind == ELMDDM_POINTS_INTERIOR) v = &P->int_pts;
    else if (kind == ELMDDM_POINTS_BOUNDARY) v = &P->bnd_pts;
    else if (kind == ELMDDM_POINTS_INTERFACE) v = &P->ifc_pts;
    else return fail(ELMDDM_INVALID_ARG, "unknown point kind");
    if (capacity < (int64_t)(v->size() / 2)) return fail(ELMDDM_INVALID_ARG, "capacity too small");
    std::memcpy(xy, v->data(), v->size() * sizeof(double));
    return ELMDDM_OK;
}

elmddm_status elmddm_assemble(elmddm_plan* P, const double* W, const double* b, const double* f,
                              const double* g, const double* coef, double* K, double* A, double* F,
                              void* stream)
{
    if (!P || !W || !b || !f || !K || !A || !F) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (P->nB > 0 && !g) return fail(ELMDDM_INVALID_ARG, "g is NULL but the problem has boundary points");
    if (P->p.op == ELMDDM_OP_VARCOEF && !coef) return fail(ELMDDM_INVALID_ARG, "coef is NULL for VARCOEF");
    hipStream_t st = (hipStream_t)stream;
    assemble(st, P->NT, P->N, P->nB, P->ldx, P->n, row_table(P), sub_geom(P), P->p.op, W, b, f, g,
             coef, P->q2, nullptr, F, P->max_rows, K, P->max_rows, A, std::max(P->maxk, 1));
    return check_launch("assemble");
}

elmddm_status elmddm_plan_keep_schur(elmddm_plan* P, int32_t keep)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (keep && P->mfree) return fail(ELMDDM_UNSUPPORTED, "a matrix-free plan never forms S");
    if (keep && !P->Skeep) {
        elmddm_status st = P->dalloc(&P->Skeep, (size_t)P->lds * std::max(P->nG, 1));
        if (st != ELMDDM_OK) return st;
    }
    P->keep_schur = keep != 0;
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_set_cg(elmddm_plan* P, double tol, int32_t maxit)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (!(tol > 0.0 && tol < 1.0) || maxit < 1) return fail(ELMDDM_INVALID_ARG, "need 0 < tol < 1 and maxit >= 1");
    P->cg_tol = tol;
    P->cg_maxit = maxit;
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_set_cg_precond(elmddm_plan* P, int32_t kind)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (kind != 0 && kind != 1) return fail(ELMDDM_INVALID_ARG, "preconditioner kind must be 0 or 1");
    P->cg_precond = kind;
    P->factors_valid = false;   // the preconditioner is set up by the next solve
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_cg_stats(const elmddm_plan* P, int32_t* iters, double* relres)
{
    if (!P || !iters || !relres) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (!P->mfree) return fail(ELMDDM_UNSUPPORTED, "the plan factors the interface system directly");
    for (int q = 0; q < P->B; ++q) {
        iters[q] = q < (int)P->cg_iters.size() ? P->cg_iters[q] : 0;
        relres[q] = q < (int)P->cg_relres.size() ? P->cg_relres[q] : 0.0;
    }
    return ELMDDM_OK;
}

int32_t elmddm_plan_is_matrix_free(const elmddm_plan* P) { return P && P->mfree ? 1 : 0; }

elmddm_status elmddm_plan_set_passes(elmddm_plan* P, int32_t npass)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (npass < 3 || npass > 5) return fail(ELMDDM_INVALID_ARG, "npass must be 3, 4 or 5");
    for (int i = 0; i < npass; ++i)
        if (!P->Linv[i]) {
            const size_t cnt = (size_t)P->NT * P->sL;
            elmddm_status st = P->dalloc(&P->Linv[i], cnt);
            if (st != ELMDDM_OK) return st;
            if (hipMemset(P->Linv[i], 0, cnt * sizeof(double)) != hipSuccess)
                return fail(ELMDDM_HIP_ERROR, "hipMemset failed");
        }
    P->npass = npass;
    P->factors_valid = false;
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_set_mode(elmddm_plan* P, int32_t mode)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (mode != ELMDDM_MODE_FP64 && mode != ELMDDM_MODE_MIXED) return fail(ELMDDM_INVALID_ARG, "unknown precision mode");
    P->mode = mode;
    return ELMDDM_OK;
}

elmddm_status elmddm_get_schur(elmddm_plan* P, double* S, double* rhs, void* stream)
{
    if (!P || !S || !rhs) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (!P->schur_valid) return fail(ELMDDM_INVALID_ARG, "no Schur system kept (call elmddm_plan_keep_schur before solving)");
    hipStream_t st = (hipStream_t)stream;
    if (P->nG == 0) return ELMDDM_OK;
    // The kept copy is in the permuted edge order: S in the first nG rows, rhs in row nG.
    unpermute_matrix(st, P->nE, P->mg, P->d_perm, P->Skeep, P->lds, S);
    copy_row(st, P->Skeep + P->nG, P->lds, 0, P->uperm, 1, 0, P->nG, 1);
    unpermute(st, P->nE, P->mg, P->d_perm, P->uperm, rhs, 1);
    return check_launch("get_schur");
}

namespace {

struct CgBufs {
    double *r, *p, *q, *state, *t, *w, *z;
};

// y = S x for R systems with the matrix-free operator (Section 3, eq. schur
// applied without forming S).  shared: one operator (instance 0) for all R.
void apply_mfree(elmddm_plan* P, hipStream_t st, const double* x, double* y, int R, bool shared, const CgBufs& cb)
{
    const int N = P->N;
    const long long sM = shared ? 0 : (long long)P->n_mblocks * P->mg * P->mg;
    mf_tpart(st, N * R, N, P->kpad, P->P, P->ldp, P->sP, P->d_gidx, x, P->nG, cb.t, P->kpad, shared);
    mf_mv4(st, P->nE, P->mg, P->d_mstart, P->d_mE, P->Mbuf, sM, x, P->nG, cb.w, (long long)P->nE * P->mg, R);
    mf_mtv4(st, P->nE, P->mg, P->d_qdesc, P->d_gptr, P->d_gdesc, cb.t, P->kpad, P->MbT, sM, cb.w,
            (long long)P->nE * P->mg, y, P->nG, N, R);
}

// CG (stop at ||b - S x|| <= tol ||b||) for R systems on the matrix-free
// operator, block-Jacobi preconditioned if the plan says so (the inverse
// edge-block factors of instance 0 serve all systems when shared); x holds
// the start.  Polls the convergence flags every 32 steps.
elmddm_status run_cg(elmddm_plan* P, hipStream_t st, const double* b, double* x, int R, double tol, int maxit,
                     bool shared, const CgBufs& cb)
{
    const int nG = P->nG;
    const bool pre = P->cg_precond != 0;
    const long long sD = shared ? 0 : (long long)P->nE * 4096;
    apply_mfree(P, st, x, cb.q, R, shared, cb);
    if (pre) {
        pcg_init1(st, nG, b, cb.q, cb.r, cb.state, R);
        mf_bjacobi(st, P->nE, P->mg, P->DEinv, sD, cb.r, cb.z, nG, R);
        pcg_init2(st, nG, cb.r, cb.z, cb.p, cb.state, tol, R);
    } else {
        cg_init(st, nG, b, cb.q, cb.r, cb.p, cb.state, tol, R);
    }
    const int ss = pre ? 8 : 4;   // state words per system
    std::vector<double> state(ss * R, 0.0);
    auto poll = [&]() -> elmddm_status {
        if (hipMemcpyAsync(state.data(), cb.state, ss * R * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return check_launch("CG poll");
        return ELMDDM_OK;
    };
    elmddm_status est = poll();
    if (est != ELMDDM_OK) return est;
    auto all_done = [&]() {
        for (int q = 0; q < R; ++q)
            if (state[ss * q + 2] == 0.0) return false;
        return true;
    };
    for (int it = 0; it < maxit && !all_done(); ++it) {
        apply_mfree(P, st, cb.p, cb.q, R, shared, cb);
        if (pre) {
            pcg_step1(st, nG, x, cb.r, cb.p, cb.q, cb.state, tol, R);
            mf_bjacobi(st, P->nE, P->mg, P->DEinv, sD, cb.r, cb.z, nG, R);
            pcg_step2(st, nG, cb.r, cb.z, cb.p, cb.state, R);
        } else {
            cg_step(st, nG, x, cb.r, cb.p, cb.q, cb.state, tol, R);
        }
        if ((it & 31) == 31 || it + 1 == maxit) {
            est = poll();
            if (est != ELMDDM_OK) return est;
        }
    }
    est = poll();
    if (est != ELMDDM_OK) return est;
    P->cg_iters.assign(R, 0);
    P->cg_relres.assign(R, 0.0);
    P->cg_failed = false;
    for (int q = 0; q < R; ++q) {
        const double rr = pre ? state[ss * q + 4] : state[ss * q];
        P->cg_iters[q] = (int32_t)state[ss * q + 3];
        P->cg_relres[q] = state[ss * q + 1] > 0.0 ? std::sqrt(rr / state[ss * q + 1]) : 0.0;
        if (state[ss * q + 2] != 1.0) P->cg_failed = true;
    }
    return check_launch("CG");
}

// Edge blocks of S and their inverse Cholesky factors (block-Jacobi).
void setup_bjacobi(elmddm_plan* P, hipStream_t st)
{
    const long long sM = (long long)P->n_mblocks * P->mg * P->mg;
    mf_diag_blocks(st, P->nE, P->mg, P->d_qdesc, P->d_gptr, P->d_gdesc, P->P, P->ldp, P->sP, P->Mbuf, sM, P->DE,
                   P->N, P->B);
    potrf_diag(st, P->DE, 64, 4096, 0, P->mg, P->DEinv, 4096, nullptr, 0, 0, P->d_info, -1, P->B * P->nE, nullptr,
               0, 0.0, nullptr, 0);
}

}  // namespace

elmddm_status elmddm_solve(elmddm_plan* P, const double* W, const double* b, const double* f,
                           const double* g, const double* coef, double* u_gamma, double* c,
                           void* stream)
{
    if (!P || !W || !b || !f || !c) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (P->nB > 0 && !g) return fail(ELMDDM_INVALID_ARG, "g is NULL but the problem has boundary points");
    if (P->nG > 0 && !u_gamma) return fail(ELMDDM_INVALID_ARG, "u_gamma is NULL");
    if (P->p.op == ELMDDM_OP_VARCOEF && !coef) return fail(ELMDDM_INVALID_ARG, "coef is NULL for VARCOEF");
    hipStream_t st = (hipStream_t)stream;
    if (P->timing) P->harvest();
    P->last_stream = st;
    P->solved = true;
    P->factors_valid = false;
    const int N = P->NT, n = P->n, ldx = P->ldx, ldg = P->ldg;
    const int B = P->B;
    const long long sS = (long long)P->lds * std::max(P->nG, 1);
    init_info(st, P->d_info);
    P->mark(0, st);

    // Feature assembly: X0 = [K rows | interface rows | flux rows], column n = F.
    assemble(st, N, P->N, P->nB, ldx, n, row_table(P), sub_geom(P), P->p.op, W, b, f, g, coef, P->q2,
             P->X0, nullptr, 0, nullptr, 0, nullptr, 0);
    // the last pass reads X1 when the pass count is even: give it the F column too
    if (P->npass % 2 == 0 &&
        hipMemcpy2DAsync(P->X1 + (size_t)n * ldx, P->sX * sizeof(double), P->X0 + (size_t)n * ldx,
                         P->sX * sizeof(double), (size_t)ldx * sizeof(double), N, hipMemcpyDeviceToDevice,
                         st) != hipSuccess)
        return check_launch("F column copy");
    P->mark(1, st);

    // Three-pass shifted CholeskyQR of every K^s (Fukaya et al., SIAM J. Sci.
    // Comput. 42 (2020)); the flux rows ride along through the triangular
    // solves but stay out of the Gram matrices.  Pass 1 shifts the Gram
    // diagonal by s * diag(G) (column-scaled shift), pass 3 also factors the
    // extra row F^T Q2, which becomes h = Q^T F.
    const double u = 0x1p-53;
    const bool mixed = P->mode == ELMDDM_MODE_MIXED;
    // FP64: the bound of Fukaya et al. for column-scaled X; mixed: a shift that
    // covers the FP32 rounding of the pass-1 Gram entries (errors of order
    // sqrt(m) u32 relative to |k_i||k_j|, spectral norm a few sqrt(n) times that).
    const double shift64 = 11.0 * ((double)P->gram_rows * n + (double)n * (n + 1)) * u * n;
    const double shift32 = 16.0 * std::sqrt((double)P->gram_rows * n) * 0x1p-24;
    double* src = P->X0;
    double* dst = P->X1;
    const int np = P->npass;
    for (int pass = 1; pass <= np; ++pass) {
        const bool last = pass == np;
        const int ncol = last ? n + 1 : n;
        if (P->timing) (void)hipEventRecord(P->pev[3 * (pass - 1)], st);
        // The last pass takes the Gram of [Q F] (F is column n): its row n is
        // the right-hand side row F^T Q that the factorisation turns into h
        // (n + 1 columns fall in the same 64-wide tiles as n unless n % 64 == 0).
        if (pass == 1 && mixed)
            gram_product_f32(st, n, P->gram_rows, src, ldx, P->sX, P->G, ldg, P->sG, N);
        else
            gram_product(st, P->gram_code, last ? n + 1 : n, P->gram_rows, src, ldx, P->sX, P->G, ldg, P->sG, N);
        if (P->timing) (void)hipEventRecord(P->pev[3 * (pass - 1) + 1], st);
        if (pass <= np - 2) scale_diag(st, P->G, ldg, P->sG, n, 1.0 + (pass == 1 && mixed ? shift32 : shift64), N);
        // breakdown threshold on pivot / original diagonal: 64 n u, except for
        // the unshifted middle pass of the mixed mode, whose input has
        // kappa(Q1) up to ~1e8 after the larger FP32 shift and legitimately
        // meets pivots down to ~1e-12 of the diagonal; there only pivots at
        // the rounding level (<= 64 u, e.g. from duplicate neurons) are flagged
        const double tau = (mixed && !last && pass > np - 2) ? 64.0 * u : 64.0 * n * u;
        blocked_potrf(st, P->G, ldg, P->sG, ncol, n, P->Dinv, P->sD, P->Linv[pass - 1], ldg, P->sL,
                      P->Tbuf, P->d_info, pass, N, P->dsave, n, tau);
        if (P->timing) (void)hipEventRecord(P->pev[3 * (pass - 1) + 2], st);
        const int r0 = last ? P->mI : 0;
        trsm_product(st, P->trsm_code, ldx - r0, n, src + r0, ldx, P->sX, P->Linv[pass - 1], ldg, P->sL,
                     dst + r0, P->sX, N);
        if (!last) std::swap(src, dst);
    }
    if (P->timing) (void)hipEventRecord(P->pev[3 * np], st);
    P->Qprev = src;
    P->Xfin = dst;
    // dst now holds the last pass's interface rows and Z^T = A R^{-1}; put h^T in its row.
    copy_row(st, P->G + n, ldg, P->sG, dst + P->hrow, ldx, P->sX, n, N);
    P->mark(4, st);
    elmddm_status est = check_launch("local factorisation");
    if (est != ELMDDM_OK) return est;

    if (P->nG > 0) {
        // P_s = [Y^T; h^T; Z^T] [Y h]  -> T_s, q_s, C_s, a_s
        gemm_f64(st, false, true, 0, false, 2 * P->kpad + 16, P->kpad + 1, n, 1.0, dst + P->mI, ldx,
                 P->sX, dst + P->mI, ldx, P->sX, 0.0, P->P, P->ldp, P->sP, N);
        const int cbase = P->kpad + 16;
        const long long sM = (long long)P->n_mblocks * P->mg * P->mg;
        schur_mblocks(st, P->n_mblocks, P->d_mdesc, P->P, P->ldp, P->sP, cbase, P->mg, P->Mbuf, P->N, B);
        schur_avec(st, P->nE, P->d_adesc, P->P, P->ldp, P->sP, cbase, P->kpad, P->mg, P->abuf, P->N, B);
        if (P->mfree) {
            // the paper's interface solver: CG on the matrix-free operator, in
            // the interface numbering (identity edge order), zero start
            schur_rhs(st, P->nE, P->mg, P->d_qdesc, P->d_gptr, P->d_gdesc, P->P, P->ldp, P->sP, P->kpad,
                      P->Mbuf, P->abuf, P->yvec, 1, P->d_ident, P->N, sM, (long long)P->nE * P->mg, P->nG, B);
            P->mark(5, st);
            P->mark(6, st);
            transpose_blocks(st, (long long)B * P->n_mblocks, P->mg, P->Mbuf, P->MbT);
            if (P->cg_precond) setup_bjacobi(P, st);
            est = check_launch("Schur pieces");
            if (est != ELMDDM_OK) return est;
            if (hipMemsetAsync(P->mfX, 0, (size_t)B * P->nG * sizeof(double), st) != hipSuccess)
                return check_launch("CG start");
            est = run_cg(P, st, P->yvec, P->mfX, B, P->cg_tol, P->cg_maxit, false,
                         CgBufs{P->mfR, P->mfP, P->mfQ, P->mfS, P->tbuf, P->wbuf, P->uperm});
            if (est != ELMDDM_OK) return est;
            if (hipMemcpyAsync(u_gamma, P->mfX, (size_t)B * P->nG * sizeof(double), hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                return check_launch("CG result copy");
        } else {
            // a kept S is copied whole: then every zero block is written
            const bool all_zero = P->keep_schur && P->Skeep;
            schur_sblocks(st, P->nE, P->mg, P->d_nzb, P->n_nzb, all_zero ? P->d_zb : P->d_zb_env,
                          all_zero ? P->n_zb : P->n_zb_env, P->d_tptr, P->d_tdesc, P->d_mptr, P->d_mlist, P->P,
                          P->ldp, P->sP, P->Mbuf, P->Sx, P->lds, P->d_perm, P->N, sM, sS, B);
            schur_rhs(st, P->nE, P->mg, P->d_qdesc, P->d_gptr, P->d_gdesc, P->P, P->ldp, P->sP, P->kpad,
                      P->Mbuf, P->abuf, P->yvec, 1, P->d_perm, P->N, sM, (long long)P->nE * P->mg,
                      P->nG, B);
            P->mark(5, st);
            if (P->keep_schur && P->Skeep) {
                (void)hipMemcpyAsync(P->Skeep, P->Sx, (size_t)P->lds * P->nG * sizeof(double),
                                     hipMemcpyDeviceToDevice, st);
                copy_row(st, P->yvec, 1, 0, P->Skeep + P->nG, P->lds, 0, P->nG, 1);
                P->schur_valid = true;
            }
            // Interface solve in the permuted order: envelope Cholesky with the
            // forward substitution fused (yvec <- L^{-1} rhs), then L^T u = y
            // block by block, then back to the interface numbering.
            const long long sDS = (long long)P->nblkS * NB * NB;
            // the lookahead's side stream is used only outside stream capture
            // (captured solves keep the single-stream order)
            hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
            const bool look = cap == hipStreamCaptureStatusNone;
            envelope_potrf(st, P->Sx, P->lds, sS, P->SL, P->lds, sS, P->nG, P->rend.data(), P->DinvS, sDS,
                           P->d_info, -1, P->dsave, P->yvec, P->nG, B, P->env_fused, look ? P->side : nullptr,
                           P->ev_fork, P->ev_join);
            P->mark(6, st);
            const int BR = 4 * NB;
            for (int j0 = (P->nG - 1) / BR * BR; j0 >= 0; j0 -= BR) {
                const int br = std::min(BR, P->nG - j0);
                trsv_lower_t_block(st, P->SL, P->lds, sS, j0, br, P->kbeg[j0 / NB], P->DinvS, sDS,
                                   P->yvec, P->uperm, P->nG, B);
            }
            unpermute(st, P->nE, P->mg, P->d_perm, P->uperm, u_gamma, B);
            est = check_launch("interface solve");
            if (est != ELMDDM_OK) return est;
        }
    } else {
        P->mark(5, st);
        P->mark(6, st);
    }
    P->mark(7, st);
    local_backsolve(st, N, P->N, P->nG, n, P->kpad, dst, ldx, P->sX, P->mI, P->hrow, P->d_gidx, u_gamma,
                    P->Linv, np, ldg, P->sL, c, P->bs1, P->bs2);
    const long long nc = (long long)N * n;
    P->mark(8, st);
    check_finite(st, c, nc, P->d_info);
    if (P->nG > 0) check_finite(st, u_gamma, (long long)B * P->nG, P->d_info);
    if (P->timing) P->ev_pending = true;
    est = check_launch("back-solve");
    P->factors_valid = est == ELMDDM_OK;
    return est;
}

elmddm_status elmddm_plan_reserve_rhs(elmddm_plan* P, int32_t max_rhs)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (P->B != 1) return fail(ELMDDM_UNSUPPORTED, "further right-hand sides need a plan with batch 1");
    if (max_rhs < 1 || max_rhs > 4096) return fail(ELMDDM_INVALID_ARG, "max_rhs must be in [1, 4096]");
    if (max_rhs <= P->rhs_cap) return ELMDDM_OK;
    for (double** q : {&P->Fr, &P->Tm, &P->Hm, &P->Ph, &P->abufR, &P->yR, &P->uR, &P->Vm, &P->cgX, &P->cgR,
                       &P->cgP, &P->cgQ, &P->cgS, &P->tbufR, &P->wbufR}) {
        if (*q) {
            P->allocs.erase(std::find(P->allocs.begin(), P->allocs.end(), (void*)*q));
            (void)hipFree(*q);
            *q = nullptr;
        }
    }
    P->rhs_cap = 0;
    const size_t R = max_rhs, N = P->N, n = P->n, nGm = std::max(P->nG, 1);
    elmddm_status st;
    if ((st = P->dalloc(&P->Fr, N * R * P->gram_rows)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->Tm, N * R * n)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->Hm, N * R * n)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->Vm, N * R * n)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->Ph, R * N * P->ldp)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->abufR, R * std::max(P->nE, 1) * P->mg)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->yR, R * nGm)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->uR, R * nGm)) != ELMDDM_OK) return st;
    for (double** q : {&P->cgX, &P->cgR, &P->cgP, &P->cgQ})
        if ((st = P->dalloc(q, R * nGm)) != ELMDDM_OK) return st;
    if ((st = P->dalloc(&P->cgS, 8 * R)) != ELMDDM_OK) return st;
    if (P->mfree) {
        if ((st = P->dalloc(&P->tbufR, N * R * std::max(P->kpad, 1))) != ELMDDM_OK) return st;
        if ((st = P->dalloc(&P->wbufR, R * std::max(P->nE, 1) * P->mg)) != ELMDDM_OK) return st;
    }
    if (!P->mfree && !P->d_rb && P->nblkS > 0) {
        if ((st = P->upload(&P->d_rb, P->kbeg)) != ELMDDM_OK) return st;
        if ((st = P->upload(&P->d_re, P->rend)) != ELMDDM_OK) return st;
    }
    P->rhs_cap = max_rhs;
    return ELMDDM_OK;
}

namespace {

elmddm_status rhs_checks(elmddm_plan* P, int32_t nrhs, const void* f)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (P->B != 1) return fail(ELMDDM_UNSUPPORTED, "further right-hand sides need a plan with batch 1");
    if (nrhs < 0 || !f) return fail(ELMDDM_INVALID_ARG, "bad nrhs or NULL input");
    if (!P->factors_valid) return fail(ELMDDM_INVALID_ARG, "no factors: call elmddm_solve on this plan first");
    if (P->rhs_cap < 1) return fail(ELMDDM_INVALID_ARG, "call elmddm_plan_reserve_rhs first");
    return ELMDDM_OK;
}

// For R sources starting at f (g may be NULL): Hm = h = Q^T F per subdomain
// and, if the problem has an interface, the Schur right-hand side of eq.
// schur in the envelope order in yR.
void rhs_stage(elmddm_plan* P, hipStream_t st, int R, const double* f, const double* g)
{
    const int N = P->N, n = P->n, ldx = P->ldx, ldg = P->ldg, ldf = P->gram_rows, nG = P->nG;
    const int ldp = P->ldp, mg = P->mg, kp = P->kpad;
    const long long nf = (long long)N * P->q2;
    // after a solve: X0 = Q2 (all rows), X1 rows [mI, ldx) = Q3 interface rows, h row, Z^T rows
    rhs_assemble(st, row_table(P), ldx, P->gram_rows, ldf, f, g, N, R, nf, P->nB, P->Fr);
    // h = L3^{-1} Q2^T F
    gemm_f64(st, true, false, 0, false, n, R, P->gram_rows, 1.0, P->Qprev, ldx, P->sX, P->Fr, ldf, (long long)R * ldf,
             0.0, P->Tm, n, (long long)R * n, N);
    gemm_f64(st, false, false, 0, false, n, R, n, 1.0, P->Linv[P->npass - 1], ldg, P->sL, P->Tm, n,
             (long long)R * n, 0.0, P->Hm, n, (long long)R * n, N);
    if (nG == 0) return;
    // [q; a] = [Q_Gamma^T h; Z h] per subdomain, laid out [rhs][subdomain][ldp]
    gemm_f64(st, false, false, 0, false, 2 * kp + 16, R, n, 1.0, P->Xfin + P->mI, ldx, P->sX, P->Hm, n,
             (long long)R * n, 0.0, P->Ph, N * ldp, ldp, N);
    schur_avec(st, P->nE, P->d_adesc, P->Ph, ldp, ldp, kp + 16, 0, mg, P->abufR, N, R);
    schur_rhs(st, P->nE, mg, P->d_qdesc, P->d_gptr, P->d_gdesc, P->Ph, ldp, ldp, 0, P->Mbuf, P->abufR, P->yR, 1,
              P->mfree ? P->d_ident : P->d_perm, N, 0, (long long)P->nE * mg, nG, R);
}

}  // namespace

elmddm_status elmddm_solve_rhs(elmddm_plan* P, int32_t nrhs, const double* f, const double* g,
                               double* u_gamma, double* c, void* stream)
{
    elmddm_status est = rhs_checks(P, nrhs, f);
    if (est != ELMDDM_OK) return est;
    if (P->nG > 0 && !u_gamma) return fail(ELMDDM_INVALID_ARG, "u_gamma is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int N = P->N, n = P->n, ldx = P->ldx, ldg = P->ldg, nG = P->nG, mg = P->mg, kp = P->kpad;
    const long long nf = (long long)N * P->q2;
    for (int r0 = 0; r0 < nrhs; r0 += P->rhs_cap) {
        const int R = std::min(P->rhs_cap, nrhs - r0);
        rhs_stage(P, st, R, f + r0 * nf, g ? g + r0 * P->nB : nullptr);
        if (nG > 0 && P->mfree) {
            // CG from zero on the shared matrix-free operator
            double* ur = u_gamma + (long long)r0 * nG;
            if (hipMemsetAsync(ur, 0, (size_t)R * nG * sizeof(double), st) != hipSuccess)
                return check_launch("CG start");
            est = run_cg(P, st, P->yR, ur, R, P->cg_tol, P->cg_maxit, true,
                         CgBufs{P->cgR, P->cgP, P->cgQ, P->cgS, P->tbufR, P->wbufR, P->uR});
            if (est != ELMDDM_OK) return est;
            if (P->cg_failed) return fail(ELMDDM_NOT_CONVERGED, "interface CG did not reach the tolerance");
        } else if (nG > 0) {
            // L y = g, then L^T u = y, with the envelope factor of S
            const int BR = 4 * NB;
            for (int j0 = 0; j0 < nG; j0 += BR) {
                const int br = std::min(BR, nG - j0);
                const int r1 = std::max(j0 + br, P->rend[(j0 + br - 1) / NB]);
                trsv_lower_block(st, P->SL, P->lds, 0, j0, br, r1, P->DinvS, 0, P->yR, nG, R);
            }
            for (int j0 = (nG - 1) / BR * BR; j0 >= 0; j0 -= BR) {
                const int br = std::min(BR, nG - j0);
                trsv_lower_t_block(st, P->SL, P->lds, 0, j0, br, P->kbeg[j0 / NB], P->DinvS, 0, P->yR, P->uR,
                                   nG, R);
            }
            unpermute(st, P->nE, mg, P->d_perm, P->uR, u_gamma + (long long)r0 * nG, R);
        }
        if (c) {
            // c = Linv1^T ... Linv_npass^T (h + Q_Gamma^T u)
            backsolve_rhs_multi(st, N, n, kp, P->Xfin, ldx, P->sX, P->mI, P->d_gidx,
                                nG > 0 ? u_gamma + (long long)r0 * nG : nullptr, nG, P->Hm, P->Vm, R);
            double* cur = P->Vm;
            double* nxt = P->Tm;
            for (int q = P->npass - 1; q >= 0; --q) {
                double* out = q == 0 ? c + (long long)r0 * N * n : nxt;
                gemm_f64(st, true, false, 0, false, n, R, n, 1.0, P->Linv[q], ldg, P->sL, cur, n, (long long)R * n,
                         0.0, out, q == 0 ? N * n : n, q == 0 ? (long long)n : (long long)R * n, N);
                std::swap(cur, nxt);
            }
        }
    }
    return check_launch("solve_rhs");
}

elmddm_status elmddm_schur_rhs(elmddm_plan* P, int32_t nrhs, const double* f, const double* g, double* rhs,
                               void* stream)
{
    elmddm_status est = rhs_checks(P, nrhs, f);
    if (est != ELMDDM_OK) return est;
    if (P->nG > 0 && !rhs) return fail(ELMDDM_INVALID_ARG, "rhs is NULL");
    hipStream_t st = (hipStream_t)stream;
    const long long nf = (long long)P->N * P->q2;
    for (int r0 = 0; r0 < nrhs && P->nG > 0; r0 += P->rhs_cap) {
        const int R = std::min(P->rhs_cap, nrhs - r0);
        rhs_stage(P, st, R, f + r0 * nf, g ? g + r0 * P->nB : nullptr);
        unpermute(st, P->nE, P->mg, P->mfree ? P->d_ident : P->d_perm, P->yR, rhs + (long long)r0 * P->nG, R);
    }
    return check_launch("schur_rhs");
}

elmddm_status elmddm_interface_cg(elmddm_plan* P, int32_t nrhs, const double* rhs, double* u, double tol,
                                  int32_t maxit, int32_t* iters, double* relres, void* stream)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (nrhs < 0 || (P->nG > 0 && (!rhs || !u))) return fail(ELMDDM_INVALID_ARG, "bad nrhs or NULL vector");
    if (!(tol > 0.0) || maxit < 0) return fail(ELMDDM_INVALID_ARG, "tol must be > 0 and maxit >= 0");
    if (P->B != 1) return fail(ELMDDM_UNSUPPORTED, "interface CG needs a plan with batch 1");
    if (P->rhs_cap < 1) return fail(ELMDDM_INVALID_ARG, "call elmddm_plan_reserve_rhs first");
    hipStream_t st = (hipStream_t)stream;
    const int nG = P->nG, mg = P->mg;
    if (P->mfree) {
        if (!P->factors_valid) return fail(ELMDDM_INVALID_ARG, "no factors: call elmddm_solve on this plan first");
        bool ok = true;
        for (int r0 = 0; r0 < nrhs && nG > 0; r0 += P->rhs_cap) {
            const int R = std::min(P->rhs_cap, nrhs - r0);
            const size_t bytes = (size_t)R * nG * sizeof(double);
            if (hipMemcpyAsync(P->yR, rhs + (long long)r0 * nG, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(P->cgX, u + (long long)r0 * nG, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return check_launch("interface_cg copy");
            elmddm_status est = run_cg(P, st, P->yR, P->cgX, R, tol, maxit, true,
                                       CgBufs{P->cgR, P->cgP, P->cgQ, P->cgS, P->tbufR, P->wbufR, P->uR});
            if (est != ELMDDM_OK) return est;
            for (int q = 0; q < R; ++q) {
                if (iters) iters[r0 + q] = P->cg_iters[q];
                if (relres) relres[r0 + q] = P->cg_relres[q];
            }
            ok = ok && !P->cg_failed;
            if (hipMemcpyAsync(u + (long long)r0 * nG, P->cgX, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return check_launch("interface_cg copy");
        }
        elmddm_status est = check_launch("interface_cg");
        if (est != ELMDDM_OK) return est;
        if (!ok) return fail(ELMDDM_NOT_CONVERGED, "interface CG did not reach the tolerance");
        return ELMDDM_OK;
    }
    if (!P->schur_valid) return fail(ELMDDM_INVALID_ARG, "no kept Schur matrix (elmddm_plan_keep_schur before the solve)");
    bool all_done = true;
    std::vector<double> state;
    for (int r0 = 0; r0 < nrhs && nG > 0; r0 += P->rhs_cap) {
        const int R = std::min(P->rhs_cap, nrhs - r0);
        permute(st, P->nE, mg, P->d_perm, rhs + (long long)r0 * nG, P->yR, R);
        permute(st, P->nE, mg, P->d_perm, u + (long long)r0 * nG, P->cgX, R);
        band_symv(st, nG, P->Skeep, P->lds, P->d_rb, P->d_re, P->cgX, P->cgQ, R);
        cg_init(st, nG, P->yR, P->cgQ, P->cgR, P->cgP, P->cgS, tol, R);
        state.assign(4 * R, 0.0);
        for (int it = 0; it < maxit; ++it) {
            band_symv(st, nG, P->Skeep, P->lds, P->d_rb, P->d_re, P->cgP, P->cgQ, R);
            cg_step(st, nG, P->cgX, P->cgR, P->cgP, P->cgQ, P->cgS, tol, R);
            if ((it & 15) == 15 || it + 1 == maxit) {
                if (hipMemcpyAsync(state.data(), P->cgS, 4 * R * sizeof(double), hipMemcpyDeviceToHost, st) !=
                        hipSuccess || hipStreamSynchronize(st) != hipSuccess)
                    return check_launch("interface_cg poll");
                bool done = true;
                for (int q = 0; q < R; ++q) done = done && state[4 * q + 2] != 0.0;
                if (done) break;
            }
        }
        if (hipMemcpyAsync(state.data(), P->cgS, 4 * R * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return check_launch("interface_cg state");
        for (int q = 0; q < R; ++q) {
            if (iters) iters[r0 + q] = (int32_t)state[4 * q + 3];
            if (relres) relres[r0 + q] = state[4 * q + 1] > 0.0 ? std::sqrt(state[4 * q] / state[4 * q + 1]) : 0.0;
            all_done = all_done && state[4 * q + 2] == 1.0;
        }
        unpermute(st, P->nE, mg, P->d_perm, P->cgX, u + (long long)r0 * nG, R);
    }
    elmddm_status est = check_launch("interface_cg");
    if (est != ELMDDM_OK) return est;
    if (!all_done) return fail(ELMDDM_NOT_CONVERGED, "interface CG did not reach the tolerance");
    return ELMDDM_OK;
}

elmddm_status elmddm_autotune(elmddm_plan* P, void* stream, int32_t* choice)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    P->factors_valid = false;
    hipStream_t st = (hipStream_t)stream;
    const int N = P->NT, n = P->n, ldx = P->ldx, ldg = P->ldg;
    // timing only: operand values do not matter, but must be finite
    if (hipMemsetAsync(P->X0, 0, (size_t)N * P->sX * sizeof(double), st) != hipSuccess)
        return check_launch("autotune memset");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return check_launch("autotune events");
    // XCD-aware tile order first (it reads X once per XCD instead of up to
    // eight times); a later candidate replaces the kept one only if it is 2%
    // faster, so candidates within timing noise of each other do not flip
    // between runs
    const int codes[] = {-4, -2, -3, -1, 8, 7, 6, 5, 4};
    auto time_it = [&](auto&& fn) {
        fn();
        (void)hipEventRecord(e0, st);
        fn();
        fn();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    float best_g = 1e30f, best_t = 1e30f;
    for (int ci = 0; ci < 9; ++ci) {
        const int code = codes[ci];
        const float tg = time_it([&] {
            gram_product(st, code, n, P->gram_rows, P->X0, ldx, P->sX, P->G, ldg, P->sG, N);
        });
        if (tg < 0.98f * best_g) {
            best_g = tg;
            P->gram_code = code;
        }
        const float tt = time_it([&] {
            trsm_product(st, code, ldx, n, P->X0, ldx, P->sX, P->Linv[0], ldg, P->sL, P->X1, P->sX, N);
        });
        if (tt < 0.98f * best_t) {
            best_t = tt;
            P->trsm_code = code;
        }
        P->tune_ms[0][ci] = 0.5f * tg;
        P->tune_ms[1][ci] = 0.5f * tt;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (choice) {
        choice[0] = P->gram_code;
        choice[1] = P->trsm_code;
    }
    return check_launch("autotune");
}

elmddm_status elmddm_solve_info(elmddm_plan* P, elmddm_info* info)
{
    if (!P || !info) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (!P->solved) return fail(ELMDDM_INVALID_ARG, "no solve has been enqueued on this plan");
    if (hipStreamSynchronize(P->last_stream) != hipSuccess) return check_launch("solve_info sync");
    DevInfo h{};
    if (hipMemcpy(&h, P->d_info, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return check_launch("solve_info copy");
    info->status = h.status;
    if (h.status == ELMDDM_OK && P->mfree && P->cg_failed) info->status = ELMDDM_NOT_CONVERGED;
    info->bad_subdomain = h.bad_subdomain == INT_MAX ? -1 : h.bad_subdomain % P->N;
    info->bad_pass = h.bad_pass;
    info->bad_instance = h.bad_subdomain == INT_MAX ? -1 : h.bad_subdomain / P->N;
    return ELMDDM_OK;
}

elmddm_status elmddm_eval(elmddm_plan* P, const double* W, const double* b, const double* c,
                          const double* xy, int64_t npts, double* u, void* stream)
{
    if (!P || !W || !b || !c || (npts > 0 && (!xy || !u))) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (npts < 0 || npts > INT_MAX) return fail(ELMDDM_INVALID_ARG, "npts out of range");
    eval_points((hipStream_t)stream, (int)npts, xy, P->nx, P->ny, P->p.x0, P->p.x1, P->p.y0, P->p.y1,
                P->n, W, b, c, u);
    return check_launch("eval");
}

elmddm_status elmddm_eval_grad(elmddm_plan* P, const double* W, const double* b, const double* c,
                               const double* xy, int64_t npts, double* u, double* dudx, double* dudy, void* stream)
{
    if (!P || !W || !b || !c || (npts > 0 && (!xy || !dudx || !dudy))) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (npts < 0 || npts > INT_MAX) return fail(ELMDDM_INVALID_ARG, "npts out of range");
    eval_points_grad((hipStream_t)stream, (int)npts, xy, P->nx, P->ny, P->p.x0, P->p.x1, P->p.y0, P->p.y1, P->n, W,
                     b, c, u, dudx, dudy);
    return check_launch("eval_grad");
}

elmddm_status elmddm_set_timing(elmddm_plan* P, int32_t enable)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    if (enable && !P->ev_ready) {
        for (auto& e : P->ev)
            if (hipEventCreate(&e) != hipSuccess) return check_launch("hipEventCreate");
        for (auto& e : P->pev)
            if (hipEventCreate(&e) != hipSuccess) return check_launch("hipEventCreate");
        P->ev_ready = true;
    }
    if (P->ev_pending && P->last_stream) (void)hipStreamSynchronize(P->last_stream);
    P->ev_pending = false;
    P->timing = enable != 0;
    for (double& v : P->stage_ms) v = 0.0;
    for (double& v : P->pass_ms) v = 0.0;
    P->timed_solves = 0;
    return ELMDDM_OK;
}

elmddm_status elmddm_stage_times(elmddm_plan* P, double* ms, int32_t* solves)
{
    if (!P || !ms) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    P->harvest();
    for (int i = 0; i < ELMDDM_NUM_STAGES; ++i) ms[i] = P->stage_ms[i];
    if (solves) *solves = P->timed_solves;
    return ELMDDM_OK;
}

elmddm_status elmddm_plan_set_kernels(elmddm_plan* P, int32_t gram_code, int32_t trsm_code)
{
    if (!P) return fail(ELMDDM_INVALID_ARG, "NULL plan");
    auto ok = [](int c) { return (c >= -4 && c <= -1) || (c >= 4 && c <= 8); };
    if (!ok(gram_code) || !ok(trsm_code)) return fail(ELMDDM_INVALID_ARG, "kernel code out of range");
    P->gram_code = gram_code;
    P->trsm_code = trsm_code;
    return ELMDDM_OK;
}

elmddm_status elmddm_autotune_times(const elmddm_plan* P, int32_t* codes, double* gram_ms, double* trsm_ms)
{
    if (!P || !codes || !gram_ms || !trsm_ms) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    const int cs[] = {-4, -2, -3, -1, 8, 7, 6, 5, 4};
    for (int i = 0; i < 9; ++i) {
        codes[i] = cs[i];
        gram_ms[i] = P->tune_ms[0][i];
        trsm_ms[i] = P->tune_ms[1][i];
    }
    return ELMDDM_OK;
}

elmddm_status elmddm_pass_times(elmddm_plan* P, double* ms, int32_t* solves)
{
    if (!P || !ms) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    P->harvest();
    for (int i = 0; i < 15; ++i) ms[i] = i < 3 * P->npass ? P->pass_ms[i] : 0.0;
    if (solves) *solves = P->timed_solves;
    return ELMDDM_OK;
}

const char* elmddm_status_string(elmddm_status s)
{
    switch (s) {
        case ELMDDM_OK: return "ok";
        case ELMDDM_INVALID_ARG: return "invalid argument";
        case ELMDDM_OOM: return "out of memory";
        case ELMDDM_NOT_SPD: return "local Gram matrix not positive definite";
        case ELMDDM_SCHUR_NOT_SPD: return "interface Schur matrix not positive definite";
        case ELMDDM_NOT_CONVERGED: return "iteration did not converge";
        case ELMDDM_NONFINITE: return "non-finite values in the result";
        case ELMDDM_HIP_ERROR: return "HIP runtime error";
        case ELMDDM_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char* elmddm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Whole solves captured into one HIP graph.
// ---------------------------------------------------------------------------
struct elmddm_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<elmddm_plan*> plans;     // per captured solve
    DevInfo* d_infos = nullptr;          // per captured solve: copy of its status word
    hipStream_t last = nullptr;
    bool launched = false;
    ~elmddm_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_infos) (void)hipFree(d_infos);
    }
};

elmddm_status elmddm_graph_capture(elmddm_plan* const* plans, const elmddm_solve_args* args, int32_t nsolves,
                                   elmddm_graph** out)
{
    if (!out) return fail(ELMDDM_INVALID_ARG, "graph output pointer is NULL");
    *out = nullptr;
    if (!plans || !args || nsolves < 1) return fail(ELMDDM_INVALID_ARG, "no solves to capture");
    for (int i = 0; i < nsolves; ++i) {
        if (!plans[i]) return fail(ELMDDM_INVALID_ARG, "NULL plan");
        if (plans[i]->timing) return fail(ELMDDM_INVALID_ARG, "stage timing must be off while capturing");
        if (plans[i]->mfree)
            return fail(ELMDDM_UNSUPPORTED, "matrix-free plans poll their CG from the host and cannot be captured");
    }
    elmddm_graph* G = new (std::nothrow) elmddm_graph();
    if (!G) return fail(ELMDDM_OOM, "host allocation failed");
    if (hipMalloc((void**)&G->d_infos, nsolves * sizeof(DevInfo)) != hipSuccess) {
        (void)hipGetLastError();
        delete G;
        return fail(ELMDDM_OOM, "hipMalloc of the graph status words failed");
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete G;
        return check_launch("graph capture stream");
    }
    elmddm_status est = ELMDDM_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        est = check_launch("hipStreamBeginCapture");
    } else {
        for (int i = 0; i < nsolves && est == ELMDDM_OK; ++i) {
            const elmddm_solve_args& a = args[i];
            est = elmddm_solve(plans[i], a.W, a.b, a.f, a.g, a.coef, a.u_gamma, a.c, cs);
            if (est == ELMDDM_OK &&
                hipMemcpyAsync(G->d_infos + i, plans[i]->d_info, sizeof(DevInfo), hipMemcpyDeviceToDevice, cs) !=
                    hipSuccess)
                est = check_launch("graph status copy");
            G->plans.push_back(plans[i]);
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (est == ELMDDM_OK && e != hipSuccess) est = check_launch("hipStreamEndCapture");
        G->graph = g;
        if (est == ELMDDM_OK && hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0) != hipSuccess)
            est = check_launch("hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cs);
    // the workspaces hold nothing until the graph runs
    for (int i = 0; i < nsolves; ++i) {
        plans[i]->factors_valid = false;
        plans[i]->schur_valid = false;
        plans[i]->last_stream = nullptr;
        plans[i]->solved = false;
    }
    if (est != ELMDDM_OK) {
        delete G;
        return est;
    }
    *out = G;
    return ELMDDM_OK;
}

elmddm_status elmddm_graph_launch(elmddm_graph* G, void* stream)
{
    if (!G || !G->exec) return fail(ELMDDM_INVALID_ARG, "NULL graph");
    hipStream_t st = (hipStream_t)stream;
    if (hipGraphLaunch(G->exec, st) != hipSuccess) return check_launch("hipGraphLaunch");
    G->last = st;
    G->launched = true;
    // every plan's workspace now holds the factors of its last solve in the graph
    for (elmddm_plan* P : G->plans) {
        P->factors_valid = true;
        P->schur_valid = P->keep_schur && P->Skeep;
        P->last_stream = st;
        P->solved = true;
    }
    return ELMDDM_OK;
}

elmddm_status elmddm_graph_info(elmddm_graph* G, int32_t i, elmddm_info* info)
{
    if (!G || !info) return fail(ELMDDM_INVALID_ARG, "NULL argument");
    if (i < 0 || i >= (int)G->plans.size()) return fail(ELMDDM_INVALID_ARG, "solve index out of range");
    if (!G->launched) return fail(ELMDDM_INVALID_ARG, "the graph has not been launched");
    if (hipStreamSynchronize(G->last) != hipSuccess) return check_launch("graph_info sync");
    DevInfo h{};
    if (hipMemcpy(&h, G->d_infos + i, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return check_launch("graph_info copy");
    const elmddm_plan* P = G->plans[i];
    info->status = h.status;
    info->bad_subdomain = h.bad_subdomain == INT_MAX ? -1 : h.bad_subdomain % P->N;
    info->bad_pass = h.bad_pass;
    info->bad_instance = h.bad_subdomain == INT_MAX ? -1 : h.bad_subdomain / P->N;
    return ELMDDM_OK;
}

elmddm_status elmddm_graph_destroy(elmddm_graph* G)
{
    delete G;
    return ELMDDM_OK;
}
