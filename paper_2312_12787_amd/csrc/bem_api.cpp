// bem_api.cpp -- host runtime behind the C ABI of include/bem.h.
//
// Host work is validation and integer bookkeeping (element ranges, equation
// blocks, tiles, buffer offsets) plus the control flow of GMRES; every step
// of the numerical method runs in the gfx950 kernels (assemble.hip,
// linalg.hip).  The library never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bem.h"
#include "internal.h"
#include "launch.h"

using bemk::GeomLayout;
using bemk::IfacePlan;
using bemk::Tile;

namespace {

thread_local std::string g_err;

bem_status fail(bem_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

bem_status hip_fail(hipError_t e, const char* where)
{
    return fail(BEM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OK(call)                                           \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// BEM_MIXED matrix buffer: the FP64 matrix, then its FP32 copy (same lda).
size_t mixed_offset(size_t n, size_t lda) { return align256(lda * n * sizeof(double2)); }

}  // namespace

// HIP-event timing of the main kernels (bem_profile_enable / bem_profile_read).
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipEvent_t pending[bemk::N_KINDS] = {};
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    hipError_t err = hipSuccess;
};

void prof_cb(void* ctx, int kind, int phase, hipStream_t s)
{
    Prof* P = static_cast<Prof*>(ctx);
    if (!P->on) return;
    if (P->used == P->pool.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            P->err = r;
            return;
        }
        P->pool.push_back(e);
    }
    hipEvent_t e = P->pool[P->used++];
    hipError_t r = hipEventRecord(e, s);
    if (r != hipSuccess) P->err = r;
    if (kind < 0 || kind >= bemk::N_KINDS) return;
    if (phase == 0)
        P->pending[kind] = e;
    else if (P->pending[kind])
        P->recs.push_back({kind, P->pending[kind], e});
}

struct bem_problem {
    mutable Prof prof;
    bemk::KernelHook hook{prof_cb, nullptr};
    const bemk::KernelHook* hk() const { return prof.on ? &hook : nullptr; }
    int n_dom = 0, n_if = 0, N = 0, quad = 8, form = 0;
    std::vector<std::complex<double>> k;
    std::vector<int> dl, dr, n_nodes, closed;
    std::vector<double> xy;
    std::vector<IfacePlan> iface;
    std::vector<int> sigma;        // [d * n_if + m]
    std::vector<Tile> rtiles, cchunks;
    std::vector<int> vtiles;                     // row-tile ids grouped by assembly variant
    int vcount[bemk::ASM_VARIANTS] = {0}, voff[bemk::ASM_VARIANTS] = {0};
    std::vector<int> npairs;  // (row tile * 4 + wave, column chunk, part) items that may hold near pairs, by variant
    int ncount[bemk::ASM_VARIANTS] = {0}, noff[bemk::ASM_VARIANTS] = {0};
    std::vector<int> elif;          // interface of each element
    std::vector<int> elnodes;       // (a, b) node indices per element
    bemk::DomIn dummy{};
    std::vector<bemk::DomIn> dom_in;
    bemk::GlobalIn glob{};
    GeomLayout L{};
    // pinned host slots for the asynchronous read-back of the GMRES flags
    int* pinned = nullptr;      // host address
    int* pinned_dev = nullptr;  // the same memory as the kernels address it
    size_t pinned_ints = 0;
    hipEvent_t flag_ev[bemk::FLAG_RING] = {};
    bool lent = false;  // pinned / flag_ev belong to the caller (request server slot)
    // Arnoldi segments captured as HIP graphs (bem_solve_opts.graph_steps), by
    // segment index, and everything their launches bake in
    struct StepGraphs {
        std::vector<hipGraphExec_t> seg;
        const void *A = nullptr, *A32 = nullptr;
        const char* w = nullptr;
        const int* flags = nullptr;
        size_t lda = 0, ldv = 0;
        int prec = -1, n = 0, nr = 0, m = 0, S = 0, maxit = 0;
        bemk::MvShapes shapes{};
    } graphs;
    hipStream_t cap = nullptr;  // private stream the segments are captured on (never runs work)
    hipStream_t asm_side = nullptr;       // second stream of the assembly launches
    hipEvent_t asm_ev[2] = {};            // its fork and join events
    // device state recorded by the calls
    char* geom = nullptr;
    void* A = nullptr;      // FP64 or FP32 matrix (BEM_MIXED: the FP64 one)
    void* A32 = nullptr;    // BEM_MIXED: the FP32 copy (leading dimension lda)
    size_t lda = 0;
    int prec = -1;
    // launch shapes of this problem's products, resolved at bem_assemble from
    // `frozen` (a request server's copy of the shape sources) or else from the
    // live tuned table and environment; bem_tune of this problem updates them
    mutable bemk::MvShapes shapes{};
    std::shared_ptr<const bemk::ShapeSnapshot> frozen;
};

namespace {

void drop_graphs(bem_problem* p)
{
    for (hipGraphExec_t e : p->graphs.seg)
        if (e) (void)hipGraphExecDestroy(e);
    p->graphs.seg.clear();
}

int sigma_of(const bem_problem* p, int d, int m)
{
    if (p->dr[m] == d) return 1;
    if (p->dl[m] == d) return -1;
    return 0;
}

GeomLayout make_layout(const bem_problem* p)
{
    GeomLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    size_t nn = p->xy.size() / 2;
    L.nodes = take(nn * sizeof(double2));
    L.elnodes = take((size_t)p->N * sizeof(int2));
    L.elif = take((size_t)p->N * sizeof(int));
    L.iface = take((size_t)p->n_if * sizeof(IfacePlan));
    L.rtiles = take(p->rtiles.size() * sizeof(Tile));
    L.cchunks = take(p->cchunks.size() * sizeof(Tile));
    L.sigma = take((size_t)p->n_dom * p->n_if * sizeof(int));
    L.dom_in = take((size_t)p->n_dom * sizeof(bemk::DomIn));
    L.glob_in = take(sizeof(bemk::GlobalIn));
    L.vtiles = take(p->vtiles.size() * sizeof(int) + sizeof(int));
    L.npairs = take(p->npairs.size() * sizeof(int) + 3 * sizeof(int));
    size_t upload_end = off;
    (void)upload_end;
    L.elem = take((size_t)p->N * sizeof(bemk::ElemRec));
    L.gauss = take((size_t)p->N * sizeof(bemk::GaussRec));
    L.gauss32 = take((size_t)p->N * sizeof(bemk::GaussRec32));
    L.gl = take(2 * bemk::QMAX * sizeof(double));
    L.dom = take((size_t)p->n_dom * sizeof(bemk::DomConst));
    L.wave = take((size_t)p->n_dom * sizeof(bemk::WaveConst));
    L.wave32 = take((size_t)p->n_dom * sizeof(bemk::WaveConst32));
    L.self = take((size_t)p->n_dom * p->N * sizeof(double2));
    L.total = off;
    return L;
}

// Workspace of the solver and products (byte offsets into work_dev).
struct WorkLayout {
    size_t V, W, R, Ro, D, mv_part, dot_part, dot_part2, upd_part, y, H, Hraw, cs, sn, gvec, norm_part, hnorm,
        rnorm, bnorm, thr, active, kdim, iters, total;
    int ldv, nblk, anblk;
};

WorkLayout make_work(int n, int nr, int m)
{
    WorkLayout W{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    W.ldv = (n + 63) / 64 * 64;
    W.nblk = (n + 255) / 256;
    const size_t vec = (size_t)W.ldv * nr * sizeof(double2);
    W.V = take((size_t)(m + 1) * vec);
    W.W = take(vec);
    W.R = take(vec);
    W.Ro = take(vec);
    W.D = take(vec);
    W.mv_part = take(bemk::matvec_part_elems(n, nr) * sizeof(double2));
    W.anblk = bemk::arnoldi_blocks(n);
    W.dot_part = take((size_t)nr * W.anblk * (m + 1) * sizeof(double2));
    W.dot_part2 = take((size_t)nr * W.anblk * (m + 1) * sizeof(double2));
    W.upd_part = take((size_t)nr * W.anblk * sizeof(double));
    W.thr = take((size_t)nr * sizeof(double));
    W.iters = take((size_t)nr * sizeof(int));
    W.y = take((size_t)nr * (m + 1) * sizeof(double2));
    W.H = take((size_t)nr * (m + 1) * m * sizeof(double2));
    W.Hraw = take((size_t)nr * (m + 1) * m * sizeof(double2));
    W.cs = take((size_t)nr * m * sizeof(double2));
    W.sn = take((size_t)nr * m * sizeof(double2));
    W.gvec = take((size_t)nr * (m + 1) * sizeof(double2));
    W.norm_part = take((size_t)nr * std::max(W.nblk, 64) * sizeof(double));
    W.hnorm = take((size_t)nr * sizeof(double));
    W.rnorm = take((size_t)nr * sizeof(double));
    W.bnorm = take((size_t)nr * sizeof(double));
    W.active = take((size_t)nr * sizeof(int));
    W.kdim = take((size_t)nr * sizeof(int));
    W.total = off;
    return W;
}

bem_status check_problem(const bem_problem* p)
{
    if (!p) return fail(BEM_E_ARG, "null problem");
    return BEM_OK;
}

}  // namespace

extern "C" {

const char* bem_last_error(void) { return g_err.c_str(); }

bem_status bem_create(const bem_desc* desc, bem_problem** out)
{
    if (!desc || !out) return fail(BEM_E_ARG, "null argument");
    *out = nullptr;
    if (desc->n_dom < 2 || desc->n_dom > 64) return fail(BEM_E_ARG, "n_dom must be in [2, 64]");
    if (desc->n_if < 1) return fail(BEM_E_ARG, "n_if must be >= 1");
    if (desc->quad < 1 || desc->quad > bemk::QMAX) return fail(BEM_E_ARG, "quad must be in [1, 16]");
    if (desc->form < 0 || desc->form > 3) return fail(BEM_E_ARG, "unknown form");
    if (!desc->k || !desc->n_nodes || !desc->closed || !desc->xy || !desc->dom_left || !desc->dom_right)
        return fail(BEM_E_ARG, "null array in the description");
    auto p = new bem_problem();
    p->hook.ctx = &p->prof;
    p->n_dom = desc->n_dom;
    p->n_if = desc->n_if;
    p->quad = desc->quad;
    p->form = desc->form;
    for (int d = 0; d < p->n_dom; ++d) {
        const std::complex<double> kd(desc->k[d].re, desc->k[d].im);
        if (!std::isfinite(kd.real()) || !std::isfinite(kd.imag())) {
            delete p;
            return fail(BEM_E_ARG, "non-finite wavenumber");
        }
        if (d == 0 && !(kd.real() > 0.0 && kd.imag() == 0.0)) {
            delete p;
            return fail(BEM_E_ARG, "k[0] (host medium) must be real and positive");
        }
        if (kd.imag() < 0.0) {
            delete p;
            return fail(BEM_E_ARG, "Im k must be >= 0");
        }
        // The large-argument Hankel form evaluates amplitude polynomials fitted
        // on the real axis at the complex argument (XS/k r)^2; their error
        // grows with arg k (relative 1e-14 at 3.2 deg, 1.7e-12 at 10 deg,
        // 1.5e-10 at 20 deg against 150-digit values), so lossy media are
        // accepted up to arg k = 10 deg.
        if (kd.imag() > 0.0 && !(kd.imag() <= bemk::MAX_TAN_ARG_K * kd.real())) {
            delete p;
            return fail(BEM_E_ARG, "arg k must be <= 10 degrees (Im k <= tan(10 deg) Re k)");
        }
        if (std::abs(kd) == 0.0) {
            delete p;
            return fail(BEM_E_ARG, "k must be nonzero");
        }
        p->k.push_back(kd);
    }
    int node0 = 0, total = 0;
    for (int m = 0; m < p->n_if; ++m) {
        const int nn = desc->n_nodes[m], cl = desc->closed[m] ? 1 : 0;
        const int l = desc->dom_left[m], r = desc->dom_right[m];
        if (l < 0 || l >= p->n_dom || r < 0 || r >= p->n_dom || l == r) {
            delete p;
            return fail(BEM_E_GEOMETRY, "interface " + std::to_string(m) + ": bad domain ids");
        }
        if (l == 0) {
            delete p;
            return fail(BEM_E_GEOMETRY, "interface " + std::to_string(m) +
                                            ": the normal must leave the host medium (dom_right = 0)");
        }
        if (nn < (cl ? 3 : 2)) {
            delete p;
            return fail(BEM_E_GEOMETRY, "interface " + std::to_string(m) + ": too few nodes");
        }
        const int ne = cl ? nn : nn - 1;
        IfacePlan P{};
        P.off = total;
        P.count = ne;
        P.dl = l;
        P.dr = r;
        for (int e = 0; e < ne; ++e) {
            const int a = node0 + e, b = node0 + (e + 1) % nn;
            const double dx = desc->xy[2 * b] - desc->xy[2 * a], dy = desc->xy[2 * b + 1] - desc->xy[2 * a + 1];
            if (!std::isfinite(dx) || !std::isfinite(dy) || dx * dx + dy * dy == 0.0) {
                delete p;
                return fail(BEM_E_GEOMETRY, "interface " + std::to_string(m) + ": zero-length or non-finite element " +
                                                std::to_string(e));
            }
            p->elnodes.push_back(a);
            p->elnodes.push_back(b);
            p->elif.push_back(m);
        }
        p->iface.push_back(P);
        p->n_nodes.push_back(nn);
        p->closed.push_back(cl);
        p->dl.push_back(l);
        p->dr.push_back(r);
        node0 += nn;
        total += ne;
    }
    p->xy.assign(desc->xy, desc->xy + 2 * node0);
    p->N = total;
    // the device's phase reduction (k r reduced by pi/2) is exact below 2^30:
    // bound max |k| times the diameter of the nodes' bounding box
    {
        double x0 = p->xy[0], x1 = x0, y0 = p->xy[1], y1 = y0, kmax = 0.0;
        for (int a = 0; a < node0; ++a) {
            x0 = std::min(x0, p->xy[2 * a]);
            x1 = std::max(x1, p->xy[2 * a]);
            y0 = std::min(y0, p->xy[2 * a + 1]);
            y1 = std::max(y1, p->xy[2 * a + 1]);
        }
        for (const auto& kd : p->k) kmax = std::max(kmax, std::abs(kd));
        if (kmax * std::hypot(x1 - x0, y1 - y0) >= 0x1p29) {
            delete p;
            return fail(BEM_E_ARG, "max |k| times the boundary's diameter must stay below 2^29");
        }
    }
    // eps_left / eps_right = -1 puts the accumulation point at 0 (end of Sec. 5)
    for (int m = 0; m < p->n_if; ++m) {
        const auto el = (p->k[p->dl[m]] / p->k[0]) * (p->k[p->dl[m]] / p->k[0]);
        const auto er = (p->k[p->dr[m]] / p->k[0]) * (p->k[p->dr[m]] / p->k[0]);
        if (std::abs(1.0 + el / er) < 1e-12) {
            delete p;
            return fail(BEM_E_GEOMETRY, "eps_left / eps_right = -1 on interface " + std::to_string(m));
        }
    }
    p->sigma.assign((size_t)p->n_dom * p->n_if, 0);
    for (int d = 0; d < p->n_dom; ++d)
        for (int m = 0; m < p->n_if; ++m) p->sigma[(size_t)d * p->n_if + m] = sigma_of(p, d, m);
    // equation blocks
    const int N = p->N;
    if (p->form == BEM_CONVENTIONAL) {
        // eq. (naive_bie) / (3dom_conv_bie): domain by domain, host medium first
        int row = 0;
        for (int d = 0; d < p->n_dom; ++d)
            for (int m = 0; m < p->n_if; ++m) {
                if (p->dr[m] == d) {
                    p->iface[m].row_r = row;
                    row += p->iface[m].count;
                }
                if (p->dl[m] == d) {
                    p->iface[m].row_l = row;
                    row += p->iface[m].count;
                }
            }
        for (int m = 0; m < p->n_if; ++m) p->iface[m].bm_r = (p->dr[m] == 0);
    } else {
        // standard-type equations in the upper half, Burton-Miller ones in the lower
        for (int m = 0; m < p->n_if; ++m) {
            p->iface[m].row_l = p->iface[m].off;
            p->iface[m].row_r = N + p->iface[m].off;
            p->iface[m].bm_r = (p->form == BEM_CALDERON_ORIG) ? (p->dr[m] == 0) : 1;
        }
    }
    for (int m = 0; m < p->n_if; ++m) {
        const IfacePlan& P = p->iface[m];
        for (int s = 0; s < P.count; s += bemk::ROW_TILE)
            p->rtiles.push_back(Tile{m, P.off + s, std::min(bemk::ROW_TILE, P.count - s), 0});
        for (int s = 0; s < P.count; s += bemk::COL_CHUNK)
            p->cchunks.push_back(Tile{m, P.off + s, std::min(bemk::COL_CHUNK, P.count - s), 0});
    }
    // row tiles grouped by assembly variant (side, row type, complex wavenumber)
    {
        std::vector<std::vector<int>> lists(bemk::ASM_VARIANTS);
        for (size_t t = 0; t < p->rtiles.size(); ++t) {
            const IfacePlan& P = p->iface[p->rtiles[t].iface];
            for (int side = 0; side < 2; ++side) {
                const int d = side ? P.dr : P.dl;
                const int bm = side ? P.bm_r : 0;
                const int cplx = p->k[d].imag() != 0.0;
                lists[side * 4 + bm * 2 + cplx].push_back((int)t);
            }
        }
        for (int v = 0; v < bemk::ASM_VARIANTS; ++v) {
            p->voff[v] = (int)p->vtiles.size();
            p->vcount[v] = (int)lists[v].size();
            p->vtiles.insert(p->vtiles.end(), lists[v].begin(), lists[v].end());
        }
        // Near list of each variant: (row tile * 4 + 64-row wave of the tile,
        // column chunk, part) triples -- a part being NEAR_PART consecutive
        // elements of the chunk -- whose bounding boxes (collocation points;
        // element midpoints widened by the largest half length) come within
        // the series radius XS/|k_d| of the rows' domain (the larger FP64
        // radius; relative margin 1e-6).  Only these can hold an element the
        // assembly's per-wave test calls near, so the near-element launch runs
        // over them alone, one wave per item.
        struct Box {
            double x0, x1, y0, y1, hh;
        };
        auto box = [&](int e0, int cnt) {
            Box b{1e300, -1e300, 1e300, -1e300, 0.0};
            for (int e = e0; e < e0 + cnt; ++e) {
                const int a = p->elnodes[2 * e], c = p->elnodes[2 * e + 1];
                const double ax = p->xy[2 * a], ay = p->xy[2 * a + 1], cx = p->xy[2 * c], cy = p->xy[2 * c + 1];
                const double mx = 0.5 * (ax + cx), my = 0.5 * (ay + cy);
                b.x0 = std::min(b.x0, mx);
                b.x1 = std::max(b.x1, mx);
                b.y0 = std::min(b.y0, my);
                b.y1 = std::max(b.y1, my);
                b.hh = std::max(b.hh, 0.5 * std::hypot(cx - ax, cy - ay));
            }
            return b;
        };
        constexpr int NP = bemk::COL_CHUNK / bemk::NEAR_PART;
        constexpr int NW = bemk::ROW_TILE / 64;
        std::vector<Box> rb(p->rtiles.size() * NW), cb(p->cchunks.size() * NP);
        for (size_t t = 0; t < p->rtiles.size(); ++t)
            for (int w = 0; w < NW; ++w) {
                const int s0 = 64 * w, cnt = std::min(64, p->rtiles[t].count - s0);
                rb[t * NW + w] = cnt > 0 ? box(p->rtiles[t].start + s0, cnt) : Box{1e300, 1e300, 1e300, 1e300, 0.0};
            }
        for (size_t c = 0; c < p->cchunks.size(); ++c)
            for (int q = 0; q < NP; ++q) {
                const int s0 = q * bemk::NEAR_PART, cnt = std::min(bemk::NEAR_PART, p->cchunks[c].count - s0);
                cb[c * NP + q] = cnt > 0 ? box(p->cchunks[c].start + s0, cnt) : Box{1e300, 1e300, 1e300, 1e300, 0.0};
            }
        for (int v = 0; v < bemk::ASM_VARIANTS; ++v) {
            p->noff[v] = (int)p->npairs.size() / 3;
            const int side = v >> 2 & 1;
            for (int t : lists[v]) {
                const IfacePlan& P = p->iface[p->rtiles[t].iface];
                const int d = side ? P.dr : P.dl;
                const double rs = std::max(bemk::XS_SERIES_F64, bemk::XS_SERIES_F32) / std::abs(p->k[d]);
                for (int w = 0; w < NW && 64 * w < p->rtiles[t].count; ++w)
                    for (size_t c = 0; c < p->cchunks.size(); ++c) {
                        if (p->sigma[(size_t)d * p->n_if + p->cchunks[c].iface] == 0) continue;
                        for (int q = 0; q < NP; ++q) {
                            if (q * bemk::NEAR_PART >= p->cchunks[c].count) break;
                            const Box &a = rb[t * NW + w], &b = cb[c * NP + q];
                            const double dx = std::max(0.0, std::max(a.x0 - b.x1, b.x0 - a.x1));
                            const double dy = std::max(0.0, std::max(a.y0 - b.y1, b.y0 - a.y1));
                            const double lim = (rs + b.hh) * (1.0 + 1e-6) + 1e-12;
                            if (dx * dx + dy * dy < lim * lim) {
                                p->npairs.push_back(t * NW + w);
                                p->npairs.push_back((int)c);
                                p->npairs.push_back(q);
                            }
                        }
                    }
            }
            p->ncount[v] = (int)p->npairs.size() / 3 - p->noff[v];
        }
    }
    // inputs for the device-side constant tables
    p->dom_in.resize(p->n_dom);
    for (int d = 0; d < p->n_dom; ++d) {
        p->dom_in[d].k[0] = p->k[d].real();
        p->dom_in[d].k[1] = p->k[d].imag();
        p->dom_in[d].has_bm = desc->bm_coef ? 1 : 0;
        p->dom_in[d].bm[0] = desc->bm_coef ? desc->bm_coef[d].re : 0.0;
        p->dom_in[d].bm[1] = desc->bm_coef ? desc->bm_coef[d].im : 0.0;
    }
    p->glob.has_alpha = desc->alpha ? 1 : 0;
    p->glob.alpha[0] = desc->alpha ? desc->alpha->re : 0.0;
    p->glob.alpha[1] = desc->alpha ? desc->alpha->im : 0.0;
    p->glob.has_beta = desc->beta ? 1 : 0;
    p->glob.beta[0] = desc->beta ? desc->beta->re : 0.0;
    p->glob.beta[1] = desc->beta ? desc->beta->im : 0.0;
    p->glob.form = p->form;
    p->glob.n_dom = p->n_dom;
    p->L = make_layout(p);
    *out = p;
    return BEM_OK;
}

void bem_destroy(bem_problem* p)
{
    if (!p) return;
    for (hipEvent_t e : p->prof.pool) (void)hipEventDestroy(e);
    drop_graphs(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (hipEvent_t e : p->asm_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->asm_side) (void)hipStreamDestroy(p->asm_side);
    if (!p->lent) {
        for (hipEvent_t e : p->flag_ev)
            if (e) (void)hipEventDestroy(e);
        if (p->pinned) (void)hipHostFree(p->pinned);
    }
    delete p;
}

bem_status bem_profile_enable(bem_problem* p, int on)
{
    if (bem_status s = check_problem(p)) return s;
    p->prof.on = on != 0;
    return BEM_OK;
}

bem_status bem_profile_read(bem_problem* p, bem_profile* out, int reset)
{
    if (bem_status s = check_problem(p)) return s;
    if (!out) return fail(BEM_E_ARG, "null output");
    Prof& P = p->prof;
    if (P.err != hipSuccess) return hip_fail(P.err, "profiling events");
    std::memset(out, 0, sizeof *out);
    for (const auto& r : P.recs) {
        HIP_OK(hipEventSynchronize(r.b));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.kind == bemk::KIND_ASSEMBLE) {
            out->assemble_launches += 1;
            out->assemble_ms += ms;
        } else if (r.kind == bemk::KIND_MATVEC) {
            out->matvec_launches += 1;
            out->matvec_ms += ms;
        } else {
            out->residual_launches += 1;
            out->residual_ms += ms;
        }
    }
    if (reset) {
        P.recs.clear();
        P.used = 0;
        for (hipEvent_t& e : P.pending) e = nullptr;
    }
    return BEM_OK;
}

int bem_n_elements(const bem_problem* p) { return p ? p->N : -1; }
int bem_order(const bem_problem* p) { return p ? 2 * p->N : -1; }

bem_status bem_sizes(const bem_problem* p, int prec, int nrhs, int restart, size_t* geom_bytes,
                     size_t* matrix_bytes, size_t* work_bytes)
{
    if (bem_status s = check_problem(p)) return s;
    if (prec != BEM_F64 && prec != BEM_F32 && prec != BEM_MIXED)
        return fail(BEM_E_ARG, "prec must be BEM_F64, BEM_F32 or BEM_MIXED");
    if (nrhs < 1) return fail(BEM_E_ARG, "nrhs must be >= 1");
    if (restart < 1 || restart > BEM_MAX_RESTART)
        return fail(BEM_E_ARG, "restart must be in [1, " + std::to_string(BEM_MAX_RESTART) + "]");
    const size_t n = 2 * (size_t)p->N;
    if (geom_bytes) *geom_bytes = p->L.total;
    if (matrix_bytes) *matrix_bytes = bemk::matrix_bytes_ld(prec, n, n);
    if (work_bytes) *work_bytes = make_work((int)n, nrhs, restart).total;
    return BEM_OK;
}

bem_status bem_geometry(bem_problem* p, void* geom_dev, size_t geom_bytes, hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!geom_dev) return fail(BEM_E_ARG, "null geometry buffer");
    if (geom_bytes < p->L.total) return fail(BEM_E_NOMEM, "geometry buffer smaller than bem_sizes asked for");
    const GeomLayout& L = p->L;
    // one host image of everything uploaded
    std::vector<char> img(L.elem, 0);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + off, src, bytes);
    };
    put(L.nodes, p->xy.data(), p->xy.size() * sizeof(double));
    put(L.elnodes, p->elnodes.data(), p->elnodes.size() * sizeof(int));
    put(L.elif, p->elif.data(), p->elif.size() * sizeof(int));
    put(L.iface, p->iface.data(), p->iface.size() * sizeof(IfacePlan));
    put(L.rtiles, p->rtiles.data(), p->rtiles.size() * sizeof(Tile));
    put(L.cchunks, p->cchunks.data(), p->cchunks.size() * sizeof(Tile));
    put(L.sigma, p->sigma.data(), p->sigma.size() * sizeof(int));
    put(L.dom_in, p->dom_in.data(), p->dom_in.size() * sizeof(bemk::DomIn));
    put(L.glob_in, &p->glob, sizeof(bemk::GlobalIn));
    put(L.vtiles, p->vtiles.data(), p->vtiles.size() * sizeof(int));
    put(L.npairs, p->npairs.data(), p->npairs.size() * sizeof(int));
    char* g = static_cast<char*>(geom_dev);
    HIP_OK(hipMemcpyAsync(g, img.data(), img.size(), hipMemcpyHostToDevice, stream));
    HIP_OK(bemk::launch_setup(g, L, p->N, p->n_dom, p->quad, stream));
    // the host image must outlive the asynchronous copy
    HIP_OK(hipStreamSynchronize(stream));
    p->geom = g;
    p->A = nullptr;
    p->prec = -1;
    return BEM_OK;
}

bem_status bem_geometry_update(bem_problem* p, hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->geom) return fail(BEM_E_STATE, "bem_geometry must run before bem_geometry_update");
    HIP_OK(bemk::launch_setup(p->geom, p->L, p->N, p->n_dom, p->quad, stream));
    p->A = nullptr;
    p->prec = -1;
    return BEM_OK;
}

bem_status bem_assemble(bem_problem* p, int prec, void* A_dev, size_t lda, hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->geom) return fail(BEM_E_STATE, "bem_geometry must run before bem_assemble");
    if (prec != BEM_F64 && prec != BEM_F32 && prec != BEM_MIXED)
        return fail(BEM_E_ARG, "prec must be BEM_F64, BEM_F32 or BEM_MIXED");
    const size_t n = 2 * (size_t)p->N;
    if (!A_dev) return fail(BEM_E_ARG, "null matrix");
    if (lda < n) return fail(BEM_E_ARG, "lda < n");
    const int nrt = (int)p->rtiles.size(), ncc = (int)p->cchunks.size();
    if (nrt > 65535 || ncc > 65535) return fail(BEM_E_ARG, "problem too large for one assembly grid");
    const int* lists[bemk::ASM_VARIANTS];
    const int* pairs[bemk::ASM_VARIANTS];
    for (int v = 0; v < bemk::ASM_VARIANTS; ++v) {
        lists[v] = reinterpret_cast<const int*>(p->geom + p->L.vtiles) + p->voff[v];
        pairs[v] = reinterpret_cast<const int*>(p->geom + p->L.npairs) + 3 * (size_t)p->noff[v];
    }
    bemk::resolve_shapes(p->frozen.get(), (int)n, p->shapes);
    bemk::hook_call(p->hk(), bemk::KIND_ASSEMBLE, 0, stream);
    float2* A32 = prec == BEM_MIXED ? reinterpret_cast<float2*>(static_cast<char*>(A_dev) + mixed_offset(n, lda))
                                    : nullptr;
    // The equation-block variants write disjoint rows, so every second one
    // runs on the problem's side stream (forked from the caller's stream and
    // joined back below): one variant's launches fill the other's tails.
    int nvar = 0;
    for (int v = 0; v < bemk::ASM_VARIANTS; ++v) nvar += p->vcount[v] > 0;
    hipStream_t side = stream;
    static const bool one_stream = [] {
        const char* e = getenv("BEM_ASM_ONE_STREAM");  // measurement switch: every variant on the caller's stream
        return e && e[0] == '1';
    }();
    if (nvar >= 2 && !one_stream) {
        if (!p->asm_side) HIP_OK(hipStreamCreateWithFlags(&p->asm_side, hipStreamNonBlocking));
        for (hipEvent_t& e : p->asm_ev)
            if (!e) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_OK(hipEventRecord(p->asm_ev[0], stream));
        HIP_OK(hipStreamWaitEvent(p->asm_side, p->asm_ev[0], 0));
        side = p->asm_side;
    }
    if (prec == BEM_F32)
        HIP_OK(bemk::launch_assemble_f32(p->geom, p->L, p->N, p->n_if, ncc, p->quad, lists, p->vcount, pairs,
                                         p->ncount, static_cast<float2*>(A_dev), lda, stream, side));
    else
        HIP_OK(bemk::launch_assemble_f64(p->geom, p->L, p->N, p->n_if, ncc, p->quad, lists, p->vcount, pairs,
                                         p->ncount, static_cast<double2*>(A_dev), lda, A32, lda, stream, side));
    if (side != stream) {
        HIP_OK(hipEventRecord(p->asm_ev[1], side));
        HIP_OK(hipStreamWaitEvent(stream, p->asm_ev[1], 0));
    }
    bemk::hook_call(p->hk(), bemk::KIND_ASSEMBLE, 1, stream);
    p->A = A_dev;
    p->A32 = A32;
    p->lda = lda;
    p->prec = prec;
    return BEM_OK;
}


bem_status bem_rhs(const bem_problem* p, int nang, const double* angles, void* B_dev, size_t ldb,
                   hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->geom) return fail(BEM_E_STATE, "bem_geometry must run before bem_rhs");
    if (nang < 1 || !angles || !B_dev) return fail(BEM_E_ARG, "bad right-hand-side arguments");
    if (ldb < 2 * (size_t)p->N) return fail(BEM_E_ARG, "ldb < n");
    HIP_OK(bemk::launch_rhs(p->geom, p->L, p->N, angles, nang, static_cast<double2*>(B_dev), ldb, stream));
    return BEM_OK;
}

bem_status bem_matvec(const bem_problem* p, int nrhs, const void* X_dev, size_t ldx, void* Y_dev, size_t ldy,
                      void* work_dev, size_t work_bytes, hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->A) return fail(BEM_E_STATE, "bem_assemble must run before bem_matvec");
    const int n = 2 * p->N;
    if (nrhs < 1 || !X_dev || !Y_dev || !work_dev) return fail(BEM_E_ARG, "bad matvec arguments");
    if (ldx < (size_t)n || ldy < (size_t)n) return fail(BEM_E_ARG, "leading dimension < n");
    const size_t need = bemk::matvec_part_elems(n, nrhs) * sizeof(double2);
    if (work_bytes < need) return fail(BEM_E_NOMEM, "work buffer smaller than bem_sizes asked for");
    char* w = static_cast<char*>(work_dev);
    if (p->prec != BEM_F32)
        HIP_OK(bemk::launch_matvec_f64(static_cast<const double2*>(p->A), p->lda, n,
                                       static_cast<const double2*>(X_dev), ldx, nrhs, static_cast<double2*>(Y_dev),
                                       ldy, reinterpret_cast<double2*>(w), stream, p->hk(), &p->shapes));
    else
        HIP_OK(bemk::launch_matvec_f32(static_cast<const float2*>(p->A), p->lda, n, static_cast<const float2*>(X_dev),
                                       ldx, nrhs, static_cast<float2*>(Y_dev), ldy,
                                       reinterpret_cast<float2*>(w), stream, p->hk(), &p->shapes));
    return BEM_OK;
}

}  // extern "C"

namespace {

// Device memory of the allocation-free product: the split-K partial sums and
// the packed right-hand sides of one product at a time per GPU.  Host code
// uses the device address from hipGetSymbolAddress, looked up once per device.
constexpr size_t SCRATCH_BYTES = BEM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

bem_status scratch_ptr(void** out)
{
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(BEM_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(BEM_E_DEVICE, "hipGetSymbolAddress gave a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BEM_OK;
}

}  // namespace

extern "C" {

bem_status bem_matvec_noalloc(const bem_problem* p, int nrhs, const void* X_dev, size_t ldx, void* Y_dev, size_t ldy,
                              hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->A) return fail(BEM_E_STATE, "bem_assemble must run before bem_matvec_noalloc");
    const int n = 2 * p->N;
    if (nrhs < 1 || !X_dev || !Y_dev) return fail(BEM_E_ARG, "bad matvec arguments");
    if (ldx < (size_t)n || ldy < (size_t)n) return fail(BEM_E_ARG, "leading dimension < n");
    const bool f64 = p->prec != BEM_F32;
    const size_t need = bemk::matvec_part_elems_shaped(p->shapes, f64 ? 3 : 0, n, nrhs) *
                        (f64 ? sizeof(double2) : sizeof(float2));
    if (need > SCRATCH_BYTES)
        return fail(BEM_E_ARG, "bem_matvec_noalloc: the product needs " + std::to_string(need) +
                                   " bytes of partial sums, more than the library's " +
                                   std::to_string(SCRATCH_BYTES) + "-byte device scratch; use bem_matvec");
    void* w = nullptr;
    if (bem_status s = scratch_ptr(&w)) return s;
    if (f64)
        HIP_OK(bemk::launch_matvec_f64(static_cast<const double2*>(p->A), p->lda, n,
                                       static_cast<const double2*>(X_dev), ldx, nrhs, static_cast<double2*>(Y_dev),
                                       ldy, static_cast<double2*>(w), stream, nullptr, &p->shapes));
    else
        HIP_OK(bemk::launch_matvec_f32(static_cast<const float2*>(p->A), p->lda, n, static_cast<const float2*>(X_dev),
                                       ldx, nrhs, static_cast<float2*>(Y_dev), ldy, static_cast<float2*>(w), stream,
                                       nullptr, &p->shapes));
    return BEM_OK;
}

bem_status bem_tune(const bem_problem* p, int nrhs, const void* X_dev, size_t ldx, void* Y_dev, size_t ldy,
                    void* work_dev, size_t work_bytes, int reps, bem_tune_info* info, hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->A) return fail(BEM_E_STATE, "bem_assemble must run before bem_tune");
    const int n = 2 * p->N;
    if (nrhs < 1 || !X_dev || !Y_dev || !work_dev) return fail(BEM_E_ARG, "bad tuning arguments");
    if (reps < 1 || reps > 100) return fail(BEM_E_ARG, "reps must be in [1, 100]");
    if (ldx < (size_t)n || ldy < (size_t)n) return fail(BEM_E_ARG, "leading dimension < n");
    const size_t need = bemk::matvec_part_elems(n, nrhs) * sizeof(double2);
    if (work_bytes < need) return fail(BEM_E_NOMEM, "work buffer smaller than bem_sizes asked for");
    const int nr = std::min(nrhs, 64);
    const int ng = nr > 4 ? (nr + 15) / 16 : 0;
    const bool f64 = p->prec == BEM_F64;
    const int types = f64 ? 3 : 0;  // FP64 matrix and sums, or FP32 matrix and sums (FP64 vectors)
    const double2* X = static_cast<const double2*>(X_dev);
    double2* Y = static_cast<double2*>(Y_dev);
    auto product = [&]() -> hipError_t {
        if (f64)
            return bemk::launch_matvec_f64(static_cast<const double2*>(p->A), p->lda, n, X, ldx, nr, Y, ldy,
                                           static_cast<double2*>(work_dev), stream, nullptr);
        const float2* A32 = static_cast<const float2*>(p->prec == BEM_MIXED ? p->A32 : p->A);
        return bemk::launch_matvec_f32x64(A32, p->lda, n, X, ldx, nr, Y, ldy, static_cast<float2*>(work_dev), stream,
                                          nullptr);
    };
    const std::vector<bemk::MvShape> cand = bemk::candidate_shapes(types, ng, n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    // average of `reps` products after one untimed, per candidate
    auto timed = [&](const bemk::MvShape& sh, double& avg) -> hipError_t {
        bemk::force_shape(&sh);
        hipError_t e = product();
        if (e == hipSuccess) e = hipEventRecord(e0, stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = product();
        if (e == hipSuccess) e = hipEventRecord(e1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        avg = (double)ms / reps;
        return e;
    };
    std::vector<double> t(cand.size(), 1e300);
    for (size_t c = 0; c < cand.size() && err == hipSuccess; ++c) err = timed(cand[c], t[c]);
    const double def = t[0];  // the built-in shape is the first candidate
    // the fastest few again, twice each in turn, keeping each one's best
    // time: candidates within timing noise of each other are then ranked on
    // more than one short sample
    std::vector<size_t> order(cand.size());
    for (size_t c = 0; c < order.size(); ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return t[a] < t[b]; });
    const size_t top = std::min<size_t>(4, order.size());
    for (int pass = 0; pass < 2 && err == hipSuccess; ++pass)
        for (size_t k = 0; k < top && err == hipSuccess; ++k) {
            double again = 0.0;
            err = timed(cand[order[k]], again);
            t[order[k]] = std::min(t[order[k]], again);
        }
    size_t bi = 0;
    for (size_t c = 1; c < cand.size(); ++c)
        if (t[c] < t[bi]) bi = c;
    const double best = t[bi];
    const bemk::MvShape bestc = cand[bi];
    bemk::force_shape(nullptr);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(BEM_E_DEVICE, std::string("bem_tune: ") + hipGetErrorString(err));
    bemk::set_tuned_shape(types, ng, n, bestc);
    // this problem runs the tuned shape from now on (others when assembled next)
    p->shapes.s[types][ng] = bemk::current_shape(types, ng, n);
    if (info) {
        info->rt = bestc.rt;
        info->u = bestc.u;
        info->splits = bestc.splits;
        info->g3 = bestc.g3;
        info->candidates = (int)cand.size();
        info->best_ms = best;
        info->default_ms = def;
    }
    return BEM_OK;
}

size_t bem_tune_export(char* buf, size_t len)
{
    const std::string t = bemk::export_tuned_shapes();
    if (buf && len > 0) {
        const size_t c = std::min(len - 1, t.size());
        std::memcpy(buf, t.data(), c);
        buf[c] = '\0';
    }
    return t.size();
}

bem_status bem_tune_import(const char* text)
{
    if (!text || !bemk::import_tuned_shapes(text)) return fail(BEM_E_ARG, "malformed launch-shape table");
    return BEM_OK;
}

void bem_tune_reset(void) { bemk::clear_tuned_shapes(); }

}  // extern "C"

namespace {

// Shared state of one bem_solve call.
struct Solver {
    bem_problem* p;
    WorkLayout W;
    char* w;
    hipStream_t s;
    int n, nr, m;
    int graph = 0;  // Krylov steps per captured graph (0: kernel-by-kernel launches)
    template <class T>
    T* at(size_t off) const
    {
        return reinterpret_cast<T*>(w + off);
    }
    // The Krylov basis: complex128, or complex64 when the products run in FP32
    // (the inner solves of BEM_F32 / BEM_MIXED; same element offsets, half
    // the bytes of the region)
    bool v32() const { return p->prec != BEM_F64; }
    double2* V(int i) const { return at<double2>(W.V) + (size_t)i * nr * W.ldv; }
    float2* V32(int i) const { return at<float2>(W.V) + (size_t)i * nr * W.ldv; }
};

// The Krylov step's product Y = A v_j: with more than 4 right-hand sides the
// matrix-core kernel reads v_j packed (written by the kernel that produced
// v_j: the cycle start or the previous step's normalisation), with up to 4
// the vector kernel reads v_j itself.  FP64 product, or the FP32 one on the
// complex64 basis (FP32 matrix, or the FP32 copy of a BEM_MIXED one), Y in
// FP64 either way.
bemk::ProductPlan step_plan(const Solver& c)
{
    return bemk::product_plan(&c.p->shapes, c.v32() ? 0 : 3, c.n, c.nr);
}

bem_status apply_basis(const Solver& c, int j, double2* Y, size_t ldy)
{
    const bem_problem* p = c.p;
    const bemk::ProductPlan pl = step_plan(c);
    if (pl.ng > 0) {
        // from step 1 on the packed inputs are w of the previous step, and the
        // product normalises them (the Arnoldi launches skip the normalisation)
        bemk::StepNorm sn{};
        if (j >= 1) {
            sn.norm_part = c.at<double>(c.W.upd_part);
            sn.nu = bemk::update_blocks(c.n);
            sn.V = c.v32() ? static_cast<void*>(c.V32(j)) : static_cast<void*>(c.V(j));
            sn.ldv = c.W.ldv;
            sn.v32 = c.v32();
            sn.hnorm = c.at<double>(c.W.hnorm);
            sn.active = c.at<int>(c.W.active);
        }
        const bemk::StepNorm* snp = j >= 1 ? &sn : nullptr;
        if (!c.v32())
            HIP_OK(bemk::launch_product_packed_f64(pl, static_cast<const double2*>(p->A), p->lda, c.n, c.nr,
                                                   c.at<double2>(c.W.mv_part), Y, ldy, snp, c.s, p->hk()));
        else
            HIP_OK(bemk::launch_product_packed_f32(
                pl, static_cast<const float2*>(p->prec == BEM_MIXED ? p->A32 : p->A), p->lda, c.n, c.nr,
                reinterpret_cast<float2*>(c.at<double2>(c.W.mv_part)), Y, ldy, snp, c.s, p->hk()));
        return BEM_OK;
    }
    if (!c.v32()) {
        HIP_OK(bemk::launch_matvec_f64(static_cast<const double2*>(p->A), p->lda, c.n, c.V(j), c.W.ldv, c.nr, Y, ldy,
                                       c.at<double2>(c.W.mv_part), c.s, p->hk(), &p->shapes));
        return BEM_OK;
    }
    const float2* A32 = static_cast<const float2*>(p->prec == BEM_MIXED ? p->A32 : p->A);
    HIP_OK(bemk::launch_matvec_f32v(A32, p->lda, c.n, c.V32(j), c.W.ldv, c.nr, Y, ldy,
                                    reinterpret_cast<float2*>(c.at<double2>(c.W.mv_part)), c.s, p->hk(), &p->shapes));
    return BEM_OK;
}

// R = B - A X with FP64 accumulation: the FP64 matrix (BEM_F64, BEM_MIXED) or
// the FP32 one widened on load (BEM_F32).
bem_status residual(const Solver& c, const double2* B, size_t ldb, const double2* X, size_t ldx, double2* R,
                    size_t ldr)
{
    const bem_problem* p = c.p;
    if (p->prec != BEM_F32)
        HIP_OK(bemk::launch_residual_f64(static_cast<const double2*>(p->A), p->lda, c.n, X, ldx, c.nr, B, ldb, R, ldr,
                                         c.at<double2>(c.W.mv_part), c.s, p->hk(), &p->shapes));
    else
        HIP_OK(bemk::launch_residual_f32A(static_cast<const float2*>(p->A), p->lda, c.n, X, ldx, c.nr, B, ldb, R,
                                          ldr, c.at<double2>(c.W.mv_part), c.s, p->hk(), &p->shapes));
    return BEM_OK;
}

bem_status col_norms(const Solver& c, const double2* X, size_t ldx, double* dev_out, std::vector<double>& host)
{
    HIP_OK(bemk::launch_col_norms(X, ldx, c.n, c.nr, c.at<double>(c.W.norm_part), dev_out, c.s));
    host.resize(c.nr);
    HIP_OK(hipMemcpyAsync(host.data(), dev_out, c.nr * sizeof(double), hipMemcpyDeviceToHost, c.s));
    HIP_OK(hipStreamSynchronize(c.s));
    return BEM_OK;
}

bem_status upload_ints(const Solver& c, size_t off, const std::vector<int>& v)
{
    HIP_OK(hipMemcpyAsync(c.w + off, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, c.s));
    return BEM_OK;
}

// Steps the host runs ahead of the GPU's stopping flags: 1 for matrices of
// 128 MB and more (a product outlasts the host's work for a step), up to
// FLAG_RING - 1 for small ones.
int flag_lag(int n, int prec)
{
    const double bytes = (double)n * n * (prec == BEM_F64 ? 16.0 : 8.0);
    if (bytes >= 128e6) return 1;
    if (bytes >= 32e6) return 2;
    return bemk::FLAG_RING - 1;
}

// The executable graph of Arnoldi segment sg: steps j = sg S .. min(m, sg S + S - 1),
// each the product V_j -> W (none for j = m) and the orthogonalisation kernels,
// the stopping flags of step j going to pinned slot j % ring.  Captured on the
// problem's private stream the first time the segment is reached (capture only
// records the launches), instantiated, and kept for later cycles and calls
// while nothing the launches bake in has changed.
bem_status segment_graph(Solver& c, bemk::ArnoldiArgs arn, int sg, int S, int ring, hipGraphExec_t& out)
{
    bem_problem* p = c.p;
    auto& G = p->graphs;
    if (G.A != p->A || G.A32 != p->A32 || G.lda != p->lda || G.prec != p->prec || G.w != c.w ||
        G.ldv != c.W.ldv || G.n != c.n || G.nr != c.nr || G.m != c.m || G.S != S || G.maxit != arn.maxit ||
        G.flags != p->pinned_dev || std::memcmp(&G.shapes, &p->shapes, sizeof G.shapes) != 0 || G.seg.empty()) {
        drop_graphs(p);
        G.A = p->A;
        G.A32 = p->A32;
        G.lda = p->lda;
        G.prec = p->prec;
        G.w = c.w;
        G.ldv = c.W.ldv;
        G.n = c.n;
        G.nr = c.nr;
        G.m = c.m;
        G.S = S;
        G.maxit = arn.maxit;
        G.flags = p->pinned_dev;
        G.shapes = p->shapes;
        G.seg.assign((size_t)(c.m + S) / S, nullptr);
    }
    if (!G.seg[sg]) {
        if (!p->cap) HIP_OK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        HIP_OK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
        Solver cc = c;
        cc.s = p->cap;
        bem_status st = BEM_OK;
        hipError_t e = hipSuccess;
        const int j1 = std::min(c.m, sg * S + S - 1);
        for (int j = sg * S; j <= j1 && st == BEM_OK && e == hipSuccess; ++j) {
            if (j < c.m) st = apply_basis(cc, j, c.at<double2>(c.W.W), c.W.ldv);
            if (st != BEM_OK) break;
            arn.flags_out = p->pinned_dev + (size_t)(j % ring) * c.nr;
            e = bemk::launch_arnoldi(arn, j, p->cap);
        }
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(p->cap, &g);
        if (st == BEM_OK && e == hipSuccess) e = ee;
        if (st == BEM_OK && e == hipSuccess) e = hipGraphInstantiateWithFlags(&G.seg[sg], g, 0);
        if (g) (void)hipGraphDestroy(g);
        if (st != BEM_OK) return st;
        if (e != hipSuccess) {
            G.seg[sg] = nullptr;
            return hip_fail(e, "capturing an Arnoldi segment");
        }
    }
    out = G.seg[sg];
    return BEM_OK;
}

// GMRES(m) from X = 0 on the columns with want[r] != 0 (Sec. 3.2).  Arnoldi
// with delayed re-orthogonalisation (launch_arnoldi: steps 0..m, the last one
// only completes column m - 1); the true residual is recomputed at the end of
// each cycle with FP64 accumulation.  Columns with want[r] == 0 are left
// untouched.  iters[r] counts completed Krylov steps; tol[r] is the relative
// tolerance of column r.
//
// A batch runs several problems (same restart length and basis precision, one
// stream) in step: each step launches every running problem's product, then
// one fused set of orthogonalisation launches for all of them
// (launch_arnoldi_set); a problem whose columns have all stopped leaves the
// step loop, and at the end of a cycle each problem restarts or finishes on
// its own.  A problem's results do not depend on the batch it runs in.
struct GmItem {
    Solver* c = nullptr;
    const double2* B = nullptr;
    size_t ldb = 0;
    double2* X = nullptr;
    size_t ldx = 0;
    std::vector<double> tol;
    int maxit = 0;
    std::vector<int> want;
    std::vector<int>* iters = nullptr;
    std::vector<int>* conv = nullptr;
    std::vector<double>* rel = nullptr;
    std::vector<int>* cycles = nullptr;
    bool nonfinite = false;
    // run state
    std::vector<double> bnorm, rnorm;
    std::vector<int> alive;
    bemk::ArnoldiArgs arn{};
    bemk::ProductPlan pl{};
    void* xt = nullptr;
    bool run = false;  // still stepping in the current cycle
    bool any_alive() const { return std::count(alive.begin(), alive.end(), 1) > 0; }
};

// Start of a GMRES run: X = 0 on the wanted columns, R = B, norms, stopping
// thresholds, the flag ring (ring slots per column) and the step arguments.
bem_status gmres_begin(GmItem& g, int ring, int nev)
{
    Solver& c = *g.c;
    const int n = c.n, nr = c.nr, m = c.m;
    const size_t ldv = c.W.ldv;
    double2* R = c.at<double2>(c.W.R);
    for (int r = 0; r < nr; ++r)
        if (g.want[r]) HIP_OK(hipMemsetAsync(g.X + (size_t)r * g.ldx, 0, (size_t)n * sizeof(double2), c.s));
    HIP_OK(hipMemcpy2DAsync(R, ldv * sizeof(double2), g.B, g.ldb * sizeof(double2), (size_t)n * sizeof(double2), nr,
                            hipMemcpyDeviceToDevice, c.s));
    if (bem_status st = col_norms(c, g.B, g.ldb, c.at<double>(c.W.bnorm), g.bnorm)) return st;
    g.rnorm = g.bnorm;
    HIP_OK(hipMemcpyAsync(c.at<double>(c.W.rnorm), g.rnorm.data(), nr * sizeof(double), hipMemcpyHostToDevice, c.s));
    g.alive.assign(nr, 0);
    for (int r = 0; r < nr; ++r) {
        if (!g.want[r]) continue;
        if (!std::isfinite(g.bnorm[r])) {
            g.nonfinite = true;
            continue;
        }
        if (g.bnorm[r] == 0.0) {
            (*g.conv)[r] = 1;
            (*g.rel)[r] = 0.0;
            continue;
        }
        g.alive[r] = 1;
    }
    // device-side stopping thresholds and counters
    std::vector<double> thr(nr);
    for (int r = 0; r < nr; ++r) thr[r] = g.tol[(size_t)r] * g.bnorm[r];
    HIP_OK(hipMemcpyAsync(c.at<double>(c.W.thr), thr.data(), nr * sizeof(double), hipMemcpyHostToDevice, c.s));
    HIP_OK(hipMemcpyAsync(c.at<int>(c.W.iters), g.iters->data(), nr * sizeof(int), hipMemcpyHostToDevice, c.s));
    bem_problem* p = c.p;
    if (p->pinned_ints < (size_t)ring * nr) {
        if (p->lent) return fail(BEM_E_ARG, "lent flag buffer smaller than the flag ring times nrhs");
        if (p->pinned) HIP_OK(hipHostFree(p->pinned));
        p->pinned = nullptr;
        p->pinned_dev = nullptr;
        HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&p->pinned), (size_t)ring * nr * sizeof(int),
                             hipHostMallocMapped | hipHostMallocCoherent));
        p->pinned_ints = (size_t)ring * nr;
    }
    if (!p->pinned_dev) HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void**>(&p->pinned_dev), p->pinned, 0));
    for (int k = 0; k < nev; ++k)
        if (!p->flag_ev[k]) {
            if (p->lent) return fail(BEM_E_ARG, "lent flag events fewer than the flag ring");
            HIP_OK(hipEventCreateWithFlags(&p->flag_ev[k], hipEventDisableTiming));
        }
    bemk::ArnoldiArgs& arn = g.arn;
    arn = bemk::ArnoldiArgs{};
    arn.V = c.V(0);
    arn.v32 = c.v32();
    arn.ldv = ldv;
    arn.nr = nr;
    arn.m = m;
    arn.n = n;
    arn.W = c.at<double2>(c.W.W);
    arn.ldw = ldv;
    arn.partP = c.at<double2>(c.W.dot_part);
    arn.partQ = c.at<double2>(c.W.dot_part2);
    arn.Hraw = c.at<double2>(c.W.Hraw);
    arn.H = c.at<double2>(c.W.H);
    arn.cs = c.at<double2>(c.W.cs);
    arn.sn = c.at<double2>(c.W.sn);
    arn.gvec = c.at<double2>(c.W.gvec);
    arn.hnorm = c.at<double>(c.W.hnorm);
    arn.norm_part = c.at<double>(c.W.upd_part);
    arn.thr = c.at<double>(c.W.thr);
    arn.maxit = g.maxit;
    arn.iters = c.at<int>(c.W.iters);
    arn.kdim = c.at<int>(c.W.kdim);
    arn.active = c.at<int>(c.W.active);
    g.pl = step_plan(c);
    // the products read v_j packed (more than 4 right-hand sides), written by
    // the cycle start and the step's normalisation kernel
    g.xt = nullptr;
    if (g.pl.ng > 0) {
        if (c.v32())
            g.xt = reinterpret_cast<float2*>(c.at<double2>(c.W.mv_part)) + g.pl.xt_offset;
        else
            g.xt = c.at<double2>(c.W.mv_part) + g.pl.xt_offset;
        arn.xt = g.xt;
        arn.xw = g.pl.xw;
    }
    return BEM_OK;
}

// Start of a cycle: the active flags, v_0 = r / |r| (and its packed copy), g.
bem_status gmres_cycle_start(GmItem& g)
{
    Solver& c = *g.c;
    const size_t ldv = c.W.ldv;
    double2* R = c.at<double2>(c.W.R);
    if (bem_status st = upload_ints(c, c.W.active, g.alive)) return st;
    HIP_OK(hipMemsetAsync(c.at<int>(c.W.kdim), 0, c.nr * sizeof(int), c.s));
    if (c.v32())
        HIP_OK(bemk::launch_start_cycle(R, ldv, c.n, c.nr, c.at<double>(c.W.rnorm), c.m, c.V32(0), ldv,
                                        c.at<double2>(c.W.gvec), c.at<int>(c.W.active), static_cast<float2*>(g.xt),
                                        g.pl.xw, c.s));
    else
        HIP_OK(bemk::launch_start_cycle(R, ldv, c.n, c.nr, c.at<double>(c.W.rnorm), c.m, c.V(0), ldv,
                                        c.at<double2>(c.W.gvec), c.at<int>(c.W.active), static_cast<double2*>(g.xt),
                                        g.pl.xw, c.s));
    return BEM_OK;
}

// End of a cycle: the least-squares solution, X update, true residual and its
// norms, and each column's fate.
bem_status gmres_cycle_end(GmItem& g)
{
    Solver& c = *g.c;
    const int n = c.n, nr = c.nr, m = c.m;
    const size_t ldv = c.W.ldv;
    double2* R = c.at<double2>(c.W.R);
    HIP_OK(bemk::launch_backsolve(nr, m, c.at<double2>(c.W.H), c.at<double2>(c.W.gvec), c.at<int>(c.W.kdim),
                                  c.at<double2>(c.W.y), c.s));
    if (c.v32())
        HIP_OK(bemk::launch_xupdate(c.V32(0), ldv, nr, n, m, c.at<double2>(c.W.y), c.at<int>(c.W.kdim), g.X, g.ldx,
                                    c.s));
    else
        HIP_OK(bemk::launch_xupdate(c.V(0), ldv, nr, n, m, c.at<double2>(c.W.y), c.at<int>(c.W.kdim), g.X, g.ldx,
                                    c.s));
    // FP64 accumulation also inside the refinement: with FP32 products the
    // rounding of the restart residual (about 1e-7 kappa ||b||) can exceed
    // the inner tolerance of an ill-conditioned problem, which then never
    // stops
    if (bem_status st = residual(c, g.B, g.ldb, g.X, g.ldx, R, ldv)) return st;
    std::vector<int> dev_iters(nr);
    HIP_OK(hipMemcpyAsync(dev_iters.data(), c.at<int>(c.W.iters), nr * sizeof(int), hipMemcpyDeviceToHost, c.s));
    if (bem_status st = col_norms(c, R, ldv, c.at<double>(c.W.rnorm), g.rnorm)) return st;
    std::vector<int>& iters = *g.iters;
    for (int r = 0; r < nr; ++r)
        if (g.alive[r]) iters[r] = dev_iters[r];
    for (int r = 0; r < nr; ++r) {
        if (!g.alive[r]) continue;
        double& rel = (*g.rel)[r];
        rel = g.rnorm[r] / g.bnorm[r];
        if (!std::isfinite(rel)) {
            g.nonfinite = true;
            g.alive[r] = 0;
        } else if (rel <= g.tol[(size_t)r]) {
            (*g.conv)[r] = 1;
            g.alive[r] = 0;
        } else if (iters[r] >= g.maxit) {
            g.alive[r] = 0;
        } else {
            ++(*g.cycles)[r];
        }
    }
    return BEM_OK;
}

bem_status gmres_batch(const std::vector<GmItem*>& items)
{
    Solver& c0 = *items[0]->c;
    const int m = c0.m;
    // The GPU decides per right-hand side when to stop (the step blocks, which also
    // writes the decision into a ring of pinned host slots); the host reads
    // the flags `lag` steps behind, so the queue never drains.  A
    // small matrix gets a longer lag (its steps are shorter than the host's
    // launch work); steps enqueued after every column stopped do nothing but
    // an unused product.  A batch takes the lag of its largest matrix and the
    // events of its first problem.
    // With captured segments of S steps (one problem) the host reads the
    // flags of a segment's last step one segment late: S + 1 slots keep that
    // slot clear of the segment running meanwhile; two events mark segment
    // ends.
    const bool graphs = items.size() == 1 && c0.graph > 0 && !c0.p->prof.on;
    const int S = graphs ? c0.graph : 0;
    int nmax = 0;
    for (GmItem* g : items) nmax = std::max(nmax, g->c->n);
    const int lag = graphs ? 1 : flag_lag(nmax, c0.p->prec);
    const int ring = graphs ? S + 1 : lag + 1;
    const int nev = graphs ? 2 : ring;
    for (GmItem* g : items)
        if (bem_status st = gmres_begin(*g, ring, g == items[0] ? nev : 0)) return st;
    hipEvent_t* ev = c0.p->flag_ev;
    hipStream_t s = c0.s;
    std::vector<bemk::ArnoldiArgs> set;
    for (;;) {
        std::vector<GmItem*> cyc;
        for (GmItem* g : items)
            if (g->any_alive()) cyc.push_back(g);
        if (cyc.empty()) break;
        for (GmItem* g : cyc) {
            if (bem_status st = gmres_cycle_start(*g)) return st;
            g->run = true;
        }
        if (graphs) {
            GmItem& g = *cyc[0];
            Solver& c = *g.c;
            for (int sg = 0; sg < (m + S) / S; ++sg) {
                hipGraphExec_t ex = nullptr;
                if (bem_status st = segment_graph(c, g.arn, sg, S, ring, ex)) return st;
                HIP_OK(hipGraphLaunch(ex, s));
                HIP_OK(hipEventRecord(ev[sg & 1], s));
                if (sg >= 1) {
                    HIP_OK(hipEventSynchronize(ev[(sg - 1) & 1]));
                    const int jl = sg * S - 1;  // last step of the previous segment
                    const int* prev = c.p->pinned + (size_t)(jl % ring) * c.nr;
                    bool any = false;
                    for (int r = 0; r < c.nr; ++r) any = any || prev[r];
                    if (!any) break;
                }
            }
        }
        for (int j = 0; !graphs && j <= m; ++j) {
            set.clear();
            for (GmItem* g : cyc) {
                if (!g->run) continue;
                Solver& c = *g->c;
                if (j < m)
                    if (bem_status st = apply_basis(c, j, c.at<double2>(c.W.W), c.W.ldv)) return st;
                g->arn.flags_out = c.p->pinned_dev + (size_t)(j % ring) * c.nr;
                set.push_back(g->arn);
            }
            for (size_t k = 0; k < set.size(); k += bemk::MAX_FUSED)
                HIP_OK(bemk::launch_arnoldi_set(set.data() + k, (int)std::min(set.size() - k, (size_t)bemk::MAX_FUSED), j,
                                                s));
            HIP_OK(hipEventRecord(ev[j % ring], s));
            if (j >= lag) {
                HIP_OK(hipEventSynchronize(ev[(j - lag) % ring]));
                bool any_run = false;
                for (GmItem* g : cyc) {
                    if (!g->run) continue;
                    const int* prev = g->c->p->pinned + (size_t)((j - lag) % ring) * g->c->nr;
                    bool any = false;
                    for (int r = 0; r < g->c->nr; ++r) any = any || prev[r];
                    // every column stopped at step j - lag: the later steps were no-ops for it
                    if (!any) g->run = false;
                    any_run = any_run || g->run;
                }
                if (!any_run) break;
            }
        }
        for (GmItem* g : cyc)
            if (bem_status st = gmres_cycle_end(*g)) return st;
    }
    return BEM_OK;
}

}  // namespace

extern "C" {

bem_status bem_solve(bem_problem* p, int nrhs, const void* B_dev, size_t ldb, const bem_solve_opts* opts,
                     void* X_dev, size_t ldx, void* work_dev, size_t work_bytes, bem_solve_info* info,
                     hipStream_t stream)
{
    return bem_solve_batch(1, &p, &nrhs, &B_dev, &ldb, opts, &X_dev, &ldx, &work_dev, &work_bytes, &info, stream);
}

}  // extern "C"

namespace {

// One problem of bem_solve_batch: its solver state and per-column results.
struct SolveItem {
    Solver c;
    const double2* B;
    size_t ldb;
    double2* X;
    size_t ldx;
    std::vector<int> iters, conv, cycles, want;
    std::vector<double> rel;
    bool nonfinite = false;
    // mixed precision: outer refinement state
    std::vector<double> bnorm, rnorm;
    std::vector<int> active;
    std::vector<int> it2, conv2, cyc2;
    std::vector<double> rel2;
};

}  // namespace

extern "C" {

bem_status bem_solve_batch(int np, bem_problem* const* ps, const int* nrhs_v, const void* const* B_dev,
                           const size_t* ldb_v, const bem_solve_opts* opts, void* const* X_dev, const size_t* ldx_v,
                           void* const* work_dev, const size_t* work_bytes, bem_solve_info* const* info,
                           hipStream_t stream)
{
    if (np < 1 || np > bemk::MAX_FUSED) return fail(BEM_E_ARG, "np must be in [1, 8]");
    if (!ps || !nrhs_v || !B_dev || !ldb_v || !opts || !X_dev || !ldx_v || !work_dev || !work_bytes || !info)
        return fail(BEM_E_ARG, "bad solve arguments");
    if (opts->restart < 1 || opts->restart > BEM_MAX_RESTART)
        return fail(BEM_E_ARG, "restart must be in [1, " + std::to_string(BEM_MAX_RESTART) + "]");
    if (!(opts->tol > 0.0) || opts->max_iter < 1) return fail(BEM_E_ARG, "tol must be > 0 and max_iter >= 1");
    if (opts->graph_steps < 0 || opts->graph_steps > bemk::GRAPH_MAX_STEPS)
        return fail(BEM_E_ARG, "graph_steps must be in [0, " + std::to_string(bemk::GRAPH_MAX_STEPS) + "]");
    std::vector<SolveItem> it((size_t)np);
    for (int k = 0; k < np; ++k) {
        bem_problem* p = ps[k];
        if (bem_status s = check_problem(p)) return s;
        if (!p->A) return fail(BEM_E_STATE, "bem_assemble must run before bem_solve");
        const int nrhs = nrhs_v[k];
        if (nrhs < 1 || !B_dev[k] || !X_dev[k] || !work_dev[k] || !info[k]) return fail(BEM_E_ARG, "bad solve arguments");
        const int n = 2 * p->N;
        if (ldb_v[k] < (size_t)n || ldx_v[k] < (size_t)n) return fail(BEM_E_ARG, "leading dimension < n");
        if ((p->prec == BEM_F64) != (ps[0]->prec == BEM_F64))
            return fail(BEM_E_ARG, "a batch mixes FP64 and FP32-product problems");
        for (int q = 0; q < k; ++q)
            if (ps[q] == p) return fail(BEM_E_ARG, "a problem appears twice in the batch");
        SolveItem& t = it[(size_t)k];
        t.c = Solver{p, make_work(n, nrhs, opts->restart), static_cast<char*>(work_dev[k]), stream, n, nrhs,
                     opts->restart, np == 1 ? opts->graph_steps : 0};
        if (work_bytes[k] < t.c.W.total) return fail(BEM_E_NOMEM, "work buffer smaller than bem_sizes asked for");
        t.B = static_cast<const double2*>(B_dev[k]);
        t.ldb = ldb_v[k];
        t.X = static_cast<double2*>(X_dev[k]);
        t.ldx = ldx_v[k];
        t.iters.assign(nrhs, 0);
        t.conv.assign(nrhs, 0);
        t.cycles.assign(nrhs, 0);
        t.want.assign(nrhs, 1);
        t.rel.assign(nrhs, 1.0);
    }
    auto item = [&](SolveItem& t, const double2* B, size_t ldb, double2* X, size_t ldx, const std::vector<double>& tol,
                    const std::vector<int>& want, std::vector<int>& iters, std::vector<int>& conv,
                    std::vector<double>& rel, std::vector<int>& cycles) {
        GmItem g;
        g.c = &t.c;
        g.B = B;
        g.ldb = ldb;
        g.X = X;
        g.ldx = ldx;
        g.tol = tol;
        g.maxit = opts->max_iter;
        g.want = want;
        g.iters = &iters;
        g.conv = &conv;
        g.rel = &rel;
        g.cycles = &cycles;
        return g;
    };
    if (ps[0]->prec == BEM_F64) {
        std::vector<GmItem> gs;
        gs.reserve((size_t)np);
        for (SolveItem& t : it)
            gs.push_back(item(t, t.B, t.ldb, t.X, t.ldx, std::vector<double>((size_t)t.c.nr, opts->tol), t.want,
                              t.iters, t.conv, t.rel, t.cycles));
        std::vector<GmItem*> gp;
        for (GmItem& g : gs) gp.push_back(&g);
        if (bem_status st = gmres_batch(gp)) return st;
        for (size_t k = 0; k < gs.size(); ++k)
            if (gs[k].nonfinite) it[k].nonfinite = true;
    } else {
        // FP32 products inside GMRES, FP64 outer iterative refinement:
        //   r = b - A x (FP64 accumulation), solve A d = r loosely, x += d.
        const double inner_tol = opts->inner_tol > 0.0 ? opts->inner_tol : 1e-5;
        const int max_refine = opts->max_refine > 0 ? opts->max_refine : 20;
        for (SolveItem& t : it) {
            Solver& c = t.c;
            const size_t ldv = c.W.ldv;
            for (int r = 0; r < c.nr; ++r)
                HIP_OK(hipMemsetAsync(t.X + (size_t)r * t.ldx, 0, (size_t)c.n * sizeof(double2), stream));
            if (bem_status st = col_norms(c, t.B, t.ldb, c.at<double>(c.W.bnorm), t.bnorm)) return st;
            HIP_OK(hipMemcpy2DAsync(c.at<double2>(c.W.Ro), ldv * sizeof(double2), t.B, t.ldb * sizeof(double2),
                                    (size_t)c.n * sizeof(double2), c.nr, hipMemcpyDeviceToDevice, stream));
            t.rnorm = t.bnorm;
            t.active.assign(c.nr, 1);
        }
        for (int step = 0; step <= max_refine; ++step) {
            std::vector<GmItem> gs;
            std::vector<SolveItem*> in;
            gs.reserve((size_t)np);
            for (SolveItem& t : it) {
                bool any = false;
                for (int r = 0; r < t.c.nr; ++r) {
                    if (!t.active[r]) continue;
                    t.rel[r] = t.bnorm[r] > 0.0 ? t.rnorm[r] / t.bnorm[r] : 0.0;
                    if (!std::isfinite(t.rel[r])) {
                        t.nonfinite = true;
                        t.active[r] = 0;
                    } else if (t.rel[r] <= opts->tol) {
                        t.conv[r] = 1;
                        t.active[r] = 0;
                    } else if (t.iters[r] >= opts->max_iter || step == max_refine) {
                        t.active[r] = 0;
                    } else {
                        any = true;
                    }
                }
                if (!any) continue;
                // inner tolerance: inner_tol, or less if that already takes the
                // outer residual below half the target
                std::vector<double> tols((size_t)t.c.nr, inner_tol);
                for (int r = 0; r < t.c.nr; ++r)
                    if (t.active[r] && t.rnorm[r] > 0.0)
                        tols[(size_t)r] = std::max(inner_tol, 0.5 * opts->tol * t.bnorm[r] / t.rnorm[r]);
                t.it2.assign(t.c.nr, 0);
                t.conv2.assign(t.c.nr, 0);
                t.cyc2.assign(t.c.nr, 0);
                t.rel2.assign(t.c.nr, 1.0);
                const size_t ldv = t.c.W.ldv;
                gs.push_back(item(t, t.c.at<double2>(t.c.W.Ro), ldv, t.c.at<double2>(t.c.W.D), ldv, tols, t.active,
                                  t.it2, t.conv2, t.rel2, t.cyc2));
                in.push_back(&t);
            }
            if (in.empty()) break;
            std::vector<GmItem*> gp;
            for (GmItem& g : gs) gp.push_back(&g);
            if (bem_status st = gmres_batch(gp)) return st;
            for (size_t k = 0; k < in.size(); ++k) {
                SolveItem& t = *in[k];
                Solver& c = t.c;
                const size_t ldv = c.W.ldv;
                if (gs[k].nonfinite) t.nonfinite = true;
                for (int r = 0; r < c.nr; ++r) {
                    t.iters[r] += t.it2[r];
                    if (t.active[r]) ++t.cycles[r];
                }
                if (bem_status st = upload_ints(c, c.W.active, t.active)) return st;
                HIP_OK(bemk::launch_add_f64(c.at<double2>(c.W.D), ldv, c.n, c.nr, t.X, t.ldx, c.at<int>(c.W.active),
                                            stream));
                if (bem_status st = residual(c, t.B, t.ldb, t.X, t.ldx, c.at<double2>(c.W.Ro), ldv)) return st;
                if (bem_status st = col_norms(c, c.at<double2>(c.W.Ro), ldv, c.at<double>(c.W.rnorm), t.rnorm))
                    return st;
            }
        }
    }
    bool all = true, nonfinite = false;
    for (int k = 0; k < np; ++k) {
        const SolveItem& t = it[(size_t)k];
        for (int r = 0; r < t.c.nr; ++r) {
            info[k][r].iters = t.iters[r];
            info[k][r].restarts = t.cycles[r];
            info[k][r].converged = t.conv[r];
            info[k][r].rel_residual = t.rel[r];
            all = all && t.conv[r];
        }
        nonfinite = nonfinite || t.nonfinite;
    }
    if (nonfinite) return fail(BEM_E_NONFINITE, "non-finite residual");
    if (!all) return fail(BEM_E_NOCONV, "GMRES reached max_iter before tol on some right-hand side");
    return BEM_OK;
}

bem_status bem_farfield(const bem_problem* p, int nrhs, const void* X_dev, size_t ldx, int ndir, const double* dirs,
                        void* F_dev, size_t ldf, void* work_dev, size_t work_bytes, hipStream_t stream)
{
    (void)work_dev;
    (void)work_bytes;
    if (bem_status s = check_problem(p)) return s;
    if (!p->geom) return fail(BEM_E_STATE, "bem_geometry must run before bem_farfield");
    if (nrhs < 1 || ndir < 1 || ndir > bemk::MAX_DIRS || !X_dev || !dirs || !F_dev)
        return fail(BEM_E_ARG, "bad far-field arguments");
    if (ldx < 2 * (size_t)p->N || ldf < (size_t)ndir) return fail(BEM_E_ARG, "leading dimension too small");
    if (nrhs > 65535 * 8) return fail(BEM_E_ARG, "too many right-hand sides");
    HIP_OK(bemk::launch_farfield(p->geom, p->L, p->N, p->n_if, p->n_dom, static_cast<const double2*>(X_dev), ldx, nrhs,
                                 dirs, ndir, static_cast<double2*>(F_dev), ldf, stream));
    return BEM_OK;
}

bem_status bem_nearfield(const bem_problem* p, int nrhs, const void* X_dev, size_t ldx, const double* angles,
                         int npts, const double* xy_dev, const int* dom_dev, void* U_dev, size_t ldu,
                         hipStream_t stream)
{
    if (bem_status s = check_problem(p)) return s;
    if (!p->geom) return fail(BEM_E_STATE, "bem_geometry must run before bem_nearfield");
    if (nrhs < 1 || npts < 0 || !X_dev || (npts > 0 && (!xy_dev || !dom_dev || !U_dev)))
        return fail(BEM_E_ARG, "bad near-field arguments");
    if (ldx < 2 * (size_t)p->N || ldu < (size_t)npts) return fail(BEM_E_ARG, "leading dimension too small");
    if (npts == 0) return BEM_OK;
    std::vector<int> cplx((size_t)p->n_dom);
    for (int d = 0; d < p->n_dom; ++d) cplx[(size_t)d] = p->k[(size_t)d].imag() != 0.0;
    HIP_OK(bemk::launch_nearfield(p->geom, p->L, p->n_if, p->n_dom, p->N, p->quad, cplx.data(),
                                  static_cast<const double2*>(X_dev), ldx, nrhs, angles, xy_dev, dom_dev, npts,
                                  static_cast<double2*>(U_dev), ldu, stream));
    return BEM_OK;
}

}  // extern "C"

namespace bemk {

// Bytes of a matrix buffer of order n with leading dimension lda (the
// BEM_MIXED buffer holds the FP64 matrix, then its FP32 copy, same lda).
size_t matrix_bytes_ld(int prec, size_t n, size_t lda)
{
    return prec == BEM_F64   ? lda * n * sizeof(double2)
           : prec == BEM_F32 ? lda * n * sizeof(float2)
                             : mixed_offset(n, lda) + lda * n * sizeof(float2);
}

// The request server keeps one pinned flag buffer and FLAG_RING events per slot and
// lends them to each problem it runs, so that no request allocates or frees
// pinned memory (hipHostFree may wait for the whole device).
void lend_flag_buffers(bem_problem* p, int* pinned, size_t ints, const hipEvent_t* ev)
{
    p->pinned = pinned;
    p->pinned_dev = nullptr;
    p->pinned_ints = ints;
    for (int k = 0; k < FLAG_RING; ++k) p->flag_ev[k] = ev[k];
    p->lent = true;
}

// The request server's frozen shape sources: every request it runs resolves
// its launch shapes from the copy taken when the server was created.
void freeze_shapes(bem_problem* p, std::shared_ptr<const ShapeSnapshot> snap) { p->frozen = std::move(snap); }

// bem_last_error() text for the calls of the request server.
void set_last_error(const std::string& msg) { g_err = msg; }

}  // namespace bemk
