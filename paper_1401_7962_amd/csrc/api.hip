// api.hip -- the C ABI of libgj (see include/gj.h): argument checks, path
// selection, workspace layout and kernel launches.  No C++ exception leaves
// this file.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gj_launch.h"

namespace gj {
namespace {

constexpr int kOnchipMax = 128;     // largest order held in registers
constexpr int kMaxN = 16384;        // logical indices are packed in 16 bits
constexpr double kEps64 = 0x1p-52;  // default zero threshold scale (FP64 elimination)

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Opts {
    int precision = GJ_PREC_FP64;
    int want_resid = 0;
    int max_refine_iters = 10;
    int flags = 0;
    double zero_tol = -1.0;
    void *const *events = nullptr;
};

bool read_opts(const gj_opts *o, Opts &out) {
    out = Opts();
    if (!o) return true;
    if (o->precision != GJ_PREC_FP64 && o->precision != GJ_PREC_FP32_REFINED) return false;
    if (o->want_resid != 0 && o->want_resid != 1) return false;
    if (o->max_refine_iters < 0 || o->max_refine_iters > 100) return false;
    if (o->flags & ~GJ_FLAG_REUSE_PLAN) return false;
    if (std::isnan(o->zero_tol)) return false;
    out.precision = o->precision;
    out.want_resid = o->want_resid;
    out.max_refine_iters = o->max_refine_iters;
    out.flags = o->flags;
    out.zero_tol = o->zero_tol;
    out.events = (o->step_events[0] || o->step_events[1]) ? o->step_events : nullptr;
    return true;
}

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

// ------------------------------------------------------ streaming-path plan
struct BigShape {
    int n, nt, tpr, R, nblk;
    int64_t ldw;
};

int big_threads(int n, bool fp32) {
    const int ve = fp32 ? 4 : 2;
    const int per = 8 * ve;  // columns per thread
    int need = (n + per - 1) / per;
    if (need <= 256) return 256;
    if (need <= 512) return 512;
    return 1024;
}

BigShape big_shape(int n, bool fp32, int nt) {
    BigShape s;
    const int ve = fp32 ? 4 : 2;
    s.n = n;
    s.nt = nt;
    int need = (n + 8 * ve - 1) / (8 * ve);
    int tpr = 64;
    while (tpr < need) tpr <<= 1;
    if (tpr > nt) tpr = nt;
    s.tpr = tpr;
    const int rg = nt / tpr;
    int R = env_int("GJ_BIG_ROWS", 0);
    if (R <= 0) R = std::max(1, n / 512);
    R = std::max(R, rg);
    R = std::min(R, 64);
    s.R = R;
    s.nblk = (n + R - 1) / R;
    const int64_t chunk = (int64_t)tpr * ve;
    s.ldw = ((int64_t)n + chunk - 1) / chunk * chunk + env_int("GJ_BIG_PAD", 0) * ve;
    return s;
}

// Byte layout of one matrix's streaming-path buffers, relative to `base`.
struct BigBufs {
    size_t W, part, rowlog, collog, rowphys, colphys, steps, hdr, end;
};

BigBufs big_bufs(const BigShape &s, bool fp32, size_t base) {
    BigBufs b;
    const size_t es = fp32 ? 4 : 8;
    size_t c = a256(base);
    b.W = c; c = a256(c + (size_t)s.n * s.ldw * es);
    b.part = c; c = a256(c + 2 * (size_t)s.nblk * sizeof(BigPart));
    b.rowlog = c; c = a256(c + 2 * (size_t)s.ldw * 4);
    b.collog = c; c = a256(c + 2 * (size_t)s.ldw * 4);
    b.rowphys = c; c = a256(c + (size_t)s.n * 4);
    b.colphys = c; c = a256(c + (size_t)s.n * 4);
    b.steps = c; c = a256(c + (size_t)s.n * sizeof(StepRec));
    b.hdr = c; c = a256(c + sizeof(BigHdr));
    b.end = c;
    return b;
}

BigDesc make_desc(const BigShape &s, const BigBufs &b, char *ws, const double *A, int64_t lda,
                  double *X, int64_t ldx, int32_t *ipiv, int32_t *jpiv, gj_result *res) {
    BigDesc d;
    std::memset(&d, 0, sizeof(d));
    d.W = ws + b.W;
    d.ldw = s.ldw;
    d.part = reinterpret_cast<BigPart *>(ws + b.part);
    d.rowlog = reinterpret_cast<int32_t *>(ws + b.rowlog);
    d.collog = reinterpret_cast<int32_t *>(ws + b.collog);
    d.rowphys = reinterpret_cast<int32_t *>(ws + b.rowphys);
    d.colphys = reinterpret_cast<int32_t *>(ws + b.colphys);
    d.steps = reinterpret_cast<StepRec *>(ws + b.steps);
    d.hdr = reinterpret_cast<BigHdr *>(ws + b.hdr);
    d.A = A;
    d.lda = lda;
    d.X = X;
    d.ldx = ldx;
    d.ipiv = ipiv;
    d.jpiv = jpiv;
    d.res = res;
    d.mstride = s.ldw;
    d.n = s.n;
    d.R = s.R;
    d.nblk = s.nblk;
    d.tpr = s.tpr;
    return d;
}

// --------------------------------------------------------- batched plan
struct BatchPlan {
    // host copies of the device tables
    std::vector<MatDesc> mats;
    std::vector<OnchipTask> tasks;
    std::vector<int> big_members;  // member ids on the streaming path, n descending
    std::vector<BigShape> big_shapes;
    std::vector<BigBufs> big_bufs;
    std::vector<int2> bmap;
    std::vector<int> grid_per_step;
    int big_nt = 256, big_max_n = 0;
    // byte offsets in the workspace
    size_t off_mats = 0, off_tasks = 0, off_queue = 0, off_descs = 0, off_bmap = 0, total = 0;
};

bool plan_batch(int batch, const int32_t *n_host, bool fp32, BatchPlan &P) {
    P = BatchPlan();
    std::vector<int> small_k1, small_k0;
    for (int b = 0; b < batch; ++b) {
        const int n = n_host[b];
        if (n < 1 || n > kMaxN) return false;
        if (n <= 64) small_k1.push_back(b);
        else if (n <= kOnchipMax) small_k0.push_back(b);
        else P.big_members.push_back(b);
    }
    auto by_n_desc = [&](int x, int y) {
        return n_host[x] != n_host[y] ? n_host[x] > n_host[y] : x < y;
    };
    std::sort(small_k1.begin(), small_k1.end(), by_n_desc);
    std::sort(small_k0.begin(), small_k0.end(), by_n_desc);
    std::sort(P.big_members.begin(), P.big_members.end(), by_n_desc);
    // tasks, most expensive first (cost ~ n^3; a kind-1 task runs its four
    // members side by side, so it costs as much as its largest)
    struct T2 { double cost; OnchipTask t; };
    std::vector<T2> tl;
    for (int m : small_k0) {
        OnchipTask t{0, {m, -1, -1, -1}};
        tl.push_back({std::pow((double)n_host[m], 3.0) / 4.0, t});
    }
    for (size_t x = 0; x < small_k1.size(); x += 4) {
        OnchipTask t{1, {-1, -1, -1, -1}};
        for (int w = 0; w < 4 && x + w < small_k1.size(); ++w) t.m[w] = small_k1[x + w];
        tl.push_back({std::pow((double)n_host[t.m[0]], 3.0), t});
    }
    std::stable_sort(tl.begin(), tl.end(), [](const T2 &a, const T2 &b) { return a.cost > b.cost; });
    for (auto &x : tl) P.tasks.push_back(x.t);
    // layout
    size_t c = 0;
    P.off_mats = c; c = a256(c + sizeof(MatDesc) * (size_t)batch);
    P.off_tasks = c; c = a256(c + sizeof(OnchipTask) * std::max<size_t>(1, P.tasks.size()));
    P.off_queue = c; c = a256(c + 256);
    if (!P.big_members.empty()) {
        P.big_max_n = n_host[P.big_members[0]];
        P.big_nt = big_threads(P.big_max_n, fp32);
        P.off_descs = c; c = a256(c + sizeof(BigDesc) * P.big_members.size());
        size_t nb = 0;
        for (int m : P.big_members) {
            BigShape s = big_shape(n_host[m], fp32, P.big_nt);
            P.big_shapes.push_back(s);
            nb += s.nblk;
        }
        P.off_bmap = c; c = a256(c + sizeof(int2) * nb);
        for (size_t x = 0; x < P.big_members.size(); ++x) {
            BigBufs bb = big_bufs(P.big_shapes[x], fp32, c);
            P.big_bufs.push_back(bb);
            c = bb.end;
        }
        // block map: members in n-descending order, so the blocks still
        // active at step k are a prefix
        for (size_t x = 0; x < P.big_members.size(); ++x)
            for (int rb = 0; rb < P.big_shapes[x].nblk; ++rb) P.bmap.push_back(make_int2((int)x, rb));
        P.grid_per_step.assign(P.big_max_n, 0);
        for (int k = 0; k < P.big_max_n; ++k) {
            int g = 0;
            for (size_t x = 0; x < P.big_members.size(); ++x)
                if (P.big_shapes[x].n > k) g += P.big_shapes[x].nblk;
            P.grid_per_step[k] = g;
        }
    }
    P.total = std::max<size_t>(c, 256);
    return true;
}

thread_local char g_last_error[256] = {0};

gj_status hip_fail(hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "HIP error %d: %s", (int)e,
                  hipGetErrorString(e));
    return GJ_E_HIP;
}

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bn && y < x + an;
}

size_t single_ws(int n, const Opts &o, bool det_only) {
    (void)det_only;
    const bool fp32 = (o.precision == GJ_PREC_FP32_REFINED);
    if (n <= kOnchipMax) return 256;
    BigShape s = big_shape(n, fp32, big_threads(n, fp32));
    return big_bufs(s, fp32, 0).end;
}

gj_status run_single(int n, const double *A, int64_t lda, double *X, int64_t ldx, int32_t *ipiv,
                     int32_t *jpiv, gj_result *res, const Opts &o, void *ws, size_t ws_bytes,
                     hipStream_t s, bool det_only) {
    const bool fp32 = (o.precision == GJ_PREC_FP32_REFINED);
    const double eps_default = fp32 ? 0.0 : kEps64;
    if (n <= kOnchipMax) {
        MatDesc md;
        md.a_off = 0;
        md.x_off = 0;
        md.piv_off = 0;
        md.n = n;
        md.lda = (int32_t)lda;
        md.ldx = (int32_t)(det_only ? n : ldx);
        md.res_idx = 0;
        if (o.events && o.events[0]) {
            hipError_t e = hipEventRecord((hipEvent_t)o.events[0], s);
            if (e != hipSuccess) return hip_fail(e);
        }
        hipError_t e = launch_onchip(fp32, nullptr, nullptr, 0, nullptr, md, 1, A, X, ipiv, jpiv,
                                     res, o.zero_tol, eps_default, det_only ? 1 : 0, s);
        if (e != hipSuccess) return hip_fail(e);
        if (o.events && o.events[1]) {
            e = hipEventRecord((hipEvent_t)o.events[1], s);
            if (e != hipSuccess) return hip_fail(e);
        }
        return GJ_OK;
    }
    const int nt = big_threads(n, fp32);
    BigShape sh = big_shape(n, fp32, nt);
    BigBufs bb = big_bufs(sh, fp32, 0);
    if (ws_bytes < bb.end) return GJ_E_WORKSPACE;
    BigDesc d = make_desc(sh, bb, (char *)ws, A, lda, X, ldx, ipiv, jpiv, res);
    hipError_t e = launch_big(fp32, nt, nullptr, nullptr, d, nullptr, sh.nblk, sh.nblk, n,
                              det_only ? 0 : sh.nblk, o.zero_tol, eps_default, det_only ? 1 : 0,
                              o.events, s);
    if (e != hipSuccess) return hip_fail(e);
    return GJ_OK;
}

}  // namespace
}  // namespace gj

using namespace gj;

extern "C" {

const char *gj_status_string(int32_t code) {
    switch (code) {
        case GJ_OK: return "GJ_OK";
        case GJ_E_INVALID_ARG: return "GJ_E_INVALID_ARG: invalid argument";
        case GJ_E_WORKSPACE: return "GJ_E_WORKSPACE: workspace too small or misaligned";
        case GJ_E_HIP: return g_last_error[0] ? g_last_error : "GJ_E_HIP: HIP runtime error";
        case GJ_E_UNSUPPORTED: return "GJ_E_UNSUPPORTED: size or option not supported";
        case 100 + GJ_RES_OK: return "GJ_RES_OK";
        case 100 + GJ_RES_SINGULAR: return "GJ_RES_SINGULAR: every candidate pivot below the zero threshold";
        case 100 + GJ_RES_NONFINITE: return "GJ_RES_NONFINITE: NaN or infinity among the candidates";
        case 100 + GJ_RES_REFINE_FALLBACK: return "GJ_RES_REFINE_FALLBACK: refinement fell back to FP64";
    }
    return "unknown code";
}

int32_t gj_onchip_max_n(int32_t precision) {
    (void)precision;
    return kOnchipMax;
}

size_t gj_workspace_size(int32_t op, int32_t n_or_batch, const int32_t *n_host,
                         const gj_opts *opts) {
    Opts o;
    if (!read_opts(opts, o)) return 0;
    if (op == GJ_OP_INVERT || op == GJ_OP_DET) {
        if (n_or_batch < 1 || n_or_batch > kMaxN) return 0;
        return single_ws(n_or_batch, o, op == GJ_OP_DET);
    }
    if (op == GJ_OP_INVERT_BATCHED) {
        if (n_or_batch < 1 || !n_host) return 0;
        BatchPlan P;
        if (!plan_batch(n_or_batch, n_host, o.precision == GJ_PREC_FP32_REFINED, P)) return 0;
        return P.total;
    }
    return 0;
}

gj_status gj_invert(int32_t n, const double *A, int64_t lda, double *X, int64_t ldx,
                    int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts, void *ws,
                    size_t ws_bytes, void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (n < 1 || lda < n || ldx < n || !A || !X || !ipiv || !jpiv || !res)
            return GJ_E_INVALID_ARG;
        if (n > kMaxN) return GJ_E_UNSUPPORTED;
        if (o.precision != GJ_PREC_FP64) return GJ_E_UNSUPPORTED;
        const size_t abytes = ((size_t)(n - 1) * lda + n) * 8, xbytes = ((size_t)(n - 1) * ldx + n) * 8;
        if (overlaps(A, abytes, X, xbytes)) return GJ_E_INVALID_ARG;
        const size_t need = single_ws(n, o, false);
        if (n > kOnchipMax) {
            if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
            if (ws_bytes < need) return GJ_E_WORKSPACE;
            if (overlaps(ws, ws_bytes, X, xbytes) || overlaps(ws, ws_bytes, A, abytes))
                return GJ_E_INVALID_ARG;
        }
        return run_single(n, A, lda, X, ldx, ipiv, jpiv, res, o, ws, ws_bytes,
                          (hipStream_t)stream, false);
    } catch (...) {
        return GJ_E_HIP;
    }
}

gj_status gj_det(int32_t n, const double *A, int64_t lda, int32_t *ipiv, int32_t *jpiv,
                 gj_result *res, const gj_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (n < 1 || lda < n || !A || !ipiv || !jpiv || !res) return GJ_E_INVALID_ARG;
        if (n > kMaxN) return GJ_E_UNSUPPORTED;
        if (o.precision != GJ_PREC_FP64) return GJ_E_UNSUPPORTED;
        const size_t need = single_ws(n, o, true);
        if (n > kOnchipMax) {
            if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
            if (ws_bytes < need) return GJ_E_WORKSPACE;
        }
        return run_single(n, A, lda, nullptr, n, ipiv, jpiv, res, o, ws, ws_bytes,
                          (hipStream_t)stream, true);
    } catch (...) {
        return GJ_E_HIP;
    }
}

gj_status gj_invert_batched(int32_t batch, const int32_t *n_host, const int64_t *off_host,
                            const double *A, double *X, const int64_t *piv_off_host,
                            int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts,
                            void *ws, size_t ws_bytes, void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (batch < 1 || !n_host || !off_host || !piv_off_host || !A || !X || !ipiv || !jpiv ||
            !res)
            return GJ_E_INVALID_ARG;
        if (o.precision != GJ_PREC_FP64) return GJ_E_UNSUPPORTED;
        if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
        const bool fp32 = false;
        BatchPlan P;
        if (!plan_batch(batch, n_host, fp32, P)) return GJ_E_INVALID_ARG;
        if (ws_bytes < P.total) return GJ_E_WORKSPACE;
        for (int b = 0; b < batch; ++b)
            if (off_host[b] < 0 || piv_off_host[b] < 0) return GJ_E_INVALID_ARG;
        hipStream_t s = (hipStream_t)stream;
        char *w = (char *)ws;
        // device tables
        P.mats.resize(batch);
        for (int b = 0; b < batch; ++b) {
            MatDesc &m = P.mats[b];
            m.a_off = off_host[b];
            m.x_off = off_host[b];
            m.piv_off = piv_off_host[b];
            m.n = n_host[b];
            m.lda = n_host[b];
            m.ldx = n_host[b];
            m.res_idx = b;
        }
        std::vector<BigDesc> descs;
        for (size_t x = 0; x < P.big_members.size(); ++x) {
            const int m = P.big_members[x];
            descs.push_back(make_desc(P.big_shapes[x], P.big_bufs[x], w, A + off_host[m],
                                      n_host[m], X + off_host[m], n_host[m],
                                      ipiv + piv_off_host[m], jpiv + piv_off_host[m], res + m));
        }
        if (!(o.flags & GJ_FLAG_REUSE_PLAN)) {
            std::vector<char> stage(P.off_queue, 0);
            std::memcpy(stage.data() + P.off_mats, P.mats.data(), sizeof(MatDesc) * batch);
            if (!P.tasks.empty())
                std::memcpy(stage.data() + P.off_tasks, P.tasks.data(),
                            sizeof(OnchipTask) * P.tasks.size());
            hipError_t e = hipMemcpyAsync(w, stage.data(), stage.size(), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e);
            if (!descs.empty()) {
                e = hipMemcpyAsync(w + P.off_descs, descs.data(), sizeof(BigDesc) * descs.size(),
                                   hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return hip_fail(e);
                e = hipMemcpyAsync(w + P.off_bmap, P.bmap.data(), sizeof(int2) * P.bmap.size(),
                                   hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return hip_fail(e);
            }
            // the host tables die with this call: wait for the copies
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e);
        }
        const double eps_default = fp32 ? 0.0 : kEps64;
        if (!P.tasks.empty()) {
            int dev = 0, cus = 256;
            hipGetDevice(&dev);
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            const int per_cu = std::max(1, env_int("GJ_ONCHIP_WG_PER_CU", 2));
            const int grid = std::min<int>((int)P.tasks.size(), cus * per_cu);
            hipError_t e = launch_onchip(fp32, reinterpret_cast<const MatDesc *>(w + P.off_mats),
                                         reinterpret_cast<const OnchipTask *>(w + P.off_tasks),
                                         (int)P.tasks.size(),
                                         reinterpret_cast<uint32_t *>(w + P.off_queue), MatDesc(),
                                         grid, A, X, ipiv, jpiv, res, o.zero_tol, eps_default, 0, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        if (!P.big_members.empty()) {
            const int nb = (int)P.bmap.size();
            hipError_t e = launch_big(fp32, P.big_nt, reinterpret_cast<const BigDesc *>(w + P.off_descs),
                                      reinterpret_cast<const int2 *>(w + P.off_bmap), BigDesc(),
                                      P.grid_per_step.data(), nb, nb, P.big_max_n, nb, o.zero_tol,
                                      eps_default, 0, o.events, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        return GJ_OK;
    } catch (...) {
        return GJ_E_HIP;
    }
}

}  // extern "C"
