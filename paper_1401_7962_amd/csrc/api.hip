// api.hip -- the C ABI of libgj (see include/gj.h): argument checks, path
// selection, workspace layout and kernel launches.  No C++ exception leaves
// this file.
#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <optional>
#include <string>
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
    int rule = 0;   // pivot rule: 0 full, 1 partial on |a|, 2 the program's
};

bool read_opts(const gj_opts *o, Opts &out) {
    out = Opts();
    if (!o) return true;
    if (o->precision != GJ_PREC_FP64 && o->precision != GJ_PREC_FP32_REFINED) return false;
    if (o->want_resid != 0 && o->want_resid != 1) return false;
    if (o->max_refine_iters < 0 || o->max_refine_iters > 100) return false;
    if (o->flags & ~(GJ_FLAG_REUSE_PLAN | GJ_FLAG_PIVOT_PARTIAL | GJ_FLAG_PIVOT_PROGRAM | GJ_FLAG_ACCURATE |
                     GJ_FLAG_BLOCKED))
        return false;
    if ((o->flags & GJ_FLAG_ACCURATE) && o->precision != GJ_PREC_FP32_REFINED) return false;
    if ((o->flags & GJ_FLAG_BLOCKED) && (o->flags & (GJ_FLAG_PIVOT_PARTIAL | GJ_FLAG_PIVOT_PROGRAM)))
        return false;
    if ((o->flags & GJ_FLAG_PIVOT_PARTIAL) && (o->flags & GJ_FLAG_PIVOT_PROGRAM)) return false;
    if (std::isnan(o->zero_tol)) return false;
    out.precision = o->precision;
    out.want_resid = o->want_resid;
    out.max_refine_iters = o->max_refine_iters;
    out.flags = o->flags;
    out.zero_tol = o->zero_tol;
    out.events = (o->step_events[0] || o->step_events[1]) ? o->step_events : nullptr;
    out.rule = (o->flags & GJ_FLAG_PIVOT_PARTIAL) ? 1 : (o->flags & GJ_FLAG_PIVOT_PROGRAM) ? 2 : 0;
    return true;
}

}  // namespace

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

namespace {

// ------------------------------------------------------------ tuning table
// Written by the project's autotuner (paper_1401_7962_amd/tune.py) as lines
//     big_rows <f32|f64> <n_min> <n_max> <rows per workgroup> [<counted %> [<chunks>]]
// and read once from $GJ_TUNE_FILE, else from gj_tune.txt beside libgj.so.
// The optional fields are the share of a step's work units handed out by
// the step kernel's counter (default 0: every unit taken by index) and the
// register chunks a thread aims to fill (default 8; fewer means more threads
// per row).  $GJ_BIG_ROWS, $GJ_BIG_COUNTED and $GJ_BIG_CHUNKS, when set,
// override the three fields (the autotuner uses them to sweep);
// $GJ_BIG_STATIC sets the units taken by index per workgroup directly.
struct TuneEntry { int fp32, nmin, nmax, rows, counted, chunks; };
std::vector<TuneEntry> g_tune;
std::once_flag g_tune_once;

void load_tune_table() {
    std::string path;
    if (const char *f = std::getenv("GJ_TUNE_FILE")) {
        path = f;
    } else {
        Dl_info info;
        if (dladdr((void *)&load_tune_table, &info) && info.dli_fname) {
            path = info.dli_fname;
            const size_t slash = path.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/gj_tune.txt";
        }
    }
    FILE *fp = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!fp) return;
    char line[256];
    while (std::fgets(line, sizeof(line), fp)) {
        char key[64], prec[16];
        int lo, hi, v, pct = 0, ch = 8;
        const int got = std::sscanf(line, "%63s %15s %d %d %d %d %d", key, prec, &lo, &hi, &v, &pct, &ch);
        if (got >= 5 && std::strcmp(key, "big_rows") == 0 && v >= 1 && v <= 64 && lo <= hi) {
            if (got < 6 || pct < 0 || pct > 90) pct = 0;
            if (got < 7 || ch < 1 || ch > 8) ch = 8;
            g_tune.push_back(TuneEntry{std::strcmp(prec, "f32") == 0 ? 1 : 0, lo, hi, v, pct, ch});
        }
    }
    std::fclose(fp);
}

const TuneEntry *tuned(bool fp32, int n) {
    std::call_once(g_tune_once, load_tune_table);
    for (const TuneEntry &e : g_tune)
        if (e.fp32 == (fp32 ? 1 : 0) && n >= e.nmin && n <= e.nmax) return &e;
    return nullptr;
}

// ------------------------------------------------------ streaming-path plan
struct BigShape {
    int n, ncol, nt, tpr, R, nblk;   // ncol: columns of W in use (n, or rhs0 + m for a solve)
    int rhs0;                        // column of W holding B's first column (n when not solving)
    int nunits, share;   // work units of a step; units per workgroup
    int ustat;           // units per workgroup taken by index (the rest by counter)
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

BigShape big_shape(int n, bool fp32, int nt, int ncol = 0, int rows = 0, int chunks_want = 0) {
    BigShape s;
    const int ve = fp32 ? 4 : 2;
    if (ncol < n) ncol = n;
    s.n = n;
    s.ncol = ncol;
    s.rhs0 = n;
    s.nt = nt;
    // threads per row: just enough for the tuned number of vector chunks per
    // thread (8 by default, so that every thread's registers are used; a
    // wavefront may span several rows)
    const TuneEntry *te = tuned(fp32, n);
    int chunks = chunks_want > 0 ? chunks_want : env_int("GJ_BIG_CHUNKS", 0);
    if (chunks < 1 || chunks > 8) chunks = te ? te->chunks : 8;
    int need = (ncol + chunks * ve - 1) / (chunks * ve);
    int tpr = 4;
    while (tpr < need) tpr <<= 1;
    if (tpr > nt) tpr = nt;
    s.tpr = tpr;
    const int rg = nt / tpr;
    int R = rows > 0 ? rows : env_int("GJ_BIG_ROWS", 0);
    if (R <= 0 && te) R = te->rows;
    if (R <= 0) R = std::max(1, n / 512);
    // a work unit of the step kernel is one register group (2 rows per
    // thread below 1024 threads, else 1), or the workgroup's rows if fewer;
    // a workgroup covers whole units.  All are powers of two, so R stays
    // <= 64 rows: the kernel's LDS tables.
    R = std::max(std::min(R, 64), rg);
    const int unit = std::min((nt < 1024 ? 2 : 1) * rg, R);
    R = (R + unit - 1) / unit * unit;
    s.R = R;
    s.nblk = (n + R - 1) / R;
    s.nunits = (n + unit - 1) / unit;
    s.share = R / unit;
    // units taken by index per workgroup: all of its share, less the tuned
    // share left to the counter (GJ_BIG_STATIC overrides); the counter is
    // compiled only into the full-chunk kernels below 1024 threads
    const int per = tpr * (fp32 ? 4 : 2);
    const bool cnt_ok = (ncol + per - 1) / per == 8 && nt < 1024;
    int pct = env_int("GJ_BIG_COUNTED", -1);
    if (pct < 0 || pct > 90) pct = te ? te->counted : 0;
    int S = env_int("GJ_BIG_STATIC", 0);
    if (S <= 0) S = s.share - (s.share * pct + 50) / 100;
    s.ustat = cnt_ok ? std::max(1, std::min(S, s.share)) : s.share;
    const int64_t chunk = (int64_t)tpr * ve;
    s.ldw = ((int64_t)ncol + chunk - 1) / chunk * chunk + env_int("GJ_BIG_PAD", 0) * ve;
    return s;
}


// Nontemporal row loads and stores once the array swept per step clearly
// outgrows the 256 MB Infinity Cache.  Measured on MI355X (FP64, ms per
// inversion, cached / nontemporal): 6144^2 = 288 MiB 758 / 841, 6656^2 =
// 338 MiB 1077 / 1050, 7168^2 1219 / 1180, 8192^2 1661 / 1540.  Arrays the
// cache holds lose with them (8192^2 FP32, 256 MiB: 13%; 4096^2 FP64: 9% with
// the loads alone, 6% with the stores alone).  GJ_BIG_NT=0/1 overrides.
bool big_nt_loads(size_t swept_bytes) {
    const int e = env_int("GJ_BIG_NT", -1);
    return e >= 0 ? e != 0 : swept_bytes > ((size_t)320 << 20);
}
size_t big_swept_bytes(const BigShape &s, bool fp32) {
    return (size_t)s.n * (size_t)s.ldw * (fp32 ? 4 : 8);
}
// Some work units of a step are handed out by the step kernel's counter.
bool big_counted(const BigShape &s) {
    return (int64_t)s.nblk * s.ustat < s.nunits;
}
// Every thread of the row uses all 8 of its vector chunks (the step kernel
// then compiles without the per-chunk tests).
bool big_full(const BigShape &s, bool fp32) {
    const int64_t per = (int64_t)s.tpr * (fp32 ? 4 : 2);
    return (s.ncol + per - 1) / per == 8;
}
// The step kernel's chunk count for one matrix: the number of chunks its rows
// fill, 8 or (below 1024 threads; such shapes have no counted units) 1-7, so
// that no unused chunk is loaded or looped over; else 0 (the 8-chunk kernel
// with per-chunk tests).
int big_full_chunks(const BigShape &s, bool fp32) {
    const int64_t per = (int64_t)s.tpr * (fp32 ? 4 : 2);
    const int64_t ch = (s.ncol + per - 1) / per;
    if (ch == 8) return 8;
    if (ch >= 1 && ch < 8 && s.nt < 1024 && !big_counted(s)) return (int)ch;
    return 0;
}

// Row shape of a single matrix.  The table's buckets up to 1024 were tuned on
// packed batches, where many members share a launch and few workgroups per
// member pay; one matrix of that order needs the most workgroups instead: FP64
// us per step, table rows / one register group per workgroup: 512: 20.7 / 10.4,
// 768: 20.3 / 10.7, 1024: 21.2 / 11.0 (FP32: 22.3 / 15.1, 19.9 / 14.3,
// 22.6 / 15.4); above 1024 the table's single-matrix rows stay (1536: 14.3
// against 19.7).  Up to 2048 the rows are also spread over more threads (fewer
// register chunks each, on the kernel of the chunk count they fill): FP64 us
// per step with 8 / 4 / 2 chunks asked for: 256: 10.2 / 7.6 / 6.4, 512: 10.3 /
// 7.7 / 6.4, 768: 9.4 / 7.9 / 8.7, 1024: 11.0 / 9.3 / 10.5, 2048: 15.8 / 14.2 /
// 14.2; FP32 (4 / 2 / 1): 256: 10.1 / 7.7 / 6.6, 512: 10.1 / 7.7 / 6.8, 768:
// 8.9 / 8.5 / 8.9, 1024: 10.5 / 8.8 / 10.4, 2048: 14.1 / 12.5 / 12.5.
// allow_wide = false keeps the 8-chunk shape (the solve's extra right-hand-
// side chunk needs it).  GJ_BIG_ROWS and GJ_BIG_CHUNKS still override.
int wide_chunks(int n, bool fp32) {
    if (fp32) return n <= 512 ? 1 : 2;
    return n <= 512 ? 2 : 4;
}
BigShape single_shape(int n, bool fp32, int nt, int ncol = 0, bool allow_wide = true) {
    const int rows = (n <= 1024 && env_int("GJ_BIG_ROWS", 0) <= 0) ? 1 : 0;
    int chunks = 0;
    if (allow_wide && n <= 2048 && env_int("GJ_BIG_CHUNKS", 0) <= 0) chunks = wide_chunks(n, fp32);
    BigShape s = big_shape(n, fp32, nt, ncol, rows, chunks);
    if (chunks && big_full_chunks(s, fp32) == 0) s = big_shape(n, fp32, nt, ncol, rows);
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
    d.ustat = s.ustat;
    d.ncol = s.ncol;
    d.rhs0 = s.rhs0;
    return d;
}

// --------------------------------------------------------- batched plan
// Streaming members that share a launch sequence: the same chunk count filled
// exactly (the step kernel of that count), or none (the 8-chunk kernel with
// per-chunk tests).
struct BigGroup {
    int full = 0;             // launch_big's `full`
    bool counted = false;     // some member leaves units to the counter (full == 8 only)
    size_t bmap0 = 0;         // the group's first block-map entry
    int nb = 0, max_n = 0;    // its blocks, its largest order
    size_t swept = 0;         // bytes of W its steps sweep
    std::vector<int> grid_per_step;
};

struct BatchPlan {
    // host copies of the device tables
    std::vector<MatDesc> mats;
    std::vector<OnchipTask> tasks;
    std::vector<int> big_members;  // member ids on the streaming path, n descending
    std::vector<BigShape> big_shapes;
    std::vector<BigBufs> big_bufs;
    std::vector<int2> bmap;        // the groups' block maps, one after another
    std::vector<BigGroup> groups;
    int big_nt = 256, big_max_n = 0;
    int cls_start[kOnchipClasses] = {0}, cls_count[kOnchipClasses] = {0};
    // byte offsets in the workspace
    size_t off_mats = 0, off_tasks = 0, off_queue = 0, off_descs = 0, off_bmap = 0, total = 0;
};

bool plan_batch(int batch, const int32_t *n_host, bool fp32, BatchPlan &P) {
    P = BatchPlan();
    std::vector<int> by_cls[kOnchipClasses];
    for (int b = 0; b < batch; ++b) {
        const int n = n_host[b];
        if (n < 1 || n > kMaxN) return false;
        if (n <= kOnchipMax) by_cls[onchip_class_of(n, false)].push_back(b);
        else P.big_members.push_back(b);
    }
    auto by_n_desc = [&](int x, int y) {
        return n_host[x] != n_host[y] ? n_host[x] > n_host[y] : x < y;
    };
    std::sort(P.big_members.begin(), P.big_members.end(), by_n_desc);
    // one task list per class, most expensive first; a kind-1 task runs four
    // members of the class side by side (one per wavefront)
    for (int c = 0; c < kOnchipClasses; ++c) {
        auto &v = by_cls[c];
        std::sort(v.begin(), v.end(), by_n_desc);
        P.cls_start[c] = (int)P.tasks.size();
        if (onchip_class_kind(c) == 0) {
            for (int m : v) P.tasks.push_back(OnchipTask{0, {m, -1, -1, -1}});
        } else {
            for (size_t x = 0; x < v.size(); x += 4) {
                OnchipTask t{1, {-1, -1, -1, -1}};
                for (int w = 0; w < 4 && x + w < v.size(); ++w) t.m[w] = v[x + w];
                P.tasks.push_back(t);
            }
        }
        P.cls_count[c] = (int)P.tasks.size() - P.cls_start[c];
    }
    // layout
    size_t c = 0;
    P.off_mats = c; c = a256(c + sizeof(MatDesc) * (size_t)batch);
    P.off_tasks = c; c = a256(c + sizeof(OnchipTask) * std::max<size_t>(1, P.tasks.size()));
    P.off_queue = c; c = a256(c + 4 * kOnchipClasses);
    if (!P.big_members.empty()) {
        P.big_max_n = n_host[P.big_members[0]];
        P.big_nt = big_threads(P.big_max_n, fp32);
        P.off_descs = c; c = a256(c + sizeof(BigDesc) * P.big_members.size());
        size_t nb = 0;
        std::vector<int> key;   // launch_big's `full` for each member
        for (int m : P.big_members) {
            BigShape s = big_shape(n_host[m], fp32, P.big_nt);
            const int f = big_full_chunks(s, fp32);
            if (f != 8) s.ustat = s.share;   // the counter: 8 full chunks only
            key.push_back(f);
            P.big_shapes.push_back(s);
            nb += s.nblk;
        }
        P.off_bmap = c; c = a256(c + sizeof(int2) * nb);
        for (size_t x = 0; x < P.big_members.size(); ++x) {
            BigBufs bb = big_bufs(P.big_shapes[x], fp32, c);
            P.big_bufs.push_back(bb);
            c = bb.end;
        }
        // one launch sequence per chunk count (the groups run one after
        // another; members are independent).  Within a group the members stay
        // in n-descending order, so the blocks still active at step k are a
        // prefix of the group's block map.  20k members of orders 32-512:
        // plain FP64 1078 -> 1037 ms against one launch sequence for all,
        // FP32 + refinement 926 -> 883 ms.  Splitting the groups further into
        // parts of 96-640 MB (the Infinity Cache's size) gave no consistent
        // gain (FP64 981-1109 ms, FP32 stage 895-1033 ms).
        // every key a member has, largest first (so no member is left out)
        std::vector<int> fulls(key);
        std::sort(fulls.begin(), fulls.end(), std::greater<int>());
        fulls.erase(std::unique(fulls.begin(), fulls.end()), fulls.end());
        for (int f : fulls) {
            BigGroup G;
            G.full = f;
            G.bmap0 = P.bmap.size();
            for (size_t x = 0; x < P.big_members.size(); ++x) {
                if (key[x] != f) continue;
                const BigShape &sh = P.big_shapes[x];
                for (int rb = 0; rb < sh.nblk; ++rb) P.bmap.push_back(make_int2((int)x, rb));
                G.max_n = std::max(G.max_n, sh.n);
                G.swept += big_swept_bytes(sh, fp32);
                G.counted = G.counted || big_counted(sh);
            }
            G.nb = (int)(P.bmap.size() - G.bmap0);
            if (G.nb == 0) continue;
            G.grid_per_step.assign(G.max_n, 0);
            for (int k = 0; k < G.max_n; ++k)
                for (size_t x = 0; x < P.big_members.size(); ++x)
                    if (key[x] == f && P.big_shapes[x].n > k) G.grid_per_step[k] += P.big_shapes[x].nblk;
            P.groups.push_back(std::move(G));
        }
    }
    P.total = std::max<size_t>(c, 256);
    return true;
}

// The streaming members of a batch: each group's init, steps, finish and
// gather; the step events bracket the first group's steps to the last's.
hipError_t launch_big_groups(bool fp32, const BatchPlan &P, const BigDesc *descs, const int2 *bmap,
                             double zero_tol, double eps_default, void *const *events,
                             hipStream_t s) {
    for (size_t g = 0; g < P.groups.size(); ++g) {
        const BigGroup &G = P.groups[g];
        void *ev[2] = {events && g == 0 ? events[0] : nullptr,
                       events && g + 1 == P.groups.size() ? events[1] : nullptr};
        const hipError_t e = launch_big(fp32, P.big_nt, big_nt_loads(G.swept), G.full, G.counted,
                                        false, 0, descs, bmap + G.bmap0, BigDesc(),
                                        G.grid_per_step.data(), G.nb, G.nb, G.max_n, G.nb, zero_tol,
                                        eps_default, 0, ev, nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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

size_t resid_ws(int n);
struct RefinedLayout;
size_t refined_ws(int n, bool acc, bool blocked = false);

// ------------------------------------------------ blocked elimination
// Panels of kBlkNb steps on the trailing block, then the delayed updates as
// FP64 matrix-core products (blocked.hip).  Measured on MI355X (ms per
// inversion, 4096^2 / 8192^2 FP64, rows per workgroup m / 256): 128-step
// panels 109.6 / 721.8, 256-step panels 107.9 / 712.8.  The array's row stride covers
// every panel's row shape from its block's first column (a block of order m
// at column k0 sweeps k0 + ldw(m) columns); two arrays alternate, one
// panel's pivot-ordered copy being the next one's input.
constexpr int kBlkNb = 256;

// Row shape of a panel's trailing block of order m.  The table's rows were
// tuned on whole inversions (up to 1024 on packed batches); for the trailing
// blocks, rows per workgroup m / kBlkRowDiv measured better (at least one
// register group; the kernel rounds to whole work units).  ms per 4096^2 /
// 8192^2 inversion with 128-step panels: m / 256 109.6 / 721.8, m / 512
// 120.2 / 734.9, m / 1024 139.0 / 799.6, the table's rows 117.9 / 731.8;
// with 256-step panels: m / 256 108.0 / 715.1, m / 128 128.7 / 739.1, the
// table's rows above m = 2048 (m / 256 below) 107.5 / 713.3.
constexpr int kBlkRowDiv = 256;
BigShape blk_shape(int m, bool fp32) {
    const int div = env_int("GJ_BLK_RDIV", kBlkRowDiv);   // experiments
    int rows = 1;
    while (rows * 2 <= m / std::max(div, 1)) rows *= 2;
    // FP32 blocks above 6144 take the table's rows (whole-inversion tuning):
    // refined 8192^2 with FP32 delayed updates 679.7 ms against 693.9 with
    // m / 256 everywhere (402.5 / 409.9 ms for the FP32 stage; table rows
    // above 4096: 686.9, above 7000: 687.2)
    if (fp32 && m > 6144) rows = 0;
    if (env_int("GJ_BIG_ROWS", 0) > 0) rows = 0;
    // blocks up to 2048 spread each row over more threads, as single matrices
    // of that order do: ms per 4096^2 / 8192^2 FP64, refined 4096^2 with FP32
    // delayed updates: 101.3 / 689.8, 128.0 without; 98.3 / 687.1, 120.9 up to
    // 1024; 97.4 / 686.3, 121.9 up to 2048; 97.5 / 686.3, 121.1 up to 4096
    const int wide = env_int("GJ_BLK_WIDE", 2048);   // experiments
    if (m <= wide && env_int("GJ_BIG_CHUNKS", 0) <= 0) {
        const BigShape s = big_shape(m, fp32, big_threads(m, fp32), 0, rows, wide_chunks(m, fp32));
        if (big_full_chunks(s, fp32) != 0) return s;
    }
    return big_shape(m, fp32, big_threads(m, fp32), 0, rows);
}

struct BlkLayout {
    BigBufs bb;      // streaming buffers (W: the first array), sized for the largest panel
    int64_t ldw;
    int nb, nblk;    // panel width; most workgroups of any panel's step
    size_t W2, tA, tB, perm, end;
};

// base: the layout's first byte (the refined path places it after its own
// control block); an FP32 layout holds FP32 arrays.
BlkLayout blk_layout(int n, bool fp32 = false, size_t base = 0) {
    BlkLayout L;
    int nb = env_int("GJ_BLK_NB", kBlkNb);   // panel width (experiments)
    L.nb = std::max(2, std::min(nb, 1024)) & ~1;   // even: block starts stay 16-byte aligned
    int64_t ldw = n;
    int nblk = 1;
    for (int k0 = 0; k0 < n; k0 += L.nb) {
        const int m = n - k0;
        const BigShape s = blk_shape(m, fp32);
        ldw = std::max<int64_t>(ldw, k0 + s.ldw);
        nblk = std::max(nblk, s.nblk);
    }
    L.ldw = (ldw + 15) / 16 * 16;
    L.nblk = nblk;
    BigShape s0 = big_shape(n, fp32, big_threads(n, fp32));
    s0.ldw = L.ldw;
    s0.nblk = nblk;
    L.bb = big_bufs(s0, fp32, base);
    const size_t es = fp32 ? 4 : 8;
    size_t c = L.bb.end;
    L.W2 = c; c = a256(c + (size_t)n * L.ldw * es);
    L.tA = c; c = a256(c + (size_t)n * L.nb * es);    // k0 x nb, ld nb
    L.tB = c; c = a256(c + (size_t)n * L.nb * es);    // nb x k0, ld n
    L.perm = c; c = a256(c + (size_t)6 * n * 4);      // prow[2], pcol[2], rowinv, colinv
    L.end = c;
    return L;
}

// One product of the panel's delayed update, in the elimination's precision.
hipError_t blk_gemm(bool fp32, int M, int N, int K, double alpha, const void *A, int64_t lda,
                    const void *B, int64_t ldb, double beta, const void *C, int64_t ldc, void *D,
                    int64_t ldd, hipStream_t s) {
    if (fp32) {
        GemmArgsT<float> g;
        std::memset(&g, 0, sizeof(g));
        g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.beta = beta;
        g.A = (const float *)A; g.lda = lda; g.B = (const float *)B; g.ldb = ldb;
        g.C = (const float *)C; g.ldc = ldc; g.D = (float *)D; g.ldd = ldd;
        return launch_gemm_f32(g, s);
    }
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.beta = beta;
    g.A = (const double *)A; g.lda = lda; g.B = (const double *)B; g.ldb = ldb;
    g.C = (const double *)C; g.ldc = ldc; g.D = (double *)D; g.ldd = ldd;
    return launch_gemm_f64(g, s);
}

// fp32: the first stage of the refined path (zero threshold 0, as its
// unblocked FP32 elimination); X may be null (no gather).  rows / cols, when
// given, receive the device addresses of the final pivot-order maps
// (position -> original row / column).
gj_status run_blocked(bool fp32, int n, const double *A, int64_t lda, double *X, int64_t ldx,
                      int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                      double eps_default, void *ws, size_t ws_bytes, size_t base, hipStream_t s,
                      const int32_t **rows = nullptr, const int32_t **cols = nullptr) {
    const BlkLayout L = blk_layout(n, fp32, base);
    if (ws_bytes < L.end) return GJ_E_WORKSPACE;
    char *w = (char *)ws;
    const int64_t ldw = L.ldw;
    const size_t es = fp32 ? 4 : 8;
    char *Wb[2] = {w + L.bb.W, w + L.W2};
    char *tA = w + L.tA, *tB = w + L.tB;
    int32_t *perm = reinterpret_cast<int32_t *>(w + L.perm);
    int32_t *prow[2] = {perm, perm + n}, *pcol[2] = {perm + 2 * n, perm + 3 * n};
    int32_t *rowinv = perm + 4 * n, *colinv = perm + 5 * n;
    StepRec *steps = reinterpret_cast<StepRec *>(w + L.bb.steps);
    BigHdr *hdr = reinterpret_cast<BigHdr *>(w + L.bb.hdr);
    hipError_t e = launch_blk_init_perm(prow[0], pcol[0], n, s);
    if (e != hipSuccess) return hip_fail(e);
    int cur = 0;
    auto at = [&](char *base_, int64_t row, int64_t col) { return base_ + (row * ldw + col) * (int64_t)es; };
    for (int k0 = 0; k0 < n; k0 += L.nb) {
        const int m = n - k0, nbp = std::min(L.nb, m);
        const BigShape sh = blk_shape(m, fp32);
        const int nt = sh.nt;
        // the block's row shape and candidate list fit the layout
        if (k0 + sh.ldw > ldw || sh.nblk > L.nblk) return GJ_E_WORKSPACE;
        BigDesc d = make_desc(sh, L.bb, w, A, lda, X, ldx, ipiv, jpiv, res);
        d.W = at(Wb[cur], k0, k0);
        d.ldw = ldw;
        d.mstride = ldw;
        d.steps = steps + k0;
        d.k0 = k0;
        d.inplace = k0 > 0;
        // nbp steps on the trailing block, no finish
        e = launch_big(fp32, nt, big_nt_loads(big_swept_bytes(sh, fp32)), big_full_chunks(sh, fp32),
                       big_counted(sh), false, 0, nullptr, nullptr, d, nullptr, sh.nblk, 0, nbp, 0,
                       zero_tol, eps_default, 0, nullptr, nullptr, s);
        if (e != hipSuccess) return hip_fail(e);
        e = launch_blk_panel_end(fp32, hdr, d.rowlog + (size_t)(nbp & 1) * ldw,
                                 d.collog + (size_t)(nbp & 1) * ldw, m, d.rowphys, d.colphys,
                                 steps + k0, nbp, k0, Wb[cur], Wb[cur ^ 1], ldw, n, tA, L.nb, tB,
                                 n, prow[cur], pcol[cur], prow[cur ^ 1], pcol[cur ^ 1], s);
        if (e != hipSuccess) return hip_fail(e);
        cur ^= 1;
        if (k0 == 0) continue;
        // the panel's steps on the other rows and columns (b: the panel's
        // pivots, 1: the k0 earlier ones, 3: the rest)
        char *Wc = Wb[cur];
        // W_b1 = T W_b1(old)
        e = blk_gemm(fp32, nbp, k0, nbp, 1.0, at(Wc, k0, k0), ldw, tB, n, 0.0, nullptr, 0,
                     at(Wc, k0, 0), ldw, s);
        if (e != hipSuccess) return hip_fail(e);
        // W_31 += W_3b W_b1(old), W_3b = -W_3b(old) T from the panel
        if (m > nbp) {
            e = blk_gemm(fp32, m - nbp, k0, nbp, 1.0, at(Wc, k0 + nbp, k0), ldw, tB, n, 1.0,
                         at(Wc, k0 + nbp, 0), ldw, at(Wc, k0 + nbp, 0), ldw, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        // W_1* -= W_1b(old) W_b* (W_1b zeroed by the copy: it becomes -W_1b(old) T)
        e = blk_gemm(fp32, k0, n, nbp, -1.0, tA, L.nb, at(Wc, k0, 0), ldw, 1.0, Wc, ldw, Wc, ldw, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = launch_blk_finish(fp32, hdr, steps, n, ipiv, jpiv, res, prow[cur], pcol[cur], rowinv, colinv,
                          Wb[cur], ldw, X, ldx, s);
    if (e != hipSuccess) return hip_fail(e);
    if (rows) *rows = prow[cur];
    if (cols) *cols = pcol[cur];
    return GJ_OK;
}

bool use_blocked(int n, const Opts &o, bool det_only) {
    return (o.flags & GJ_FLAG_BLOCKED) && !det_only && n > kOnchipMax;
}

size_t single_ws(int n, const Opts &o, bool det_only) {
    if (o.precision == GJ_PREC_FP32_REFINED)
        return refined_ws(n, (o.flags & GJ_FLAG_ACCURATE) && !det_only, use_blocked(n, o, det_only));
    size_t need = 256;
    if (use_blocked(n, o, det_only)) {
        need = blk_layout(n).end;
    } else if (n > kOnchipMax || o.rule != 0) {
        BigShape s = single_shape(n, false, big_threads(n, false));
        need = big_bufs(s, false, 0).end;
    }
    if (o.want_resid && !det_only) need = a256(need) + resid_ws(n);
    return need;
}

// A X = B through the streaming elimination on [A | B] (every order; the
// on-chip kernels hold no right-hand sides).  When A alone fills all 8
// register chunks of its own row shape and B fits one more chunk, B becomes
// that extra partial chunk and the inversion's row shape is kept (rhs);
// otherwise [A | B] is shaped as one wider array, B right after A.
BigShape big_shape_solve(int n, int m, int rule, bool &rhs) {
    const int nt = big_threads(n, false);
    BigShape s = single_shape(n, false, nt, 0, false);
    rhs = rule == 0 && big_full(s, false) && nt < 1024 && m <= s.tpr * 2;
    if (rhs) {
        s.rhs0 = 8 * s.tpr * 2;
        s.ncol = s.rhs0 + m;
        s.ldw = s.rhs0 + (m + 15) / 16 * 16;   // rows stay 128-byte aligned
        s.ustat = s.share;                     // the extra chunk is built without the counter
        return s;
    }
    return single_shape(n, false, big_threads(n + m, false), n + m, false);
}

size_t solve_ws(int n, int m, int rule) {
    bool rhs;
    return big_bufs(big_shape_solve(n, m, rule, rhs), false, 0).end;
}

gj_status run_solve(int n, int m, const double *A, int64_t lda, const double *B, int64_t ldb,
                    double *X, int64_t ldx, int32_t *ipiv, int32_t *jpiv, gj_result *res,
                    const Opts &o, void *ws, size_t ws_bytes, hipStream_t s) {
    bool rhs;
    BigShape sh = big_shape_solve(n, m, o.rule, rhs);
    if (o.rule != 0) sh.ustat = sh.share;   // the other rules are built without the counter
    BigBufs bb = big_bufs(sh, false, 0);
    if (ws_bytes < bb.end) return GJ_E_WORKSPACE;
    BigDesc d = make_desc(sh, bb, (char *)ws, A, lda, X, ldx, ipiv, jpiv, res);
    d.B = B;
    d.ldb = ldb;
    d.rule = o.rule;
    const int full = (o.rule == 0 && (rhs || big_full(sh, false))) ? 8 : 0;
    hipError_t e = launch_big(false, sh.nt, big_nt_loads(big_swept_bytes(sh, false)),
                              full, o.rule == 0 && !rhs && big_counted(sh), rhs, o.rule, nullptr,
                              nullptr, d, nullptr, sh.nblk, sh.nblk, n, sh.nblk, o.zero_tol,
                              kEps64, 0, o.events, nullptr, s);
    if (e != hipSuccess) return hip_fail(e);
    return GJ_OK;
}

gj_status run_single(int n, const double *A, int64_t lda, double *X, int64_t ldx, int32_t *ipiv,
                     int32_t *jpiv, gj_result *res, const Opts &o, void *ws, size_t ws_bytes,
                     hipStream_t s, bool det_only) {
    const bool fp32 = (o.precision == GJ_PREC_FP32_REFINED);
    const double eps_default = fp32 ? 0.0 : kEps64;
    if (n <= kOnchipMax && o.rule == 0) {
        MatDesc md;
        md.a_off = 0;
        md.x_off = 0;
        md.piv_off = 0;
        md.n = n;
        md.lda = (int32_t)lda;
        md.ldx = (int32_t)(det_only ? n : ldx);
        md.res_idx = 0;
        md.run = nullptr;
        if (o.events && o.events[0]) {
            hipError_t e = hipEventRecord((hipEvent_t)o.events[0], s);
            if (e != hipSuccess) return hip_fail(e);
        }
        hipError_t e = launch_onchip(fp32, nullptr, nullptr, 0, nullptr, md, 1, A, X, ipiv, jpiv,
                                     res, o.zero_tol, eps_default, det_only ? 1 : 0, nullptr, s);
        if (e != hipSuccess) return hip_fail(e);
        if (o.events && o.events[1]) {
            e = hipEventRecord((hipEvent_t)o.events[1], s);
            if (e != hipSuccess) return hip_fail(e);
        }
        return GJ_OK;
    }
    const int nt = big_threads(n, fp32);
    BigShape sh = single_shape(n, fp32, nt);
    if (o.rule != 0) sh.ustat = sh.share;   // the other rules are built without the counter
    BigBufs bb = big_bufs(sh, fp32, 0);
    if (ws_bytes < bb.end) return GJ_E_WORKSPACE;
    BigDesc d = make_desc(sh, bb, (char *)ws, A, lda, X, ldx, ipiv, jpiv, res);
    d.rule = o.rule;
    hipError_t e = launch_big(fp32, nt, big_nt_loads(big_swept_bytes(sh, fp32)),
                              o.rule == 0 ? big_full_chunks(sh, fp32) : 0, o.rule == 0 && big_counted(sh),
                              false, o.rule, nullptr, nullptr,
                              d, nullptr, sh.nblk, sh.nblk, n,
                              det_only ? 0 : sh.nblk, o.zero_tol, eps_default, det_only ? 1 : 0,
                              o.events, nullptr, s);
    if (e != hipSuccess) return hip_fail(e);
    return GJ_OK;
}


// ------------------------------------------------------------ refined path
constexpr int kDetBlock = 128;          // diagonal blocks of the FP64 determinant
constexpr double kAcceptResid = 1e-2;   // ||I - A X||_F above this: fall back to FP64
constexpr double kStall = 0.5;          // rounding floor: a kept update that neither halves
                                         // ||R||_F nor comes within 2 ||R||_F^2 ends the loop
// accurate-residual phase: slices of 19 bits keep every partial sum of the
// exact products below 2^53 units for n <= 16384; at most 2 updates (from an
// accepted FP64 iterate with residual R_0 they leave an error of about
// ||R_0||^4 + u; a third residual only confirmed the floor in every case
// measured, at 8 products of n^3)
constexpr int kAccBeta = 19;
constexpr int kAccIters = 2;

struct RefinedLayout {
    size_t ctl, big32, xw, r, over64, t, dinv, part_r, part_a, part_x, blockres, rows, cols, bpiv, acc, end;
    int nparts;
};

RefinedLayout refined_layout(int n, bool acc = false, bool blocked = false) {
    RefinedLayout L;
    size_t c = 0;
    const size_t n2 = (size_t)n * n * 8;
    L.ctl = c; c = a256(c + refine_ctl_bytes());
    L.big32 = c;
    if (n > kOnchipMax && blocked) {
        c = blk_layout(n, true, c).end;             // FP32 elimination with delayed updates
    } else if (n > kOnchipMax) {
        BigShape s = single_shape(n, true, big_threads(n, true));
        c = big_bufs(s, true, c).end;
    }
    // the FP64 fallback's buffers overlay the second iterate and R: it runs
    // only when neither is needed any more
    L.xw = c;
    L.over64 = c;
    size_t over = 2 * n2;
    if (n > kOnchipMax) {
        BigShape s = single_shape(n, false, big_threads(n, false));
        over = std::max(over, big_bufs(s, false, 0).end);
    }
    L.r = a256(c + n2);
    c = a256(c + std::max(over, a256(n2) + n2));
    L.t = c; c = a256(c + (size_t)kDetBlock * n * 8);
    L.dinv = c; c = a256(c + (size_t)kDetBlock * kDetBlock * 8);
    L.nparts = std::max(gemm_tiles(n, n), sumsq_blocks(n));
    L.part_r = c; c = a256(c + (size_t)L.nparts * 8);
    L.part_a = c; c = a256(c + (size_t)L.nparts * 8);
    L.part_x = c; c = a256(c + (size_t)L.nparts * 8);
    L.blockres = c; c = a256(c + (size_t)((n + kDetBlock - 1) / kDetBlock) * sizeof(gj_result));
    L.rows = c; c = a256(c + (size_t)n * 4);
    L.cols = c; c = a256(c + (size_t)n * 4);
    L.bpiv = c; c = a256(c + 2 * kDetBlock * 4);
    // accurate-residual phase: three slices of A and three of X
    L.acc = c;
    if (acc) c = a256(c + 6 * n2);
    L.end = c;
    return L;
}

#define GJ_TRY(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) return hip_fail(e_); } while (0)

// A second stream per device, for work that can overlap the caller's stream:
// * the refined path's FP64 fallback beside its determinant stage: the two
//   exclude each other (both flags are set before either runs, and each
//   touches the buffers they share only when its flag is set); when the
//   fallback is not needed its n step launches return at once (about 1.8 us
//   each), time the determinant stage hides (outside graph capture only);
// * a batch's one-matrix-per-wavefront on-chip classes beside the others and
//   the streaming members (disjoint members, their own queue counters), so
//   that their persistent launches fill the other classes' tails (also under
//   capture, once the stream exists).
// gj_invert_noalloc (which creates nothing) keeps everything in order on the
// caller's stream.
thread_local bool g_no_side = false;

// One side stream per device with its fork and join events, created once
// outside graph capture.  A fork holds the device's lock until it has joined
// back, so that concurrent callers do not interleave on the shared events.
struct SideRes {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool failed = false;
    std::mutex mu;
};
SideRes g_side_res[64];

// The fork of the caller's stream s onto the side stream (fs) and the join
// back; fs == s when there is none (gj_invert_noalloc, another device's
// stream, capture without allow_capture or before the side stream exists).
struct SideFork {
    hipStream_t s, fs;
    SideRes *r = nullptr;
    std::unique_lock<std::mutex> lock;
    SideFork(hipStream_t s_, bool allow_capture) : s(s_), fs(s_) {
        if (g_no_side) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess) return;
        const bool capturing = cs != hipStreamCaptureStatusNone;
        if (capturing && !allow_capture) return;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
        if (s) {
            hipDevice_t sd = 0;
            if (hipStreamGetDevice(s, &sd) != hipSuccess || (int)sd != dev) return;
        }
        SideRes *x = &g_side_res[dev];
        std::unique_lock<std::mutex> l(x->mu);
        if (!x->s) {
            if (capturing || x->failed) return;
            hipStream_t st = nullptr;
            hipEvent_t f = nullptr, j = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
                x->failed = true;
                return;
            }
            x->s = st; x->fork = f; x->join = j;
        }
        if (hipEventRecord(x->fork, s) != hipSuccess || hipStreamWaitEvent(x->s, x->fork, 0) != hipSuccess)
            return;
        r = x;
        lock = std::move(l);
        fs = x->s;
    }
    hipError_t join_back() {
        if (fs == s) return hipSuccess;
        hipError_t e = hipEventRecord(r->join, fs);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, r->join, 0);
        fs = s;
        lock.unlock();
        return e;
    }
    ~SideFork() { (void)join_back(); }   // an early error return still joins
};

// Eliminate in FP32 (the pivots and X0), refine X in FP64, FP64 determinant.
gj_status run_refined_single(int n, const double *A, int64_t lda, double *X, int64_t ldx,
                             int32_t *ipiv, int32_t *jpiv, gj_result *res, const Opts &o, char *w,
                             hipStream_t s, bool det_only) {
    const bool acc = (o.flags & GJ_FLAG_ACCURATE) && !det_only;
    const bool blk = use_blocked(n, o, det_only);
    const RefinedLayout L = refined_layout(n, acc, blk);
    void *ctl = w + L.ctl;
    double *Xw = reinterpret_cast<double *>(w + L.xw);
    double *R = reinterpret_cast<double *>(w + L.r);
    double *T = reinterpret_cast<double *>(w + L.t);
    double *Dinv = reinterpret_cast<double *>(w + L.dinv);
    double *pr = reinterpret_cast<double *>(w + L.part_r);
    double *pa = reinterpret_cast<double *>(w + L.part_a);
    double *px = reinterpret_cast<double *>(w + L.part_x);
    gj_result *blockres = reinterpret_cast<gj_result *>(w + L.blockres);
    int32_t *rows = reinterpret_cast<int32_t *>(w + L.rows);
    int32_t *cols = reinterpret_cast<int32_t *>(w + L.cols);
    int32_t *bpiv = reinterpret_cast<int32_t *>(w + L.bpiv);
    const int nparts = gemm_tiles(n, n);
    const int row_blocks = std::min(n, 1024);

    // 1. FP32 elimination (zero threshold 0): X0 in X, pivots, FP32 status
    BigDesc d32;
    std::memset(&d32, 0, sizeof(d32));
    const int32_t *blk_rows = nullptr, *blk_cols = nullptr;
    if (blk) {
        // with delayed updates (FP32 products); the pivots are the unblocked
        // FP32 elimination's, and the pivot-order maps come out of it
        if (o.events && o.events[0]) GJ_TRY(hipEventRecord((hipEvent_t)o.events[0], s));
        const gj_status bs = run_blocked(true, n, A, lda, X, ldx, ipiv, jpiv, res, 0.0, 0.0, w, L.end,
                                         L.big32, s, &blk_rows, &blk_cols);
        if (bs != GJ_OK) return bs;
        if (o.events && o.events[1]) GJ_TRY(hipEventRecord((hipEvent_t)o.events[1], s));
    } else if (n <= kOnchipMax) {
        MatDesc md{0, 0, 0, n, (int32_t)lda, (int32_t)(det_only ? n : ldx), 0, nullptr};
        if (o.events && o.events[0]) GJ_TRY(hipEventRecord((hipEvent_t)o.events[0], s));
        GJ_TRY(launch_onchip(true, nullptr, nullptr, 0, nullptr, md, 1, A, det_only ? nullptr : X,
                             ipiv, jpiv, res, 0.0, 0.0, det_only ? 1 : 0, nullptr, s));
        if (o.events && o.events[1]) GJ_TRY(hipEventRecord((hipEvent_t)o.events[1], s));
    } else {
        const int nt = big_threads(n, true);
        BigShape sh = single_shape(n, true, nt);
        BigBufs bb = big_bufs(sh, true, L.big32);
        d32 = make_desc(sh, bb, w, A, lda, det_only ? nullptr : X, ldx, ipiv, jpiv, res);
        GJ_TRY(launch_big(true, nt, big_nt_loads(big_swept_bytes(sh, true)), big_full_chunks(sh, true), big_counted(sh), false, 0,
                          nullptr, nullptr, d32,
                          nullptr, sh.nblk, sh.nblk, n,
                          det_only ? 0 : sh.nblk, 0.0, 0.0, det_only ? 1 : 0, o.events, nullptr, s));
    }
    GJ_TRY(launch_refine_bind(ctl, res, pr, nparts, s));
    GJ_TRY(launch_refine_start(ctl, 1, s));

    RefMember m;
    std::memset(&m, 0, sizeof(m));
    m.A = A; m.lda = lda; m.X = X; m.ldx = ldx; m.Xw = Xw; m.B = R;
    m.ipiv = ipiv; m.jpiv = jpiv;
    if (blk) {
        m.rows = blk_rows; m.cols = blk_cols;
    } else if (n <= kOnchipMax) {
        m.rows = rows; m.cols = cols; m.rows_buf = rows; m.cols_buf = cols;
    } else {
        m.rows = d32.rowphys; m.cols = d32.colphys;
    }
    m.blockres = blockres;
    m.n = n;
    m.nblocks = (n + kDetBlock - 1) / kDetBlock;

    // 2. Newton-Schulz: R = I - A X; X' = X + X R; keep while ||R||_F drops
    if (!det_only) {
        GemmArgs g;
        std::memset(&g, 0, sizeof(g));
        g.M = g.N = g.K = n;
        g.A = A; g.lda = lda; g.B = X; g.ldb = ldx; g.D = R; g.ldd = n;
        g.alpha = -1.0; g.beta = 0.0; g.gamma = 1.0;
        g.norm_partials = pr; g.run_flag = ctl_run_ns(ctl);
        GJ_TRY(launch_gemm_f64(g, s));
        GJ_TRY(launch_refine_resid0(ctl, 1, s));
        for (int it = 1; it <= o.max_refine_iters; ++it) {
            double *Xs = ((it - 1) & 1) ? Xw : X;
            double *Xd = (it & 1) ? Xw : X;
            const int64_t lds = ((it - 1) & 1) ? n : ldx, ldd = (it & 1) ? n : ldx;
            GemmArgs u;
            std::memset(&u, 0, sizeof(u));
            u.M = u.N = u.K = n;
            u.A = Xs; u.lda = lds; u.B = R; u.ldb = n; u.C = Xs; u.ldc = lds; u.D = Xd; u.ldd = ldd;
            u.alpha = 1.0; u.beta = 1.0; u.gamma = 0.0;
            u.run_flag = ctl_run_ns(ctl);
            GJ_TRY(launch_gemm_f64(u, s));
            GemmArgs r2 = g;
            r2.B = Xd; r2.ldb = ldd;
            GJ_TRY(launch_gemm_f64(r2, s));
            GJ_TRY(launch_refine_after_update(ctl, 1, it, o.max_refine_iters, kStall, s));
        }
        GJ_TRY(launch_refine_finish(ctl, 1, kAcceptResid, 1, s));
        GJ_TRY(launch_copy_back(nullptr, m, ctl, 1, row_blocks, s));
        if (acc) {
            // accurate residuals (error-free split products on the matrix
            // cores) for a few more updates; skipped when the FP64 result
            // falls back.  Buffers: R for the residual, Xw for the update.
            const size_t nn = (size_t)n * n;
            double *As = reinterpret_cast<double *>(w + L.acc), *Xs = As + 3 * nn;
            GJ_TRY(launch_acc_prepare(ctl, 1, s));
            const int32_t *ra = ctl_run_acc(ctl);
            GJ_TRY(launch_slice_rows(A, lda, n, As, kAccBeta, ra, s));
            // R = I - sum of A_s X_t over every slice pair but A3 X3
            static const int terms[8][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}, {0, 2}, {2, 0}, {1, 2}, {2, 1}};
            for (int j = 0; j < kAccIters; ++j) {
                GJ_TRY(launch_slice_global(X, ldx, n, ctl, Xs, kAccBeta, s));
                for (int q = 0; q < 8; ++q) {
                    GemmArgs a;
                    std::memset(&a, 0, sizeof(a));
                    a.M = a.N = a.K = n;
                    a.A = As + terms[q][0] * nn; a.lda = n;
                    a.B = Xs + terms[q][1] * nn; a.ldb = n;
                    a.D = R; a.ldd = n;
                    a.alpha = -1.0;
                    if (q == 0) {
                        a.gamma = 1.0;
                    } else {
                        a.C = R; a.ldc = n; a.beta = 1.0;
                    }
                    if (q == 7) a.norm_partials = pr;
                    a.run_flag = ra;
                    GJ_TRY(launch_gemm_f64(a, s));
                }
                GJ_TRY(launch_acc_check(ctl, j, s));
                GemmArgs u;
                std::memset(&u, 0, sizeof(u));
                u.M = u.N = u.K = n;
                u.A = X; u.lda = ldx; u.B = R; u.ldb = n; u.C = X; u.ldc = ldx; u.D = Xw; u.ldd = n;
                u.alpha = 1.0; u.beta = 1.0;
                u.run_flag = ra;
                GJ_TRY(launch_gemm_f64(u, s));
                GJ_TRY(launch_acc_copy(Xw, n, X, ldx, ctl, s));
            }
            GJ_TRY(launch_acc_finish(ctl, s));
        }
    } else {
        GJ_TRY(launch_refine_finish(ctl, 1, __builtin_inf(), 1, s));
    }

    // 3. fallback: the plain FP64 elimination, only when flagged (on the side
    // stream where there is one, beside the determinant stage)
    SideFork fork(s, false);
    if (n <= kOnchipMax) {
        MatDesc md{0, 0, 0, n, (int32_t)lda, (int32_t)(det_only ? n : ldx), 0, nullptr};
        GJ_TRY(launch_onchip(false, nullptr, nullptr, 0, nullptr, md, 1, A, det_only ? nullptr : X,
                             ipiv, jpiv, res, o.zero_tol, kEps64, det_only ? 1 : 0,
                             ctl_run_fallback(ctl), fork.fs));
    } else {
        const int nt = big_threads(n, false);
        BigShape sh = single_shape(n, false, nt);
        BigBufs bb = big_bufs(sh, false, L.over64);
        BigDesc d = make_desc(sh, bb, w, A, lda, det_only ? nullptr : X, ldx, ipiv, jpiv, res);
        GJ_TRY(launch_big(false, nt, big_nt_loads(big_swept_bytes(sh, false)), big_full_chunks(sh, false), big_counted(sh), false, 0,
                          nullptr, nullptr, d,
                          nullptr, sh.nblk, sh.nblk, n,
                          det_only ? 0 : sh.nblk, o.zero_tol, kEps64, det_only ? 1 : 0, nullptr,
                          ctl_run_fallback(ctl), fork.fs));
    }
    GJ_TRY(launch_fallback_mark(ctl, 1, fork.fs));

    // 4. FP64 determinant: permute A with the FP32 order, block elimination
    const int32_t *fdet = ctl_run_det(ctl);
    GJ_TRY(launch_perms_from_pivots(nullptr, m, ctl, 1, s));
    GJ_TRY(launch_gather_perm(nullptr, m, ctl, 1, row_blocks, s));
    double *B = R;
    for (int kb = 0, bi = 0; kb < n; kb += kDetBlock, ++bi) {
        const int nbk = std::min(kDetBlock, n - kb);
        MatDesc md{(int64_t)kb * n + kb, 0, 0, nbk, n, kDetBlock, 0, nullptr};
        // the block in the FP32 pivot order: static pivots (an exact zero only
        // counts as singular, as in an LU in that order)
        GJ_TRY(launch_onchip(false, nullptr, nullptr, 0, nullptr, md, 1, B, Dinv, bpiv,
                             bpiv + kDetBlock, blockres + bi, 0.0, kEps64, kOnchipStaticPivots,
                             fdet, s));
        const int mm = n - kb - nbk;
        if (mm > 0) {
            GemmArgs g1;
            std::memset(&g1, 0, sizeof(g1));
            g1.M = nbk; g1.N = mm; g1.K = nbk;
            g1.A = Dinv; g1.lda = kDetBlock;
            g1.B = B + (int64_t)kb * n + kb + nbk; g1.ldb = n;
            g1.D = T; g1.ldd = n;
            g1.alpha = 1.0; g1.run_flag = fdet;
            GJ_TRY(launch_gemm_f64(g1, s));
            // one refinement step of the block solve T = D^-1 S12 (S12 is not
            // needed afterwards and takes the residual): with the explicit
            // inverse alone the Schur complement, and so log|det|, carries an
            // error of order cond(D) u; the corrected T makes it as accurate
            // as an LU in the same order
            GemmArgs gr;
            std::memset(&gr, 0, sizeof(gr));
            gr.M = nbk; gr.N = mm; gr.K = nbk;
            gr.A = B + (int64_t)kb * n + kb; gr.lda = n;
            gr.B = T; gr.ldb = n;
            gr.C = B + (int64_t)kb * n + kb + nbk; gr.ldc = n;
            gr.D = const_cast<double *>(gr.C); gr.ldd = n;
            gr.alpha = -1.0; gr.beta = 1.0; gr.run_flag = fdet;
            GJ_TRY(launch_gemm_f64(gr, s));
            GemmArgs gc;
            std::memset(&gc, 0, sizeof(gc));
            gc.M = nbk; gc.N = mm; gc.K = nbk;
            gc.A = Dinv; gc.lda = kDetBlock;
            gc.B = gr.C; gc.ldb = n;
            gc.C = T; gc.ldc = n;
            gc.D = T; gc.ldd = n;
            gc.alpha = 1.0; gc.beta = 1.0; gc.run_flag = fdet;
            GJ_TRY(launch_gemm_f64(gc, s));
            GemmArgs g2;
            std::memset(&g2, 0, sizeof(g2));
            g2.M = mm; g2.N = mm; g2.K = nbk;
            g2.A = B + (int64_t)(kb + nbk) * n + kb; g2.lda = n;
            g2.B = T; g2.ldb = n;
            g2.C = B + (int64_t)(kb + nbk) * n + kb + nbk; g2.ldc = n;
            g2.D = const_cast<double *>(g2.C); g2.ldd = n;
            g2.alpha = -1.0; g2.beta = 1.0; g2.run_flag = fdet;
            GJ_TRY(launch_gemm_f64(g2, s));
        }
    }
    GJ_TRY(launch_det_combine(nullptr, m, ctl, 1, s));
    GJ_TRY(launch_refine_iters(ctl, 1, s));
    GJ_TRY(fork.join_back());

    // 5. optional residual of the returned inverse
    if (o.want_resid && !det_only) {
        GemmArgs g;
        std::memset(&g, 0, sizeof(g));
        g.M = g.N = g.K = n;
        g.A = A; g.lda = lda; g.B = X; g.ldb = ldx; g.D = R; g.ldd = n;
        g.alpha = -1.0; g.gamma = 1.0; g.norm_partials = pr;
        GJ_TRY(launch_gemm_f64(g, s));
        GJ_TRY(launch_sumsq(A, lda, n, pa, s));
        GJ_TRY(launch_sumsq(X, ldx, n, px, s));
        GJ_TRY(launch_resid(pr, nparts, pa, sumsq_blocks(n), px, sumsq_blocks(n), res, s));
    }
    return GJ_OK;
}

// ------------------------------------------------------ batched refined
// One grouped-GEMM problem list and its workgroup -> (problem, tile) map.
struct GemmList {
    std::vector<GemmArgs> probs;
    std::vector<int2> tiles;
    size_t off_probs = 0, off_tiles = 0;
    void add(const GemmArgs &g) {
        const int p = (int)probs.size();
        probs.push_back(g);
        const int nt = gemm_tiles(g.M, g.N);
        for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(p, t));
    }
};

// An on-chip task set (classes as in plan_batch) over a descriptor array.
struct OnchipSet {
    std::vector<MatDesc> mats;
    std::vector<OnchipTask> tasks;
    int cls_start[kOnchipClasses] = {0}, cls_count[kOnchipClasses] = {0};
    size_t off_mats = 0, off_tasks = 0;
    void build() {   // tasks over all mats, grouped by class, largest first
        std::vector<int> by_cls[kOnchipClasses];
        for (int i = 0; i < (int)mats.size(); ++i) by_cls[onchip_class_of(mats[i].n, false)].push_back(i);
        tasks.clear();
        for (int c = 0; c < kOnchipClasses; ++c) {
            auto &v = by_cls[c];
            std::sort(v.begin(), v.end(), [&](int x, int y) {
                return mats[x].n != mats[y].n ? mats[x].n > mats[y].n : x < y; });
            cls_start[c] = (int)tasks.size();
            if (onchip_class_kind(c) == 0) {
                for (int i : v) tasks.push_back(OnchipTask{0, {i, -1, -1, -1}});
            } else {
                for (size_t x = 0; x < v.size(); x += 4) {
                    OnchipTask t{1, {-1, -1, -1, -1}};
                    for (int q = 0; q < 4 && x + q < v.size(); ++q) t.m[q] = v[x + q];
                    tasks.push_back(t);
                }
            }
            cls_count[c] = (int)tasks.size() - cls_start[c];
        }
    }
};

struct RefBatchPlan {
    BatchPlan e32;                       // FP32 elimination (starts at offset 0)
    std::vector<size_t> region, xw, r, t, dinv, parts, rows, cols, bpiv;
    std::vector<int> nblocks, blockres_start;
    size_t off_ctl = 0, off_mem = 0, off_blockres = 0;
    // FP64 fallback
    OnchipSet fb;                        // on-chip members (run flag: run_fallback)
    std::vector<BigShape> fb_shapes;
    std::vector<BigBufs> fb_bufs;
    std::vector<int2> fb_bmap;
    std::vector<int> fb_grid;
    int fb_nt = 256;
    size_t fb_swept = 0;
    bool fb_full = true;
    bool fb_counted = false;
    size_t off_fb_descs = 0, off_fb_bmap = 0;
    // Newton-Schulz product lists
    GemmList r0, upd[2], res[2];
    // determinant block steps
    std::vector<OnchipSet> det_blocks;
    std::vector<GemmList> det_t, det_r, det_c, det_s;   // T, residual, correction, Schur update
    size_t total = 0;
};

// Byte layout only (pointers are formed at call time from the workspace base).
bool plan_refined_batch(int batch, const int32_t *n_host, RefBatchPlan &P) {
    if (!plan_batch(batch, n_host, true, P.e32)) return false;
    size_t c = a256(P.e32.total);
    P.region.resize(batch); P.xw.resize(batch); P.r.resize(batch); P.t.resize(batch);
    P.dinv.resize(batch); P.parts.resize(batch); P.rows.resize(batch); P.cols.resize(batch);
    P.bpiv.resize(batch); P.nblocks.resize(batch); P.blockres_start.resize(batch);
    int nbtot = 0;
    for (int b = 0; b < batch; ++b) {
        const int n = n_host[b];
        const size_t n2 = a256((size_t)n * n * 8);
        size_t reg = 2 * n2;
        if (n > kOnchipMax) {
            BigShape s = big_shape(n, false, big_threads(P.e32.big_max_n, false));
            reg = std::max(reg, big_bufs(s, false, 0).end);
        }
        P.region[b] = c;
        P.xw[b] = c;
        P.r[b] = c + n2;
        c = a256(c + reg);
        const int nb = std::min(n, kDetBlock);
        P.t[b] = c; c = a256(c + (n > kDetBlock ? (size_t)kDetBlock * n * 8 : 0));
        P.dinv[b] = c; c = a256(c + (size_t)nb * nb * 8);
        P.parts[b] = c; c = a256(c + (size_t)gemm_tiles(n, n) * 8);
        P.rows[b] = c; c = a256(c + (size_t)n * 4);
        P.cols[b] = c; c = a256(c + (size_t)n * 4);
        P.bpiv[b] = c; c = a256(c + 2 * kDetBlock * 4);
        P.nblocks[b] = (n + kDetBlock - 1) / kDetBlock;
        P.blockres_start[b] = nbtot;
        nbtot += P.nblocks[b];
    }
    P.off_blockres = c; c = a256(c + (size_t)nbtot * sizeof(gj_result));
    P.off_ctl = c; c = a256(c + (size_t)batch * refine_ctl_bytes());
    P.off_mem = c; c = a256(c + (size_t)batch * refine_member_bytes());
    // FP64 fallback tables
    P.fb.mats.resize(batch);
    P.fb.off_mats = c; c = a256(c + sizeof(MatDesc) * batch);
    P.fb.off_tasks = c; c = a256(c + sizeof(OnchipTask) * std::max<size_t>(1, P.e32.tasks.size()));
    if (!P.e32.big_members.empty()) {
        P.fb_nt = big_threads(P.e32.big_max_n, false);
        P.off_fb_descs = c; c = a256(c + sizeof(BigDesc) * P.e32.big_members.size());
        size_t nb = 0;
        for (int m : P.e32.big_members) {
            BigShape s = big_shape(n_host[m], false, P.fb_nt);
            P.fb_shapes.push_back(s);
            P.fb_swept += big_swept_bytes(s, false);
            P.fb_full = P.fb_full && big_full(s, false);
            P.fb_bufs.push_back(big_bufs(s, false, P.region[m]));
            nb += s.nblk;
        }
        for (BigShape &s : P.fb_shapes) {
            if (!P.fb_full) s.ustat = s.share;
            P.fb_counted = P.fb_counted || big_counted(s);
        }
        P.off_fb_bmap = c; c = a256(c + sizeof(int2) * nb);
        for (size_t x = 0; x < P.e32.big_members.size(); ++x)
            for (int rb = 0; rb < P.fb_shapes[x].nblk; ++rb) P.fb_bmap.push_back(make_int2((int)x, rb));
        P.fb_grid.assign(P.e32.big_max_n, 0);
        for (int k = 0; k < P.e32.big_max_n; ++k)
            for (size_t x = 0; x < P.e32.big_members.size(); ++x)
                if (P.fb_shapes[x].n > k) P.fb_grid[k] += P.fb_shapes[x].nblk;
    }
    // product lists (shapes only here; pointers filled at call time)
    int maxn = 0;
    for (int b = 0; b < batch; ++b) maxn = std::max(maxn, (int)n_host[b]);
    const int nsteps = (maxn + kDetBlock - 1) / kDetBlock;
    P.det_blocks.resize(nsteps);
    P.det_t.resize(nsteps);
    P.det_r.resize(nsteps);
    P.det_c.resize(nsteps);
    P.det_s.resize(nsteps);
    auto list_bytes = [&](GemmList &L, int count_probs, int count_tiles) {
        L.off_probs = c; c = a256(c + sizeof(GemmArgs) * std::max(1, count_probs));
        L.off_tiles = c; c = a256(c + sizeof(int2) * std::max(1, count_tiles));
    };
    int tiles_all = 0;
    for (int b = 0; b < batch; ++b) tiles_all += gemm_tiles(n_host[b], n_host[b]);
    list_bytes(P.r0, batch, tiles_all);
    for (int p = 0; p < 2; ++p) {
        list_bytes(P.upd[p], batch, tiles_all);
        list_bytes(P.res[p], batch, tiles_all);
    }
    for (int s = 0; s < nsteps; ++s) {
        int nprob = 0, tt = 0, ts = 0, nmat = 0;
        for (int b = 0; b < batch; ++b) {
            const int n = n_host[b], kb = s * kDetBlock;
            if (n <= kb) continue;
            ++nmat;
            const int nbk = std::min(kDetBlock, n - kb), mm = n - kb - nbk;
            if (mm > 0) { ++nprob; tt += gemm_tiles(nbk, mm); ts += gemm_tiles(mm, mm); }
        }
        P.det_blocks[s].off_mats = c; c = a256(c + sizeof(MatDesc) * std::max(1, nmat));
        P.det_blocks[s].off_tasks = c; c = a256(c + sizeof(OnchipTask) * std::max(1, nmat));
        list_bytes(P.det_t[s], nprob, tt);
        list_bytes(P.det_r[s], nprob, tt);
        list_bytes(P.det_c[s], nprob, tt);
        list_bytes(P.det_s[s], nprob, ts);
    }
    P.total = c;
    return true;
}

gj_status run_refined_batched(int batch, const int32_t *n_host, const int64_t *off_host,
                              const double *A, double *X, const int64_t *piv_off_host,
                              int32_t *ipiv, int32_t *jpiv, gj_result *res, const Opts &o,
                              char *w, size_t ws_bytes, hipStream_t s) {
    RefBatchPlan P;
    if (!plan_refined_batch(batch, n_host, P)) return GJ_E_INVALID_ARG;
    if (ws_bytes < P.total) return GJ_E_WORKSPACE;
    BatchPlan &E = P.e32;
    double *wd = reinterpret_cast<double *>(w);
    char *ctl = w + P.off_ctl;
    gj_result *blockres = reinterpret_cast<gj_result *>(w + P.off_blockres);
    const size_t cb = refine_ctl_bytes();

    // ---- host copies of every device table
    E.mats.resize(batch);
    for (int b = 0; b < batch; ++b)
        E.mats[b] = MatDesc{off_host[b], off_host[b], piv_off_host[b], n_host[b], n_host[b], n_host[b], b, nullptr};
    std::vector<BigDesc> d32, d64;
    for (size_t x = 0; x < E.big_members.size(); ++x) {
        const int m = E.big_members[x];
        d32.push_back(make_desc(E.big_shapes[x], E.big_bufs[x], w, A + off_host[m], n_host[m],
                                X + off_host[m], n_host[m], ipiv + piv_off_host[m],
                                jpiv + piv_off_host[m], res + m));
        BigDesc d = make_desc(P.fb_shapes[x], P.fb_bufs[x], w, A + off_host[m], n_host[m],
                              X + off_host[m], n_host[m], ipiv + piv_off_host[m],
                              jpiv + piv_off_host[m], res + m);
        d.run = ctl_run_fallback(ctl + (size_t)m * cb);
        d64.push_back(d);
    }
    std::vector<int> big_index(batch, -1);
    for (size_t x = 0; x < E.big_members.size(); ++x) big_index[E.big_members[x]] = (int)x;
    // control records (pointers only; the state is reset on the device)
    std::vector<char> ctl_host((size_t)batch * cb, 0);
    std::vector<RefMember> mem(batch);
    for (int b = 0; b < batch; ++b) {
        const int n = n_host[b];
        RefineCtl h;
        std::memset(&h, 0, sizeof(h));
        h.nparts = gemm_tiles(n, n);
        h.partials = reinterpret_cast<double *>(w + P.parts[b]);
        h.res = res + b;
        std::memcpy(ctl_host.data() + (size_t)b * cb, &h, sizeof(h));
        RefMember &m = mem[b];
        std::memset(&m, 0, sizeof(m));
        m.A = A + off_host[b]; m.lda = n; m.X = X + off_host[b]; m.ldx = n;
        m.Xw = reinterpret_cast<double *>(w + P.xw[b]);
        m.B = reinterpret_cast<double *>(w + P.r[b]);
        m.ipiv = ipiv + piv_off_host[b]; m.jpiv = jpiv + piv_off_host[b];
        if (big_index[b] >= 0) {
            m.rows = d32[big_index[b]].rowphys; m.cols = d32[big_index[b]].colphys;
        } else {
            m.rows_buf = reinterpret_cast<int32_t *>(w + P.rows[b]);
            m.cols_buf = reinterpret_cast<int32_t *>(w + P.cols[b]);
            m.rows = m.rows_buf; m.cols = m.cols_buf;
        }
        m.blockres = blockres + P.blockres_start[b];
        m.n = n; m.nblocks = P.nblocks[b];
        P.fb.mats[b] = E.mats[b];
        P.fb.mats[b].run = ctl_run_fallback(ctl + (size_t)b * cb);
    }
    // Newton-Schulz lists
    for (int b = 0; b < batch; ++b) {
        const int n = n_host[b];
        const void *cm = ctl + (size_t)b * cb;
        double *Xb = X + off_host[b], *Xwb = reinterpret_cast<double *>(w + P.xw[b]);
        double *Rb = reinterpret_cast<double *>(w + P.r[b]);
        double *pb = reinterpret_cast<double *>(w + P.parts[b]);
        GemmArgs g;
        std::memset(&g, 0, sizeof(g));
        g.M = g.N = g.K = n;
        g.A = A + off_host[b]; g.lda = n; g.B = Xb; g.ldb = n; g.D = Rb; g.ldd = n;
        g.alpha = -1.0; g.gamma = 1.0; g.norm_partials = pb; g.run_flag = ctl_run_ns(cm);
        P.r0.add(g);
        for (int p = 0; p < 2; ++p) {   // p = iteration parity: odd reads X, writes Xw
            double *Xs = p ? Xb : Xwb, *Xd = p ? Xwb : Xb;
            GemmArgs u;
            std::memset(&u, 0, sizeof(u));
            u.M = u.N = u.K = n;
            u.A = Xs; u.lda = n; u.B = Rb; u.ldb = n; u.C = Xs; u.ldc = n; u.D = Xd; u.ldd = n;
            u.alpha = 1.0; u.beta = 1.0; u.run_flag = ctl_run_ns(cm);
            P.upd[p].add(u);
            GemmArgs r2 = g;
            r2.B = Xd;
            P.res[p].add(r2);
        }
    }
    // determinant block steps
    for (size_t st = 0; st < P.det_blocks.size(); ++st) {
        OnchipSet &S = P.det_blocks[st];
        S.mats.clear();
        const int kb = (int)st * kDetBlock;
        for (int b = 0; b < batch; ++b) {
            const int n = n_host[b];
            if (n <= kb) continue;
            const void *cm = ctl + (size_t)b * cb;
            const int nbk = std::min(kDetBlock, n - kb), mm = n - kb - nbk;
            const int ldd = std::min(n, kDetBlock);
            MatDesc md;
            md.a_off = (int64_t)(P.r[b] / 8) + (int64_t)kb * n + kb;
            md.x_off = (int64_t)(P.dinv[b] / 8);
            md.piv_off = (int64_t)(P.bpiv[b] / 4);
            md.n = nbk; md.lda = n; md.ldx = ldd;
            md.res_idx = P.blockres_start[b] + (int)st;
            md.run = ctl_run_det(cm);
            S.mats.push_back(md);
            if (mm > 0) {
                double *Bb = reinterpret_cast<double *>(w + P.r[b]);
                double *Tb = reinterpret_cast<double *>(w + P.t[b]);
                GemmArgs g1;
                std::memset(&g1, 0, sizeof(g1));
                g1.M = nbk; g1.N = mm; g1.K = nbk;
                g1.A = reinterpret_cast<double *>(w + P.dinv[b]); g1.lda = ldd;
                g1.B = Bb + (int64_t)kb * n + kb + nbk; g1.ldb = n;
                g1.D = Tb; g1.ldd = n;
                g1.alpha = 1.0; g1.run_flag = ctl_run_det(cm);
                P.det_t[st].add(g1);
                // one refinement step of T (see the single-matrix path)
                GemmArgs gr;
                std::memset(&gr, 0, sizeof(gr));
                gr.M = nbk; gr.N = mm; gr.K = nbk;
                gr.A = Bb + (int64_t)kb * n + kb; gr.lda = n;
                gr.B = Tb; gr.ldb = n;
                gr.C = Bb + (int64_t)kb * n + kb + nbk; gr.ldc = n;
                gr.D = const_cast<double *>(gr.C); gr.ldd = n;
                gr.alpha = -1.0; gr.beta = 1.0; gr.run_flag = ctl_run_det(cm);
                P.det_r[st].add(gr);
                GemmArgs gc;
                std::memset(&gc, 0, sizeof(gc));
                gc.M = nbk; gc.N = mm; gc.K = nbk;
                gc.A = g1.A; gc.lda = ldd;
                gc.B = gr.C; gc.ldb = n;
                gc.C = Tb; gc.ldc = n;
                gc.D = Tb; gc.ldd = n;
                gc.alpha = 1.0; gc.beta = 1.0; gc.run_flag = ctl_run_det(cm);
                P.det_c[st].add(gc);
                GemmArgs g2;
                std::memset(&g2, 0, sizeof(g2));
                g2.M = mm; g2.N = mm; g2.K = nbk;
                g2.A = Bb + (int64_t)(kb + nbk) * n + kb; g2.lda = n;
                g2.B = Tb; g2.ldb = n;
                g2.C = Bb + (int64_t)(kb + nbk) * n + kb + nbk; g2.ldc = n;
                g2.D = const_cast<double *>(g2.C); g2.ldd = n;
                g2.alpha = -1.0; g2.beta = 1.0; g2.run_flag = ctl_run_det(cm);
                P.det_s[st].add(g2);
            }
        }
        S.build();
    }

    // ---- upload (host tables die with this call: synchronise once)
    if (!(o.flags & GJ_FLAG_REUSE_PLAN)) {
        std::vector<std::pair<size_t, std::pair<const void *, size_t>>> up;
        auto put = [&](size_t off, const void *p, size_t bytes) { if (bytes) up.push_back({off, {p, bytes}}); };
        put(E.off_mats, E.mats.data(), sizeof(MatDesc) * batch);
        put(E.off_tasks, E.tasks.data(), sizeof(OnchipTask) * E.tasks.size());
        put(E.off_descs, d32.data(), sizeof(BigDesc) * d32.size());
        put(E.off_bmap, E.bmap.data(), sizeof(int2) * E.bmap.size());
        put(P.off_ctl, ctl_host.data(), ctl_host.size());
        put(P.off_mem, mem.data(), sizeof(RefMember) * batch);
        put(P.fb.off_mats, P.fb.mats.data(), sizeof(MatDesc) * batch);
        put(P.fb.off_tasks, E.tasks.data(), sizeof(OnchipTask) * E.tasks.size());
        put(P.off_fb_descs, d64.data(), sizeof(BigDesc) * d64.size());
        put(P.off_fb_bmap, P.fb_bmap.data(), sizeof(int2) * P.fb_bmap.size());
        auto put_list = [&](GemmList &L) {
            put(L.off_probs, L.probs.data(), sizeof(GemmArgs) * L.probs.size());
            put(L.off_tiles, L.tiles.data(), sizeof(int2) * L.tiles.size());
        };
        put_list(P.r0);
        for (int p = 0; p < 2; ++p) { put_list(P.upd[p]); put_list(P.res[p]); }
        for (size_t st = 0; st < P.det_blocks.size(); ++st) {
            put(P.det_blocks[st].off_mats, P.det_blocks[st].mats.data(), sizeof(MatDesc) * P.det_blocks[st].mats.size());
            put(P.det_blocks[st].off_tasks, P.det_blocks[st].tasks.data(), sizeof(OnchipTask) * P.det_blocks[st].tasks.size());
            put_list(P.det_t[st]);
            put_list(P.det_r[st]);
            put_list(P.det_c[st]);
            put_list(P.det_s[st]);
        }
        for (auto &u : up)
            GJ_TRY(hipMemcpyAsync(w + u.first, u.second.first, u.second.second, hipMemcpyHostToDevice, s));
        GJ_TRY(hipStreamSynchronize(s));
    }
    uint32_t *queues = reinterpret_cast<uint32_t *>(w + E.off_queue);
    auto run_onchip_set = [&](bool fp32, const MatDesc *mats, const OnchipTask *tasks,
                              const int *cstart, const int *ccount, const double *Ab, double *Xb,
                              int32_t *ip, int32_t *jp, gj_result *rs, double tol, double eps,
                              int mode) -> gj_status {
        GJ_TRY(launch_zero_u32(queues, kOnchipClasses, s));
        for (int c = 0; c < kOnchipClasses; ++c) {
            if (!ccount[c]) continue;
            GJ_TRY(launch_onchip_class(fp32, c, mats, tasks + cstart[c], ccount[c], queues + c, MatDesc(),
                                       Ab, Xb, ip, jp, rs, tol, eps, mode, nullptr, s));
        }
        return GJ_OK;
    };
    auto grouped = [&](GemmList &L) -> gj_status {
        GJ_TRY(launch_gemm_f64_grouped(reinterpret_cast<const GemmArgs *>(w + L.off_probs),
                                       reinterpret_cast<const int2 *>(w + L.off_tiles),
                                       (int)L.tiles.size(), s));
        return GJ_OK;
    };
    gj_status st;

    // 1. FP32 elimination of every member
    if (!E.tasks.empty()) {
        st = run_onchip_set(true, reinterpret_cast<const MatDesc *>(w + E.off_mats),
                            reinterpret_cast<const OnchipTask *>(w + E.off_tasks), E.cls_start,
                            E.cls_count, A, X, ipiv, jpiv, res, 0.0, 0.0, 0);
        if (st != GJ_OK) return st;
    }
    if (!E.big_members.empty())
        GJ_TRY(launch_big_groups(true, E, reinterpret_cast<const BigDesc *>(w + E.off_descs),
                                 reinterpret_cast<const int2 *>(w + E.off_bmap), 0.0, 0.0, o.events,
                                 s));
    GJ_TRY(launch_refine_start(ctl, batch, s));
    // 2. Newton-Schulz on grouped MFMA products
    if ((st = grouped(P.r0)) != GJ_OK) return st;
    GJ_TRY(launch_refine_resid0(ctl, batch, s));
    for (int it = 1; it <= o.max_refine_iters; ++it) {
        if ((st = grouped(P.upd[it & 1])) != GJ_OK) return st;
        if ((st = grouped(P.res[it & 1])) != GJ_OK) return st;
        GJ_TRY(launch_refine_after_update(ctl, batch, it, o.max_refine_iters, kStall, s));
    }
    GJ_TRY(launch_refine_finish(ctl, batch, kAcceptResid, 1, s));
    GJ_TRY(launch_copy_back(reinterpret_cast<const RefMember *>(w + P.off_mem), RefMember(), ctl,
                            batch, 4, s));
    // 3. FP64 elimination for the members whose refinement failed
    if (!E.tasks.empty()) {
        st = run_onchip_set(false, reinterpret_cast<const MatDesc *>(w + P.fb.off_mats),
                            reinterpret_cast<const OnchipTask *>(w + P.fb.off_tasks), E.cls_start,
                            E.cls_count, A, X, ipiv, jpiv, res, o.zero_tol, kEps64, 0);
        if (st != GJ_OK) return st;
    }
    if (!E.big_members.empty()) {
        const int nb = (int)P.fb_bmap.size();
        GJ_TRY(launch_big(false, P.fb_nt, big_nt_loads(P.fb_swept), P.fb_full ? 8 : 0, P.fb_counted, false, 0,
                          reinterpret_cast<const BigDesc *>(w + P.off_fb_descs),
                          reinterpret_cast<const int2 *>(w + P.off_fb_bmap), BigDesc(),
                          P.fb_grid.data(), nb, nb, E.big_max_n, nb, o.zero_tol, kEps64, 0, nullptr,
                          nullptr, s));
    }
    GJ_TRY(launch_fallback_mark(ctl, batch, s));
    // 4. FP64 determinants: permuted copies, block elimination in lock step
    const RefMember *memd = reinterpret_cast<const RefMember *>(w + P.off_mem);
    GJ_TRY(launch_perms_from_pivots(memd, RefMember(), ctl, batch, s));
    GJ_TRY(launch_gather_perm(memd, RefMember(), ctl, batch, 4, s));
    for (size_t sb = 0; sb < P.det_blocks.size(); ++sb) {
        OnchipSet &S = P.det_blocks[sb];
        st = run_onchip_set(false, reinterpret_cast<const MatDesc *>(w + S.off_mats),
                            reinterpret_cast<const OnchipTask *>(w + S.off_tasks), S.cls_start,
                            S.cls_count, wd, wd, reinterpret_cast<int32_t *>(w),
                            reinterpret_cast<int32_t *>(w) + kDetBlock, blockres, 0.0, kEps64,
                            kOnchipStaticPivots);
        if (st != GJ_OK) return st;
        if ((st = grouped(P.det_t[sb])) != GJ_OK) return st;
        if ((st = grouped(P.det_r[sb])) != GJ_OK) return st;
        if ((st = grouped(P.det_c[sb])) != GJ_OK) return st;
        if ((st = grouped(P.det_s[sb])) != GJ_OK) return st;
    }
    GJ_TRY(launch_det_combine(memd, RefMember(), ctl, batch, s));
    GJ_TRY(launch_refine_iters(ctl, batch, s));
    return GJ_OK;
}

size_t refined_ws(int n, bool acc, bool blocked) { return refined_layout(n, acc, blocked).end; }

// Residual of a plain FP64 result (want_resid): needs n^2 + partial sums.
size_t resid_ws(int n) {
    return a256((size_t)n * n * 8) + 3 * a256((size_t)std::max(gemm_tiles(n, n), sumsq_blocks(n)) * 8);
}

gj_status run_resid(int n, const double *A, int64_t lda, const double *X, int64_t ldx,
                    gj_result *res, char *w, hipStream_t s) {
    double *R = reinterpret_cast<double *>(w);
    const size_t np = a256((size_t)std::max(gemm_tiles(n, n), sumsq_blocks(n)) * 8);
    double *pr = reinterpret_cast<double *>(w + a256((size_t)n * n * 8));
    double *pa = reinterpret_cast<double *>((char *)pr + np);
    double *px = reinterpret_cast<double *>((char *)pa + np);
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = g.N = g.K = n;
    g.A = A; g.lda = lda; g.B = X; g.ldb = ldx; g.D = R; g.ldd = n;
    g.alpha = -1.0; g.gamma = 1.0; g.norm_partials = pr;
    GJ_TRY(launch_gemm_f64(g, s));
    GJ_TRY(launch_sumsq(A, lda, n, pa, s));
    GJ_TRY(launch_sumsq(X, ldx, n, px, s));
    GJ_TRY(launch_resid(pr, gemm_tiles(n, n), pa, sumsq_blocks(n), px, sumsq_blocks(n), res, s));
    return GJ_OK;
}

}  // namespace
}  // namespace gj

// ------------------------------------------------ uploaded batched plans
// The tables a batched call uploads into the workspace hold the caller's
// buffer addresses.  A GJ_FLAG_REUSE_PLAN call is therefore accepted only
// with the workspace, buffers, precision and batch description of the upload
// it reuses: the library keeps a signature of the last upload into each
// workspace (at most kPlanSlots workspaces, the oldest forgotten first).
namespace gj {
namespace {

constexpr size_t kPlanSlots = 64;
struct PlanSig { const void *ws; uint64_t sig; };
std::mutex g_plan_mu;
std::vector<PlanSig> g_plans;

uint64_t fnv1a(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t plan_signature(int batch, const int32_t *n_host, const int64_t *off_host,
                        const int64_t *piv_off_host, const void *A, const void *X,
                        const void *ipiv, const void *jpiv, const void *res, int precision,
                        size_t ws_bytes) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &batch, sizeof(batch));
    h = fnv1a(h, n_host, sizeof(int32_t) * (size_t)batch);
    h = fnv1a(h, off_host, sizeof(int64_t) * (size_t)batch);
    h = fnv1a(h, piv_off_host, sizeof(int64_t) * (size_t)batch);
    const void *ptrs[5] = {A, X, ipiv, jpiv, res};
    h = fnv1a(h, ptrs, sizeof(ptrs));
    h = fnv1a(h, &precision, sizeof(precision));
    h = fnv1a(h, &ws_bytes, sizeof(ws_bytes));
    return h;
}

void plan_record(const void *ws, uint64_t sig) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    for (PlanSig &p : g_plans)
        if (p.ws == ws) { p.sig = sig; return; }
    if (g_plans.size() >= kPlanSlots) g_plans.erase(g_plans.begin());
    g_plans.push_back(PlanSig{ws, sig});
}

bool plan_matches(const void *ws, uint64_t sig) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    for (const PlanSig &p : g_plans)
        if (p.ws == ws) return p.sig == sig;
    return false;
}

}  // namespace
}  // namespace gj

// ------------------------------------------------------- built-in scratch
// The workspace of gj_invert_noalloc: one array in the code object, which
// every GPU the library runs on holds from module load until the process ends
// (each at its own device address).  In host code the name is only a stand-in
// for the symbol: the device address comes from hipGetSymbolAddress, once per
// device, with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[GJ_NOALLOC_SCRATCH_BYTES];

namespace gj {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the calling thread's current device's array.
hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
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

gj_status gj_dgemm(int32_t M, int32_t N, int32_t K, double alpha, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double beta, const double *C, int64_t ldc,
                   double gamma, double *D, int64_t ldd, void *stream) {
    try {
        if (M < 0 || N < 0 || K < 0 || !D || ldd < N) return GJ_E_INVALID_ARG;
        if (K > 0 && (!A || !B || lda < K || ldb < N)) return GJ_E_INVALID_ARG;
        if (beta != 0.0 && (!C || ldc < N)) return GJ_E_INVALID_ARG;
        GemmArgs g;
        std::memset(&g, 0, sizeof(g));
        g.M = M; g.N = N; g.K = K;
        g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
        g.alpha = alpha; g.beta = beta; g.gamma = gamma;
        hipError_t e = launch_gemm_f64(g, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e);
        return GJ_OK;
    } catch (...) {
        return GJ_E_HIP;
    }
}

gj_status gj_sgemm(int32_t M, int32_t N, int32_t K, float alpha, const float *A, int64_t lda,
                   const float *B, int64_t ldb, float beta, const float *C, int64_t ldc,
                   float gamma, float *D, int64_t ldd, void *stream) {
    try {
        if (M < 0 || N < 0 || K < 0 || !D || ldd < N) return GJ_E_INVALID_ARG;
        if (K > 0 && (!A || !B || lda < K || ldb < N)) return GJ_E_INVALID_ARG;
        if (beta != 0.0f && (!C || ldc < N)) return GJ_E_INVALID_ARG;
        GemmArgsT<float> g;
        std::memset(&g, 0, sizeof(g));
        g.M = M; g.N = N; g.K = K;
        g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
        g.alpha = alpha; g.beta = beta; g.gamma = gamma;
        hipError_t e = launch_gemm_f32(g, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e);
        return GJ_OK;
    } catch (...) {
        return GJ_E_HIP;
    }
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
        if (o.rule != 0 && o.precision != GJ_PREC_FP64) return 0;
        if (op == GJ_OP_DET && (o.flags & GJ_FLAG_BLOCKED)) return 0;
        return single_ws(n_or_batch, o, op == GJ_OP_DET);
    }
    if (op == GJ_OP_SOLVE) {
        if (n_or_batch < 1 || !n_host || n_host[0] < 1 || n_or_batch + n_host[0] > kMaxN) return 0;
        if (o.precision != GJ_PREC_FP64 || o.want_resid || (o.flags & GJ_FLAG_BLOCKED)) return 0;
        return solve_ws(n_or_batch, n_host[0], o.rule);
    }
    if (op == GJ_OP_INVERT_BATCHED) {
        if (n_or_batch < 1 || !n_host || o.rule != 0 || (o.flags & (GJ_FLAG_ACCURATE | GJ_FLAG_BLOCKED)))
            return 0;
        if (o.precision == GJ_PREC_FP32_REFINED) {
            RefBatchPlan R;
            if (!plan_refined_batch(n_or_batch, n_host, R)) return 0;
            return R.total;
        }
        BatchPlan P;
        if (!plan_batch(n_or_batch, n_host, false, P)) return 0;
        return P.total;
    }
    return 0;
}

static bool needs_ws(int n, const Opts &o, bool det_only) {
    return n > kOnchipMax || o.rule != 0 || o.precision == GJ_PREC_FP32_REFINED ||
           (o.want_resid && !det_only);
}

gj_status gj_invert(int32_t n, const double *A, int64_t lda, double *X, int64_t ldx,
                    int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts, void *ws,
                    size_t ws_bytes, void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (n < 1 || lda < n || ldx < n || !A || !X || !ipiv || !jpiv || !res)
            return GJ_E_INVALID_ARG;
        if (n > kMaxN || (o.rule != 0 && o.precision != GJ_PREC_FP64)) return GJ_E_UNSUPPORTED;
        const size_t abytes = ((size_t)(n - 1) * lda + n) * 8, xbytes = ((size_t)(n - 1) * ldx + n) * 8;
        if (overlaps(A, abytes, X, xbytes)) return GJ_E_INVALID_ARG;
        const size_t need = single_ws(n, o, false);
        if (needs_ws(n, o, false)) {
            if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
            if (ws_bytes < need) return GJ_E_WORKSPACE;
            if (overlaps(ws, ws_bytes, X, xbytes) || overlaps(ws, ws_bytes, A, abytes))
                return GJ_E_INVALID_ARG;
        }
        hipStream_t s = (hipStream_t)stream;
        if (o.precision == GJ_PREC_FP32_REFINED)
            return run_refined_single(n, A, lda, X, ldx, ipiv, jpiv, res, o, (char *)ws, s, false);
        const bool blocked = use_blocked(n, o, false);
        gj_status st = blocked ? run_blocked(false, n, A, lda, X, ldx, ipiv, jpiv, res, o.zero_tol, kEps64,
                                             ws, ws_bytes, 0, s)
                               : run_single(n, A, lda, X, ldx, ipiv, jpiv, res, o, ws, ws_bytes, s, false);
        if (st != GJ_OK || !o.want_resid) return st;
        size_t off = 0;
        if (blocked)
            off = a256(blk_layout(n).end);
        else if (n > kOnchipMax || o.rule != 0)
            off = a256(big_bufs(single_shape(n, false, big_threads(n, false)), false, 0).end);
        return run_resid(n, A, lda, X, ldx, res, (char *)ws + off, s);
    } catch (...) {
        return GJ_E_HIP;
    }
}

gj_status gj_invert_noalloc(int32_t n, const double *A, int64_t lda, double *X, int64_t ldx,
                            int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts,
                            void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (n < 1 || n > kMaxN) return n < 1 ? GJ_E_INVALID_ARG : GJ_E_UNSUPPORTED;
        if (o.rule != 0 && o.precision != GJ_PREC_FP64) return GJ_E_UNSUPPORTED;
        // the whole workspace the call would need must fit the built-in array
        if (single_ws(n, o, false) > (size_t)GJ_NOALLOC_SCRATCH_BYTES) return GJ_E_UNSUPPORTED;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e);
        if (stream) {   // the array used is the stream's device's
            hipDevice_t sdev = 0;
            e = hipStreamGetDevice((hipStream_t)stream, &sdev);
            if (e != hipSuccess) return hip_fail(e);
            if ((int)sdev != dev) return GJ_E_INVALID_ARG;
        }
        void *ws = nullptr;
        e = scratch_address(dev, &ws);
        if (e != hipSuccess) return hip_fail(e);
        struct NoSide {   // no side stream or event is created for this call
            NoSide() { g_no_side = true; }
            ~NoSide() { g_no_side = false; }
        } no_side;
        return gj_invert(n, A, lda, X, ldx, ipiv, jpiv, res, opts, ws,
                         (size_t)GJ_NOALLOC_SCRATCH_BYTES, stream);
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
        if (n > kMaxN || (o.rule != 0 && o.precision != GJ_PREC_FP64)) return GJ_E_UNSUPPORTED;
        if (o.flags & GJ_FLAG_BLOCKED) return GJ_E_UNSUPPORTED;
        const size_t need = single_ws(n, o, true);
        if (needs_ws(n, o, true)) {
            if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
            if (ws_bytes < need) return GJ_E_WORKSPACE;
        }
        hipStream_t s = (hipStream_t)stream;
        if (o.precision == GJ_PREC_FP32_REFINED)
            return run_refined_single(n, A, lda, nullptr, n, ipiv, jpiv, res, o, (char *)ws, s, true);
        return run_single(n, A, lda, nullptr, n, ipiv, jpiv, res, o, ws, ws_bytes, s, true);
    } catch (...) {
        return GJ_E_HIP;
    }
}

gj_status gj_solve(int32_t n, int32_t m, const double *A, int64_t lda, const double *B,
                   int64_t ldb, double *X, int64_t ldx, int32_t *ipiv, int32_t *jpiv,
                   gj_result *res, const gj_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    try {
        Opts o;
        if (!read_opts(opts, o)) return GJ_E_INVALID_ARG;
        if (n < 1 || m < 1 || lda < n || ldb < m || ldx < m || !A || !B || !X || !ipiv || !jpiv ||
            !res)
            return GJ_E_INVALID_ARG;
        if ((int64_t)n + m > kMaxN || o.precision != GJ_PREC_FP64 || o.want_resid ||
            (o.flags & GJ_FLAG_BLOCKED))
            return GJ_E_UNSUPPORTED;
        const size_t abytes = ((size_t)(n - 1) * lda + n) * 8;
        const size_t bbytes = ((size_t)(n - 1) * ldb + m) * 8, xbytes = ((size_t)(n - 1) * ldx + m) * 8;
        if (overlaps(A, abytes, X, xbytes) || overlaps(B, bbytes, X, xbytes)) return GJ_E_INVALID_ARG;
        if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
        if (ws_bytes < solve_ws(n, m, o.rule)) return GJ_E_WORKSPACE;
        if (overlaps(ws, ws_bytes, X, xbytes) || overlaps(ws, ws_bytes, A, abytes) ||
            overlaps(ws, ws_bytes, B, bbytes))
            return GJ_E_INVALID_ARG;
        return run_solve(n, m, A, lda, B, ldb, X, ldx, ipiv, jpiv, res, o, ws, ws_bytes,
                         (hipStream_t)stream);
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
        if (o.rule != 0) return GJ_E_UNSUPPORTED;   // the batch kernels search the full block
        if (o.flags & (GJ_FLAG_ACCURATE | GJ_FLAG_BLOCKED)) return GJ_E_UNSUPPORTED;   // single matrices only
        if (!ws || ((uintptr_t)ws & 255)) return GJ_E_WORKSPACE;
        size_t mat_end = 0;   // elements of A (and of X) the members span
        for (int b = 0; b < batch; ++b) {
            if (n_host[b] < 1 || n_host[b] > kMaxN || off_host[b] < 0 || piv_off_host[b] < 0)
                return GJ_E_INVALID_ARG;
            mat_end = std::max(mat_end, (size_t)off_host[b] + (size_t)n_host[b] * n_host[b]);
        }
        if (overlaps(A, mat_end * 8, X, mat_end * 8) || overlaps(ws, ws_bytes, A, mat_end * 8) ||
            overlaps(ws, ws_bytes, X, mat_end * 8))
            return GJ_E_INVALID_ARG;
        const uint64_t sig = plan_signature(batch, n_host, off_host, piv_off_host, A, X, ipiv,
                                            jpiv, res, o.precision, ws_bytes);
        if ((o.flags & GJ_FLAG_REUSE_PLAN) && !plan_matches(ws, sig)) return GJ_E_INVALID_ARG;
        if (o.precision == GJ_PREC_FP32_REFINED) {
            const gj_status st = run_refined_batched(batch, n_host, off_host, A, X, piv_off_host,
                                                     ipiv, jpiv, res, o, (char *)ws, ws_bytes,
                                                     (hipStream_t)stream);
            if (st == GJ_OK && !(o.flags & GJ_FLAG_REUSE_PLAN)) plan_record(ws, sig);
            return st;
        }
        const bool fp32 = false;
        BatchPlan P;
        if (!plan_batch(batch, n_host, fp32, P)) return GJ_E_INVALID_ARG;
        if (ws_bytes < P.total) return GJ_E_WORKSPACE;
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
            m.run = nullptr;
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
            plan_record(ws, sig);
        }
        const double eps_default = fp32 ? 0.0 : kEps64;
        std::optional<SideFork> fork;   // the one-matrix-per-wavefront classes beside the rest
        if (!P.tasks.empty()) {
            uint32_t *queues = reinterpret_cast<uint32_t *>(w + P.off_queue);
            hipError_t e = launch_zero_u32(queues, kOnchipClasses, s);
            if (e != hipSuccess) return hip_fail(e);
            fork.emplace(s, true);
            const MatDesc *mats = reinterpret_cast<const MatDesc *>(w + P.off_mats);
            const OnchipTask *tasks = reinterpret_cast<const OnchipTask *>(w + P.off_tasks);
            for (int c = 0; c < kOnchipClasses; ++c) {
                if (!P.cls_count[c]) continue;
                e = launch_onchip_class(fp32, c, mats, tasks + P.cls_start[c], P.cls_count[c],
                                        queues + c, MatDesc(), A, X, ipiv, jpiv, res, o.zero_tol,
                                        eps_default, 0, nullptr, onchip_class_kind(c) == 1 ? fork->fs : s);
                if (e != hipSuccess) return hip_fail(e);
            }
        }
        if (!P.big_members.empty()) {
            hipError_t e = launch_big_groups(fp32, P, reinterpret_cast<const BigDesc *>(w + P.off_descs),
                                             reinterpret_cast<const int2 *>(w + P.off_bmap), o.zero_tol,
                                             eps_default, o.events, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        if (fork) {
            const hipError_t e = fork->join_back();
            if (e != hipSuccess) return hip_fail(e);
        }
        return GJ_OK;
    } catch (...) {
        return GJ_E_HIP;
    }
}

}  // extern "C"
