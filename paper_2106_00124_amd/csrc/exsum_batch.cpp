// exsum_batch.cpp -- batched form: many tensors of uneven shapes, ranks,
// boxes, dtypes and operators in one hipGraph launch of persistent work-list
// kernels, with an autotuner for the work granularity.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Each job is planned by the same planner as the plain call (exsum_plan.hpp),
// but its steps are recorded instead of launched.  Step p of every job goes
// to phase p (a job's recorded order respects its dependencies); within a
// phase, steps of one kind, dtype, operator and register bucket share one
// work-list launch (exsum_worklist.hip).  Every job gets its own region of
// the batch workspace.  The whole sequence is captured once per workspace
// into a hipGraph and replayed.
//
// Autotuning: the work granularity (minimum tasks per step, which sets how
// many chunks a row or axis-0 stream is cut into) and the persistent grid
// size (workgroups per CU) are chosen by timing candidate settings on the
// batch itself; the winner is cached in a JSON file keyed by a signature of
// the batch's shapes, boxes, dtypes, operators and modes.  A file at that
// path that is not such a cache is neither used nor overwritten.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>
#include <string>
#include <vector>

#include "exsum_internal.hpp"
#include "exsum_plan.hpp"
#include "exsum_tasks.hpp"
#include "exsum_tunecache.hpp"

namespace exs {

struct TuneCfg {
    i64 min_tasks = 16384;  // minimum tasks per bdbs / axis-0 step
    int wg_per_cu = 4;      // persistent workgroups per CU
};

struct Rec {
    Step s;
    int dtype, op, kb;
};

// Records the planner's steps (the generic kernels only).
template <typename T, class Op>
struct ListSink {
    std::vector<Rec>* out;
    int dtype, op;
    TuneCfg cfg;
    bool fused_ok = false;
    void level(int) {}
    // the fused 2-D stream has no work-list form
    bool row_ok(i64, i64, i64, i64) const { return false; }
    void row_axis0(const T*, const T*, const T*, const T*, T*, T*, i64, i64, i64, i64, i64) {}
    // the single-workgroup kernel for a short last level has no work-list form
    bool small1d_ok(i64) const { return false; }
    // nor the one-workgroup rank-2 kernel
    bool small2d_ok(i64, i64, i64, i64) const { return false; }
    void small2d(const T*, T*, T*, i64, i64, i64, i64) {}
    // the fused levels are off here, and with them the fused aggregate pass
    bool aggmid_ok() const { return false; }
    void aggmid(const T*, T*, T*, T*, i64, i64, i64, i64, i64, i64, i64) {}
    // the staged multi-axis BDBS has no work-list form
    i64 tail_box_max() const { return 0; }
    void bdbs_tail(const T*, T*, i64, int, const i64*, const i64*) {}
    bool long1d_ok(i64, i64) const { return false; }
    void long1d(const T*, T*, T*, i64, i64, T*, T*, T*, T*) {}
    void ex1d_small(const T*, T*, i64, i64) {}
    // weak excluded sums are rejected when the batch is created
    void total(const T*, i64, void*, T*) {}
    void weak_exc(const T*, const T*, T*, i64) {}
    void plane_weak(const T*, T*, const T*, T*, i64, i64, i64, i64, i64, i64, i64) {}
    // 4-byte generic BDBS and axis-0 steps with boxes up to 8 share the
    // bucket of 8 (every such kernel runs at full occupancy): fewer launches
    void push(const Step& s, int kb) {
        if (sizeof(T) == 4 && (s.kind == SK_BDBS || s.kind == SK_AX0) && kb < 8) kb = 8;
        out->push_back(Rec{s, dtype, op, kb});
    }
    void bdbs(const T* in, T* o, i64 O, i64 n, i64 I, i64 k) {
        Step s{};
        s.k = (int)k;
        s.in0 = in;
        s.out0 = o;
        s.O = O;
        s.n = n;
        s.I = I;
        const int kb = bucket_for(k);
        if (kb == 0) {
            s.kind = SK_BDBS2;
            s.ntasks = O * I;
            push(s, 1);
            return;
        }
        const i64 rcb = I == 1 ? rows_blocks(O, n, k, ROWS_MIN_TASKS) : 0;
        // (the same choice as the plain call's launch_bdbs)
        const bool rows_lds = I == 1 && O >= rows_per_task(k) &&
                              (kb > COOP_CS || n > 256 ||
                               rows_tasks(O, n, k, rcb) >= ROWS_MIN_TASKS);
        if (I == 1 && !rows_lds && n <= 256 && narrow_ok(O * n, (int)sizeof(T), 32)) {
            // short rows of the contiguous axis, too few for the LDS-staged
            // tasks: one wavefront per task, segmented scans across the lanes
            s.kind = SK_BDBSV;
            s.cb = wave_rows_per_task(O);
            s.ntasks = (O + s.cb - 1) / s.cb * 64;
            push(s, 1);
            return;
        }
        if (rows_lds) {
            // rows of the contiguous axis of a large tensor: wavefront tasks
            // through LDS
            s.kind = SK_BDBSR;
            const i64 nbr = (n + k - 1) / k;
            s.cb = rcb;
            s.nchunks = (nbr + s.cb - 1) / s.cb;
            s.ntasks = ((O + rows_per_task(k) - 1) / rows_per_task(k)) * s.nchunks;
            push(s, kb);
            return;
        }
        const i64 nb = (n + k - 1) / k, cols = O * I;
        if (kb >= 32 && I > 1 && O * n * I * (i64)sizeof(T) < ((i64)1 << 31)) {
            // boxes of 17 to 64 along a strided axis: lanes share a column
            s.kind = SK_BDBSC;
            const i64 C = 64 / coop_g(kb, (int)sizeof(T), false);
            const i64 groups = (cols + C - 1) / C;
            s.cb = coop_run_blocks(groups, nb);
            s.nchunks = (nb + s.cb - 1) / s.cb;
            s.ntasks = groups * s.nchunks * 64;
            push(s, kb);
            return;
        }
        s.kind = narrow_ok(O * n * I, (int)sizeof(T), kb) ? SK_BDBS : SK_BDBSW;
        i64 nch = (cfg.min_tasks + cols - 1) / cols;
        if (nch > nb) nch = nb;
        if (nch < 1) nch = 1;
        s.cb = (nb + nch - 1) / nch;
        s.nchunks = (nb + s.cb - 1) / s.cb;
        s.ntasks = cols * s.nchunks;
        push(s, kb);
    }
    void segtot(const T* Gw, const T* Ga, T* Tw, T* Ta, i64 Q, i64 M, i64 L) {
        Step s{};
        s.kind = SK_SEGTOT;
        s.in0 = Gw;
        s.in1 = Ga;
        s.out0 = Tw;
        s.out1 = Ta;
        s.Q = Q;
        s.I = M;
        s.cb = L;
        s.ntasks = ((Q + L - 1) / L) * M;
        push(s, 1);
    }
    void segexp(const T* Gw, const T* SPX, const T* SSX, T* PX, T* SX, i64 Q, i64 M, i64 L,
                i64) {
        Step s{};
        s.kind = SK_SEGEXP;
        s.in0 = Gw;
        s.in1 = SPX;
        s.in2 = SSX;
        s.out0 = PX;
        s.out1 = SX;
        s.Q = Q;
        s.I = M;
        s.cb = L;
        s.ntasks = ((Q + L - 1) / L) * M;
        push(s, 1);
    }
    void blockagg(const T* X, T* Ga, i64 n0, i64 M, i64 k0, i64 Q) {
        Step s{};
        s.kind = SK_AGG;
        s.k = (int)k0;
        s.in0 = X;
        s.out0 = Ga;
        s.n = n0;
        s.I = M;
        s.Q = Q;
        s.ntasks = Q * M;
        push(s, 1);
    }
    // (pxe is 1 here: the fused levels, whose streams read PX at run starts
    // only, are off)
    void blockscan(const T* Gw, const T* Ga, T* PX, T* SX, T* R, i64 Q, i64 M, i64) {
        Step s{};
        s.kind = SK_SCAN;
        s.in0 = Gw;
        s.in1 = Ga;
        s.out0 = PX;
        s.out1 = SX;
        s.out2 = R;
        s.Q = Q;
        s.I = M;
        s.ntasks = M;
        push(s, 1);
    }
    // (ex2t, the chunk totals of the plain call's chunked long-box sweep, is
    // not used: the work-list runs the per-column sweep)
    void axis0(const T* W, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
               i64 M, i64 k0, i64 Q, T*) {
        const int kb = bucket_for(k0);
        if (kb == 0) {
            if (exc) {
                Step s{};
                s.kind = SK_EX2;
                s.k = (int)k0;
                s.in0 = W;
                s.in3 = Trest;
                s.out0 = exc;
                s.n = n0;
                s.I = M;
                s.ntasks = M;
                push(s, 1);
            }
            if (inc) bdbs(W, inc, 1, n0, M, k0);
            return;
        }
        Step s{};
        const bool coop = kb >= 32 && n0 * M * (i64)sizeof(T) < ((i64)1 << 31);
        s.kind = coop ? SK_AX0C : narrow_ok(n0 * M, (int)sizeof(T), kb) ? SK_AX0 : SK_AX0W;
        s.k = (int)k0;
        s.in0 = W;
        s.in1 = PX;
        s.in2 = SX;
        s.in3 = Trest;
        s.out0 = exc;
        s.out1 = inc;
        s.n = n0;
        s.I = M;
        s.Q = Q;
        if (coop) {
            // boxes of 17 to 64 along axis 0: lanes share a point
            const i64 C = 64 / coop_g(kb, (int)sizeof(T), true);
            const i64 groups = (M + C - 1) / C;
            s.cb = coop_run_blocks(groups, Q);
            s.nchunks = (Q + s.cb - 1) / s.cb;
            s.ntasks = groups * s.nchunks * 64;
            push(s, kb);
            return;
        }
        i64 nseg = (cfg.min_tasks + M - 1) / M;
        if (nseg > Q) nseg = Q;
        if (nseg < 1) nseg = 1;
        s.cb = (Q + nseg - 1) / nseg;
        s.nchunks = (Q + s.cb - 1) / s.cb;
        s.ntasks = M * s.nchunks;
        push(s, kb);
    }
    // blocks per run of a split-block step: runs enough for min_tasks threads
    i64 coop_run_blocks(i64 groups, i64 nb) const {
        i64 runs = (cfg.min_tasks + 64 * groups - 1) / (64 * groups);
        if (runs > nb) runs = nb;
        if (runs < 1) runs = 1;
        return (nb + runs - 1) / runs;
    }
    void plane_axis0(const T*, const T*, const T*, const T*, T*, T*, i64, i64, i64, i64, i64, i64,
                     i64, i64) {}
    void plane_bdbs(const T*, T*, i64, i64, i64, i64, i64) {}
    void plane_scan(const T*, const T*, T*, T*, T*, T*, i64, i64, i64, i64, i64, i64, i64) {}
    bool tail_ok(i64, i64, i64) const { return false; }
    void tail_scan(const T*, T*, T*, T*, i64, i64, i64, i64) {}
};

template <typename T, class Op>
static exs_status plan_into(const exs_job* job, Arena& ar, std::vector<Rec>* out,
                            const TuneCfg& cfg) {
    ListSink<T, Op> sink{out, job->dtype, job->op, cfg};
    return plan_job<T>(job, ar, sink);
}

template <typename T>
static exs_status plan_op(const exs_job* job, Arena& ar, std::vector<Rec>* out,
                          const TuneCfg& cfg) {
    if (job->op == EXS_SUM) return plan_into<T, OpSum>(job, ar, out, cfg);
    if (job->op == EXS_MAX) return plan_into<T, OpMax>(job, ar, out, cfg);
    return plan_into<T, OpMin>(job, ar, out, cfg);
}

static exs_status plan_any(const exs_job* job, Arena& ar, std::vector<Rec>* out,
                           const TuneCfg& cfg) {
    switch (job->dtype) {
        case EXS_F32: return plan_op<float>(job, ar, out, cfg);
        case EXS_F64: return plan_op<double>(job, ar, out, cfg);
        case EXS_I32: return plan_op<int>(job, ar, out, cfg);
        case EXS_I64: return plan_op<long long>(job, ar, out, cfg);
    }
    return set_error(EXS_EINVAL, "unknown dtype");
}

struct Launch {
    int es, kind, kb;  // element size, step kind, register bucket
    WlParts parts;     // (type, operator) parts: codes and chunk ranges
    size_t first;  // index of the first step in the device array
    int nsteps;
    size_t table;  // offset of its chunk table (task table for row tasks)
    i64 units;     // chunks of WL_CHUNK tasks (tasks, for row tasks)
    size_t lds;    // dynamic LDS bytes per workgroup (row tasks)
};

}  // namespace exs

using namespace exs;

struct exs_batch {
    std::vector<exs_job> jobs;
    std::vector<size_t> ws_off;
    size_t ws_total = 0;
    TuneCfg cfg;
    int num_cu = 256;
    // built for one workspace
    void* ws_base = nullptr;
    std::vector<std::vector<Launch>> phases;
    Step* dev_steps = nullptr;
    size_t dev_cap = 0;
    int* dev_table = nullptr;  // per launch: the step of every chunk (or row task)
    size_t table_cap = 0;
    i64 items = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_nodes = 0;
};

namespace exs {

static void drop_graph(exs_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_nodes = 0;
}

// Record every job's steps for workspace `ws`, group them into phases and
// upload the step array.
static exs_status build(exs_batch* b, void* ws, const TuneCfg& cfg) {
    std::vector<std::vector<Rec>> recs(b->jobs.size());
    size_t maxlen = 0;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        Arena ar;
        ar.dry = false;
        ar.base = (char*)ws + b->ws_off[j];
        exs_status s = plan_any(&b->jobs[j], ar, &recs[j], cfg);
        if (s != EXS_OK) return s;
        maxlen = std::max(maxlen, recs[j].size());
    }
    std::vector<Step> all;
    std::vector<int> table;
    b->phases.assign(maxlen, {});
    b->items = 0;
    for (size_t p = 0; p < maxlen; ++p) {
        // one launch per (element size, kind, register bucket): the steps
        // carry their element type and operator
        std::map<std::tuple<int, int, int>, std::vector<const Rec*>> groups;
        for (auto& r : recs)
            if (p < r.size())
                groups[std::make_tuple((int)dtype_size(r[p].dtype), r[p].s.kind, r[p].kb)]
                    .push_back(&r[p]);
        for (auto& g : groups) {
            // parts of one (type, operator) each, in code order
            std::stable_sort(g.second.begin(), g.second.end(), [](const Rec* a, const Rec* b) {
                return a->dtype * 4 + a->op < b->dtype * 4 + b->op;
            });
            Launch L;
            L.es = std::get<0>(g.first);
            L.kind = std::get<1>(g.first);
            L.kb = std::get<2>(g.first);
            L.parts = WlParts{};
            L.first = all.size();
            L.nsteps = (int)g.second.size();
            L.table = table.size();
            // row tasks: one table entry per task; other kinds: every step
            // starts at a chunk boundary and each chunk names its step
            const bool rows = L.kind == SK_BDBSR;
            i64 tb = 0;
            L.lds = 0;
            for (const Rec* r : g.second) {
                Step s = r->s;
                const int code = r->dtype * 4 + r->op;
                WlParts& P = L.parts;
                if (P.n == 0 || P.code[P.n - 1] != code) {
                    if (P.n == WL_MAX_PARTS)
                        return set_error(EXS_EINVAL, "too many (type, operator) parts in a launch");
                    P.code[P.n] = code;
                    P.unit0[P.n] = rows ? tb : tb / WL_CHUNK;
                    ++P.n;
                }
                s.task_begin = tb;
                const i64 span = rows ? s.ntasks : (s.ntasks + WL_CHUNK - 1) / WL_CHUNK * WL_CHUNK;
                tb += span;
                const int local = (int)(all.size() - L.first);
                for (i64 u = 0; u < (rows ? span : span / WL_CHUNK); ++u) table.push_back(local);
                all.push_back(s);
                if (rows)
                    L.lds = std::max(L.lds, (size_t)rows_per_task(s.k) * rows_pitch(s.cb, s.k) *
                                                (size_t)L.es);
            }
            L.units = rows ? tb : tb / WL_CHUNK;
            L.parts.unit0[L.parts.n] = L.units;
            b->items += (i64)g.second.size();
            b->phases[p].push_back(L);
        }
    }
    // the tables are rewritten in place: earlier launches of this batch, on
    // any stream, must be done with them
    if ((b->dev_steps || b->dev_table) && hipDeviceSynchronize() != hipSuccess)
        return set_error(EXS_EDEVICE, "hipDeviceSynchronize failed before rewriting the tables");
    const size_t bytes = all.size() * sizeof(Step);
    if (bytes > b->dev_cap) {
        if (b->dev_steps) (void)hipFree(b->dev_steps);
        b->dev_steps = nullptr;
        b->dev_cap = 0;
        if (hipMalloc(&b->dev_steps, bytes) != hipSuccess)
            return set_error(EXS_ENOMEM, "cannot allocate the batch step table");
        b->dev_cap = bytes;
    }
    if (bytes && hipMemcpy(b->dev_steps, all.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(EXS_EDEVICE, "cannot upload the batch step table");
    const size_t tbytes = table.size() * sizeof(int);
    if (tbytes > b->table_cap) {
        if (b->dev_table) (void)hipFree(b->dev_table);
        b->dev_table = nullptr;
        b->table_cap = 0;
        if (hipMalloc(&b->dev_table, tbytes) != hipSuccess)
            return set_error(EXS_ENOMEM, "cannot allocate the batch chunk table");
        b->table_cap = tbytes;
    }
    if (tbytes && hipMemcpy(b->dev_table, table.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(EXS_EDEVICE, "cannot upload the batch chunk table");
    b->ws_base = ws;
    return EXS_OK;
}

static void enqueue(exs_batch* b, const TuneCfg& cfg, hipStream_t st) {
    const i64 cap = (i64)cfg.wg_per_cu * b->num_cu;
    for (auto& ph : b->phases)
        for (auto& L : ph) {
            // one chunk (one row task) per workgroup at a time
            i64 g = L.kind == SK_BDBSR ? (L.units < 4 * cap ? L.units : 4 * cap)
                                       : (L.units < cap ? L.units : cap);
            if (g < 1) g = 1;
            // the workgroups split over the parts by their chunk counts (at
            // least one each, never more than a part has chunks)
            WlParts& P = L.parts;
            P.wg0[0] = 0;
            for (int i = 0; i < P.n; ++i) {
                const i64 u = P.unit0[i + 1] - P.unit0[i];
                i64 w = L.units > 0 ? g * u / L.units : 1;
                if (w < 1) w = 1;
                if (w > u && u > 0) w = u;
                P.wg0[i + 1] = P.wg0[i] + (int)w;
            }
            launch_worklist(L.es, L.kind, L.kb, b->dev_steps + L.first, b->dev_table + L.table, P,
                            L.lds, st);
        }
}

// ---------------------------------------------------------------------------
// Autotune cache (format and parser in exsum_tunecache.hpp)
// ---------------------------------------------------------------------------
static std::string signature(const std::vector<exs_job>& jobs) {
    uint64_t h = 1469598103934665603ULL;  // FNV-1a over the shape description
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ULL;
        }
    };
    for (auto& j : jobs) {
        mix(j.d);
        mix(j.dtype);
        mix(j.op);
        mix(j.mode);
        for (int i = 0; i < j.d; ++i) {
            mix(j.dims[i]);
            mix(j.box[i]);
        }
    }
    char buf[40];
    std::snprintf(buf, sizeof(buf), "batch-%016llx-n%zu", (unsigned long long)h, jobs.size());
    return buf;
}

// Cache file state: absent, a valid cache (entries read), or something else
// (then it is neither used nor overwritten).
enum class CacheFile { ABSENT, OK, FOREIGN };

static CacheFile read_cache(const char* path, tunecache::Entries* m) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return CacheFile::ABSENT;
    std::stringstream ss;
    ss << f.rdbuf();
    return tunecache::parse(ss.str(), m) ? CacheFile::OK : CacheFile::FOREIGN;
}

static void write_cache(const char* path, const tunecache::Entries& m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f << tunecache::render(m);
        if (!f) return;
    }
    std::rename(tmp.c_str(), path);
}

static exs_status autotune(exs_batch* b, const char* path) {
    const std::string sig = signature(b->jobs);
    tunecache::Entries cache;
    const CacheFile state = read_cache(path, &cache);
    auto it = cache.find(sig);
    if (it != cache.end()) {
        auto mt = it->second.find("min_tasks"), wg = it->second.find("wg_per_cu");
        // only values the tuner itself can choose are taken
        if (mt != it->second.end() && wg != it->second.end() && mt->second >= 1 &&
            mt->second <= (double)(1 << 30) && wg->second >= 1 && wg->second <= 64) {
            b->cfg.min_tasks = (i64)mt->second;
            b->cfg.wg_per_cu = (int)wg->second;
            return EXS_OK;
        }
    }
    // the tuning runs read the jobs' inputs on a stream of its own: whatever
    // the caller enqueued to produce them must be complete first
    if (hipDeviceSynchronize() != hipSuccess)
        return set_error(EXS_EDEVICE, "hipDeviceSynchronize failed before autotuning");
    void* ws = nullptr;
    if (b->ws_total && hipMalloc(&ws, b->ws_total) != hipSuccess)
        return set_error(EXS_ENOMEM, "cannot allocate the autotuning workspace");
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) {
        if (ws) (void)hipFree(ws);
        return set_error(EXS_EDEVICE, "hipStreamCreate failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipStreamDestroy(st);
        if (ws) (void)hipFree(ws);
        return set_error(EXS_EDEVICE, "hipEventCreate failed");
    }
    const i64 mts[] = {4096, 16384, 65536};
    const int wgs[] = {2, 4, 8};
    TuneCfg best = b->cfg;
    float best_ms = 1e30f;
    exs_status rc = EXS_OK;
    for (i64 mt : mts)
        for (int wg : wgs) {
            TuneCfg c;
            c.min_tasks = mt;
            c.wg_per_cu = wg;
            rc = build(b, ws, c);
            if (rc != EXS_OK) break;
            enqueue(b, c, st);  // warm-up
            bool ok = hipEventRecord(e0, st) == hipSuccess;
            for (int r = 0; r < 3; ++r) enqueue(b, c, st);
            ok = ok && hipEventRecord(e1, st) == hipSuccess;
            float ms = 0.f;
            if (!ok || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = set_error(EXS_EDEVICE, "autotuning run failed");
                break;
            }
            ms /= 3.f;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (ws) (void)hipFree(ws);
    b->ws_base = nullptr;  // the tuning build pointed into the freed workspace
    if (rc != EXS_OK) return rc;
    b->cfg = best;
    if (state != CacheFile::FOREIGN) {
        cache[sig] = {{"min_tasks", (double)best.min_tasks},
                      {"wg_per_cu", (double)best.wg_per_cu},
                      {"ms", (double)best_ms}};
        write_cache(path, cache);
    }
    return EXS_OK;
}

}  // namespace exs

extern "C" {

exs_status exs_batch_create(const exs_job* jobs, int32_t n, const char* tune_cache,
                            exs_batch** out) {
    if (!out) return set_error(EXS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !jobs) return set_error(EXS_EINVAL, "a batch needs at least one job");
    exs_batch* b = new (std::nothrow) exs_batch();
    if (!b) return set_error(EXS_ENOMEM, "out of host memory");
    b->jobs.assign(jobs, jobs + n);
    size_t off = 0;
    for (int j = 0; j < n; ++j) {
        exs_status s = validate_job(&b->jobs[j], true);
        if (s == EXS_OK && (b->jobs[j].mode & EXS_WEAK))
            s = set_error(EXS_EUNSUPPORTED, "weak excluded sums are not batched");
        if (s == EXS_OK && b->jobs[j].dtype == EXS_VALIDX)
            s = set_error(EXS_EUNSUPPORTED, "(value, index) pairs are not batched");
        if (s != EXS_OK) {
            delete b;
            return set_error(s, "job " + std::to_string(j) + ": " + exs_last_error());
        }
        Arena ar;
        ar.dry = true;
        std::vector<Rec> none;
        s = plan_any(&b->jobs[j], ar, &none, b->cfg);
        if (s != EXS_OK) {
            delete b;
            return s;
        }
        b->ws_off.push_back(off);
        off += (ar.off + 255) & ~(size_t)255;
    }
    b->ws_total = off;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cu > 0)
            b->num_cu = cu;
    }
    if (tune_cache) {
        exs_status s = autotune(b, tune_cache);
        if (s != EXS_OK) {
            exs_batch_destroy(b);
            return s;
        }
    }
    *out = b;
    return EXS_OK;
}

exs_status exs_batch_workspace_size(const exs_batch* b, size_t* bytes) {
    if (!b || !bytes) return set_error(EXS_EINVAL, "NULL argument");
    *bytes = b->ws_total;
    return EXS_OK;
}

static exs_status check_ws(exs_batch* b, void* ws, size_t ws_bytes) {
    if (ws_bytes < b->ws_total)
        return set_error(EXS_ENOMEM, "batch workspace too small: need " +
                                         std::to_string(b->ws_total) + " bytes");
    if (b->ws_total && !ws) return set_error(EXS_EINVAL, "ws is NULL");
    if (((uintptr_t)ws & 255) != 0) return set_error(EXS_EINVAL, "ws must be 256-byte aligned");
    if (ws != b->ws_base || b->phases.empty()) {
        drop_graph(b);
        exs_status s = build(b, ws, b->cfg);
        if (s != EXS_OK) return s;
    }
    return EXS_OK;
}

exs_status exs_batch_launch_eager(exs_batch* b, void* ws, size_t ws_bytes, void* stream) {
    if (!b) return set_error(EXS_EINVAL, "batch is NULL");
    exs_status s = check_ws(b, ws, ws_bytes);
    if (s != EXS_OK) return s;
    enqueue(b, b->cfg, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(EXS_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
    return EXS_OK;
}

exs_status exs_batch_launch(exs_batch* b, void* ws, size_t ws_bytes, void* stream) {
    if (!b) return set_error(EXS_EINVAL, "batch is NULL");
    exs_status s = check_ws(b, ws, ws_bytes);
    if (s != EXS_OK) return s;
    if (!b->exec) {
        if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return set_error(EXS_EDEVICE, "hipStreamCreate failed");
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return set_error(EXS_EDEVICE, "hipStreamBeginCapture failed");
        enqueue(b, b->cfg, b->cap_stream);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(b->cap_stream, &g) != hipSuccess || !g)
            return set_error(EXS_EDEVICE, "hipStreamEndCapture failed");
        b->graph = g;
        size_t nn = 0;
        if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess) b->graph_nodes = (int)nn;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            return set_error(EXS_EDEVICE, "hipGraphInstantiate failed");
        }
    }
    if (hipGraphLaunch(b->exec, (hipStream_t)stream) != hipSuccess)
        return set_error(EXS_EDEVICE, "hipGraphLaunch failed");
    return EXS_OK;
}

exs_status exs_batch_info(const exs_batch* b, int32_t* graph_nodes, int64_t* work_items) {
    if (!b) return set_error(EXS_EINVAL, "batch is NULL");
    if (graph_nodes) *graph_nodes = b->graph_nodes;
    if (work_items) *work_items = b->items;
    return EXS_OK;
}

void exs_batch_destroy(exs_batch* b) {
    if (!b) return;
    drop_graph(b);
    if (b->dev_steps) (void)hipFree(b->dev_steps);
    if (b->dev_table) (void)hipFree(b->dev_table);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

}  // extern "C"
