// batched.cpp -- many uneven GEMMs in one launch.
//
// Persistent mode: the host cuts every GEMM of the batch into output tiles
// (of the configured shape, or 64 x 64 for GEMMs too small for it), estimates
// each tile's cost from its shape and K depth, and packs the tiles into one
// bin per resident workgroup with the longest-processing-time-first rule
// (largest tile to the currently least-loaded bin).  With a direct-to-LDS
// tile, one copy kernel first packs the operands into aligned, zero-padded
// buffers (one launch for the whole batch).  The device then runs one
// grid of exactly that many workgroups; workgroup b walks its own task range,
// so there is no device-side queue, counter or reset.  Every tile runs the
// same code as a plain launch of its tile shape with split_k = 1, so results
// equal per-GEMM launches of that shape bit for bit.
//
// Each GEMM may have its own tile configuration: in persistent mode the GEMMs
// are grouped by kernel and each group is one persistent launch.
//
// Graph mode: the launch(es) are captured once into a hipGraph on a private
// stream and replayed on the caller's stream; the graph and its device task
// lists are cached per (descriptors, configurations, flags), at most 16
// batches (least recently used freed first), and freed by mlk_release().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mlk {

namespace {

struct Plan {
    // GemmArgs[count] | Task[ntasks] | int32 bounds[nblk + 1] | PackJob[njobs] |
    // int64 seg_start[njobs + 1] | packed operands
    void* dev = nullptr;
    GemmArgs* gemms = nullptr;
    Task* tasks = nullptr;
    int32_t* bounds = nullptr;
    int nblk = 0;
    PackJob* jobs = nullptr;
    int64_t* seg_start = nullptr;
    int njobs = 0;
    int64_t pack_segs = 0;
    int esize = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

void free_plan(Plan& p) {
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.dev) (void)hipFree(p.dev);
    p = Plan();
}

// The GEMMs of a batch whose configurations share one compiled kernel: in
// persistent mode each group is one persistent launch over the whole device,
// the groups launched one after another on the stream.
struct Group {
    const KernelEntry* e = nullptr;
    mlk_tile_config c{};
    std::vector<int64_t> idx;  // the group's GEMMs (indices into the batch)
    Plan plan;
};

struct BatchPlan {
    std::vector<Group> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* ws = nullptr;  // graph of per-GEMM launches: their packing workspace (one GEMM at a time)
    size_t ws_bytes = 0;
};

void free_batch(BatchPlan& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    for (Group& g : b.groups) free_plan(g.plan);
    if (b.ws) (void)hipFree(b.ws);
    b = BatchPlan();
}

std::mutex g_mu;
std::map<std::string, BatchPlan> g_plans;
std::map<int, hipStream_t> g_capture_streams;
// Cached batches (each holds device task lists and packed operand copies) are
// kept up to this many; the least recently used one is freed beyond it.
constexpr size_t kMaxCachedBatches = 16;
std::vector<std::string> g_lru;  // keys, least recently used first

void touch(const std::string& key) {
    auto it = std::find(g_lru.begin(), g_lru.end(), key);
    if (it != g_lru.end()) g_lru.erase(it);
    g_lru.push_back(key);
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

std::string plan_key(int dt, int64_t count, const mlk_gemm_desc* d, const std::vector<mlk_tile_config>& cf,
                     int accumulate, uint32_t flags, int device) {
    std::string k;
    k.append((const char*)&dt, sizeof dt);
    k.append((const char*)&accumulate, sizeof accumulate);
    k.append((const char*)&flags, sizeof flags);
    k.append((const char*)&device, sizeof device);
    k.append((const char*)cf.data(), sizeof(mlk_tile_config) * cf.size());
    k.append((const char*)d, sizeof(mlk_gemm_desc) * (size_t)count);
    return k;
}

GemmArgs args_for(int dt, const mlk_gemm_desc& d, const mlk_tile_config& c, int accumulate) {
    GemmArgs g;
    memset(&g, 0, sizeof g);
    const int es = dt == DT_F32 ? 4 : dt == DT_BF16 ? 2 : 1;
    g.M = d.M;
    g.N = d.N;
    g.K = d.K;
    g.A = d.A;
    g.lda = d.lda;
    g.B = d.B;
    g.ldb = d.ldb;
    g.C = d.C;
    g.ldc = d.ldc;
    g.accumulate = accumulate;
    g.atomic = 0;
    g.split_k = 1;
    g.vec_a = ((uintptr_t)d.A % 16 == 0) && ((d.lda * es) % 16 == 0);
    g.vec_b = ((uintptr_t)d.B % 16 == 0) && ((d.ldb * es) % 16 == 0);
    g.tiles_m = (int32_t)cdiv(d.M, c.bm);
    g.tiles_n = (int32_t)cdiv(d.N, c.bn);
    g.group_m = 1;
    g.xcd_remap = 0;
    return g;
}

// Workgroups of the persistent kernel that are resident on the device at once
// (the runtime's occupancy for its registers, LDS and waves): one bin each.
int resident_blocks(const KernelEntry* e, int cus) {
    return cus * (e->occupancy ? e->occupancy() : 1);
}

int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Build the LPT schedule on the host and upload it.  For a direct-to-LDS tile
// every operand that is not already in its form (16-byte rows, K a multiple of
// the stage depth; for B also N a multiple of 16 bytes) gets a zero-padded copy: A as M x Kp, B as Kp x Np, with Kp
// K rounded up to the stage depth and Np N rounded up to 16 bytes.  The padded
// K columns of A and rows of B are zero, so they add nothing.
mlk_status build_plan(int dt, int64_t count, const mlk_gemm_desc* d, const KernelEntry* e,
                      const mlk_tile_config& c, int accumulate, Plan* plan) {
    std::vector<GemmArgs> gemms((size_t)count);
    const int es = dt == DT_F32 ? 4 : dt == DT_BF16 ? 2 : 1;
    const bool pack = e->stages >= 2;
    std::vector<PackJob> jobs;
    std::vector<int64_t> dst_off;  // byte offset of each job's block in the packed area
    int64_t packed_bytes = 0;
    struct Fix {
        int64_t gemm;
        int which;  // 0: A, 1: B
        int64_t job;
    };
    std::vector<Fix> fixes;
    struct T {
        double cost;
        Task t;
    };
    std::vector<T> all;
    // A register-staged kernel whose configured tile has 4 waves also carries
    // a 64 x 64 tile;
    // each GEMM takes the shape with the smaller estimated time: padded tile
    // work plus a fixed prologue / epilogue of about two K stages, with the
    // small tile's stages taken as 1.5x less efficient per flop.
    const bool pair = e->stages == 0 && e->threads == 256 && !(c.bm == 64 && c.bn == 64);
    const int sbk = dt == DT_F32 ? 32 : 64;
    for (int64_t i = 0; i < count; ++i) {
        gemms[i] = args_for(dt, d[i], c, accumulate);
        if (d[i].M == 0 || d[i].N == 0) continue;
        if (pack && d[i].K > 0) {
            GemmArgs& g = gemms[i];
            const int64_t Kp = round_up(d[i].K, e->bk), Np = round_up(d[i].N, 16 / es);
            const bool kfit = d[i].K % e->bk == 0;
            if (!(kfit && g.vec_a)) {
                jobs.push_back(PackJob{d[i].A, nullptr, d[i].lda, Kp, (int32_t)d[i].M, (int32_t)d[i].K,
                                       (int32_t)d[i].M, 0});
                dst_off.push_back(packed_bytes);
                packed_bytes += round_up(d[i].M * Kp * es, 256);
                fixes.push_back(Fix{i, 0, (int64_t)jobs.size() - 1});
                g.lda = Kp;
            }
            // B is read in whole 16-byte chunks up to its last row's padded end
            if (!(kfit && g.vec_b && d[i].N % (16 / es) == 0)) {
                jobs.push_back(PackJob{d[i].B, nullptr, d[i].ldb, Np, (int32_t)d[i].K, (int32_t)d[i].N,
                                       (int32_t)Kp, 0});
                dst_off.push_back(packed_bytes);
                packed_bytes += round_up(Kp * Np * es, 256);
                fixes.push_back(Fix{i, 1, (int64_t)jobs.size() - 1});
                g.ldb = Np;
            }
            g.K = Kp;
            g.vec_a = g.vec_b = 1;
            if (((d[i].M - 1) * g.lda + Kp) * es >= ((int64_t)1 << 31) ||
                ((Kp - 1) * g.ldb + d[i].N) * es >= ((int64_t)1 << 31))
                return fail(MLK_ERR_CONFIG, "batched: operand of desc %lld exceeds 2 GiB for a direct-to-LDS tile",
                            (long long)i);
        }
        const int64_t K = std::max<int64_t>(d[i].K, 1);
        const int64_t tb = cdiv(d[i].M, c.bm) * cdiv(d[i].N, c.bn);
        const double cost_big = (double)(cdiv(K, c.bk) + 2) * c.bm * c.bn * c.bk;
        const int64_t ts = cdiv(d[i].M, 64) * cdiv(d[i].N, 64);
        const double cost_small = 1.5 * (double)(cdiv(K, sbk) + 2) * 64 * 64 * sbk;
        const bool small = pair && ts * cost_small < tb * cost_big;
        const int bm = small ? 64 : c.bm, bn = small ? 64 : c.bn;
        const double unit = small ? cost_small : cost_big;
        for (int32_t tm = 0; tm < (int32_t)cdiv(d[i].M, bm); ++tm)
            for (int32_t tn = 0; tn < (int32_t)cdiv(d[i].N, bn); ++tn)
                all.push_back(T{unit, Task{(int32_t)i, tm, tn, small ? 1 : 0}});
    }
    const int cus = device_cus();
    int nblk = resident_blocks(e, cus);
    if ((int64_t)nblk > (int64_t)all.size()) nblk = std::max<int>(1, (int)all.size());
    std::vector<std::vector<Task>> bins((size_t)nblk);
    // Two-level longest-processing-time-first.  Workgroup b runs on XCD b % 8
    // (workgroups are dealt to the eight XCDs in turn), and each XCD has its
    // own L2: so whole GEMMs -- or, for a GEMM heavier than a quarter of an
    // XCD's share, bands of consecutive tile rows, which share A's row panels
    // -- are first dealt to the XCDs, largest first to the least-loaded one;
    // then each XCD's tiles go to its own workgroups, largest first to the
    // least-loaded one.
    const int nx = nblk >= 8 && nblk % 8 == 0 ? 8 : 1;
    double work = 0.0;
    for (const T& x : all) work += x.cost;
    const double cap = work / (4.0 * nx);
    struct Unit {
        double cost;
        std::vector<int64_t> tiles;  // indices into `all`
    };
    std::vector<Unit> units;
    for (size_t a = 0; a < all.size();) {
        // `all` holds each GEMM's tiles together, row by row
        size_t z = a;
        double gc = 0.0;
        while (z < all.size() && all[z].t.gemm == all[a].t.gemm) gc += all[z++].cost;
        const int32_t rows = all[z - 1].t.tm + 1;
        const int32_t band = gc <= cap ? rows : std::max<int32_t>(1, (int32_t)std::floor(rows * cap / gc));
        for (size_t k = a; k < z; ++k) {
            if (k == a || all[k].t.tm / band != all[k - 1].t.tm / band) units.push_back(Unit{0.0, {}});
            units.back().cost += all[k].cost;
            units.back().tiles.push_back((int64_t)k);
        }
        a = z;
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit& u, const Unit& v) { return u.cost > v.cost; });
    typedef std::pair<double, int> LB;  // (load, index), smallest load on top
    std::priority_queue<LB, std::vector<LB>, std::greater<LB>> xh;
    for (int x = 0; x < nx; ++x) xh.push(LB(0.0, x));
    std::vector<std::vector<int64_t>> per_x((size_t)nx);
    for (const Unit& u : units) {
        LB top = xh.top();
        xh.pop();
        per_x[top.second].insert(per_x[top.second].end(), u.tiles.begin(), u.tiles.end());
        xh.push(LB(top.first + u.cost, top.second));
    }
    for (int x = 0; x < nx; ++x) {
        std::vector<int64_t>& tl = per_x[x];
        std::stable_sort(tl.begin(), tl.end(), [&](int64_t u, int64_t v) { return all[u].cost > all[v].cost; });
        std::priority_queue<LB, std::vector<LB>, std::greater<LB>> heap;
        for (int b = x; b < nblk; b += nx) heap.push(LB(0.0, b));
        for (int64_t k : tl) {
            LB top = heap.top();
            heap.pop();
            bins[top.second].push_back(all[k].t);
            heap.push(LB(top.first + all[k].cost, top.second));
        }
    }
    std::vector<Task> tasks;
    std::vector<int32_t> bounds((size_t)nblk + 1, 0);
    for (int b = 0; b < nblk; ++b) {
        bounds[b] = (int32_t)tasks.size();
        tasks.insert(tasks.end(), bins[b].begin(), bins[b].end());
    }
    bounds[nblk] = (int32_t)tasks.size();

    // pack job table: destination segments counted over all jobs
    std::vector<int64_t> seg_start(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j) seg_start[j + 1] = seg_start[j] + pack_segments(jobs[j]);

    const size_t gb = sizeof(GemmArgs) * gemms.size();
    const size_t tb = sizeof(Task) * std::max<size_t>(tasks.size(), 1);
    const size_t bb = sizeof(int32_t) * bounds.size();
    const size_t jb = sizeof(PackJob) * jobs.size();
    const size_t rb = sizeof(int64_t) * seg_start.size();
    const size_t head = (size_t)round_up((int64_t)(gb + tb + bb + jb + rb), 256);
    const size_t total = head + (size_t)packed_bytes;
    void* dev = nullptr;
    hipError_t err = hipMalloc(&dev, total);
    if (err != hipSuccess) return hip_fail(err, "batched plan allocation");
    char* base = (char*)dev;
    for (size_t j = 0; j < jobs.size(); ++j) jobs[j].dst = base + head + dst_off[j];
    for (const Fix& f : fixes) {
        if (f.which == 0) gemms[f.gemm].A = jobs[f.job].dst;
        else gemms[f.gemm].B = jobs[f.job].dst;
    }
    std::vector<char> host(head, 0);
    memcpy(host.data(), gemms.data(), gb);
    if (!tasks.empty()) memcpy(host.data() + gb, tasks.data(), sizeof(Task) * tasks.size());
    memcpy(host.data() + gb + tb, bounds.data(), bb);
    if (!jobs.empty()) memcpy(host.data() + gb + tb + bb, jobs.data(), jb);
    memcpy(host.data() + gb + tb + bb + jb, seg_start.data(), rb);
    err = hipMemcpy(dev, host.data(), head, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(err, "batched plan upload");
    }
    plan->dev = dev;
    plan->gemms = (GemmArgs*)base;
    plan->tasks = (Task*)(base + gb);
    plan->bounds = (int32_t*)(base + gb + tb);
    plan->nblk = nblk;
    plan->jobs = (PackJob*)(base + gb + tb + bb);
    plan->seg_start = (int64_t*)(base + gb + tb + bb + jb);
    plan->njobs = (int)jobs.size();
    plan->pack_segs = seg_start.back();
    plan->esize = es;
    return MLK_OK;
}

// One launch per GEMM, each with its own configuration, on the mlk_matmul path.
Shape gemm_shape(int dt, const mlk_gemm_desc& d, int accumulate) {
    Shape s;
    s.dt = dt;
    s.conv = 0;
    s.M = d.M;
    s.N = d.N;
    s.K = d.K;
    s.accumulate = accumulate;
    return s;
}

// ws: a workspace for the GEMMs' packed operand copies, used by one GEMM at a
// time (the launches are ordered on the stream); null = the library's scratch
mlk_status launch_each(int dt, int64_t count, const mlk_gemm_desc* d, const std::vector<mlk_tile_config>& cf,
                       int accumulate, hipStream_t st, void* ws = nullptr, size_t ws_bytes = 0) {
    for (int64_t i = 0; i < count; ++i) {
        Shape s;
        s.dt = dt;
        s.conv = 0;
        s.M = d[i].M;
        s.N = d[i].N;
        s.K = d[i].K;
        s.accumulate = accumulate;
        mlk_tile_config ci = cf[(size_t)i];
        const int64_t stages = cdiv(std::max<int64_t>(s.K, 1), ci.bk);
        if (ci.split_k > stages) ci.split_k = 1;
        mlk_status r = launch_dense(s, d[i].A, d[i].lda, d[i].B, d[i].ldb, d[i].C, d[i].ldc,
                                    nullptr, nullptr, ci, st, nullptr, ws, ws_bytes);
        if (r != MLK_OK) return r;
    }
    return MLK_OK;
}

// Every group's packing copy and persistent launch, in group order.
mlk_status launch_groups(BatchPlan& b, hipStream_t st) {
    for (Group& g : b.groups) {
        Plan& p = g.plan;
        if (p.nblk == 0) continue;
        hipError_t err = launch_pack(p.jobs, p.seg_start, p.njobs, p.pack_segs, p.esize, st);
        if (err != hipSuccess) return hip_fail(err, "operand packing");
        err = g.e->persist(p.gemms, p.tasks, p.bounds, p.nblk, st);
        if (err != hipSuccess) return hip_fail(err, "persistent launch");
    }
    return MLK_OK;
}

}  // namespace

}  // namespace mlk

using namespace mlk;

extern "C" {

mlk_status mlk_batched_matmul(mlk_dtype in, mlk_dtype out, int64_t count, const mlk_gemm_desc* descs,
                              const mlk_tile_config* cfgs, int64_t ncfgs, int accumulate, uint32_t flags,
                              void* stream) {
    clear_error();
    if (flags & ~(MLK_BATCH_PERSISTENT | MLK_BATCH_GRAPH))
        return fail(MLK_ERR_ARG, "batched: unknown flag bits 0x%x", flags);
    mlk_problem p;
    memset(&p, 0, sizeof p);
    p.op = MLK_OP_BATCHED;
    p.in = in;
    p.out = out;
    p.accumulate = accumulate ? 1 : 0;
    p.count = count;
    p.descs = descs;
    Shape s;
    mlk_status st = shape_of_problem(&p, &s);
    if (st != MLK_OK) return st;
    if (ncfgs != 0 && ncfgs != 1 && ncfgs != count)
        return fail(MLK_ERR_ARG, "batched: ncfgs must be 0, 1 or count (%lld), got %lld", (long long)count,
                    (long long)ncfgs);
    if (ncfgs > 0 && !cfgs) return fail(MLK_ERR_NULL, "batched: cfgs is NULL with ncfgs %lld", (long long)ncfgs);
    const int es = s.dt == DT_F32 ? 4 : s.dt == DT_BF16 ? 2 : 1;
    for (int64_t i = 0; i < count; ++i) {
        const mlk_gemm_desc& d = descs[i];
        if (d.M == 0 || d.N == 0) continue;
        if (!d.C || (d.K > 0 && (!d.A || !d.B)))
            return fail(MLK_ERR_NULL, "batched: NULL pointer in desc %lld", (long long)i);
        if (d.lda < std::max<int64_t>(d.K, 1) || d.ldb < std::max<int64_t>(d.N, 1) ||
            d.ldc < std::max<int64_t>(d.N, 1))
            return fail(MLK_ERR_LAYOUT, "batched: leading dimension too small in desc %lld", (long long)i);
        const uintptr_t c0 = (uintptr_t)d.C, c1 = c0 + (size_t)((d.M - 1) * d.ldc + d.N) * 4;
        const uintptr_t a0 = (uintptr_t)d.A, a1 = a0 + (size_t)((d.M - 1) * d.lda + d.K) * es;
        const uintptr_t b0 = (uintptr_t)d.B, b1 = b0 + (size_t)((d.K - 1) * d.ldb + d.N) * es;
        if (d.K > 0 && ((c0 < a1 && a0 < c1) || (c0 < b1 && b0 < c1)))
            return fail(MLK_ERR_LAYOUT, "batched: C overlaps A or B in desc %lld", (long long)i);
    }
    const bool persistent = (flags & MLK_BATCH_PERSISTENT) != 0;
    const bool graph = (flags & MLK_BATCH_GRAPH) != 0;
    auto zero = [](const mlk_tile_config& c) { return c.bm == 0 && c.bn == 0; };
    auto norm = [](mlk_tile_config c) {
        if (c.group_m == 0) c.group_m = 1;
        if (c.split_k == 0) c.split_k = 1;
        return c;
    };
    // the batch's own choice: its tuned configuration, else the heuristic
    mlk_tile_config batch_c;
    if (!lookup_default(problem_key(&p), &batch_c)) batch_c = heuristic_config(s, MLK_OP_BATCHED);
    // one configuration per GEMM
    std::vector<mlk_tile_config> cf((size_t)count, batch_c);
    if (ncfgs == 1 && !zero(cfgs[0])) {
        const mlk_tile_config c = norm(cfgs[0]);
        if ((st = check_config(s, MLK_OP_BATCHED, c)) != MLK_OK) return st;
        std::fill(cf.begin(), cf.end(), c);
    } else if (ncfgs == count) {
        for (int64_t i = 0; i < count; ++i) {
            mlk_problem q;
            memset(&q, 0, sizeof q);
            q.op = MLK_OP_MATMUL;
            q.in = in;
            q.out = out;
            q.accumulate = p.accumulate;
            q.M = descs[i].M;
            q.N = descs[i].N;
            q.K = descs[i].K;
            Shape si;
            if ((st = shape_of_problem(&q, &si)) != MLK_OK) return st;
            if (zero(cfgs[i])) {
                // a GEMM left to choose: its own tuned matmul configuration when the
                // launch mode can run it, else the batch's choice
                mlk_tile_config c;
                if (!persistent && lookup_default(problem_key(&q), &c)) cf[(size_t)i] = c;
                else if (!persistent) cf[(size_t)i] = heuristic_config(si, MLK_OP_MATMUL);
                continue;
            }
            const mlk_tile_config c = norm(cfgs[i]);
            if ((st = check_config(si, persistent ? MLK_OP_BATCHED : MLK_OP_MATMUL, c)) != MLK_OK)
                return fail(st, "batched: configuration of desc %lld: %s", (long long)i, mlk_last_error());
            cf[(size_t)i] = c;
        }
    }
    // kernels, and the direct-layout tiles' 32-bit output offsets
    for (int64_t i = 0; i < count; ++i) {
        const KernelEntry* e = find_kernel(s.dt, 0, cf[(size_t)i]);
        if (!e) return fail(MLK_ERR_CONFIG, "batched: no kernel for the configuration of desc %lld", (long long)i);
        if (persistent && !e->persist)
            return fail(MLK_ERR_CONFIG, "batched: tile %dx%dx%d (desc %lld) has no persistent variant", cf[i].bm,
                        cf[i].bn, cf[i].bk, (long long)i);
        if (e->stages >= 1 && (int64_t)(e->bm - 1) * descs[i].ldc + e->bn >= ((int64_t)1 << 31))
            return fail(MLK_ERR_CONFIG, "batched: ldc of desc %lld too large for a %d-row direct-layout tile",
                        (long long)i, e->bm);
    }
    hipStream_t user = (hipStream_t)stream;
    int dev = 0;
    hipError_t herr = hipGetDevice(&dev);
    if (herr != hipSuccess) return hip_fail(herr, "hipGetDevice");

    if (!persistent && !graph) return launch_each(s.dt, count, descs, cf, p.accumulate, user);
    std::lock_guard<std::mutex> g(g_mu);
    const std::string key = plan_key(s.dt, count, descs, cf, p.accumulate, flags, dev);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        BatchPlan bp;
        if (persistent) {
            // group the GEMMs by kernel, in order of first appearance
            for (int64_t i = 0; i < count; ++i) {
                const KernelEntry* e = find_kernel(s.dt, 0, cf[(size_t)i]);
                Group* gr = nullptr;
                for (Group& x : bp.groups)
                    if (x.e == e) gr = &x;
                if (!gr) {
                    bp.groups.push_back(Group());
                    gr = &bp.groups.back();
                    gr->e = e;
                    gr->c = cf[(size_t)i];
                }
                gr->idx.push_back(i);
            }
            for (Group& gr : bp.groups) {
                std::vector<mlk_gemm_desc> gd;
                for (int64_t i : gr.idx) gd.push_back(descs[i]);
                gr.plan.device = dev;
                if ((st = build_plan(s.dt, (int64_t)gd.size(), gd.data(), gr.e, gr.c, p.accumulate, &gr.plan)) !=
                    MLK_OK) {
                    free_batch(bp);
                    return st;
                }
            }
        }
        if (graph && !persistent) {
            // per-GEMM launches recorded into a graph take no scratch memory: the
            // batch owns one workspace for the largest packing any GEMM needs
            int64_t need = 0;
            for (int64_t i = 0; i < count; ++i)
                need = std::max(need, dense_workspace_bytes(gemm_shape(s.dt, descs[i], p.accumulate), descs[i].A,
                                                            descs[i].lda, descs[i].B, descs[i].ldb, cf[(size_t)i]));
            if (need > 0) {
                if ((herr = hipMalloc(&bp.ws, (size_t)need)) != hipSuccess) {
                    free_batch(bp);
                    return hip_fail(herr, "batched graph workspace");
                }
                bp.ws_bytes = (size_t)need;
            }
        }
        if (graph) {
            hipStream_t cap = nullptr;
            auto cs = g_capture_streams.find(dev);
            if (cs == g_capture_streams.end()) {
                herr = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
                if (herr != hipSuccess) {
                    free_batch(bp);
                    return hip_fail(herr, "capture stream");
                }
                g_capture_streams[dev] = cap;
            } else {
                cap = cs->second;
            }
            herr = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (herr != hipSuccess) {
                free_batch(bp);
                return hip_fail(herr, "hipStreamBeginCapture");
            }
            st = persistent ? launch_groups(bp, cap)
                            : launch_each(s.dt, count, descs, cf, p.accumulate, cap, bp.ws, bp.ws_bytes);
            hipGraph_t gr = nullptr;
            hipError_t endc = hipStreamEndCapture(cap, &gr);
            bp.graph = gr;
            if (st != MLK_OK) {
                free_batch(bp);
                return st;
            }
            if (endc != hipSuccess) {
                free_batch(bp);
                return hip_fail(endc, "hipStreamEndCapture");
            }
            herr = hipGraphInstantiate(&bp.exec, gr, nullptr, nullptr, 0);
            if (herr != hipSuccess) {
                free_batch(bp);
                return hip_fail(herr, "hipGraphInstantiate");
            }
        }
        // keep at most kMaxCachedBatches: free the least recently used (after
        // the device has finished with it)
        if (g_plans.size() >= kMaxCachedBatches && !g_lru.empty()) {
            auto old = g_plans.find(g_lru.front());
            if (old != g_plans.end()) {
                (void)hipDeviceSynchronize();
                free_batch(old->second);
                g_plans.erase(old);
            }
            g_lru.erase(g_lru.begin());
        }
        it = g_plans.emplace(key, std::move(bp)).first;
    }
    touch(key);
    BatchPlan& bp = it->second;
    if (graph) {
        herr = hipGraphLaunch(bp.exec, user);
        if (herr != hipSuccess) return hip_fail(herr, "hipGraphLaunch");
        return MLK_OK;
    }
    return launch_groups(bp, user);
}

void mlk_release(void) {
    std::lock_guard<std::mutex> g(g_mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : g_plans) free_batch(kv.second);
    g_plans.clear();
    g_lru.clear();
    for (auto& kv : g_capture_streams) (void)hipStreamDestroy(kv.second);
    g_capture_streams.clear();
    release_scratch();
}

}  // extern "C"
