// conv_batch.cpp -- many independent convolutions in one persistent launch.
//
// Every convolution of the batch (linalg.conv_2d_nchw_fchw, paper Sec. 4.1)
// is viewed as its implicit GEMM -- rows F, columns N*HO*WO, depth C*KH*KW --
// and cut into tasks of the register-loaded channel-gather conv tile: one
// output tile and one part of the convolution's K split.  The host estimates
// each task's time from its stage count, deals the tasks longest first into
// one range per resident workgroup of the persistent kernel (the least-loaded
// range takes the next task), and uploads convolutions, tasks and ranges once;
// a run is then one launch (plus, when y is overwritten, a zero fill of each
// split convolution's output).  Each task runs exactly the code of a plain
// launch's workgroup of the same tile, split and convolution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <vector>

#include "internal.hpp"

struct mlk_conv_batch {
    std::vector<mlk_conv_desc> d;
    std::vector<int32_t> split;   // per convolution
    const mlk::KernelEntry* e = nullptr;
    mlk_tile_config cfg{};
    int accumulate = 1;
    void* dev = nullptr;          // GemmArgs[count] | Task[ntasks] | int32 bounds[nblk + 1] | filters
    mlk::GemmArgs* convs = nullptr;
    mlk::Task* tasks = nullptr;
    int32_t* bounds = nullptr;
    std::vector<size_t> filter_off;  // byte offset of each transposed filter in dev (0: used in place)
    int64_t ntasks = 0;
    int nblk = 0;
    int device = 0;
};

namespace mlk {
namespace {

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up64(int64_t a, int64_t b) { return cdiv64(a, b) * b; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t x_bytes(const mlk_conv_desc& d) { return (size_t)(d.N * d.C * d.H * d.W) * 2; }
size_t w_bytes(const mlk_conv_desc& d) { return (size_t)(d.F * d.C * d.KH * d.KW) * 2; }
size_t y_bytes(const mlk_conv_desc& d) {
    return (size_t)(d.N * d.F * conv_out(d.H, d.KH, d.sh, d.ph) * conv_out(d.W, d.KW, d.sw, d.pw)) * 4;
}

// every filter larger than 1 x 1 into F x KH x KW x C, in the batch's buffer
mlk_status transpose_filters(const mlk_conv_batch* b, hipStream_t st) {
    for (size_t i = 0; i < b->d.size(); ++i) {
        const mlk_conv_desc& d = b->d[i];
        if (d.KH * d.KW == 1) continue;
        const hipError_t e = launch_transpose_pair(nullptr, nullptr, 0, 0, 0, d.w, (char*)b->dev + b->filter_off[i],
                                                   d.F, d.C, d.KH * d.KW, 2, st);
        if (e != hipSuccess) return hip_fail(e, "conv batch filter transpose");
    }
    return MLK_OK;
}

}  // namespace
}  // namespace mlk

using namespace mlk;

extern "C" {

mlk_status mlk_conv2d_batch_create(mlk_dtype in, mlk_dtype out, int64_t count, const mlk_conv_desc* descs,
                                   int accumulate, const mlk_tile_config* cfg, void* stream,
                                   mlk_conv_batch** batch) {
    clear_error();
    if (!batch) return fail(MLK_ERR_NULL, "conv batch: batch is NULL");
    *batch = nullptr;
    if (in != MLK_BF16 || out != MLK_F32)
        return fail(MLK_ERR_DTYPE, "conv batch: bf16 inputs and an fp32 output only");
    if (count < 1) return fail(MLK_ERR_ARG, "conv batch: count must be >= 1");
    if (!descs) return fail(MLK_ERR_NULL, "conv batch: descs is NULL");
    // the tile: a register-loaded conv tile with a persistent channel-gather form
    mlk_tile_config c{64, 64, 64, 2, 2, 16, 1, 0, 1, 3, 0};
    const bool choose = !cfg || (cfg->bm == 0 && cfg->bn == 0 && cfg->bk == 0 && cfg->wm == 0 && cfg->wn == 0 &&
                                 cfg->split_k == 0 && cfg->group_m == 0 && cfg->xcd_remap == 0 &&
                                 cfg->stages == 0 && cfg->layout == 0 && cfg->mfma == 0);
    if (!choose) {
        if (cfg->split_k < 1 || cfg->split_k > 32) return fail(MLK_ERR_CONFIG, "conv batch: split_k (the cap) in [1, 32]");
        if (cfg->stages != 1 || (cfg->layout != 3 && cfg->layout != 0) || cfg->xcd_remap != 0 ||
            cfg->group_m > 1 || (cfg->mfma != 0 && cfg->mfma != 16))
            return fail(MLK_ERR_CONFIG, "conv batch: a register-loaded tile (stages 1, layout 3, no raster options)");
        c = mlk_tile_config{cfg->bm, cfg->bn, 64, cfg->wm, cfg->wn, cfg->split_k, 1, 0, 1, 3, 0};
        if (cfg->bk != 0 && cfg->bk != 64) return fail(MLK_ERR_CONFIG, "conv batch: bk is 64 for bf16");
    }
    const KernelEntry* e = nullptr;
    for (const KernelEntry* k : registry())
        if (k->dt == DT_BF16 && k->conv && k->stages == 1 && k->persist_gather && k->bm == c.bm && k->bn == c.bn &&
            k->wm == c.wm && k->wn == c.wn)
            e = k;
    if (!e) return fail(MLK_ERR_CONFIG, "conv batch: no persistent channel-gather tile %dx%d (%dx%d waves)", c.bm,
                        c.bn, c.wm, c.wn);
    // every descriptor: a valid bf16 convolution with C a multiple of 8
    std::vector<Shape> shapes((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const mlk_conv_desc& d = descs[i];
        mlk_problem p;
        memset(&p, 0, sizeof p);
        p.op = MLK_OP_CONV2D;
        p.in = in;
        p.out = out;
        p.accumulate = accumulate ? 1 : 0;
        p.n = d.N;
        p.c = d.C;
        p.h = d.H;
        p.w = d.W;
        p.f = d.F;
        p.kh = d.KH;
        p.kw = d.KW;
        p.sh = d.sh;
        p.sw = d.sw;
        p.ph = d.ph;
        p.pw = d.pw;
        mlk_status st = shape_of_problem(&p, &shapes[(size_t)i]);
        if (st != MLK_OK) {
            const std::string why = mlk_last_error();
            return fail(st, "conv batch: descriptor %lld: %s", (long long)i, why.c_str());
        }
        if (d.C % 8 != 0 || d.F > 65535)
            return fail(MLK_ERR_SHAPE, "conv batch: descriptor %lld needs C a multiple of 8 and F <= 65535",
                        (long long)i);
        if (!d.x || !d.w || !d.y) return fail(MLK_ERR_NULL, "conv batch: NULL pointer in descriptor %lld", (long long)i);
    }
    for (int64_t i = 0; i < count; ++i)
        for (int64_t j = 0; j < count; ++j) {
            const mlk_conv_desc &a = descs[i], &b = descs[j];
            if (overlap(a.y, y_bytes(a), b.x, x_bytes(b)) || overlap(a.y, y_bytes(a), b.w, w_bytes(b)) ||
                (i != j && overlap(a.y, y_bytes(a), b.y, y_bytes(b))))
                return fail(MLK_ERR_LAYOUT, "conv batch: y of descriptor %lld overlaps an operand of descriptor %lld",
                            (long long)i, (long long)j);
        }
    const hipStream_t hs = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t err = hipStreamIsCapturing(hs, &cs);
    if (err != hipSuccess) return hip_fail(err, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(MLK_ERR_CONFIG, "conv batch: create batches outside stream capture (runs may be captured)");

    mlk_conv_batch* b = new mlk_conv_batch();
    b->d.assign(descs, descs + count);
    b->e = e;
    b->cfg = c;
    b->accumulate = accumulate ? 1 : 0;
    if ((err = hipGetDevice(&b->device)) != hipSuccess) {
        delete b;
        return hip_fail(err, "hipGetDevice");
    }
    // tasks: (tile, split part); cost ~ stages of the part plus a fixed two
    // for the prologue and the output
    struct T {
        double cost;
        Task t;
    };
    std::vector<T> all;
    std::vector<GemmArgs> convs((size_t)count);
    b->split.assign((size_t)count, 1);
    for (int64_t i = 0; i < count; ++i) {
        const Shape& s = shapes[(size_t)i];
        const mlk_conv_desc& d = descs[i];
        const int64_t stages = cdiv64(s.K, 64);
        const int sk = (int)std::max<int64_t>(1, std::min<int64_t>(c.split_k, cdiv64(stages, 4)));
        b->split[(size_t)i] = sk;
        GemmArgs& g = convs[(size_t)i];
        memset(&g, 0, sizeof g);
        g.M = s.M;
        g.N = s.N;
        g.K = s.K;
        g.B = d.x;
        g.C = d.y;
        g.accumulate = b->accumulate;
        g.split_k = sk;
        g.atomic = sk > 1 ? 1 : 0;
        g.tiles_m = (int32_t)cdiv64(s.M, c.bm);
        g.tiles_n = (int32_t)cdiv64(s.N, c.bn);
        g.group_m = 1;
        g.lda = d.C * d.KH * d.KW;
        g.cn = (int32_t)d.N;
        g.cc = (int32_t)d.C;
        g.ch = (int32_t)d.H;
        g.cw = (int32_t)d.W;
        g.ckh = (int32_t)d.KH;
        g.ckw = (int32_t)d.KW;
        g.csh = d.sh;
        g.csw = d.sw;
        g.cph = d.ph;
        g.cpw = d.pw;
        g.cho = (int32_t)conv_out(d.H, d.KH, d.sh, d.ph);
        g.cwo = (int32_t)conv_out(d.W, d.KW, d.sw, d.pw);
        const int64_t per = cdiv64(stages, sk);
        for (int kz = 0; kz < sk; ++kz) {
            const int64_t part = std::max<int64_t>(0, std::min<int64_t>(stages, (kz + 1) * per) - kz * per);
            if (part == 0) continue;  // e.g. 25 stages in 6 parts of 5: the last part has nothing to add
            for (int32_t tm = 0; tm < g.tiles_m; ++tm)
                for (int32_t tn = 0; tn < g.tiles_n; ++tn)
                    all.push_back(T{(double)(part + 2), Task{(int32_t)i, tm, tn, kz}});
        }
    }
    std::stable_sort(all.begin(), all.end(), [](const T& u, const T& v) { return u.cost > v.cost; });
    const int resident = device_cus() * (e->occupancy_gather ? e->occupancy_gather() : 1);
    int nblk = (int)std::min<int64_t>(resident, (int64_t)all.size());
    std::vector<std::vector<Task>> bins((size_t)nblk);
    typedef std::pair<double, int> LB;  // (load, bin), least loaded on top
    std::priority_queue<LB, std::vector<LB>, std::greater<LB>> heap;
    for (int k = 0; k < nblk; ++k) heap.push(LB(0.0, k));
    for (const T& x : all) {
        LB top = heap.top();
        heap.pop();
        bins[(size_t)top.second].push_back(x.t);
        heap.push(LB(top.first + x.cost, top.second));
    }
    std::vector<Task> tasks;
    std::vector<int32_t> bounds((size_t)nblk + 1, 0);
    for (int k = 0; k < nblk; ++k) {
        bounds[(size_t)k] = (int32_t)tasks.size();
        tasks.insert(tasks.end(), bins[(size_t)k].begin(), bins[(size_t)k].end());
    }
    bounds[(size_t)nblk] = (int32_t)tasks.size();
    // device buffer: arguments, tasks, ranges, then the transposed filters
    const size_t gb = sizeof(GemmArgs) * convs.size(), tb = sizeof(Task) * tasks.size(),
                 bb = sizeof(int32_t) * bounds.size();
    size_t off = (size_t)round_up64((int64_t)(gb + tb + bb), 256);
    b->filter_off.assign((size_t)count, 0);
    for (int64_t i = 0; i < count; ++i) {
        if (descs[i].KH * descs[i].KW == 1) continue;
        b->filter_off[(size_t)i] = off;
        off += (size_t)round_up64((int64_t)w_bytes(descs[i]), 256);
    }
    if ((err = hipMalloc(&b->dev, off)) != hipSuccess) {
        delete b;
        return hip_fail(err, "conv batch buffers");
    }
    char* base = (char*)b->dev;
    for (int64_t i = 0; i < count; ++i) {
        GemmArgs& g = convs[(size_t)i];
        g.A = descs[i].KH * descs[i].KW == 1 ? descs[i].w : (const void*)(base + b->filter_off[(size_t)i]);
        g.vec_a = (uintptr_t)g.A % 16 == 0 && (g.lda * 2) % 16 == 0;
    }
    std::vector<char> host(gb + tb + bb);
    memcpy(host.data(), convs.data(), gb);
    memcpy(host.data() + gb, tasks.data(), tb);
    memcpy(host.data() + gb + tb, bounds.data(), bb);
    err = hipMemcpyAsync(b->dev, host.data(), host.size(), hipMemcpyHostToDevice, hs);
    if (err == hipSuccess) err = hipStreamSynchronize(hs);
    if (err != hipSuccess) {
        mlk_conv2d_batch_destroy(b);
        return hip_fail(err, "conv batch upload");
    }
    b->convs = (GemmArgs*)base;
    b->tasks = (Task*)(base + gb);
    b->bounds = (int32_t*)(base + gb + tb);
    b->ntasks = (int64_t)tasks.size();
    b->nblk = nblk;
    mlk_status st = transpose_filters(b, hs);
    if (st != MLK_OK) {
        mlk_conv2d_batch_destroy(b);
        return st;
    }
    *batch = b;
    return MLK_OK;
}

mlk_status mlk_conv2d_batch_run(const mlk_conv_batch* b, void* stream) {
    clear_error();
    if (!b) return fail(MLK_ERR_NULL, "conv batch is NULL");
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
    if (dev != b->device) return fail(MLK_ERR_ARG, "conv batch: created on device %d, run on device %d", b->device, dev);
    const hipStream_t hs = (hipStream_t)stream;
    if (!b->accumulate) {
        // split parts add with atomics: their outputs start from zero
        for (size_t i = 0; i < b->d.size(); ++i) {
            if (b->split[i] <= 1) continue;
            const mlk_conv_desc& d = b->d[i];
            const int64_t hw = conv_out(d.H, d.KH, d.sh, d.ph) * conv_out(d.W, d.KW, d.sw, d.pw);
            if ((err = launch_zero_matrix(d.y, d.N * d.F, hw, hw, 4, hs)) != hipSuccess)
                return hip_fail(err, "conv batch zero output");
        }
    }
    if (b->nblk == 0) return MLK_OK;
    err = b->e->persist_gather(b->convs, b->tasks, b->bounds, b->nblk, hs);
    return err == hipSuccess ? MLK_OK : hip_fail(err, "conv batch launch");
}

mlk_status mlk_conv2d_batch_update_filters(mlk_conv_batch* b, void* stream) {
    clear_error();
    if (!b) return fail(MLK_ERR_NULL, "conv batch is NULL");
    return transpose_filters(b, (hipStream_t)stream);
}

mlk_status mlk_conv2d_batch_info(const mlk_conv_batch* b, mlk_tile_config* cfg, int64_t* tasks,
                                 int32_t* workgroups) {
    clear_error();
    if (!b) return fail(MLK_ERR_NULL, "conv batch is NULL");
    if (cfg) *cfg = b->cfg;
    if (tasks) *tasks = b->ntasks;
    if (workgroups) *workgroups = b->nblk;
    return MLK_OK;
}

void mlk_conv2d_batch_destroy(mlk_conv_batch* b) {
    if (!b) return;
    if (b->dev) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->dev);
    }
    delete b;
}

}  // extern "C"
