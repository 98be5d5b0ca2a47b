// sal_plan.cpp -- batched execution of the whole forward path over many volumes:
// window classes, tile-depth autotuning, descriptor tables and the captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sal_batch.h"

namespace sal {

namespace {

struct Class {
    sal_spec spec;
    std::vector<int> members;  // indices into the item list
    std::vector<int> candidates;
    int CT = 0;
    size_t lds = 0;
    int grid = 0;
    int64_t total = 0;
    size_t items_off = 0, prefix_off = 0;
    size_t param_bytes = 0;
    std::vector<char> params;     // host copy of the per-member kernel parameters
    std::vector<int64_t> prefix;  // first global tile of each member
    std::string timing;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int>, int> g_tuned;  // class key + log2(tiles) -> tile depth

// Tile depths tuned by earlier processes: with SAL_AUTOTUNE_CACHE naming a file, each tuned
// class is appended as one line "arch n s precision window log2(tiles) depth", and a later
// plan on the same architecture reads the depth instead of timing the candidates again.
std::string cache_path() {
    const char* v = std::getenv("SAL_AUTOTUNE_CACHE");
    return v ? std::string(v) : std::string();
}

std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool cache_lookup(const std::string& arch, int n, int s, int prec, int window, int bucket, int* ct) {
    const std::string path = cache_path();
    if (path.empty()) return false;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char a[64];
    int v[6];
    bool hit = false;
    while (std::fscanf(f, "%63s %d %d %d %d %d %d", a, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 7)
        if (arch == a && v[0] == n && v[1] == s && v[2] == prec && v[3] == window && v[4] == bucket && v[5] > 0) {
            *ct = v[5];  // the last matching line wins
            hit = true;
        }
    std::fclose(f);
    return hit;
}

void cache_store(const std::string& arch, int n, int s, int prec, int window, int bucket, int ct) {
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;  // a cache that cannot be written only costs a re-tune later
    std::fprintf(f, "%s %d %d %d %d %d %d\n", arch.c_str(), n, s, prec, window, bucket, ct);
    std::fclose(f);
}

int log2_bucket(int64_t v) {
    int b = 0;
    while (v > 1) {
        v >>= 1;
        b++;
    }
    return b;
}

}  // namespace
}  // namespace sal

struct sal_plan_s {
    std::vector<sal_batch_item> items;
    std::vector<sal::Class> classes;
    uint32_t flags = 0;
    int device = 0;
    void* dev = nullptr;
    size_t dcs_items_off = 0, dcs_first_off = 0, fuse_items_off = 0, comb_first_off = 0, adapt_off = 0, parts_off = 0,
           status_off = 0;
    int64_t dcs_blocks = 0, comb_rows = 0;
    int nadapt = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string desc;
};

namespace sal {
namespace {

sal_status build_class_params(sal_plan* plan, Class& c, int CT) {
    c.param_bytes = c.spec.precision == SAL_PREC_FP32 ? project_fp32_param_bytes() : project_lowp_param_bytes();
    c.params.assign(c.param_bytes * c.members.size(), 0);
    c.prefix.assign(c.members.size(), 0);
    int64_t total = 0;
    size_t lds = 0;
    const Tables* tb = nullptr;
    sal_status st = get_tables(nullptr, c.spec.n, c.spec.window, &tb);
    if (st) return st;
    for (size_t k = 0; k < c.members.size(); k++) {
        const sal_batch_item& it = plan->items[c.members[k]];
        int64_t nt = 0;
        size_t l = 0;
        void* dst = c.params.data() + k * c.param_bytes;
        if (c.spec.precision == SAL_PREC_FP32)
            st = project_fp32_params(c.spec.n, c.spec.s, CT, it.V, it.T, it.IL, it.XL, tb, it.E_out, dst, &nt, &l);
        else
            st = project_lowp_params(c.spec.n, c.spec.s, c.spec.precision, CT, it.V, it.T, it.IL, it.XL, tb,
                                     it.E_out, dst, &nt, &l);
        if (st) return st;
        c.prefix[k] = total;
        total += nt;
        lds = l;
    }
    c.CT = CT;
    c.total = total;
    c.lds = lds;
    int per_cu = 1, cus = 1;
    st = c.spec.precision == SAL_PREC_FP32 ? project_fp32_batch_occupancy(c.spec.n, c.spec.s, lds, &per_cu)
                                           : project_lowp_batch_occupancy(c.spec.n, c.spec.s, c.spec.precision, CT,
                                                                          lds, &per_cu);
    if (st) return st;
    if ((st = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plan->device),
                        "hipDeviceGetAttribute")))
        return st;
    per_cu = std::max(per_cu, 1);
    int64_t grid = (int64_t)cus * per_cu;
    grid = std::min<int64_t>(grid, 8 * ((total + 7) / 8));
    grid = std::max<int64_t>(8, grid / 8 * 8);
    if (c.spec.precision == SAL_PREC_FP32) grid = project_fp32_batch_grid(c.spec.n, total, grid);
    if (grid > INT32_MAX) return fail(SAL_ERR_SHAPE, "batch class too large for one launch");
    c.grid = (int)grid;
    return SAL_OK;
}

sal_status upload_class(sal_plan* plan, const Class& c) {
    char* base = (char*)plan->dev;
    sal_status st = check_hip(hipMemcpy(base + c.items_off, c.params.data(), c.params.size(), hipMemcpyHostToDevice),
                              "hipMemcpy(plan items)");
    if (st) return st;
    return check_hip(hipMemcpy(base + c.prefix_off, c.prefix.data(), c.prefix.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice),
                     "hipMemcpy(plan prefix)");
}

sal_status launch_class(sal_plan* plan, const Class& c, hipStream_t stream) {
    if (c.total == 0) return SAL_OK;
    const char* base = (const char*)plan->dev;
    const void* items = base + c.items_off;
    const int64_t* prefix = (const int64_t*)(base + c.prefix_off);
    if (c.spec.precision == SAL_PREC_FP32)
        return project_fp32_batch(c.spec.n, c.spec.s, items, prefix, (int)c.members.size(), c.total, c.lds, c.grid,
                                  stream);
    return project_lowp_batch(c.spec.n, c.spec.s, c.spec.precision, c.CT, items, prefix, (int)c.members.size(),
                              c.total, c.lds, c.grid, stream);
}

sal_status enqueue_all(sal_plan* plan, hipStream_t stream) {
    sal_status st;
    for (const Class& c : plan->classes)
        if ((st = launch_class(plan, c, stream))) return st;
    char* base = (char*)plan->dev;
    const int n = (int)plan->items.size();
    if ((st = launch_dcs_batch((const DcsItem*)(base + plan->dcs_items_off), (const int64_t*)(base + plan->dcs_first_off),
                               n, plan->dcs_blocks, stream)))
        return st;
    if ((st = launch_fuse_batch((const FuseItem*)(base + plan->fuse_items_off), n, (const int*)(base + plan->adapt_off),
                                plan->nadapt, (const int64_t*)(base + plan->comb_first_off), plan->comb_rows, stream)))
        return st;
    return launch_plan_status((const FuseItem*)(base + plan->fuse_items_off), n, (int64_t*)(base + plan->status_off),
                              stream);
}

// Time every candidate tile depth of a class on its own members; keep the fastest.
sal_status autotune_class(sal_plan* plan, Class& c) {
    const auto key = std::make_tuple(plan->device, c.spec.n, c.spec.s, c.spec.precision, c.spec.window, 0);
    int64_t tiles0 = 0;
    {
        sal_status st = build_class_params(plan, c, c.candidates[0]);
        if (st) return st;
        tiles0 = c.total;
    }
    auto key_b = std::make_tuple(std::get<0>(key), std::get<1>(key), std::get<2>(key), std::get<3>(key),
                                 std::get<4>(key), log2_bucket(tiles0));
    const std::string arch = device_arch(plan->device);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key_b);
        if (it != g_tuned.end()) {
            c.timing = "cached";
            return build_class_params(plan, c, it->second);
        }
        int ct = 0;
        if (cache_lookup(arch, c.spec.n, c.spec.s, c.spec.precision, c.spec.window, std::get<5>(key_b), &ct) &&
            std::find(c.candidates.begin(), c.candidates.end(), ct) != c.candidates.end()) {
            g_tuned[key_b] = ct;
            c.timing = "cached in " + cache_path();
            return build_class_params(plan, c, ct);
        }
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    sal_status st = check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (!st) st = check_hip(hipEventCreate(&e1), "hipEventCreate");
    float best = 1e30f;
    int best_ct = c.candidates[0];
    char buf[96];
    for (size_t k = 0; !st && k < c.candidates.size(); k++) {
        const int CT = c.candidates[k];
        if ((st = build_class_params(plan, c, CT))) break;
        if ((st = upload_class(plan, c))) break;
        if ((st = launch_class(plan, c, s))) break;  // warm-up
        float ms = 1e30f;
        for (int r = 0; !st && r < 3; r++) {
            st = check_hip(hipEventRecord(e0, s), "hipEventRecord");
            if (!st) st = launch_class(plan, c, s);
            if (!st) st = check_hip(hipEventRecord(e1, s), "hipEventRecord");
            if (!st) st = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float t = 0.f;
            if (!st) st = check_hip(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
            ms = std::min(ms, t);
        }
        snprintf(buf, sizeof(buf), "%sCT=%d:%.3fms", k ? " " : "", CT, ms);
        c.timing += buf;
        if (ms < best) {
            best = ms;
            best_ct = CT;
        }
    }
    // cleanup of the tuning stream and events; their status does not change the tuning result
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key_b] = best_ct;
        cache_store(arch, c.spec.n, c.spec.s, c.spec.precision, c.spec.window, std::get<5>(key_b), best_ct);
    }
    return build_class_params(plan, c, best_ct);
}

// Releases everything a plan owns.  A failing release cannot be acted on (the plan is gone
// either way), so its status is dropped.
void destroy(sal_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->cap) (void)hipStreamDestroy(plan->cap);
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
}

}  // namespace
}  // namespace sal

using namespace sal;

extern "C" {

static sal_status sal_plan_create_body(const sal_batch_item* items, int64_t count, uint32_t flags, sal_plan** out) {
    if (!out) return fail(SAL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!items || count < 1) return fail(SAL_ERR_ARG, "a plan needs at least one member");
    if (count > (1 << 20)) return fail(SAL_ERR_ARG, "too many members");
    if (flags & ~(SAL_PLAN_AUTOTUNE | SAL_PLAN_NO_GRAPH)) return fail(SAL_ERR_ARG, "unknown plan flags");
    std::vector<DcsStencil> stencils(count);
    for (int64_t i = 0; i < count; i++) {
        const sal_batch_item& it = items[i];
        sal_status st = check_spec(&it.spec, it.T, it.IL, it.XL);
        if (st) return fail(st, "member " + std::to_string(i) + ": " + sal_last_error());
        if (!it.V || !it.E_out || !it.Sm_out || !it.W_out || !it.S_out)
            return fail(SAL_ERR_ARG, "member " + std::to_string(i) + ": NULL buffer");
        if ((st = make_stencil(&it.stencil, it.spec.s, &stencils[i])))
            return fail(st, "member " + std::to_string(i) + ": " + sal_last_error());
        if ((st = check_fusion_args(&it.fusion, it.D)))
            return fail(st, "member " + std::to_string(i) + ": " + sal_last_error());
        if (it.spec.feature != SAL_FEATURE_MAGNITUDE)
            return fail(SAL_ERR_UNSUPPORTED, "member " + std::to_string(i) + ": the energy feature is not batched");
        if (fuse_sequential(it.fusion.mode))
            return fail(SAL_ERR_UNSUPPORTED, "member " + std::to_string(i) +
                                                 ": the LMS / NLMS / RLS rules are not batched (use sal_fuse)");
        if (it.fusion.sections != 0)
            return fail(SAL_ERR_UNSUPPORTED, "member " + std::to_string(i) +
                                                 ": sectioned re-adaptation is not batched (use sal_fuse)");
    }
    sal_plan* plan = new sal_plan();
    plan->items.assign(items, items + count);
    plan->flags = flags;
    sal_status st = check_hip(hipGetDevice(&plan->device), "hipGetDevice");
    if (st) { destroy(plan); return st; }

    // window classes in order of first appearance
    for (int64_t i = 0; i < count; i++) {
        const sal_spec& sp = items[i].spec;
        Class* c = nullptr;
        for (Class& k : plan->classes)
            if (k.spec.n == sp.n && k.spec.s == sp.s && k.spec.window == sp.window && k.spec.precision == sp.precision)
                c = &k;
        if (!c) {
            plan->classes.emplace_back();
            c = &plan->classes.back();
            c->spec = sp;
            if (sp.precision == SAL_PREC_FP32) project_fp32_ct_candidates(sp.n, sp.s, &c->candidates);
            else project_lowp_ct_candidates(sp.n, sp.s, sp.precision, &c->candidates);
            if (c->candidates.empty()) {
                destroy(plan);
                return fail(SAL_ERR_UNSUPPORTED, "no tile fits the LDS for a member's window class");
            }
        }
        c->members.push_back((int)i);
    }
    for (Class& c : plan->classes)
        if ((st = build_class_params(plan, c, c.candidates[0]))) { destroy(plan); return st; }

    // device layout: class tables, then the center-surround and fusion descriptors
    size_t off = 0;
    for (Class& c : plan->classes) {
        c.items_off = off;
        off = align256(off + c.params.size());
        c.prefix_off = off;
        off = align256(off + c.prefix.size() * sizeof(int64_t));
    }
    std::vector<DcsItem> dcs(count);
    std::vector<int64_t> dfirst(count), cfirst(count);
    std::vector<FuseItem> fus(count);
    std::vector<int> adapt;
    int64_t blocks = 0, rows = 0;
    for (int64_t i = 0; i < count; i++) {
        const sal_batch_item& it = items[i];
        const int s = it.spec.s;
        DcsItem& d = dcs[i];
        d.E = it.E_out;
        d.S = it.Sm_out;
        d.Tg = ceil_div(it.T, s); d.ILg = ceil_div(it.IL, s); d.XLg = ceil_div(it.XL, s);
        d.st = stencils[i];
        dfirst[i] = blocks;
        blocks += (d.Tg * d.ILg * d.XLg + 255) / 256;
        FuseItem& f = fus[i];
        f.Sm = it.Sm_out;
        f.D = it.D;
        f.mask = it.mask;
        f.Tg = d.Tg; f.ILg = d.ILg; f.XLg = d.XLg;
        f.T = it.T; f.IL = it.IL; f.XL = it.XL;
        f.s = s;
        f.mode = it.fusion.mode;
        f.w0 = it.fusion.w_fixed[0]; f.w1 = it.fusion.w_fixed[1]; f.w2 = it.fusion.w_fixed[2];
        f.delta = it.fusion.delta;
        f.W = it.W_out;
        f.S = it.S_out;
        f.part = nullptr;
        if (f.mode == SAL_FUSE_ADAPT_LS) adapt.push_back((int)i);
        cfirst[i] = rows;
        rows += it.T * it.IL;
    }
    if (blocks > INT32_MAX || rows > INT32_MAX) { destroy(plan); return fail(SAL_ERR_SHAPE, "batch too large"); }
    plan->dcs_blocks = blocks;
    plan->comb_rows = rows;
    plan->nadapt = (int)adapt.size();
    plan->dcs_items_off = off; off = align256(off + dcs.size() * sizeof(DcsItem));
    plan->dcs_first_off = off; off = align256(off + dfirst.size() * sizeof(int64_t));
    plan->fuse_items_off = off; off = align256(off + fus.size() * sizeof(FuseItem));
    plan->comb_first_off = off; off = align256(off + cfirst.size() * sizeof(int64_t));
    plan->adapt_off = off; off = align256(off + std::max<size_t>(1, adapt.size()) * sizeof(int));
    plan->parts_off = off; off = align256(off + adapt.size() * kBatchParts * kStats * sizeof(double));
    plan->status_off = off; off = align256(off + 2 * sizeof(int64_t));
    if ((st = check_hip(hipMalloc(&plan->dev, off), "hipMalloc(plan)"))) { destroy(plan); return st; }
    char* base = (char*)plan->dev;
    for (size_t k = 0; k < adapt.size(); k++)
        fus[adapt[k]].part = (double*)(base + plan->parts_off) + k * kBatchParts * kStats;
    st = check_hip(hipMemcpy(base + plan->dcs_items_off, dcs.data(), dcs.size() * sizeof(DcsItem), hipMemcpyHostToDevice),
                   "hipMemcpy(plan)");
    if (!st) st = check_hip(hipMemcpy(base + plan->dcs_first_off, dfirst.data(), dfirst.size() * 8, hipMemcpyHostToDevice),
                            "hipMemcpy(plan)");
    if (!st) st = check_hip(hipMemcpy(base + plan->fuse_items_off, fus.data(), fus.size() * sizeof(FuseItem),
                                      hipMemcpyHostToDevice), "hipMemcpy(plan)");
    if (!st) st = check_hip(hipMemcpy(base + plan->comb_first_off, cfirst.data(), cfirst.size() * 8, hipMemcpyHostToDevice),
                            "hipMemcpy(plan)");
    if (!st && !adapt.empty())
        st = check_hip(hipMemcpy(base + plan->adapt_off, adapt.data(), adapt.size() * sizeof(int), hipMemcpyHostToDevice),
                       "hipMemcpy(plan)");
    if (st) { destroy(plan); return st; }

    for (Class& c : plan->classes) {
        if ((flags & SAL_PLAN_AUTOTUNE) && c.candidates.size() > 1) {
            if ((st = autotune_class(plan, c))) { destroy(plan); return st; }
        }
        if ((st = upload_class(plan, c))) { destroy(plan); return st; }
    }

    // description
    char buf[256];
    for (const Class& c : plan->classes) {
        snprintf(buf, sizeof(buf), "class n=%d s=%d window=%d precision=%d: %zu members, %lld tiles, tile %dx4x4, "
                 "grid %d, LDS %zu B%s%s\n", c.spec.n, c.spec.s, c.spec.window, c.spec.precision, c.members.size(),
                 (long long)c.total, c.CT, c.grid, c.lds, c.timing.empty() ? "" : ", autotune ", c.timing.c_str());
        plan->desc += buf;
    }
    snprintf(buf, sizeof(buf), "center-surround %lld blocks, fusion %d adapted members, combine %lld rows%s\n",
             (long long)blocks, plan->nadapt, (long long)rows, (flags & SAL_PLAN_NO_GRAPH) ? "" : ", captured graph");
    plan->desc += buf;

    if (!(flags & SAL_PLAN_NO_GRAPH)) {
        st = check_hip(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking), "hipStreamCreate");
        if (!st) st = check_hip(hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (!st) {
            sal_status st2 = enqueue_all(plan, plan->cap);
            hipGraph_t g = nullptr;
            st = check_hip(hipStreamEndCapture(plan->cap, &g), "hipStreamEndCapture");
            plan->graph = g;
            if (!st) st = st2;
        }
        if (!st) st = check_hip(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        if (st) { destroy(plan); return st; }
    }
    if ((st = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize"))) { destroy(plan); return st; }
    *out = plan;
    return SAL_OK;
}

sal_status sal_plan_create(const sal_batch_item* items, int64_t count, uint32_t flags, sal_plan** out) {
    CallScope cs("sal_plan_create");
    return cs.done(sal_plan_create_body(items, count, flags, out));
}

static sal_status sal_plan_launch_body(sal_plan* plan, sal_stream stream) {
    if (!plan) return fail(SAL_ERR_ARG, "plan is NULL");
    if (plan->flags & SAL_PLAN_NO_GRAPH) return enqueue_all(plan, (hipStream_t)stream);
    return check_hip(hipGraphLaunch(plan->exec, (hipStream_t)stream), "hipGraphLaunch");
}

sal_status sal_plan_launch(sal_plan* plan, sal_stream stream) {
    CallScope cs("sal_plan_launch");
    return cs.done(sal_plan_launch_body(plan, stream));
}

sal_status sal_plan_status(const sal_plan* plan, sal_stream stream, int64_t* fallback_count, int64_t* first_fallback) {
    if (!plan) return fail(SAL_ERR_ARG, "plan is NULL");
    if (!fallback_count || !first_fallback) return fail(SAL_ERR_ARG, "NULL output");
    int64_t h[2] = {0, -1};
    sal_status st = check_hip(hipMemcpyAsync(h, (const char*)plan->dev + plan->status_off, sizeof(h),
                                             hipMemcpyDeviceToHost, (hipStream_t)stream),
                              "hipMemcpyAsync(plan status)");
    if (!st) st = check_hip(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    if (st) return st;
    *fallback_count = h[0];
    *first_fallback = h[1];
    return SAL_OK;
}

const char* sal_plan_describe(const sal_plan* plan) { return plan ? plan->desc.c_str() : ""; }

sal_status sal_plan_destroy(sal_plan* plan) {
    if (!plan) return SAL_OK;
    destroy(plan);
    return SAL_OK;
}

}  // extern "C"
