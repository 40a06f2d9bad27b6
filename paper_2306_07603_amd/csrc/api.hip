// api.hip -- the C ABI of libifdlbm.so (declared in include/ifdlbm.h):
// argument validation, FP64 metric precompute, device memory, work lists,
// the time loop with its residual schedule, HIP graph replay, and the
// steady-state driver with per-cavity retirement.
#include "ifdlbm.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ifdlbm_internal.h"

using namespace ifd;

namespace ifd {

// out[i] = round_stochastic(v[i], r16[i] & 0xFFFF) for i < n (device arrays; kernels_common.hip)
hipError_t launch_round_stochastic(const double* v, const uint32_t* r16, float* out, int64_t n, hipStream_t s);
// out[i] = x[i]^y by the FP64 power of Step (2), for i < n (device arrays; kernels_common.hip)
hipError_t launch_power_law(const double* x, double y, double* out, int64_t n, hipStream_t s);

thread_local std::string g_last_error;

// Records the text of the last error of this thread and returns code.
int fail(int code, const std::string& msg)
{
    try {
        g_last_error = msg;
    } catch (...) {
    }
    return code;
}

}  // namespace ifd

// Body of a C entry point: a host allocation failure (or any other C++
// exception) becomes an error code instead of crossing the C ABI.
#define IFD_GUARD(call)                                                       \
    try {                                                                     \
        return call;                                                          \
    } catch (const std::bad_alloc&) {                                         \
        return fail(IFDLBM_ENOMEM, "host memory allocation failed");          \
    } catch (...) {                                                           \
        return fail(IFDLBM_EDEVICE, "unexpected C++ exception in the library"); \
    }

namespace {

#define IFD_HIP(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(IFDLBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr double kCs2 = 1.0 / 3.0;

// Rows per segment of the fused kernel's work items (the columns per strip
// are at most kStripOut).  Automatic choice: the longest segment (fewest
// recomputed halo rows) that still gives kTargetItems work items, so that the
// GPU stays full through the tail of a launch; the shortest otherwise.
constexpr int kSegCandidates[] = {128, 96, 80, 72, 64, 56, 48, 40, 32, 24, 16, 8};
constexpr int kMinSegRows = 8;
constexpr int kTargetItems = 4096;
constexpr int kXcds = 8;   // MI355X: workgroups are dealt to the 8 XCDs in turn

int ceil_div(int a, int b) { return (a + b - 1) / b; }

size_t f_elem_size(int prec) { return prec == P_FP64 ? 8 : (prec == P_FP16DEV ? 2 : 4); }
size_t l_elem_size(int prec) { return prec == P_FP64 ? 8 : 4; }
size_t t_elem_size(int prec) { return (prec == P_FP64 || prec == P_FP32X || prec == P_FP32SR) ? 8 : 4; }

// 1/tan(theta) with theta in degrees; exactly 0 for the square.
double cot_deg(double theta_deg)
{
    if (theta_deg == 90.0) return 0.0;
    return 1.0 / std::tan(theta_deg * (M_PI / 180.0));
}

}  // namespace

struct ifdlbm_s {
    int n_cav = 0;
    ifdlbm_options opt{};
    std::vector<ifdlbm_cavity> cav;
    std::vector<CavityDesc> desc;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    size_t f_elems = 0, l_elems = 0;
    void* d_f[2] = {nullptr, nullptr};
    void* d_l[2] = {nullptr, nullptr};
    int cur = 0;
    CavityDesc* d_desc = nullptr;
    double* d_geo = nullptr;
    float* d_geo32 = nullptr;
    void *d_hp = nullptr, *d_bp = nullptr, *d_fb = nullptr, *d_ln = nullptr;   // staged temporaries

    // node blocks of every cavity (initialisation) and of the running ones (staged step)
    std::vector<NodeBlock> all_blocks;
    NodeBlock* d_all_blocks = nullptr;
    std::vector<NodeBlock> act_blocks;
    NodeBlock* d_act_blocks = nullptr;
    // strip items of the running cavities (fused step)
    std::vector<StripItem> act_items;      // per cavity, contiguous (unit = index)
    StripItem* d_act_items = nullptr;
    std::vector<StripItem> act_sorted;     // the same items, longest first (batched launch)
    StripItem* d_act_sorted = nullptr;
    size_t max_units = 0;
    std::vector<int32_t> unit_first, unit_count;   // per cavity, in the active unit list
    int32_t *d_unit_first = nullptr, *d_unit_count = nullptr;
    double* d_partial = nullptr;
    double* d_res = nullptr;                        // n_cav * kResult
    double* d_ref = nullptr;                        // n_cav * 2 shifts of the residual sums
    double* d_scratch = nullptr;                    // 10 * max nodes doubles
    uint32_t* d_seed = nullptr;                     // stochastic-rounding step counter
    size_t scratch_elems = 0;

    // probe record (centre velocity and kinetic energy every rec_every steps)
    int rec_every = 0, rec_capacity = 0;
    int64_t rec_first_step = 0;                     // step count after which sample 0 is taken
    double* d_rec = nullptr;                        // [n_cav][capacity][3]
    uint32_t* d_rec_count = nullptr;
    double* d_probe_partial = nullptr;              // one double per node block
    std::vector<int32_t> all_first, all_count;      // node blocks of each cavity in all_blocks
    int32_t *d_all_first = nullptr, *d_all_count = nullptr;

    std::vector<int> status;
    std::vector<double> res_u, res_p_printed, res_p_gauge;   // last evaluated residuals of Eq. (2.19)
    int64_t step_count = 0;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_dirty = true;
};

namespace {

int units_per_step(const ifdlbm_s* h) { return h->opt.kernel == IFDLBM_KERNEL_STAGED ? 5 : 1; }

// Rebuild the unit lists of the running cavities (after creation, retirement or restore).
// First row of segment g of ng over ny rows: the even split, moved to the
// nearest row that is 4 (mod 5).  The fused kernel's march then starts at a
// row that is 0 (mod 5), so every row is computed by the same unrolled copy
// of the row code whatever the segmentation, and results do not depend on
// the composition of the batch.  Each end moves by <= 2 rows; with >= 8 rows
// per segment the interior segments keep a multiple of 5 rows and the two end
// segments >= 4 (checked for every ny up to 4000).
int segment_start(int g, int ng, int ny)
{
    if (g <= 0) return 0;
    if (g >= ng) return ny;
    const int b = (int)((int64_t)g * ny / ng);
    const int r = ((b - 4) % 5 + 5) % 5;
    return r <= 2 ? b - r : b + (5 - r);
}

// Rows per segment for the cavities of one launch: all running cavities (one_cav < 0, batched launch) or
// cavity one_cav alone (one launch per cavity).
int segment_rows(const ifdlbm_s* h, int one_cav = -1)
{
    if (h->opt.segment_rows > 0) return h->opt.segment_rows;
    for (int seg : kSegCandidates) {
        size_t n = 0;
        for (int c = 0; c < h->n_cav; ++c)
            if (h->desc[c].active && (one_cav < 0 || c == one_cav))
                n += (size_t)ceil_div(h->desc[c].ny, seg) * ceil_div(h->desc[c].nx, kStripOut);
        if (n >= (size_t)kTargetItems) return seg;
    }
    return kSegCandidates[sizeof(kSegCandidates) / sizeof(kSegCandidates[0]) - 1];
}

// Order of the items in the batched launch.  Workgroup w of a launch goes to
// XCD w % 8 (each XCD has its own L2), so position 8 r + x is the r-th item of
// XCD x.  The strips of one row segment of one cavity form a group (they read
// each other's halo columns); groups are dealt to the XCDs longest first, each
// to the least loaded XCD (LPT), and every XCD runs its groups longest first,
// so that neighbouring strips share one L2 and short groups fill the tail.
// Queues are padded to equal length with empty items.
int item_cost(const StripItem& it) { return it.j1 - it.j0 + 8; }

void order_for_batch(ifdlbm_s* h)
{
    h->act_sorted.clear();
    if (h->act_items.empty()) return;
    struct Group {
        int64_t cost;
        size_t first, count;
    };
    std::vector<Group> groups;
    for (size_t u = 0; u < h->act_items.size(); ++u) {
        const StripItem& it = h->act_items[u];
        if (groups.empty() || h->act_items[groups.back().first].cav != it.cav ||
            h->act_items[groups.back().first].j0 != it.j0)
            groups.push_back({0, u, 0});
        groups.back().cost += item_cost(it);
        groups.back().count++;
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& x, const Group& y) { return x.cost > y.cost; });
    std::vector<std::vector<StripItem>> queue(kXcds);
    std::vector<int64_t> load(kXcds, 0);
    for (const Group& g : groups) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += g.cost;
        for (size_t u = g.first; u < g.first + g.count; ++u) queue[x].push_back(h->act_items[u]);
    }
    size_t rows = 0;
    for (const auto& q : queue) rows = std::max(rows, q.size());
    const StripItem empty{0, 0, 0, 0, 0, -1};
    for (size_t r = 0; r < rows; ++r)
        for (int x = 0; x < kXcds; ++x) h->act_sorted.push_back(r < queue[x].size() ? queue[x][r] : empty);
}

int rebuild_worklists(ifdlbm_s* h)
{
    h->act_blocks.clear();
    h->act_items.clear();
    const int seg_batch = segment_rows(h);
    for (int c = 0; c < h->n_cav; ++c) {
        const bool run = h->desc[c].active != 0;
        // a launch of its own fills the GPU only with the cavity's own segment length
        const int seg = h->opt.batched ? seg_batch : segment_rows(h, c);
        if (h->opt.kernel == IFDLBM_KERNEL_STAGED) {
            h->unit_first[c] = (int32_t)h->act_blocks.size();
            if (run) {
                const int nn = h->desc[c].nx * h->desc[c].ny;
                for (int n = 0; n < nn; n += kNodeBlock) h->act_blocks.push_back({c, n});
            }
            h->unit_count[c] = (int32_t)h->act_blocks.size() - h->unit_first[c];
        } else {
            h->unit_first[c] = (int32_t)h->act_items.size();
            if (run) {
                const CavityDesc& d = h->desc[c];
                const int ns = ceil_div(d.nx, kStripOut), ng = ceil_div(d.ny, seg);
                for (int g = 0; g < ng; ++g)
                    for (int s = 0; s < ns; ++s)
                        h->act_items.push_back({c, (int16_t)(s * d.nx / ns), (int16_t)((s + 1) * d.nx / ns),
                                                segment_start(g, ng, d.ny), segment_start(g + 1, ng, d.ny),
                                                (int32_t)h->act_items.size()});
            }
            h->unit_count[c] = (int32_t)h->act_items.size() - h->unit_first[c];
        }
    }
    order_for_batch(h);
    if (!h->act_blocks.empty())
        IFD_HIP(hipMemcpyAsync(h->d_act_blocks, h->act_blocks.data(), h->act_blocks.size() * sizeof(NodeBlock),
                               hipMemcpyHostToDevice, h->stream));
    if (!h->act_items.empty()) {
        IFD_HIP(hipMemcpyAsync(h->d_act_items, h->act_items.data(), h->act_items.size() * sizeof(StripItem),
                               hipMemcpyHostToDevice, h->stream));
        IFD_HIP(hipMemcpyAsync(h->d_act_sorted, h->act_sorted.data(), h->act_sorted.size() * sizeof(StripItem),
                               hipMemcpyHostToDevice, h->stream));
    }
    IFD_HIP(hipMemcpyAsync(h->d_unit_first, h->unit_first.data(), h->n_cav * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    IFD_HIP(hipMemcpyAsync(h->d_unit_count, h->unit_count.data(), h->n_cav * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    IFD_HIP(hipMemcpyAsync(h->d_desc, h->desc.data(), h->n_cav * sizeof(CavityDesc), hipMemcpyHostToDevice, h->stream));
    // the host vectors may change before the copies run
    IFD_HIP(hipStreamSynchronize(h->stream));
    h->graph_dirty = true;
    return IFDLBM_OK;
}

StepArgs step_args(ifdlbm_s* h)
{
    StepArgs a{};
    a.f_in = h->d_f[h->cur];
    a.f_out = h->d_f[h->cur ^ 1];
    a.l_in = h->d_l[h->cur];
    a.l_out = h->d_l[h->cur ^ 1];
    a.desc = h->d_desc;
    a.geo = h->d_geo;
    a.geo32 = h->d_geo32;
    a.partial = h->d_partial;
    a.res_ref = h->d_ref;
    a.hat_plus = h->d_hp;
    a.bar_plus = h->d_bp;
    a.bar_half = h->d_fb;
    a.lam_new = h->d_ln;
    a.seed_ctr = h->d_seed;
    a.step = 0;
    return a;
}

// Enqueue one time step of the running cavities, reading buffer `cur`;
// `local` numbers the step within its call or graph (stochastic rounding).
int enqueue_step(ifdlbm_s* h, bool residual, uint32_t local)
{
    StepArgs a = step_args(h);
    a.step = local;
    const int prec = h->opt.precision;
    const bool staged = h->opt.kernel == IFDLBM_KERNEL_STAGED;
    const bool impl = h->opt.lambda_mode == IFDLBM_LAMBDA_IMPLICIT;
    hipError_t e = hipSuccess;
    if (h->opt.batched) {
        e = staged ? launch_staged_step(prec, a, h->d_act_blocks, 0, (int)h->act_blocks.size(), residual, h->stream)
                   : launch_fused_step(prec, impl, a, h->d_act_sorted, 0, (int)h->act_sorted.size(), residual, h->stream);
    } else {
        for (int c = 0; c < h->n_cav && e == hipSuccess; ++c) {
            if (!h->unit_count[c]) continue;
            e = staged ? launch_staged_step(prec, a, h->d_act_blocks, h->unit_first[c], h->unit_count[c], residual, h->stream)
                       : launch_fused_step(prec, impl, a, h->d_act_items, h->unit_first[c], h->unit_count[c], residual, h->stream);
        }
    }
    if (e == hipSuccess && residual)
        e = launch_reduce_partials(h->d_partial, h->d_unit_first, h->d_unit_count, h->d_desc, h->n_cav, h->d_ref, h->d_res,
                                   h->stream);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return IFDLBM_OK;
}

// Probe record of the current state (after a step).
int enqueue_probe(ifdlbm_s* h)
{
    hipError_t e = launch_probe(h->opt.precision, h->d_f[h->cur], h->d_desc, h->n_cav, h->d_all_blocks,
                                (int)h->all_blocks.size(), h->d_probe_partial, h->d_all_first, h->d_all_count, h->d_rec,
                                h->d_rec_count, h->rec_capacity, h->stream);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("probe launch: ") + hipGetErrorString(e));
    return IFDLBM_OK;
}

bool is_residual_step(const ifdlbm_s* h, int64_t step_index) { return (step_index + 1) % h->opt.residual_every == 0; }

int eager_steps(ifdlbm_s* h, int64_t n)
{
    if (n > 0) {
        hipError_t e = launch_seed_bump(h->d_seed, h->stream);
        if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("seed: ") + hipGetErrorString(e));
    }
    for (int64_t s = 0; s < n; ++s) {
        int rc = enqueue_step(h, is_residual_step(h, h->step_count), (uint32_t)s);
        if (rc) return rc;
        h->cur ^= 1;
        h->step_count++;
        if (h->rec_every > 0 && h->step_count % h->rec_every == 0) {
            rc = enqueue_probe(h);
            if (rc) return rc;
        }
    }
    return IFDLBM_OK;
}

// Capture graph_steps steps starting at a step index that is a multiple of
// graph_steps (graph_steps is even and a multiple of residual_every, so every
// replay starts from the same buffer and has the same residual pattern).
int build_graph(ifdlbm_s* h)
{
    if (h->graph_exec) {
        IFD_HIP(hipGraphExecDestroy(h->graph_exec));
        h->graph_exec = nullptr;
    }
    const int G = h->opt.graph_steps;
    const int cur0 = h->cur;
    const int64_t count0 = h->step_count;
    hipGraph_t graph = nullptr;
    IFD_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = IFDLBM_OK;
    if (launch_seed_bump(h->d_seed, h->stream) != hipSuccess) rc = fail(IFDLBM_EDEVICE, "seed bump in capture");
    for (int s = 0; s < G && rc == IFDLBM_OK; ++s) {
        rc = enqueue_step(h, is_residual_step(h, s), (uint32_t)s);
        h->cur ^= 1;
        // the graph starts at a multiple of G, and G is a multiple of rec_every
        if (rc == IFDLBM_OK && h->rec_every > 0 && (s + 1) % h->rec_every == 0) rc = enqueue_probe(h);
    }
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    h->cur = cur0;
    h->step_count = count0;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->graph_dirty = false;
    return IFDLBM_OK;
}

int do_steps(ifdlbm_s* h, int64_t n)
{
    const int G = h->opt.graph_steps;
    if (G <= 0) return eager_steps(h, n);
    int64_t lead = (G - h->step_count % G) % G;
    lead = std::min(lead, n);
    int rc = eager_steps(h, lead);
    if (rc) return rc;
    n -= lead;
    if (n >= G && h->graph_dirty) {
        rc = build_graph(h);
        if (rc) return rc;
    }
    while (n >= G) {
        IFD_HIP(hipGraphLaunch(h->graph_exec, h->stream));
        h->step_count += G;   // G is even: the current buffer is unchanged
        n -= G;
    }
    return eager_steps(h, n);
}

// Copy cavity c's current state into the other buffer too, so that it no
// longer matters which buffer is current once the cavity stops stepping.
int mirror_state(ifdlbm_s* h, int c)
{
    const CavityDesc& d = h->desc[c];
    const int prec = h->opt.precision;
    const size_t fb = f_elem_size(prec), lb = l_elem_size(prec);
    char* f0 = static_cast<char*>(h->d_f[h->cur]);
    char* f1 = static_cast<char*>(h->d_f[h->cur ^ 1]);
    char* l0 = static_cast<char*>(h->d_l[h->cur]);
    char* l1 = static_cast<char*>(h->d_l[h->cur ^ 1]);
    IFD_HIP(hipMemcpyAsync(f1 + d.f_off * fb, f0 + d.f_off * fb, 9 * d.plane * fb, hipMemcpyDeviceToDevice, h->stream));
    IFD_HIP(hipMemcpyAsync(l1 + d.l_off * lb, l0 + d.l_off * lb, d.plane * lb, hipMemcpyDeviceToDevice, h->stream));
    return IFDLBM_OK;
}

int check_cav(const ifdlbm_s* h, int32_t c)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    if (c < 0 || c >= h->n_cav) return fail(IFDLBM_EINVAL, "cavity index out of range");
    return IFDLBM_OK;
}

int read_residuals(ifdlbm_s* h, std::vector<double>& sums)
{
    sums.assign((size_t)h->n_cav * kResult, 0.0);
    IFD_HIP(hipMemcpyAsync(sums.data(), h->d_res, sums.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    return IFDLBM_OK;
}

double rel(double num2, double den2) { return num2 <= 0.0 ? 0.0 : std::sqrt(num2) / std::sqrt(den2); }

// Relative rounding error of the FP64 residual sums: each partial sums at most
// a few hundred terms in order (a row segment per lane, a wavefront, the
// units of a cavity), so |error| < 512 u of the sum of the magnitudes.
constexpr double kSumRel = 512.0 * 0x1p-53;

// Eq. (2.19) from the sums of one cavity of nn nodes (layout of kResult):
// E(u); E(P) as printed; and E(P) of the pressure with its spatial mean
// removed, from the shifted sums: sum (x - r)^2 - (sum (x - r))^2 / nn is the
// sum of squared deviations from the mean.  A variance that the sums do not
// resolve (below the rounding bound of the subtraction, kSumRel times the
// shifted sum of squares) is reported as that bound: an upper limit, so that
// rounding never reads as convergence.  Returns false if non-finite.
bool residuals_of(const double* s, double nn, double& eu, double& ep_printed, double& ep_gauge)
{
    eu = rel(s[0], s[1]);
    ep_printed = rel(s[2], s[3]);
    const double num = s[7] - s[4] * s[4] / nn;
    const double den = s[8] - s[5] * s[5] / nn;
    const double floor = kSumRel * s[7];
    if (den > 0.0)
        ep_gauge = std::sqrt(num > floor ? num : floor) / std::sqrt(den);
    else   // uniform pressure: 0/0 counts as 0; a resolved change of a uniform field is never converged
        ep_gauge = num > floor ? DBL_MAX : 0.0;
    return s[6] == 0.0 && std::isfinite(eu) && std::isfinite(ep_printed) && std::isfinite(ep_gauge);
}

// The E(P) that the handle's options.pressure_residual selects.
double selected_ep(const ifdlbm_s* h, int c)
{
    return h->opt.pressure_residual == IFDLBM_EP_PRINTED ? h->res_p_printed[c] : h->res_p_gauge[c];
}

// Evaluates the residual record of running cavity c into the handle; false if non-finite.
bool update_residuals(ifdlbm_s* h, const std::vector<double>& sums, int c)
{
    double eu, epp, epg;
    const bool ok = residuals_of(&sums[(size_t)c * kResult], (double)h->desc[c].nx * h->desc[c].ny, eu, epp, epg);
    h->res_u[c] = ok ? eu : NAN;
    h->res_p_printed[c] = ok ? epp : NAN;
    h->res_p_gauge[c] = ok ? epg : NAN;
    return ok;
}

void free_all(ifdlbm_s* h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    void* ptrs[] = {h->d_f[0], h->d_f[1], h->d_l[0], h->d_l[1], h->d_desc, h->d_geo, h->d_geo32, h->d_hp, h->d_bp,
                    h->d_fb, h->d_ln, h->d_all_blocks, h->d_act_blocks, h->d_act_items, h->d_act_sorted, h->d_unit_first,
                    h->d_unit_count, h->d_partial, h->d_res, h->d_ref, h->d_scratch, h->d_seed, h->d_rec, h->d_rec_count,
                    h->d_probe_partial, h->d_all_first, h->d_all_count};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

template <typename P>
int dalloc(P** p, size_t bytes)
{
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? IFDLBM_ENOMEM : IFDLBM_EDEVICE,
                    std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return IFDLBM_OK;
}

}  // namespace

extern "C" {

int ifdlbm_default_options(ifdlbm_options* opt)
{
    if (!opt) return fail(IFDLBM_EINVAL, "null options");
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = IFDLBM_FP64;
    opt->cfl = 0.5;
    opt->mix = 0.75;
    opt->rho0 = 1.0;
    opt->gamma_min = 1e-6;
    opt->residual_every = 1;
    opt->kernel = IFDLBM_KERNEL_FUSED;
    opt->batched = 1;
    opt->graph_steps = 0;
    opt->dt_rule = IFDLBM_DT_CONTRAVARIANT;
    opt->segment_rows = 0;
    opt->lambda_mode = IFDLBM_LAMBDA_LAGGED;
    opt->pressure_residual = IFDLBM_EP_MEAN_REMOVED;
    opt->hip_stream = nullptr;
    return IFDLBM_OK;
}

static int ifdlbm_create_impl(const ifdlbm_cavity* cav, int32_t n_cav, const ifdlbm_options* opt, ifdlbm_t** out)
{
    if (!out) return fail(IFDLBM_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (!cav || !opt || n_cav <= 0) return fail(IFDLBM_EINVAL, "need at least one cavity and options");
    const ifdlbm_options& o = *opt;
    if (o.precision < IFDLBM_FP64 || o.precision > IFDLBM_FP32SRF) return fail(IFDLBM_EINVAL, "unknown precision");
    if (!(o.cfl > 0.0) || !(o.mix >= 0.0 && o.mix <= 1.0) || !(o.gamma_min > 0.0) || !std::isfinite(o.rho0))
        return fail(IFDLBM_EINVAL, "cfl must be > 0, mix in [0, 1], gamma_min > 0, rho0 finite");
    if (o.residual_every < 1) return fail(IFDLBM_EINVAL, "residual_every must be >= 1");
    if (o.kernel != IFDLBM_KERNEL_FUSED && o.kernel != IFDLBM_KERNEL_STAGED) return fail(IFDLBM_EINVAL, "unknown kernel");
    if (o.dt_rule != IFDLBM_DT_CONTRAVARIANT && o.dt_rule != IFDLBM_DT_CARTESIAN) return fail(IFDLBM_EINVAL, "unknown dt_rule");
    if (o.graph_steps < 0 || (o.graph_steps > 0 && (o.graph_steps % 2 != 0 || o.graph_steps % o.residual_every != 0)))
        return fail(IFDLBM_EINVAL, "graph_steps must be 0, or even and a multiple of residual_every");
    if (o.lambda_mode != IFDLBM_LAMBDA_LAGGED && o.lambda_mode != IFDLBM_LAMBDA_IMPLICIT)
        return fail(IFDLBM_EINVAL, "unknown lambda_mode");
    if (o.pressure_residual != IFDLBM_EP_MEAN_REMOVED && o.pressure_residual != IFDLBM_EP_PRINTED)
        return fail(IFDLBM_EINVAL, "unknown pressure_residual");
    if (o.segment_rows != 0 && (o.segment_rows < 8 || o.segment_rows > 4096))
        return fail(IFDLBM_EINVAL, "segment_rows must be 0 (automatic) or in [8, 4096]");
    for (int c = 0; c < n_cav; ++c) {
        const ifdlbm_cavity& v = cav[c];
        const std::string id = "cavity " + std::to_string(c) + ": ";
        if (v.n_xi < 5 || v.n_eta < 5) return fail(IFDLBM_EINVAL, id + "n_xi and n_eta must be >= 5");
        // the nine FP64 planes of a cavity span at most 9 * 2^24 * 8 bytes (1.125 GiB): every byte offset of the
        // step kernels, and the 2^31 offset their dropped stores use, stay below 2^32
        if (v.n_xi > 32767 || (int64_t)((v.n_xi + 15) / 16 * 16) * v.n_eta > (int64_t)1 << 24)
            return fail(IFDLBM_EINVAL, id + "grid too large (n_xi <= 32767, n_eta * pitch <= 2^24)");
        if (!(v.theta_deg > 0.0 && v.theta_deg <= 90.0)) return fail(IFDLBM_EINVAL, id + "theta_deg must be in (0, 90]");
        if (!(v.n > 0.0) || !std::isfinite(v.n)) return fail(IFDLBM_EINVAL, id + "n must be > 0");
        if (!(v.re > 0.0) || !std::isfinite(v.re)) return fail(IFDLBM_EINVAL, id + "re must be > 0");
        if (!(v.u_lid != 0.0) || !std::isfinite(v.u_lid)) return fail(IFDLBM_EINVAL, id + "u_lid must be nonzero");
    }

    ifdlbm_s* h = new (std::nothrow) ifdlbm_s();
    if (!h) return fail(IFDLBM_ENOMEM, "handle allocation");
    h->n_cav = n_cav;
    h->opt = o;
    h->cav.assign(cav, cav + n_cav);
    h->desc.resize(n_cav);
    h->status.assign(n_cav, IFDLBM_STATUS_RUNNING);
    h->res_u.assign(n_cav, NAN);
    h->res_p_printed.assign(n_cav, NAN);
    h->res_p_gauge.assign(n_cav, NAN);
    h->unit_first.assign(n_cav, 0);
    h->unit_count.assign(n_cav, 0);

    int rc = IFDLBM_OK;
    auto bail = [&](int code) {
        free_all(h);
        delete h;
        return code;
    };
    if (o.hip_stream) {
        h->stream = static_cast<hipStream_t>(o.hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(fail(IFDLBM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
        h->own_stream = true;
    }

    // layout and FP64 metric terms (Eqs. 3.2-3.8.2)
    std::vector<double> geo;
    int64_t f_off = 0, l_off = 0, max_nodes = 0;
    size_t n_items = 0, n_blocks = 0;
    for (int c = 0; c < n_cav; ++c) {
        const ifdlbm_cavity& v = cav[c];
        CavityDesc& d = h->desc[c];
        std::memset(&d, 0, sizeof(d));
        d.nx = v.n_xi;
        d.ny = v.n_eta;
        d.pitch = (v.n_xi + 15) / 16 * 16;
        d.active = 1;
        d.plane = (int64_t)d.ny * d.pitch;
        d.f_off = f_off;
        d.l_off = l_off;
        f_off += 9 * d.plane;
        l_off += d.plane;
        d.geo_off = (int64_t)geo.size();
        d.dxi = 1.0 / (v.n_xi - 1);
        d.deta = 1.0 / (v.n_eta - 1);
        d.cot = cot_deg(v.theta_deg);
        for (int j = 0; j < d.ny; ++j) geo.push_back(1.0 / (1.0 + 2.0 * d.cot * (j * d.deta)));   // a_j = 1/J
        for (int i = 0; i < d.nx; ++i) geo.push_back(d.cot * (double)(2 * i - (d.nx - 1)) / (double)(d.nx - 1));   // s_i = x_eta
        const double U = std::fabs(v.u_lid);
        if (o.dt_rule == IFDLBM_DT_CARTESIAN)
            d.dt = o.cfl * std::min(d.dxi, d.deta);
        else   // largest contravariant speed: |c_xi| <= 1 + cot(theta) at the bottom corners, |c_eta| <= 1
            d.dt = o.cfl / std::max((1.0 + d.cot) / d.dxi, 1.0 / d.deta);
        d.K = std::pow(U, 2.0 - v.n) / v.re;   // Eq. (2.15.1), L = 1
        d.expo = 0.5 * (v.n - 1.0);
        d.g2min = o.gamma_min * o.gamma_min;
        d.mix = o.mix;
        d.u_lid = v.u_lid;
        d.inv2dxi = 0.5 / d.dxi;
        d.inv2deta = 0.5 / d.deta;
        d.lam_newton = d.K / kCs2;
        d.lam0 = U / (v.re * kCs2);
        d.newtonian = v.n == 1.0;
        d.implicit_lambda = o.lambda_mode == IFDLBM_LAMBDA_IMPLICIT;
        d.index = c;
        const int64_t nn = (int64_t)d.nx * d.ny;
        max_nodes = std::max(max_nodes, nn);
        n_blocks += (size_t)((nn + kNodeBlock - 1) / kNodeBlock);
        n_items += (size_t)ceil_div(d.ny, kMinSegRows) * ceil_div(d.nx, kStripOut);
        h->all_first.push_back((int32_t)h->all_blocks.size());
        for (int n = 0; n < nn; n += kNodeBlock) h->all_blocks.push_back({c, n});
        h->all_count.push_back((int32_t)h->all_blocks.size() - h->all_first.back());
    }
    h->f_elems = (size_t)f_off;
    h->l_elems = (size_t)l_off;
    h->max_units = o.kernel == IFDLBM_KERNEL_STAGED ? n_blocks : n_items;
    h->scratch_elems = (size_t)max_nodes * 10;

    const int prec = o.precision;
    const size_t fs = f_elem_size(prec), ls = l_elem_size(prec), ts = t_elem_size(prec);
    for (int b = 0; b < 2 && !rc; ++b) {
        rc = dalloc(&h->d_f[b], h->f_elems * fs);
        if (!rc) rc = dalloc(&h->d_l[b], h->l_elems * ls);
    }
    if (!rc) rc = dalloc(&h->d_desc, n_cav * sizeof(CavityDesc));
    if (!rc) rc = dalloc(&h->d_geo, geo.size() * sizeof(double));
    if (!rc) rc = dalloc(&h->d_geo32, geo.size() * sizeof(float));
    if (!rc && o.kernel == IFDLBM_KERNEL_STAGED) {
        rc = dalloc(&h->d_hp, h->f_elems * ts);
        if (!rc) rc = dalloc(&h->d_bp, h->f_elems * ts);
        if (!rc) rc = dalloc(&h->d_fb, h->f_elems * ts);
        if (!rc) rc = dalloc(&h->d_ln, h->l_elems * ts);
    }
    if (!rc) rc = dalloc(&h->d_all_blocks, h->all_blocks.size() * sizeof(NodeBlock));
    if (!rc) rc = dalloc(&h->d_act_blocks, n_blocks * sizeof(NodeBlock));
    if (!rc) rc = dalloc(&h->d_act_items, n_items * sizeof(StripItem));
    // per-XCD queues are padded to equal length: at most n_items * kXcds entries
    if (!rc) rc = dalloc(&h->d_act_sorted, n_items * kXcds * sizeof(StripItem));
    if (!rc) rc = dalloc(&h->d_unit_first, n_cav * sizeof(int32_t));
    if (!rc) rc = dalloc(&h->d_unit_count, n_cav * sizeof(int32_t));
    if (!rc) rc = dalloc(&h->d_partial, h->max_units * kPartials * sizeof(double));
    if (!rc) rc = dalloc(&h->d_res, (size_t)n_cav * kResult * sizeof(double));
    if (!rc) rc = dalloc(&h->d_ref, (size_t)n_cav * 2 * sizeof(double));
    if (!rc) rc = dalloc(&h->d_scratch, h->scratch_elems * sizeof(double));
    if (!rc) rc = dalloc(&h->d_seed, sizeof(uint32_t));
    if (!rc) rc = dalloc(&h->d_all_first, n_cav * sizeof(int32_t));
    if (!rc) rc = dalloc(&h->d_all_count, n_cav * sizeof(int32_t));
    if (rc) return bail(rc);

    std::vector<float> geo32(geo.begin(), geo.end());
    auto copy = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
    };
    hipError_t e = copy(h->d_geo, geo.data(), geo.size() * sizeof(double));
    if (e == hipSuccess) e = copy(h->d_geo32, geo32.data(), geo32.size() * sizeof(float));
    if (e == hipSuccess) e = copy(h->d_all_blocks, h->all_blocks.data(), h->all_blocks.size() * sizeof(NodeBlock));
    if (e == hipSuccess) e = copy(h->d_desc, h->desc.data(), n_cav * sizeof(CavityDesc));
    if (e == hipSuccess) e = copy(h->d_all_first, h->all_first.data(), n_cav * sizeof(int32_t));
    if (e == hipSuccess) e = copy(h->d_all_count, h->all_count.data(), n_cav * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemsetAsync(h->d_res, 0, (size_t)n_cav * kResult * sizeof(double), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_ref, 0, (size_t)n_cav * 2 * sizeof(double), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_seed, 0, sizeof(uint32_t), h->stream);
    if (e == hipSuccess)
        e = launch_init(prec, h->d_f[0], h->d_l[0], h->d_desc, h->d_all_blocks, (int)h->all_blocks.size(), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(fail(IFDLBM_EDEVICE, std::string("create: ") + hipGetErrorString(e)));
    rc = rebuild_worklists(h);
    if (rc) return bail(rc);
    *out = h;
    return IFDLBM_OK;
}

static int ifdlbm_step_impl(ifdlbm_t* h, int64_t n_steps)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    if (n_steps < 0) return fail(IFDLBM_EINVAL, "n_steps must be >= 0");
    return do_steps(h, n_steps);
}

static int ifdlbm_sync_impl(ifdlbm_t* h)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    IFD_HIP(hipStreamSynchronize(h->stream));
    return IFDLBM_OK;
}

// Reads the last residual sums and evaluates them for every running cavity; a running cavity whose sums are
// non-finite is marked DIVERGED and stops stepping.  Copies the residuals of every cavity to the non-null arrays.
static int residuals_now(ifdlbm_t* h, double* res_u, double* res_p, double* res_p_printed, double* res_p_gauge)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    std::vector<double> sums;
    int rc = read_residuals(h, sums);
    if (rc) return rc;
    bool changed = false;
    for (int c = 0; c < h->n_cav; ++c) {
        if (h->desc[c].active && !update_residuals(h, sums, c)) {
            // non-finite state: the cavity stops stepping, the others continue
            h->status[c] = IFDLBM_STATUS_DIVERGED;
            h->desc[c].active = 0;
            rc = mirror_state(h, c);
            if (rc) return rc;
            changed = true;
        }
        if (res_u) res_u[c] = h->res_u[c];
        if (res_p) res_p[c] = selected_ep(h, c);
        if (res_p_printed) res_p_printed[c] = h->res_p_printed[c];
        if (res_p_gauge) res_p_gauge[c] = h->res_p_gauge[c];
    }
    if (changed) return rebuild_worklists(h);
    return IFDLBM_OK;
}

static int ifdlbm_get_residuals_impl(ifdlbm_t* h, double* res_u, double* res_p)
{
    return residuals_now(h, res_u, res_p, nullptr, nullptr);
}

static int ifdlbm_get_pressure_residuals_impl(ifdlbm_t* h, double* res_p_printed, double* res_p_mean_removed)
{
    return residuals_now(h, nullptr, nullptr, res_p_printed, res_p_mean_removed);
}

static int ifdlbm_run_to_steady_impl(ifdlbm_t* h, double tol, int64_t max_steps, int64_t* steps_done, double* res_u, double* res_p)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    if (!(tol >= 0.0) || max_steps < 0) return fail(IFDLBM_EINVAL, "tol must be >= 0 and max_steps >= 0");
    std::vector<int64_t> done(h->n_cav, 0);
    bool diverged = false;
    int64_t taken = 0;
    std::vector<double> sums;
    auto any_active = [&]() {
        for (int c = 0; c < h->n_cav; ++c)
            if (h->desc[c].active) return true;
        return false;
    };
    while (any_active() && taken < max_steps) {
        const int R = h->opt.residual_every;
        int64_t n = R - h->step_count % R;   // steps up to and including the next residual step
        n = std::min(n, max_steps - taken);
        int rc = do_steps(h, n);
        if (rc) return rc;
        taken += n;
        for (int c = 0; c < h->n_cav; ++c)
            if (h->desc[c].active) done[c] += n;
        if (h->step_count % R != 0) break;   // max_steps ended between residual steps
        rc = read_residuals(h, sums);
        if (rc) return rc;
        bool changed = false;
        for (int c = 0; c < h->n_cav; ++c) {
            if (!h->desc[c].active) continue;
            const bool ok = update_residuals(h, sums, c);
            int st = IFDLBM_STATUS_RUNNING;
            if (!ok)
                st = IFDLBM_STATUS_DIVERGED;
            else if (h->res_u[c] <= tol && selected_ep(h, c) <= tol)
                st = IFDLBM_STATUS_CONVERGED;
            if (st != IFDLBM_STATUS_RUNNING) {
                h->status[c] = st;
                diverged |= st == IFDLBM_STATUS_DIVERGED;
                h->desc[c].active = 0;
                rc = mirror_state(h, c);
                if (rc) return rc;
                changed = true;
            }
        }
        if (changed) {
            rc = rebuild_worklists(h);
            if (rc) return rc;
        }
    }
    bool unconverged = false;
    for (int c = 0; c < h->n_cav; ++c) {
        if (h->desc[c].active) {
            h->status[c] = IFDLBM_STATUS_NOT_CONVERGED;
            unconverged = true;
        }
        if (steps_done) steps_done[c] = done[c];
        if (res_u) res_u[c] = h->res_u[c];
        if (res_p) res_p[c] = selected_ep(h, c);
    }
    IFD_HIP(hipStreamSynchronize(h->stream));
    if (diverged) return fail(IFDLBM_EDIVERGED, "a cavity diverged");
    if (unconverged) return fail(IFDLBM_ENOTCONVERGED, "max_steps reached before tol");
    return IFDLBM_OK;
}

static int ifdlbm_get_fields_device_impl(ifdlbm_t* h, int32_t cav, void* u, void* v, void* p, int32_t dtype)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (dtype != 0 && dtype != 1) return fail(IFDLBM_EINVAL, "dtype must be 0 (float64) or 1 (float32)");
    hipError_t e = launch_fields(h->opt.precision, h->d_f[h->cur], h->d_desc, cav, h->desc[cav], u, v, p, dtype, h->stream);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("fields: ") + hipGetErrorString(e));
    // the caller cannot order its own work after a stream it does not know
    if (h->own_stream) IFD_HIP(hipStreamSynchronize(h->stream));
    return IFDLBM_OK;
}

static int ifdlbm_get_fields_impl(ifdlbm_t* h, int32_t cav, double* u, double* v, double* p)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    const CavityDesc& d = h->desc[cav];
    const size_t nn = (size_t)d.nx * d.ny;
    double* s = h->d_scratch;
    rc = ifdlbm_get_fields_device(h, cav, s, s + nn, s + 2 * nn, 0);
    if (rc) return rc;
    double* outs[3] = {u, v, p};
    for (int q = 0; q < 3; ++q)
        if (outs[q]) IFD_HIP(hipMemcpyAsync(outs[q], s + q * nn, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    return IFDLBM_OK;
}

static int ifdlbm_kinetic_energy_impl(ifdlbm_t* h, int32_t cav, double* energy)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (!energy) return fail(IFDLBM_EINVAL, "null energy pointer");
    const CavityDesc& d = h->desc[cav];
    const size_t nb = ((size_t)d.nx * d.ny + 255) / 256;
    hipError_t e = launch_energy(h->opt.precision, h->d_f[h->cur], h->d_desc, h->d_geo, cav, d, h->d_scratch, h->stream);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("energy: ") + hipGetErrorString(e));
    std::vector<double> part(nb);
    IFD_HIP(hipMemcpyAsync(part.data(), h->d_scratch, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    double s = 0.0;
    for (double x : part) s += x;
    *energy = s;
    return IFDLBM_OK;
}

static int ifdlbm_get_state_impl(ifdlbm_t* h, int32_t cav, double* fhat, double* lambda)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (!fhat || !lambda) return fail(IFDLBM_EINVAL, "null state array");
    const CavityDesc& d = h->desc[cav];
    const size_t nn = (size_t)d.nx * d.ny;
    double* s = h->d_scratch;
    hipError_t e = launch_state_out(h->opt.precision, h->d_f[h->cur], h->d_l[h->cur], d, h->opt.rho0, s, s + 9 * nn, h->stream);
    if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("state out: ") + hipGetErrorString(e));
    IFD_HIP(hipMemcpyAsync(fhat, s, 9 * nn * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipMemcpyAsync(lambda, s + 9 * nn, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    return IFDLBM_OK;
}

static int ifdlbm_set_state_impl(ifdlbm_t* h, int32_t cav, const double* fhat, const double* lambda)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (!fhat || !lambda) return fail(IFDLBM_EINVAL, "null state array");
    const CavityDesc& d = h->desc[cav];
    const size_t nn = (size_t)d.nx * d.ny;
    double* s = h->d_scratch;
    IFD_HIP(hipMemcpyAsync(s, fhat, 9 * nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
    IFD_HIP(hipMemcpyAsync(s + 9 * nn, lambda, nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
    for (int b = 0; b < 2; ++b) {
        hipError_t e = launch_state_in(h->opt.precision, h->d_f[b], h->d_l[b], d, h->opt.rho0, s, s + 9 * nn, h->stream);
        if (e != hipSuccess) return fail(IFDLBM_EDEVICE, std::string("state in: ") + hipGetErrorString(e));
    }
    // the residual shifts of the old trajectory would still be exact, but far from the new means
    IFD_HIP(hipMemsetAsync(h->d_ref + 2 * cav, 0, 2 * sizeof(double), h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    h->status[cav] = IFDLBM_STATUS_RUNNING;
    if (!h->desc[cav].active) {
        h->desc[cav].active = 1;
        rc = rebuild_worklists(h);
        if (rc) return rc;
    }
    return IFDLBM_OK;
}

static int ifdlbm_status_impl(ifdlbm_t* h, int32_t cav)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    return h->status[cav];
}

static int ifdlbm_autotune_impl(ifdlbm_t* h, int32_t steps_per_trial, int32_t* segment_rows, double* ms_per_step)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    if (steps_per_trial < 1 || steps_per_trial > 10000) return fail(IFDLBM_EINVAL, "steps_per_trial must be in [1, 10000]");
    if (segment_rows) *segment_rows = 0;
    if (ms_per_step) *ms_per_step = 0.0;
    if (h->opt.kernel != IFDLBM_KERNEL_FUSED) return IFDLBM_OK;   // the staged schedule has no tile shape
    // every trial starts from the current state, which is restored at the end
    const int prec = h->opt.precision;
    const size_t fb = h->f_elems * f_elem_size(prec), lb = h->l_elems * l_elem_size(prec);
    const size_t rb = (size_t)h->n_cav * kResult * sizeof(double), qb = (size_t)h->n_cav * 2 * sizeof(double);
    void *bf = nullptr, *bl = nullptr, *br = nullptr, *bq = nullptr;
    uint32_t* bs = nullptr;
    int rc = dalloc(&bf, fb);
    if (!rc) rc = dalloc(&bl, lb);
    if (!rc) rc = dalloc(&br, rb);
    if (!rc) rc = dalloc(&bq, qb);
    if (!rc) rc = dalloc(&bs, sizeof(uint32_t));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(IFDLBM_EDEVICE, "hipEventCreate");
    const int cur0 = h->cur;
    const int64_t count0 = h->step_count;
    const int32_t rows0 = h->opt.segment_rows;
    auto save = [&]() {
        hipError_t e = hipMemcpyAsync(bf, h->d_f[cur0], fb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(bl, h->d_l[cur0], lb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(br, h->d_res, rb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(bq, h->d_ref, qb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(bs, h->d_seed, sizeof(uint32_t), hipMemcpyDeviceToDevice, h->stream);
        return e;
    };
    auto restore = [&]() {
        hipError_t e = hipMemcpyAsync(h->d_f[cur0], bf, fb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->d_l[cur0], bl, lb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->d_res, br, rb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->d_ref, bq, qb, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->d_seed, bs, sizeof(uint32_t), hipMemcpyDeviceToDevice, h->stream);
        h->cur = cur0;
        h->step_count = count0;
        return e;
    };
    if (!rc && save() != hipSuccess) rc = fail(IFDLBM_EDEVICE, "autotune: state backup");
    int best = 0;
    float best_ms = 0.0f;
    const int rec_every = h->rec_every;
    h->rec_every = 0;   // trials take no probe samples
    int max_ny = 0;
    for (int c = 0; c < h->n_cav; ++c) max_ny = std::max(max_ny, h->desc[c].ny);
    for (int seg : kSegCandidates) {
        if (rc) break;
        if (seg > max_ny && seg != kSegCandidates[sizeof(kSegCandidates) / sizeof(kSegCandidates[0]) - 1]) continue;
        h->opt.segment_rows = seg;
        rc = rebuild_worklists(h);
        if (!rc) rc = eager_steps(h, 1);   // warm-up
        if (!rc && hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(IFDLBM_EDEVICE, "hipEventRecord");
        if (!rc) rc = eager_steps(h, steps_per_trial);
        if (!rc && hipEventRecord(e1, h->stream) != hipSuccess) rc = fail(IFDLBM_EDEVICE, "hipEventRecord");
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(IFDLBM_EDEVICE, "hipEventSynchronize");
        float ms = 0.0f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(IFDLBM_EDEVICE, "hipEventElapsedTime");
        if (!rc && (best == 0 || ms < best_ms)) {
            best = seg;
            best_ms = ms;
        }
        if (!rc && restore() != hipSuccess) rc = fail(IFDLBM_EDEVICE, "autotune: state restore");
    }
    h->rec_every = rec_every;
    h->opt.segment_rows = rc ? rows0 : best;
    int rc2 = rebuild_worklists(h);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(h->stream);
    for (void* p : {bf, bl, br, bq, static_cast<void*>(bs)})
        if (p) (void)hipFree(p);
    if (rc) return rc;
    if (rc2) return rc2;
    if (segment_rows) *segment_rows = best;
    if (ms_per_step) *ms_per_step = best_ms / steps_per_trial;
    return IFDLBM_OK;
}

static int ifdlbm_info_impl(ifdlbm_t* h, ifdlbm_info_t* info)
{
    if (!h || !info) return fail(IFDLBM_EINVAL, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_cavities = h->n_cav;
    for (int c = 0; c < h->n_cav; ++c)
        if (h->desc[c].active) {
            info->n_active++;
            info->nodes += (int64_t)h->desc[c].nx * h->desc[c].ny;
        }
    const int prec = h->opt.precision;
    info->state_bytes = (int64_t)(h->f_elems * f_elem_size(prec) + h->l_elems * l_elem_size(prec));
    info->alg_bytes_per_node = 2.0 * (9.0 * f_elem_size(prec) + l_elem_size(prec));
    int launches = units_per_step(h);
    if (!h->opt.batched) launches *= info->n_active;
    info->launches_per_step = launches;
    info->work_items = h->opt.kernel == IFDLBM_KERNEL_STAGED ? (int64_t)h->act_blocks.size() : (int64_t)h->act_items.size();
    return IFDLBM_OK;
}

static int ifdlbm_gradient_impl(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t objective, double* J,
                    double grad[3], bool no_alloc)
{
    if (!cav || !opt || !J || !grad) return fail(IFDLBM_EINVAL, "null argument");
    if (objective != IFDLBM_OBJ_KINETIC_ENERGY) return fail(IFDLBM_EINVAL, "unknown objective");
    if (n_steps < 1) return fail(IFDLBM_EINVAL, "n_steps must be >= 1");
    if (opt->lambda_mode != IFDLBM_LAMBDA_LAGGED)
        return fail(IFDLBM_EINVAL, "the tangent-linear gradient follows the lagged lambda of Step (2)");
    const ifdlbm_cavity& v = *cav;
    if (v.n_xi < 5 || v.n_eta < 5 || (int64_t)v.n_xi * v.n_eta > (int64_t)1 << 26)
        return fail(IFDLBM_EINVAL, "n_xi, n_eta must be >= 5 and n_xi * n_eta <= 2^26");
    if (!(v.theta_deg > 0.0 && v.theta_deg <= 90.0) || !(v.n > 0.0) || !(v.re > 0.0) || !(v.u_lid != 0.0) ||
        !std::isfinite(v.n) || !std::isfinite(v.re) || !std::isfinite(v.u_lid))
        return fail(IFDLBM_EINVAL, "cavity parameters outside their domain");
    if (!(opt->cfl > 0.0) || !(opt->mix >= 0.0 && opt->mix <= 1.0) || !(opt->gamma_min > 0.0) ||
        (opt->dt_rule != IFDLBM_DT_CONTRAVARIANT && opt->dt_rule != IFDLBM_DT_CARTESIAN))
        return fail(IFDLBM_EINVAL, "options outside their domain");
    if (no_alloc && tangent_workspace_elems(v.n_xi, v.n_eta) > tangent_scratch_capacity_elems())
        return fail(IFDLBM_EINVAL, "grid too large for the allocation-free gradient: it needs " +
                                       std::to_string(tangent_workspace_elems(v.n_xi, v.n_eta)) + " work values, the "
                                       "scratch array holds " + std::to_string(tangent_scratch_capacity_elems()) +
                                       " (48 per node)");
    hipStream_t s = static_cast<hipStream_t>(opt->hip_stream);
    bool own = false;
    if (!s && !no_alloc) {
        IFD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        own = true;
    }
    std::string err;
    hipError_t e = tangent_kinetic_energy(v.n_xi, v.n_eta, v.re, v.n, v.theta_deg, v.u_lid, opt->cfl, opt->mix,
                                          opt->gamma_min, opt->dt_rule, n_steps, s, J, grad, err, no_alloc);
    if (own) (void)hipStreamDestroy(s);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? IFDLBM_ENOMEM : IFDLBM_EDEVICE, err);
    return IFDLBM_OK;
}

static int ifdlbm_adjoint_impl(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t checkpoint_every,
                   int32_t objective, double* J, double grad[3])
{
    if (!cav || !opt || !J || !grad) return fail(IFDLBM_EINVAL, "null argument");
    if (objective != IFDLBM_OBJ_KINETIC_ENERGY) return fail(IFDLBM_EINVAL, "unknown objective");
    if (n_steps < 1) return fail(IFDLBM_EINVAL, "n_steps must be >= 1");
    if (checkpoint_every < 1) return fail(IFDLBM_EINVAL, "checkpoint_every must be >= 1");
    if ((n_steps + checkpoint_every - 1) / checkpoint_every > ((int64_t)1 << 24))
        return fail(IFDLBM_EINVAL, "more than 2^24 checkpoints: raise checkpoint_every");
    if (opt->lambda_mode != IFDLBM_LAMBDA_LAGGED)
        return fail(IFDLBM_EINVAL, "the adjoint follows the lagged lambda of Step (2)");
    ifdlbm_options o = *opt;
    o.graph_steps = 0;                 // one eager call per step: recomputation draws the same random words
    o.residual_every = 1 << 30;        // no residual work inside the sweeps
    o.batched = 1;
    ifdlbm_t* h = nullptr;
    int rc = ifdlbm_create(cav, 1, &o, &h);
    if (rc) return rc;
    const CavityDesc c = h->desc[0];
    const int prec = h->opt.precision;
    const size_t nn = (size_t)c.nx * c.ny, sd = 10 * nn;   // doubles per FP64 state
    const int64_t seg = std::min<int64_t>(checkpoint_every, n_steps);
    const int64_t n_ck = (n_steps + seg - 1) / seg;
    const size_t fbytes = h->f_elems * f_elem_size(prec), lbytes = h->l_elems * l_elem_size(prec);
    char *ck_f = nullptr, *ck_l = nullptr;
    uint32_t* ck_seed = nullptr;
    double* traj = nullptr;
    std::vector<int> ck_cur(n_ck);
    std::vector<int64_t> ck_count(n_ck);
    AdjointSweep sweep;
    hipStream_t s = h->stream;
    if (!rc) rc = dalloc(&ck_f, fbytes * n_ck);
    if (!rc) rc = dalloc(&ck_l, lbytes * n_ck);
    if (!rc) rc = dalloc(&ck_seed, sizeof(uint32_t) * n_ck);
    if (!rc) rc = dalloc(&traj, sizeof(double) * sd * (seg + 1));
    if (!rc) {
        hipError_t e = sweep.init(c, s);
        if (e != hipSuccess) rc = fail(e == hipErrorOutOfMemory ? IFDLBM_ENOMEM : IFDLBM_EDEVICE,
                                       std::string("adjoint buffers: ") + hipGetErrorString(e));
    }
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        rc = fail(IFDLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return false;
    };
    auto to_traj = [&](int64_t slot) {
        return hip_ok(launch_state_out(prec, h->d_f[h->cur], h->d_l[h->cur], c, 0.0, traj + slot * sd,
                                       traj + slot * sd + 9 * nn, s), "state out");
    };
    // forward sweep, keeping the state at every checkpoint
    for (int64_t q = 0; q < n_ck && !rc; ++q) {
        ck_cur[q] = h->cur;
        ck_count[q] = h->step_count;
        if (!hip_ok(hipMemcpyAsync(ck_f + q * fbytes, h->d_f[h->cur], fbytes, hipMemcpyDeviceToDevice, s), "checkpoint") ||
            !hip_ok(hipMemcpyAsync(ck_l + q * lbytes, h->d_l[h->cur], lbytes, hipMemcpyDeviceToDevice, s), "checkpoint") ||
            !hip_ok(hipMemcpyAsync(ck_seed + q, h->d_seed, sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "checkpoint"))
            break;
        const int64_t steps = std::min(seg, n_steps - q * seg);
        for (int64_t t = 0; t < steps && !rc; ++t) rc = eager_steps(h, 1);
    }
    // reverse sweep: recompute each segment from its checkpoint, then walk it backwards
    for (int64_t q = n_ck - 1; q >= 0 && !rc; --q) {
        h->cur = ck_cur[q];
        h->step_count = ck_count[q];
        if (!hip_ok(hipMemcpyAsync(h->d_f[h->cur], ck_f + q * fbytes, fbytes, hipMemcpyDeviceToDevice, s), "restore") ||
            !hip_ok(hipMemcpyAsync(h->d_l[h->cur], ck_l + q * lbytes, lbytes, hipMemcpyDeviceToDevice, s), "restore") ||
            !hip_ok(hipMemcpyAsync(h->d_seed, ck_seed + q, sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "restore") ||
            !to_traj(0))
            break;
        const int64_t steps = std::min(seg, n_steps - q * seg);
        for (int64_t t = 1; t <= steps && !rc; ++t)
            if (!(rc = eager_steps(h, 1))) to_traj(t);
        if (rc) break;
        if (q == n_ck - 1 && !hip_ok(sweep.objective(traj + steps * sd, s), "objective")) break;
        for (int64_t t = steps - 1; t >= 0 && !rc; --t)
            hip_ok(sweep.step_back(traj + t * sd, traj + (t + 1) * sd, s), "adjoint step");
        if (!rc && !hip_ok(hipStreamSynchronize(s), "adjoint segment")) break;
    }
    if (!rc) {
        // derivatives of the parameter rules of ifdlbm_create
        const ifdlbm_cavity& v = *cav;
        const double U = std::fabs(v.u_lid), sgn = v.u_lid < 0.0 ? -1.0 : 1.0;
        const bool contra = o.dt_rule == IFDLBM_DT_CONTRAVARIANT && !((1.0 + c.cot) / c.dxi < 1.0 / c.deta);
        const double dt_dcot = contra ? -c.dt / (1.0 + c.cot) : 0.0;
        hipError_t e = sweep.finish(c, dt_dcot, sgn / (v.re * kCs2), -c.K * std::log(U), (2.0 - v.n) * c.K / U * sgn, s,
                                    J, grad);
        if (hip_ok(e, "adjoint result") && !(std::isfinite(*J) && std::isfinite(grad[0]) && std::isfinite(grad[1]) &&
                                             std::isfinite(grad[2])))
            rc = fail(IFDLBM_EDIVERGED, "the trajectory or its adjoint became non-finite");
    }
    (void)hipStreamSynchronize(s);
    for (void* p : {static_cast<void*>(ck_f), static_cast<void*>(ck_l), static_cast<void*>(ck_seed), static_cast<void*>(traj)})
        if (p) (void)hipFree(p);
    ifdlbm_destroy(h);
    return rc;
}

static int ifdlbm_record_impl(ifdlbm_t* h, int32_t every, int32_t capacity)
{
    if (!h) return fail(IFDLBM_EINVAL, "null handle");
    if (every < 0) return fail(IFDLBM_EINVAL, "every must be >= 0");
    if (every > 0 && capacity < 1) return fail(IFDLBM_EINVAL, "capacity must be >= 1");
    if (every > 0 && h->opt.graph_steps > 0 && h->opt.graph_steps % every != 0)
        return fail(IFDLBM_EINVAL, "graph_steps must be a multiple of the recording interval");
    if (every > 0 && (int64_t)h->n_cav * capacity * 3 > ((int64_t)1 << 31))
        return fail(IFDLBM_EINVAL, "record too large (n_cavities * capacity * 3 must fit 2^31 doubles)");
    IFD_HIP(hipStreamSynchronize(h->stream));
    void* old[] = {h->d_rec, h->d_rec_count, h->d_probe_partial};
    for (void* p : old)
        if (p) IFD_HIP(hipFree(p));
    h->d_rec = nullptr;
    h->d_rec_count = nullptr;
    h->d_probe_partial = nullptr;
    h->rec_every = 0;
    h->rec_capacity = 0;
    h->graph_dirty = true;
    if (every == 0) return IFDLBM_OK;
    int rc = dalloc(&h->d_rec, (size_t)h->n_cav * capacity * 3 * sizeof(double));
    if (!rc) rc = dalloc(&h->d_rec_count, sizeof(uint32_t));
    if (!rc) rc = dalloc(&h->d_probe_partial, h->all_blocks.size() * sizeof(double));
    if (rc) return rc;
    IFD_HIP(hipMemsetAsync(h->d_rec_count, 0, sizeof(uint32_t), h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    h->rec_every = every;
    h->rec_capacity = capacity;
    h->rec_first_step = (h->step_count / every + 1) * every;
    return IFDLBM_OK;
}

static int ifdlbm_get_record_impl(ifdlbm_t* h, int32_t cav, int32_t max_samples, int32_t* n, int64_t* steps, double* u, double* v,
                      double* ke)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (!n) return fail(IFDLBM_EINVAL, "null sample count pointer");
    if (max_samples < 0) return fail(IFDLBM_EINVAL, "max_samples must be >= 0");
    *n = 0;
    if (h->rec_every == 0) return IFDLBM_OK;
    uint32_t count = 0;
    IFD_HIP(hipMemcpyAsync(&count, h->d_rec_count, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    std::vector<double> r((size_t)h->rec_capacity * 3);
    IFD_HIP(hipMemcpyAsync(r.data(), h->d_rec + (size_t)cav * h->rec_capacity * 3, r.size() * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    IFD_HIP(hipStreamSynchronize(h->stream));
    const int64_t avail = std::min<int64_t>(count, h->rec_capacity);
    const int64_t m = std::min<int64_t>(avail, max_samples);
    for (int64_t q = 0; q < m; ++q) {
        const int64_t sample = (int64_t)count - m + q;
        const size_t slot = (size_t)(sample % h->rec_capacity);
        if (steps) steps[q] = h->rec_first_step + sample * h->rec_every;
        if (u) u[q] = r[slot * 3 + 0];
        if (v) v[q] = r[slot * 3 + 1];
        if (ke) ke[q] = r[slot * 3 + 2];
    }
    *n = (int32_t)m;
    return IFDLBM_OK;
}

static int ifdlbm_time_step_impl(ifdlbm_t* h, int32_t cav, double* dt)
{
    int rc = check_cav(h, cav);
    if (rc) return rc;
    if (!dt) return fail(IFDLBM_EINVAL, "null dt pointer");
    *dt = h->desc[cav].dt;
    return IFDLBM_OK;
}

void ifdlbm_destroy(ifdlbm_t* h)
{
    try {
        if (!h) return;
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        free_all(h);
        delete h;
    } catch (...) {
    }
}

const char* ifdlbm_strerror(int code)
{
    switch (code) {
    case IFDLBM_OK: return "ok";
    case IFDLBM_EINVAL: return "invalid argument";
    case IFDLBM_ENOMEM: return "out of memory";
    case IFDLBM_EDEVICE: return "HIP device error";
    case IFDLBM_EDIVERGED: return "a cavity diverged";
    case IFDLBM_ENOTCONVERGED: return "not converged within max_steps";
    }
    return "unknown error code";
}

const char* ifdlbm_last_error(void) { return g_last_error.c_str(); }

static int ifdlbm_round_stochastic_device_impl(const double* v, const uint32_t* r16, float* out, int64_t n,
                                               void* hip_stream)
{
    if (n < 0) return fail(IFDLBM_EINVAL, "round_stochastic_device: n < 0");
    if (n > 0 && (!v || !r16 || !out)) return fail(IFDLBM_EINVAL, "round_stochastic_device: NULL array");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    IFD_HIP(launch_round_stochastic(v, r16, out, n, s));
    IFD_HIP(hipStreamSynchronize(s));
    return IFDLBM_OK;
}

static int ifdlbm_power_law_device_impl(const double* x, double y, double* out, int64_t n, void* hip_stream)
{
    if (n < 0) return fail(IFDLBM_EINVAL, "power_law_device: n < 0");
    if (n > 0 && (!x || !out)) return fail(IFDLBM_EINVAL, "power_law_device: NULL array");
    if (!std::isfinite(y)) return fail(IFDLBM_EINVAL, "power_law_device: exponent not finite");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    IFD_HIP(launch_power_law(x, y, out, n, s));
    IFD_HIP(hipStreamSynchronize(s));
    return IFDLBM_OK;
}

#ifndef IFD_SOURCE_DIGEST
#error "IFD_SOURCE_DIGEST: build the library with paper_2306_07603_amd/_build.py"
#endif
const char* ifdlbm_build_digest(void) { return IFD_SOURCE_DIGEST; }


// C entry points: no C++ exception crosses the ABI.
int ifdlbm_create(const ifdlbm_cavity* cav, int32_t n_cav, const ifdlbm_options* opt, ifdlbm_t** out)
{
    IFD_GUARD(ifdlbm_create_impl(cav, n_cav, opt, out));
}

int ifdlbm_step(ifdlbm_t* h, int64_t n_steps)
{
    IFD_GUARD(ifdlbm_step_impl(h, n_steps));
}

int ifdlbm_sync(ifdlbm_t* h)
{
    IFD_GUARD(ifdlbm_sync_impl(h));
}

int ifdlbm_get_residuals(ifdlbm_t* h, double* res_u, double* res_p)
{
    IFD_GUARD(ifdlbm_get_residuals_impl(h, res_u, res_p));
}

int ifdlbm_get_pressure_residuals(ifdlbm_t* h, double* res_p_printed, double* res_p_mean_removed)
{
    IFD_GUARD(ifdlbm_get_pressure_residuals_impl(h, res_p_printed, res_p_mean_removed));
}

int ifdlbm_run_to_steady(ifdlbm_t* h, double tol, int64_t max_steps, int64_t* steps_done, double* res_u, double* res_p)
{
    IFD_GUARD(ifdlbm_run_to_steady_impl(h, tol, max_steps, steps_done, res_u, res_p));
}

int ifdlbm_get_fields_device(ifdlbm_t* h, int32_t cav, void* u, void* v, void* p, int32_t dtype)
{
    IFD_GUARD(ifdlbm_get_fields_device_impl(h, cav, u, v, p, dtype));
}

int ifdlbm_round_stochastic_device(const double* v, const uint32_t* r16, float* out, int64_t n, void* hip_stream)
{
    IFD_GUARD(ifdlbm_round_stochastic_device_impl(v, r16, out, n, hip_stream));
}

int ifdlbm_power_law_device(const double* x, double y, double* out, int64_t n, void* hip_stream)
{
    IFD_GUARD(ifdlbm_power_law_device_impl(x, y, out, n, hip_stream));
}

int ifdlbm_get_fields(ifdlbm_t* h, int32_t cav, double* u, double* v, double* p)
{
    IFD_GUARD(ifdlbm_get_fields_impl(h, cav, u, v, p));
}

int ifdlbm_kinetic_energy(ifdlbm_t* h, int32_t cav, double* energy)
{
    IFD_GUARD(ifdlbm_kinetic_energy_impl(h, cav, energy));
}

int ifdlbm_get_state(ifdlbm_t* h, int32_t cav, double* fhat, double* lambda)
{
    IFD_GUARD(ifdlbm_get_state_impl(h, cav, fhat, lambda));
}

int ifdlbm_set_state(ifdlbm_t* h, int32_t cav, const double* fhat, const double* lambda)
{
    IFD_GUARD(ifdlbm_set_state_impl(h, cav, fhat, lambda));
}

int ifdlbm_status(ifdlbm_t* h, int32_t cav)
{
    IFD_GUARD(ifdlbm_status_impl(h, cav));
}

int ifdlbm_autotune(ifdlbm_t* h, int32_t steps_per_trial, int32_t* segment_rows, double* ms_per_step)
{
    IFD_GUARD(ifdlbm_autotune_impl(h, steps_per_trial, segment_rows, ms_per_step));
}

int ifdlbm_info(ifdlbm_t* h, ifdlbm_info_t* info)
{
    IFD_GUARD(ifdlbm_info_impl(h, info));
}

int ifdlbm_gradient(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t objective, double* J,
                    double grad[3])
{
    IFD_GUARD(ifdlbm_gradient_impl(cav, opt, n_steps, objective, J, grad, false));
}

int ifdlbm_gradient_noalloc(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t objective,
                            double* J, double grad[3])
{
    IFD_GUARD(ifdlbm_gradient_impl(cav, opt, n_steps, objective, J, grad, true));
}

int ifdlbm_adjoint(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t checkpoint_every,
                   int32_t objective, double* J, double grad[3])
{
    IFD_GUARD(ifdlbm_adjoint_impl(cav, opt, n_steps, checkpoint_every, objective, J, grad));
}

int ifdlbm_record(ifdlbm_t* h, int32_t every, int32_t capacity)
{
    IFD_GUARD(ifdlbm_record_impl(h, every, capacity));
}

int ifdlbm_get_record(ifdlbm_t* h, int32_t cav, int32_t max_samples, int32_t* n, int64_t* steps, double* u, double* v,
                      double* ke)
{
    IFD_GUARD(ifdlbm_get_record_impl(h, cav, max_samples, n, steps, u, v, ke));
}

int ifdlbm_time_step(ifdlbm_t* h, int32_t cav, double* dt)
{
    IFD_GUARD(ifdlbm_time_step_impl(h, cav, dt));
}

}  // extern "C"
