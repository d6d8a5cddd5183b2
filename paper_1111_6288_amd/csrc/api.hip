// libov host side: the context, its device memory, the drivers of the
// overlap pipeline and every extern "C" entry point of include/ov.h.
//
// Pipeline of one sign application on a batch (Sec. 2):
//   C = V^dag x, chi = x - V C                       (FP64 projection, matrix cores)
//   Clenshaw b_k = c_k chi + 2 T b_{k+1} - b_{k+2}, k = n..1,
//     T = (2 Q^2 - (1+eps)) / (1-eps), Q = H_w / norm:  two dslash launches per
//     step, the second one with the recursion fused into its epilogue
//   z = c_0 chi + T b_1 - b_2, w = Q z
//   s = w - V (V^dag w) + V sgn(lambda) C            (FP64 projection)
// D(m) = (1 - m/2)(1 + gamma5 s) + m (eq. (1) with a quark mass), and the CG
// of Sec. 3.2 runs on D(m)^dag D(m) with FP64 defect correction around an
// inner solve in the requested precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dense.h"
#include "ov.h"
#include "ov_internal.h"

using namespace ov;

// A roctx range around every entry point that launches work, so a profiler
// timeline (rocprofv3 --marker-trace) shows which API call issued each kernel;
// without a profiler attached the calls return at once.
struct OvRange {
    explicit OvRange(const char *name) { roctxRangePushA(name); }
    ~OvRange() { roctxRangePop(); }
};
#define OV_RANGE(name) OvRange ov_range_guard_(name)

// Fixed device scratch of ov_dslash_noalloc (see scratch_init below).
constexpr size_t kScratchBytes = 64ul << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

enum ProfClass { PC_DSLASH = 0, PC_CLENSHAW, PC_PROJ_DOT, PC_PROJ_EXPAND, PC_BLAS, PC_FORCE, PC_N };
const char *kProfNames[PC_N] = {"dslash", "clenshaw", "proj_dot", "proj_expand", "blas", "force"};

struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

struct Small {
    int l = 0;
    double2 *V = nullptr;     // planes [l][12][Vp]
    double *sgn = nullptr;    // [l]
};

struct Defl {
    int k = 0;
    double2 *W = nullptr;     // planes [k][12][Vp]
    std::vector<double> a, b; // ||D_ov w||^2, Re<w, D_ov w>
};

}  // namespace

struct ov_ctx {
    int device = 0;
    hipStream_t stream = nullptr;   // caller's stream; nullptr is the null stream
    int L[4] = {0, 0, 0, 0}, bc[4] = {0, 0, 0, 0};
    double mw = 0;
    Geo g{};
    std::string err;

    bool have_gauge = false;
    bool recon_allow = true;         // use two-row links when the uploaded links are SU(3)
    bool recon = false;              // kernels read two rows and rebuild the third
    double row3_dev = -1;            // max |u_2 - conj(u_0 x u_1)| of the uploaded links
    double2 *U64 = nullptr;
    float2 *U32 = nullptr;
    uint32_t *U16 = nullptr;

    int nfield = 0;
    std::vector<double> q, eta;
    cx<double> *phase = nullptr;     // [nfield][Lt]

    bool have_sign = false;
    int npoly = 0;
    double eps = 0, norm = 0;
    std::vector<double> coef;

    // norm safety: max Frobenius |U_eff - U| of the links the FP32 / BF16
    // kernels apply ([prec][0 nine entries, 1 two rows + rebuilt third]),
    // the growth bound of the current polynomial and the check mode
    double link_dev[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    std::vector<double> bound_coef;   // coefficients sign_bound2 was computed for
    double sign_bound2 = 0;
    int norm_check = 2;               // 0 off; 1 flag only; 2 flag and sign/D(m) applies synchronise

    std::vector<Small> small;
    std::vector<Defl> defl;

    // workspace arena (grow-only, sized at the start of each entry point)
    char *ws = nullptr;
    size_t ws_size = 0;
    size_t ws_top = 0;

    // content-keyed caches of small device arrays
    std::map<std::vector<int>, int *> icache;
    std::map<std::vector<double>, double *> dcache;
    std::map<std::vector<double>, double2 *> ccache;

    // dslash launch shape per precision and kind (0: plain, 1: fused Clenshaw epilogue)
    struct Launch {
        int nr = 2, block = 128, order = 0, cap = 0, stream_hint = 0, split = 1, cols = 1, wshare = 1;
    };
    Launch tune[3][2];

    // profiling
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<ProfRec> recs;

    // persistent small device scratch: [0] non-finite count, [8] row-3 deviation bits,
    // [16] norm-breach flag, [32..63] link rounding deviation bits
    int *d_count = nullptr;

    // pinned host words for the lagged reads of the CG's active flags
    int *h_pin = nullptr;
    size_t h_pin_n = 0;
    hipEvent_t ev_mask[2] = {nullptr, nullptr};

    // device address of the fixed scratch array of ov_dslash_noalloc on this device
    void *scratch = nullptr;

    size_t mem_bytes = 0;

    // captured pipelines (hipGraph), keyed by everything the launch sequence depends on
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::map<std::string, std::pair<int, hipGraphExec_t>> graphs;   // (times seen, executable)
};

namespace {

int fail(ov_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(c, OV_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                     \
    } while (0)

#define CHK(expr)                    \
    do {                             \
        int r_ = (expr);             \
        if (r_ != OV_OK) return r_;  \
    } while (0)

int dev_alloc(ov_ctx *c, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(c, OV_ENOMEM, "hipMalloc of %.3f GB failed: %s", bytes / 1e9, hipGetErrorString(e));
    }
    c->mem_bytes += bytes;
    return OV_OK;
}

void dev_free(ov_ctx *c, void *p, size_t bytes)
{
    if (p) {
        (void)hipFree(p);
        c->mem_bytes -= std::min(c->mem_bytes, bytes);
    }
}

size_t field_elems(const ov_ctx *c) { return 12ul * c->g.Vp; }

template <class S>
size_t field_bytes(const ov_ctx *c) { return field_elems(c) * sizeof(S); }

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Drop every captured pipeline: called whenever a pointer or a constant that
// a capture baked in changes (arena, phase table, small spaces, polynomial, tuning).
void invalidate_graphs(ov_ctx *c)
{
    for (auto &kv : c->graphs)
        if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
    c->graphs.clear();
}

// Two-row links are used only when every uploaded link satisfies the SU(3)
// row identity to FP64 rounding (entries of an SU(3) matrix are at most 1 in
// modulus, so the bound is absolute); the captured pipelines hold the kernel
// choice, so a change of format drops them.
constexpr double kRow3Tol = 1e-14;

void update_link_format(ov_ctx *c)
{
    const bool r = c->recon_allow && c->have_gauge && c->row3_dev >= 0 && c->row3_dev <= kRow3Tol;
    if (r != c->recon) invalidate_graphs(c);
    c->recon = r;
}

// Make sure the arena holds `bytes`; only called before any pointer is handed out.
int ws_reserve(ov_ctx *c, size_t bytes)
{
    c->ws_top = 0;
    if (bytes <= c->ws_size) return OV_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    invalidate_graphs(c);
    dev_free(c, c->ws, c->ws_size);
    c->ws = nullptr;
    c->ws_size = 0;
    CHK(dev_alloc(c, (void **)&c->ws, bytes));
    c->ws_size = bytes;
    // fresh workspace starts zeroed so that padding sites hold zeros
    HIPCHK(hipMemsetAsync(c->ws, 0, bytes, c->stream));
    return OV_OK;
}

template <class T>
T *ws_take(ov_ctx *c, size_t count)
{
    size_t bytes = align_up(count * sizeof(T));
    if (c->ws_top + bytes > c->ws_size) return nullptr;
    T *p = (T *)(c->ws + c->ws_top);
    c->ws_top += bytes;
    return p;
}

// Host-to-device copy ordered on the context stream; returns once it landed.
hipError_t h2d(ov_ctx *c, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

// Run `body` (a sequence of kernel launches on c->stream, no host sync, no
// allocation, no memset) through a cached hipGraph: the first call with a
// key runs eagerly (this fills every cache the body needs), the second one
// captures on a private stream and launches the graph on c->stream, later
// ones replay it.  Profiling turns capture off.
template <class F>
int run_graph(ov_ctx *c, const std::string &key, F &&body)
{
    if (!c->use_graphs || c->prof_on) return body();
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        c->graphs[key] = {1, nullptr};
        return body();
    }
    if (it->second.second) {
        HIPCHK(hipGraphLaunch(it->second.second, c->stream));
        return OV_OK;
    }
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = body();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    c->stream = saved;
    if (rc != OV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(c, OV_EHIP, "stream capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, OV_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    it->second.second = exec;
    HIPCHK(hipGraphLaunch(exec, c->stream));
    return OV_OK;
}

template <class T>
void key_add(std::string &k, const std::vector<T> &v)
{
    k.append((const char *)v.data(), v.size() * sizeof(T));
    k.push_back('|');
}

const int *dev_ints(ov_ctx *c, const std::vector<int> &v)
{
    if (v.empty()) return nullptr;
    auto it = c->icache.find(v);
    if (it != c->icache.end()) return it->second;
    int *p = nullptr;
    if (dev_alloc(c, (void **)&p, v.size() * sizeof(int)) != OV_OK) return nullptr;
    if (h2d(c, p, v.data(), v.size() * sizeof(int)) != hipSuccess) return nullptr;
    c->icache[v] = p;
    return p;
}

const double *dev_doubles(ov_ctx *c, const std::vector<double> &v)
{
    if (v.empty()) return nullptr;
    auto it = c->dcache.find(v);
    if (it != c->dcache.end()) return it->second;
    double *p = nullptr;
    if (dev_alloc(c, (void **)&p, v.size() * sizeof(double)) != OV_OK) return nullptr;
    if (h2d(c, p, v.data(), v.size() * sizeof(double)) != hipSuccess) return nullptr;
    c->dcache[v] = p;
    return p;
}

// complex coefficients given as interleaved (re, im) pairs
const double2 *dev_cplx(ov_ctx *c, const std::vector<double> &v)
{
    if (v.empty()) return nullptr;
    auto it = c->ccache.find(v);
    if (it != c->ccache.end()) return it->second;
    double2 *p = nullptr;
    if (dev_alloc(c, (void **)&p, v.size() * sizeof(double)) != OV_OK) return nullptr;
    if (h2d(c, p, v.data(), v.size() * sizeof(double)) != hipSuccess) return nullptr;
    c->ccache[v] = p;
    return p;
}

// ---------------------------------------------------------------- profiling
int prof_begin(ov_ctx *c)
{
    if (!c->prof_on) return -1;
    if (c->ev_used + 2 > c->ev_pool.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->ev_pool.push_back(e);
        }
    }
    hipEvent_t a = c->ev_pool[c->ev_used++];
    hipEvent_t b = c->ev_pool[c->ev_used++];
    if (hipEventRecord(a, c->stream) != hipSuccess) return -1;
    c->recs.push_back({-1, a, b, 0});
    return (int)c->recs.size() - 1;
}

void prof_end(ov_ctx *c, int idx, int cls, double bytes)
{
    if (idx < 0) return;
    c->recs[idx].cls = cls;
    c->recs[idx].bytes = bytes;
    (void)hipEventRecord(c->recs[idx].b, c->stream);
}

// ---------------------------------------------------------------- batches
// A batch names fields by storage index; groups split it by background field.
struct Batch {
    int n = 0;
    std::vector<int> slots_h;         // storage indices
    const int *slots = nullptr;       // device copy (NULL when identity 0..n-1)
    struct Grp {
        int f;
        std::vector<int> slots_h;
        const int *slots;
    };
    std::vector<Grp> groups;
};

int make_batch(ov_ctx *c, const std::vector<int> &slots, const std::vector<int> &grp_of_slot, Batch &b)
{
    b = Batch();
    b.n = (int)slots.size();
    b.slots_h = slots;
    bool ident = true;
    for (int j = 0; j < b.n; ++j) ident = ident && slots[j] == j;
    if (!ident) {
        b.slots = dev_ints(c, slots);
        if (!b.slots) return fail(c, OV_ENOMEM, "slot list upload failed");
    }
    std::map<int, std::vector<int>> by;
    for (int j = 0; j < b.n; ++j) by[grp_of_slot[slots[j]]].push_back(slots[j]);
    for (auto &kv : by) {
        Batch::Grp g;
        g.f = kv.first;
        g.slots_h = kv.second;
        g.slots = dev_ints(c, kv.second);
        if (!g.slots) return fail(c, OV_ENOMEM, "group list upload failed");
        b.groups.push_back(g);
    }
    return OV_OK;
}

// ---------------------------------------------------------------- precision map
template <class S>
struct PrecOf;
template <>
struct PrecOf<double2> {
    static constexpr int p = OV_FP64;
};
template <>
struct PrecOf<float2> {
    static constexpr int p = OV_FP32;
};
template <>
struct PrecOf<uint32_t> {
    static constexpr int p = OV_BF16;
};

template <class S>
const S *links_of(const ov_ctx *c);
template <>
const double2 *links_of<double2>(const ov_ctx *c) { return c->U64; }
template <>
const float2 *links_of<float2>(const ov_ctx *c) { return c->U32; }
template <>
const uint32_t *links_of<uint32_t>(const ov_ctx *c) { return c->U16; }

// ---------------------------------------------------------------- launch helpers
template <class S>
int dslash_launch(ov_ctx *c, const Batch &b, const int *fgroup, const S *x, S *y, double a, bool hw,
                  const S *e1 = nullptr, double c1 = 0, const S *e2 = nullptr, double c2 = 0,
                  const S *e3 = nullptr, double c3 = 0)
{
    if (b.n == 0) return OV_OK;
    DsArgs<S> d{};
    d.x = x;
    d.y = y;
    d.fstride = (long)field_elems(c);
    d.U = links_of<S>(c);
    d.slots = b.slots;
    d.n = b.n;
    d.fgroup = fgroup;
    d.phase = c->phase;
    d.g = c->g;
    d.diag = 4.0 + c->mw;
    d.a = a;
    d.e1 = e1;
    d.e2 = e2;
    d.e3 = e3;
    d.c1 = c1;
    d.c2 = c2;
    d.c3 = c3;
    const int P = PrecOf<S>::p;
    const bool epi = e1 || e2 || e3;
    const auto &tu = c->tune[P][epi ? 1 : 0];
    d.order = tu.order;
    d.blocks_per_cu = tu.cap;
    d.stream_hint = tu.stream_hint;
    d.cols = tu.cols;
    d.recon = c->recon ? 1 : 0;
    if (d.order == 2) {   // t-chunks: enough workgroups to fill the GPU, chunks of at least 4
        const int W = tu.block == 512 ? 8 : 4;   // right-hand sides per workgroup
        const long per_chunk = (long)c->g.Lz * ((c->g.Lxy + 63) / 64) * ((b.n + W - 1) / W);
        int nch = (int)std::max(1L, std::min((long)c->g.Lt / 4, (4096 + per_chunk - 1) / per_chunk));
        d.tchunk = (c->g.Lt + nch - 1) / nch;
    }
    int nr = tu.nr, split = tu.split, ws = tu.wshare;
    while (split > 1 && (split / 2) * nr >= b.n) split /= 2;
    while (nr > 1 && nr / 2 >= b.n) nr /= 2;
    while (ws > 1 && (ws / 2) * split * nr >= b.n) ws /= 2;   // no wave without a RHS
    d.wshare = ws;
    int pi = prof_begin(c);
    HIPCHK(launch_dslash<S>(d, hw || epi, epi, nr, tu.block, split, c->stream));
    const double sb = sizeof(S);
    const int nex = (e1 ? 1 : 0) + (e2 ? 1 : 0) + (e3 ? 1 : 0);
    // compulsory bytes: the links once (two rows of each when rebuilt), every
    // input and epilogue field once, the output once
    prof_end(c, pi, epi ? PC_CLENSHAW : PC_DSLASH,
             (double)c->g.V * ((c->recon ? 24.0 : 36.0) * sb + (double)b.n * 12.0 * sb * (2 + nex)));
    return OV_OK;
}

template <class SI, class SO>
int lincomb(ov_ctx *c, const Batch &b, SO *out, int nin, const SI *const *in, const double2 *const *coefs,
            const double2 *cconst, int g5mask, double *red = nullptr, int *nblk = nullptr)
{
    if (b.n == 0) return OV_OK;
    LcArgs<SI, SO> a{};
    a.nin = nin;
    for (int t = 0; t < nin; ++t) {
        a.in[t] = in[t];
        a.istride[t] = (long)field_elems(c);
        a.coef[t] = coefs ? coefs[t] : nullptr;
        a.cconst[t] = cconst ? cconst[t] : make_double2(1.0, 0.0);
    }
    a.coef_by_slot = 1;
    a.g5mask = g5mask;
    a.out = out;
    a.ostride = (long)field_elems(c);
    a.slots = b.slots;
    a.n = b.n;
    a.Vp = c->g.Vp;
    a.red = red;
    int pi = prof_begin(c);
    HIPCHK((launch_lincomb<SI, SO>(a, c->stream, nblk)));
    prof_end(c, pi, PC_BLAS, (double)b.n * field_elems(c) * (nin * sizeof(SI) + sizeof(SO)));
    return OV_OK;
}

// y = x (copy / precision conversion) for the entries of b
template <class SI, class SO>
int copy_fields(ov_ctx *c, const Batch &b, const SI *x, SO *y, int g5 = 0)
{
    const SI *in[1] = {x};
    return lincomb<SI, SO>(c, b, y, 1, in, nullptr, nullptr, g5);
}

template <class S>
int proj_dot(ov_ctx *c, const double2 *V, int l, const S *X, const Batch::Grp &gr, double2 *C, double2 *part)
{
    const int n = (int)gr.slots_h.size();
    for (int j0 = 0; j0 < n; j0 += 48) {
        const int nn = std::min(48, n - j0);
        int pi = prof_begin(c);
        HIPCHK(launch_proj_dot<S>(V, l, (long)field_elems(c), X, (long)field_elems(c), gr.slots + j0, nn, c->g.Vp,
                                  0, part, C + (long)j0 * l, c->stream));
        prof_end(c, pi, PC_PROJ_DOT, (double)field_elems(c) * (l * 16.0 + nn * (double)sizeof(S)));
    }
    return OV_OK;
}

template <class SX, class SY>
int proj_expand(ov_ctx *c, const double2 *V, int l, const SX *X, double alpha, SY *Y, const Batch::Grp &gr,
                const double2 *E, double beta)
{
    const int n = (int)gr.slots_h.size();
    for (int j0 = 0; j0 < n; j0 += 48) {
        const int nn = std::min(48, n - j0);
        int pi = prof_begin(c);
        HIPCHK((launch_proj_expand<SX, SY>(V, l, (long)field_elems(c), X, (long)field_elems(c), alpha, Y,
                                           (long)field_elems(c), gr.slots + j0, nn, c->g.Vp, E + (long)j0 * l, beta,
                                           c->stream)));
        prof_end(c, pi, PC_PROJ_EXPAND,
                 (double)field_elems(c) * (l * 16.0 + nn * (double)(sizeof(SY) + (X ? sizeof(SX) : 0))));
    }
    return OV_OK;
}

// ---------------------------------------------------------------- norm safety
int *norm_flag(const ov_ctx *c) { return (int *)((char *)c->d_count + 16); }

// Norm that the kernels of precision S divide H_w by.  The FP32 and BF16
// kernels apply rounded links U_eff with ||H_w(U_eff)|| <= ||H_w(U)|| +
// 4 max ||U_eff - U||: the hopping term of one direction has norm max ||U||
// (its two halves act on complementary spin projectors), and there are four
// directions.  A bound for the uploaded links therefore becomes one for the
// applied links after adding that margin (plus 1e-6 per link for the FP32
// evaluation of a rebuilt third row).
template <class S>
double norm_of(const ov_ctx *c)
{
    const int p = PrecOf<S>::p;
    if (p == OV_FP64) return c->norm;
    return c->norm + 4.0 * (c->link_dev[p][c->recon ? 1 : 0] + 1e-6);
}

// (slack * max_{0 <= q <= 1} |q P(q^2)|)^2 for the current coefficients, on a
// grid of q (P evaluated by Clenshaw in FP64).  The interpolant of y^{-1/2}
// gives a maximum within 1e-5 of 1; the 2 % slack covers the grid and the
// rounding of an FP32 recursion.  Outside [-1, 1] the polynomial grows like
// a Chebyshev polynomial (at degree 300 a spectrum 1 % beyond the bound
// multiplies some components by ~1e25), which is what the check detects.
void update_sign_bound(ov_ctx *c)
{
    if (c->bound_coef == c->coef) return;
    const int n = (int)c->coef.size() - 1;
    const int G = n <= 2000 ? 4001 : 1001;
    double M = 0.0;
    for (int i = 0; i <= G; ++i) {
        const double q = (double)i / G;
        const double x = (2.0 * q * q - 1.0 - c->eps) / (1.0 - c->eps);
        double b1 = 0.0, b2 = 0.0;
        for (int k = n; k >= 1; --k) {
            const double b0 = c->coef[k] + 2.0 * x * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
        const double v = q * (c->coef[0] + x * b1 - b2);
        M = std::max(M, std::fabs(v));
    }
    const double b = 1.02 * M;
    c->sign_bound2 = b * b;
    c->bound_coef = c->coef;
}

// Read and clear the norm-breach flag (synchronises).  OV_ENORM if a sign
// application since the last clear saw the polynomial grow beyond its bound.
int take_norm_flag(ov_ctx *c)
{
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, norm_flag(c), sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!h) return OV_OK;
    HIPCHK(launch_fill_int(norm_flag(c), 1, 0, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return fail(c, OV_ENORM,
                "norm bound %.6g is below ||H_w||: the Chebyshev recursion grew beyond its bound on [-1, 1] "
                "(pass a larger norm to ov_set_sign_params)",
                c->norm);
}

// Clear the flag at the start of a synchronising entry point.
int clear_norm_flag(ov_ctx *c)
{
    HIPCHK(launch_fill_int(norm_flag(c), 1, 0, c->stream));
    return OV_OK;
}

// Result of a synchronising entry point: a breach seen during the call takes
// precedence over OV_ENOCONV / OV_ENAN (both are what a breach produces).
int with_norm_status(ov_ctx *c, int rc)
{
    if (c->norm_check == 0 || !(rc == OV_OK || rc == OV_ENOCONV || rc == OV_ENAN || rc == OV_EBREAKDOWN))
        return rc;
    const int r2 = take_norm_flag(c);
    return r2 != OV_OK ? r2 : rc;
}

// ---------------------------------------------------------------- sign pipeline
template <class S>
struct SignBufs {
    S *chi = nullptr, *B[3] = {nullptr, nullptr, nullptr}, *T = nullptr;
    double2 *C = nullptr, *D = nullptr, *E = nullptr, *part = nullptr;
    double2 *npart = nullptr, *chi2 = nullptr, *w2 = nullptr;   // norm check: dot partials, |chi|^2, |w|^2
};

size_t small_arrays_bytes(const ov_ctx *c, int nstore)
{
    int lmax = 1;
    for (auto &s : c->small) lmax = std::max(lmax, s.l);
    for (auto &d : c->defl) lmax = std::max(lmax, d.k);
    const long K = 12L * c->g.Vp;
    const long nchunk = (K + proj_dot_chunk(K) - 1) / proj_dot_chunk(K);
    return 3 * align_up((size_t)nstore * lmax * 16) + align_up((size_t)nchunk * 48 * 256 * 16) +
           align_up((8192 + (size_t)nstore) * 16) + 2 * align_up((size_t)nstore * 16);
}

template <class S>
int take_sign_bufs(ov_ctx *c, int nstore, SignBufs<S> &w)
{
    const size_t fe = field_elems(c) * nstore;
    w.chi = ws_take<S>(c, fe);
    for (int i = 0; i < 3; ++i) w.B[i] = ws_take<S>(c, fe);
    w.T = ws_take<S>(c, fe);
    int lmax = 1;
    for (auto &s : c->small) lmax = std::max(lmax, s.l);
    for (auto &d : c->defl) lmax = std::max(lmax, d.k);
    w.C = ws_take<double2>(c, (size_t)nstore * lmax);
    w.D = ws_take<double2>(c, (size_t)nstore * lmax);
    w.E = ws_take<double2>(c, (size_t)nstore * lmax);
    const long K = 12L * c->g.Vp;
    const long nchunk = (K + proj_dot_chunk(K) - 1) / proj_dot_chunk(K);
    w.part = ws_take<double2>(c, (size_t)nchunk * 48 * 256);
    w.npart = ws_take<double2>(c, 8192 + (size_t)nstore);
    w.chi2 = ws_take<double2>(c, nstore);
    w.w2 = ws_take<double2>(c, nstore);
    if (!w.chi || !w.B[2] || !w.T || !w.part || !w.w2) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    return OV_OK;
}

template <class S>
size_t sign_bufs_bytes(const ov_ctx *c, int nstore)
{
    return 5 * align_up(field_bytes<S>(c) * nstore) + small_arrays_bytes(c, nstore);
}

// OUT = s(X) on the batch.  OUT may alias X.  C/D/E hold per-group blocks at
// offset (position of the group's first entry) * l.
template <class S>
int sign_batch(ov_ctx *c, const Batch &b, const int *fgroup, const S *X, S *OUT, SignBufs<S> &w)
{
    if (b.n == 0) return OV_OK;
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    bool any_small = false;
    for (auto &gr : b.groups) any_small = any_small || c->small[gr.f].l > 0;

    // 1. chi = Pi X, C = V^dag X
    const S *chi = X;
    std::vector<long> goff(b.groups.size());
    {
        long o = 0;
        for (size_t gi = 0; gi < b.groups.size(); ++gi) {
            goff[gi] = o;
            o += (long)b.groups[gi].slots_h.size() * std::max(1, c->small[b.groups[gi].f].l);
        }
    }
    if (any_small) {
        chi = w.chi;
        for (size_t gi = 0; gi < b.groups.size(); ++gi) {
            const auto &gr = b.groups[gi];
            const Small &sm = c->small[gr.f];
            Batch gb;
            gb.n = (int)gr.slots_h.size();
            gb.slots = gr.slots;
            if (sm.l > 0) {
                CHK(proj_dot<S>(c, sm.V, sm.l, X, gr, w.C + goff[gi], w.part));
                CHK((proj_expand<S, S>(c, sm.V, sm.l, X, 1.0, w.chi, gr, w.C + goff[gi], -1.0)));
            } else {
                CHK((copy_fields<S, S>(c, gb, X, w.chi)));
            }
        }
    }

    // |chi|^2 per RHS for the norm check (before OUT, which may alias X = chi, is written)
    const bool check = c->norm_check != 0;
    const long fe = (long)field_elems(c);
    if (check) {
        update_sign_bound(c);
        HIPCHK((launch_dot<S, S>(chi, fe, chi, fe, b.slots, b.n, c->g.Vp, 0, w.npart, w.chi2, b.slots, c->stream)));
    }

    // 2. Clenshaw recursion
    const double N = norm_of<S>(c);
    const double al = 2.0 / ((1.0 - c->eps) * N * N);
    const double be = (1.0 + c->eps) / (1.0 - c->eps);
    const int n = c->npoly;
    {
        const S *in[1] = {chi};
        const double2 cc[1] = {make_double2(c->coef[n], 0.0)};
        CHK((lincomb<S, S>(c, b, w.B[0], 1, in, nullptr, cc, 0)));
    }
    int i1 = 0, i2 = -1;
    for (int k = n - 1; k >= 1; --k) {
        CHK(dslash_launch<S>(c, b, fgroup, w.B[i1], w.T, 1.0, true));
        const int io = (i2 >= 0) ? i2 : (i1 + 1) % 3;
        CHK(dslash_launch<S>(c, b, fgroup, w.T, w.B[io], 2.0 * al, true, chi, c->coef[k], w.B[i1], -2.0 * be,
                             i2 >= 0 ? w.B[i2] : nullptr, -1.0));
        i2 = i1;
        i1 = io;
    }
    CHK(dslash_launch<S>(c, b, fgroup, w.B[i1], w.T, 1.0, true));
    const int iz = (i2 >= 0) ? i2 : (i1 + 1) % 3;
    CHK(dslash_launch<S>(c, b, fgroup, w.T, w.B[iz], al, true, chi, c->coef[0], w.B[i1], -be,
                         i2 >= 0 ? w.B[i2] : nullptr, -1.0));

    // 3. w = Q z
    S *wout = any_small ? w.T : OUT;
    CHK(dslash_launch<S>(c, b, fgroup, w.B[iz], wout, 1.0 / N, true));
    if (check) {   // ||w|| <= M ||chi|| holds whenever the spectrum of Q lies in [-1, 1]
        HIPCHK((launch_dot<S, S>(wout, fe, wout, fe, b.slots, b.n, c->g.Vp, 0, w.npart, w.w2, b.slots, c->stream)));
        HIPCHK(launch_norm_breach(w.chi2, w.w2, b.slots, b.n, c->sign_bound2, norm_flag(c), c->stream));
    }

    // 4. OUT = w - V (V^dag w) + V sgn C
    if (any_small) {
        for (size_t gi = 0; gi < b.groups.size(); ++gi) {
            const auto &gr = b.groups[gi];
            const Small &sm = c->small[gr.f];
            const int ng = (int)gr.slots_h.size();
            if (sm.l > 0) {
                CHK(proj_dot<S>(c, sm.V, sm.l, wout, gr, w.D + goff[gi], w.part));
                HIPCHK(launch_small_combine(w.C + goff[gi], w.D + goff[gi], sm.sgn, sm.l, ng, w.E + goff[gi],
                                            c->stream));
                CHK((proj_expand<S, S>(c, sm.V, sm.l, wout, 1.0, OUT, gr, w.E + goff[gi], 1.0)));
            } else {
                Batch gb;
                gb.n = ng;
                gb.slots = gr.slots;
                CHK((copy_fields<S, S>(c, gb, wout, OUT)));
            }
        }
    }
    return OV_OK;
}

// ---------------------------------------------------------------- D(m)
template <class S>
struct DovBufs {
    SignBufs<S> sb;
    S *XG = nullptr, *Sv = nullptr;
};

template <class S>
size_t dov_bufs_bytes(const ov_ctx *c, int nstore)
{
    return sign_bufs_bytes<S>(c, nstore) + 2 * align_up(field_bytes<S>(c) * nstore);
}

template <class S>
int take_dov_bufs(ov_ctx *c, int nstore, DovBufs<S> &w)
{
    CHK(take_sign_bufs<S>(c, nstore, w.sb));
    w.XG = ws_take<S>(c, field_elems(c) * nstore);
    w.Sv = ws_take<S>(c, field_elems(c) * nstore);
    if (!w.Sv) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    return OV_OK;
}

// Y = D(m) X or D(m)^dag X; ca = 1 + m/2, cb = 1 - m/2 per storage index.  Y may alias X.
template <class S>
int dov_batch(ov_ctx *c, const Batch &b, const int *fgroup, const double2 *ca, const double2 *cb, bool dagger,
              const S *X, S *Y, DovBufs<S> &w)
{
    if (b.n == 0) return OV_OK;
    const S *sin = X;
    if (dagger) {
        CHK((copy_fields<S, S>(c, b, X, w.XG, 1)));
        sin = w.XG;
    }
    CHK(sign_batch<S>(c, b, fgroup, sin, w.Sv, w.sb));
    // non-dagger: Y = ca X + cb gamma5 s ; dagger: Y = ca X + cb s
    const S *in[2] = {X, w.Sv};
    const double2 *cf[2] = {ca, cb};
    return lincomb<S, S>(c, b, Y, 2, in, cf, nullptr, dagger ? 0 : 2);
}

int mass_coefs(ov_ctx *c, int n, const double *mass, const double2 **ca, const double2 **cb)
{
    std::vector<double> a(2 * n), bb(2 * n);
    for (int j = 0; j < n; ++j) {
        a[2 * j] = 1.0 + 0.5 * mass[j];
        a[2 * j + 1] = 0.0;
        bb[2 * j] = 1.0 - 0.5 * mass[j];
        bb[2 * j + 1] = 0.0;
    }
    *ca = dev_cplx(c, a);
    *cb = dev_cplx(c, bb);
    if (!*ca || !*cb) return fail(c, OV_ENOMEM, "coefficient upload failed");
    return OV_OK;
}

// ---------------------------------------------------------------- validation
int check_ctx(ov_ctx *c)
{
    if (!c) return OV_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, OV_EHIP, "hipSetDevice(%d) failed", c->device);
    return OV_OK;
}

int check_fields(ov_ctx *c, int nrhs, const int *field_of_rhs, std::vector<int> &grp)
{
    if (nrhs <= 0) return fail(c, OV_EINVAL, "nrhs must be positive (got %d)", nrhs);
    if (nrhs > 4096) return fail(c, OV_EINVAL, "nrhs above 4096");
    grp.assign(nrhs, 0);
    for (int j = 0; j < nrhs; ++j) {
        int f = field_of_rhs ? field_of_rhs[j] : 0;
        if (f < 0 || f >= std::max(1, c->nfield))
            return fail(c, OV_EINVAL, "field_of_rhs[%d] = %d outside [0, %d)", j, f, std::max(1, c->nfield));
        grp[j] = f;
    }
    if (c->nfield == 0) return fail(c, OV_ESTATE, "ov_set_fields has not been called");
    return OV_OK;
}

int check_prec(ov_ctx *c, int prec)
{
    if (prec != OV_FP64 && prec != OV_FP32 && prec != OV_BF16) return fail(c, OV_EINVAL, "unknown precision %d", prec);
    return OV_OK;
}

std::vector<int> iota_vec(int n)
{
    std::vector<int> v(n);
    for (int j = 0; j < n; ++j) v[j] = j;
    return v;
}

// Chebyshev interpolant of y^{-1/2} on [eps, 1] at the n+1 Chebyshev-Gauss
// nodes, in the variable t = (2y - 1 - eps)/(1 - eps) (Sec. 2: P(x) ~ x^{-1/2}).
void cheb_interp(int n, double eps, std::vector<double> &c)
{
    const int m = n + 1;
    std::vector<double> fy(m), th(m);
    for (int j = 0; j < m; ++j) {
        th[j] = M_PI * (j + 0.5) / m;
        const double y = 0.5 * ((1.0 - eps) * std::cos(th[j]) + 1.0 + eps);
        fy[j] = 1.0 / std::sqrt(y);
    }
    c.assign(m, 0.0);
    for (int k = 0; k < m; ++k) {
        double s = 0;
        for (int j = 0; j < m; ++j) s += fy[j] * std::cos(k * th[j]);
        c[k] = 2.0 * s / m;
    }
    c[0] *= 0.5;
}

int upload_phase(ov_ctx *c)
{
    const int Lt = c->L[3];
    std::vector<cx<double>> h((size_t)c->nfield * Lt);
    for (int f = 0; f < c->nfield; ++f)
        for (int t = 0; t < Lt; ++t) {
            const double th = c->q[f] * c->eta[f] * t;
            h[(size_t)f * Lt + t] = {std::cos(th), std::sin(th)};
        }
    invalidate_graphs(c);
    if (c->phase) dev_free(c, c->phase, 0);
    c->phase = nullptr;
    CHK(dev_alloc(c, (void **)&c->phase, h.size() * sizeof(cx<double>)));
    HIPCHK(h2d(c, c->phase, h.data(), h.size() * sizeof(cx<double>)));
    return OV_OK;
}

int count_nonfinite(ov_ctx *c, const void *p, long ndouble, int *bad)
{
    HIPCHK(hipMemsetAsync(c->d_count, 0, sizeof(int), c->stream));
    HIPCHK(launch_count_nonfinite((const double *)p, ndouble, c->d_count, c->stream));
    HIPCHK(hipMemcpyAsync(bad, c->d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return OV_OK;
}

// ---------------------------------------------------------------- typed API bodies
template <class S>
int api_dslash(ov_ctx *c, int op, int nrhs, const std::vector<int> &grp, const void *x, void *y)
{
    const size_t fb = align_up(field_bytes<S>(c) * nrhs);
    CHK(ws_reserve(c, 2 * fb));
    S *X = ws_take<S>(c, field_elems(c) * nrhs);
    S *Y = ws_take<S>(c, field_elems(c) * nrhs);
    Batch b;
    CHK(make_batch(c, iota_vec(nrhs), grp, b));
    const int *fg = dev_ints(c, grp);
    HIPCHK(launch_pack_spinor<S>((const double2 *)x, X, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                 c->stream));
    CHK(dslash_launch<S>(c, b, fg, X, Y, 1.0, op == OV_OP_HW));
    HIPCHK(launch_unpack_spinor<S>(Y, (double2 *)y, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                   c->stream));
    return OV_OK;
}

// ov_dslash on the fixed scratch array instead of the arena: the field-group
// list, the packed input and the packed output live there.  No allocation:
// no arena growth, no cached device lists, no profiling events.
template <class S>
int api_dslash_noalloc(ov_ctx *c, int op, int nrhs, const std::vector<int> &grp, const void *x, void *y)
{
    const size_t ib = align_up(sizeof(int) * nrhs);
    const size_t fb = align_up(field_bytes<S>(c) * nrhs);
    if (ib + 2 * fb > kScratchBytes)
        return fail(c, OV_EINVAL, "ov_dslash_noalloc: %d RHS of %d sites need %zu bytes of scratch, the limit is %zu",
                    nrhs, c->g.V, ib + 2 * fb, kScratchBytes);
    char *base = (char *)c->scratch;
    int *fg = (int *)base;
    S *X = (S *)(base + ib);
    S *Y = (S *)(base + ib + fb);
    HIPCHK(h2d(c, fg, grp.data(), sizeof(int) * nrhs));
    Batch b;
    b.n = nrhs;
    b.slots = nullptr;
    HIPCHK(launch_pack_spinor<S>((const double2 *)x, X, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                 c->stream));
    const bool prof = c->prof_on;
    c->prof_on = false;
    const int rc = dslash_launch<S>(c, b, fg, X, Y, 1.0, op == OV_OP_HW);
    c->prof_on = prof;
    CHK(rc);
    HIPCHK(launch_unpack_spinor<S>(Y, (double2 *)y, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                   c->stream));
    return OV_OK;
}

template <class S>
int api_sign(ov_ctx *c, int nrhs, const std::vector<int> &grp, const void *x, void *y)
{
    CHK(ws_reserve(c, align_up(field_bytes<S>(c) * nrhs) + sign_bufs_bytes<S>(c, nrhs)));
    S *X = ws_take<S>(c, field_elems(c) * nrhs);
    SignBufs<S> w;
    CHK(take_sign_bufs<S>(c, nrhs, w));
    Batch b;
    CHK(make_batch(c, iota_vec(nrhs), grp, b));
    const int *fg = dev_ints(c, grp);
    HIPCHK(launch_pack_spinor<S>((const double2 *)x, X, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                 c->stream));
    std::string key = "sign|" + std::to_string(PrecOf<S>::p) + "|";
    key_add(key, grp);
    CHK(run_graph(c, key, [&]() { return sign_batch<S>(c, b, fg, X, X, w); }));
    HIPCHK(launch_unpack_spinor<S>(X, (double2 *)y, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                   c->stream));
    return c->norm_check == 2 ? take_norm_flag(c) : OV_OK;
}

template <class S>
int api_dov(ov_ctx *c, int nrhs, const std::vector<int> &grp, const double *mass, int dagger, const void *x,
            void *y)
{
    CHK(ws_reserve(c, align_up(field_bytes<S>(c) * nrhs) + dov_bufs_bytes<S>(c, nrhs)));
    S *X = ws_take<S>(c, field_elems(c) * nrhs);
    DovBufs<S> w;
    CHK(take_dov_bufs<S>(c, nrhs, w));
    Batch b;
    CHK(make_batch(c, iota_vec(nrhs), grp, b));
    const int *fg = dev_ints(c, grp);
    const double2 *ca, *cb;
    CHK(mass_coefs(c, nrhs, mass, &ca, &cb));
    HIPCHK(launch_pack_spinor<S>((const double2 *)x, X, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                 c->stream));
    std::string key = "dov|" + std::to_string(PrecOf<S>::p) + "|" + std::to_string(dagger != 0) + "|";
    key_add(key, grp);
    key_add(key, std::vector<double>(mass, mass + nrhs));
    CHK(run_graph(c, key, [&]() { return dov_batch<S>(c, b, fg, ca, cb, dagger != 0, X, X, w); }));
    HIPCHK(launch_unpack_spinor<S>(X, (double2 *)y, (long)field_elems(c), nullptr, nrhs, c->g.V, c->g.Vp,
                                   c->stream));
    return c->norm_check == 2 ? take_norm_flag(c) : OV_OK;
}

// ---------------------------------------------------------------- fixed scratch
// Device memory of the allocation-free entry point ov_dslash_noalloc: one
// array per GPU, held for the life of the process.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns for
// the current device, kept per device in g_scratch.
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Called by ov_create with the context's device current.
int scratch_init(ov_ctx *c)
{
    if (c->device >= kMaxDevices) return OV_OK;   // ov_dslash_noalloc then reports OV_ESTATE
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[c->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(c, OV_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch[c->device] = p;
    }
    c->scratch = g_scratch[c->device];
    return OV_OK;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

int ov_create(const int32_t L[4], const int32_t bc[4], double m_w, int device, ov_ctx **out)
{
    if (!out || !L || !bc) return OV_EINVAL;
    *out = nullptr;
    long V = 1;
    for (int m = 0; m < 4; ++m) {
        if (L[m] < 2 || L[m] > 4096) return OV_EINVAL;
        if (bc[m] < 0 || bc[m] > 2) return OV_EINVAL;
        V *= L[m];
    }
    if (V >= (1L << 31) / 64) return OV_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return OV_EHIP;
    if (hipSetDevice(device) != hipSuccess) return OV_EHIP;
    ov_ctx *c = new ov_ctx();
    c->device = device;
    for (int m = 0; m < 4; ++m) {
        c->L[m] = L[m];
        c->bc[m] = bc[m];
    }
    c->mw = m_w;
    Geo &g = c->g;
    g.Lx = L[0];
    g.Ly = L[1];
    g.Lz = L[2];
    g.Lt = L[3];
    g.V = (int)V;
    g.Vp = (int)((V + 63) / 64 * 64);
    g.Lxy = L[0] * L[1];
    g.Lxyz = L[0] * L[1] * L[2];
    for (int m = 0; m < 4; ++m) g.bcf[m] = bc[m] == 0 ? 1.0f : (bc[m] == 1 ? -1.0f : 0.0f);
    c->stream = nullptr;   // the null stream until ov_set_stream names another one
    if (dev_alloc(c, (void **)&c->d_count, 256) != OV_OK) {
        delete c;
        return OV_ENOMEM;
    }
    if (hipMemset(c->d_count, 0, 256) != hipSuccess || scratch_init(c) != OV_OK) {
        (void)hipFree(c->d_count);
        delete c;
        return OV_EHIP;
    }
    *out = c;
    return OV_OK;
}

int ov_destroy(ov_ctx *c)
{
    if (!c) return OV_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->U64);
    (void)hipFree(c->U32);
    (void)hipFree(c->U16);
    (void)hipFree(c->phase);
    for (auto &s : c->small) {
        (void)hipFree(s.V);
        (void)hipFree(s.sgn);
    }
    for (auto &d : c->defl) (void)hipFree(d.W);
    (void)hipFree(c->ws);
    (void)hipFree(c->d_count);
    for (auto &kv : c->icache) (void)hipFree(kv.second);
    for (auto &kv : c->dcache) (void)hipFree(kv.second);
    for (auto &kv : c->ccache) (void)hipFree(kv.second);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto e : c->ev_mask)
        if (e) (void)hipEventDestroy(e);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    invalidate_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return OV_OK;
}

int ov_set_stream(ov_ctx *c, void *stream)
{
    CHK(check_ctx(c));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)stream;
    return OV_OK;
}

const char *ov_last_error(const ov_ctx *c) { return c ? c->err.c_str() : "null context"; }

int ov_memory_used(const ov_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return OV_EINVAL;
    *bytes = (int64_t)c->mem_bytes;
    return OV_OK;
}

int ov_upload_gauge(ov_ctx *c, const void *U_dev)
{
    OV_RANGE("ov_upload_gauge");
    CHK(check_ctx(c));
    if (!U_dev) return fail(c, OV_EINVAL, "null gauge pointer");
    int bad = 0;
    CHK(count_nonfinite(c, U_dev, 4L * c->g.V * 18, &bad));
    if (bad) return fail(c, OV_ENAN, "gauge field holds %d non-finite numbers", bad);
    const size_t n = 36ul * c->g.Vp;
    if (!c->U64) {
        CHK(dev_alloc(c, (void **)&c->U64, n * sizeof(double2)));
        CHK(dev_alloc(c, (void **)&c->U32, n * sizeof(float2)));
        CHK(dev_alloc(c, (void **)&c->U16, n * sizeof(uint32_t)));
    }
    HIPCHK(launch_pack_links<double2>((const double2 *)U_dev, c->U64, c->g.V, c->g.Vp, c->stream));
    HIPCHK(launch_pack_links<float2>((const double2 *)U_dev, c->U32, c->g.V, c->g.Vp, c->stream));
    HIPCHK(launch_pack_links<uint32_t>((const double2 *)U_dev, c->U16, c->g.V, c->g.Vp, c->stream));
    unsigned long long *d_dev = (unsigned long long *)((char *)c->d_count + 8);
    unsigned long long dev_bits = 0;
    HIPCHK(hipMemsetAsync(d_dev, 0, sizeof(dev_bits), c->stream));
    HIPCHK(launch_link_row3_dev((const double2 *)U_dev, 4L * c->g.V, d_dev, c->stream));
    HIPCHK(hipMemcpyAsync(&dev_bits, d_dev, sizeof(dev_bits), hipMemcpyDeviceToHost, c->stream));
    unsigned long long *rd_dev = (unsigned long long *)((char *)c->d_count + 32);
    unsigned long long rd_bits[4] = {0, 0, 0, 0};
    HIPCHK(hipMemsetAsync(rd_dev, 0, sizeof(rd_bits), c->stream));
    HIPCHK(launch_link_round_dev((const double2 *)U_dev, 4L * c->g.V, rd_dev, c->stream));
    HIPCHK(hipMemcpyAsync(rd_bits, rd_dev, sizeof(rd_bits), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(&c->row3_dev, &dev_bits, sizeof(double));
    for (int p = 0; p < 2; ++p)
        for (int r = 0; r < 2; ++r) std::memcpy(&c->link_dev[1 + p][r], &rd_bits[2 * p + r], sizeof(double));
    invalidate_graphs(c);   // the FP32 / BF16 norms baked into captured pipelines may change
    c->have_gauge = true;
    update_link_format(c);
    return OV_OK;
}

int ov_set_link_reconstruct(ov_ctx *c, int enable)
{
    CHK(check_ctx(c));
    if (enable != 0 && enable != 1) return fail(c, OV_EINVAL, "enable must be 0 or 1");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->recon_allow = enable != 0;
    update_link_format(c);
    return OV_OK;
}

int ov_get_link_format(ov_ctx *c, int *reconstruct, double *row3_dev)
{
    CHK(check_ctx(c));
    if (reconstruct) *reconstruct = c->recon ? 1 : 0;
    if (row3_dev) *row3_dev = c->row3_dev;
    return OV_OK;
}

int ov_set_fields(ov_ctx *c, int nfield, const double *q, const double *eta)
{
    CHK(check_ctx(c));
    if (nfield < 1 || nfield > 64 || !q || !eta) return fail(c, OV_EINVAL, "need 1 <= nfield <= 64 and q, eta");
    for (int f = 0; f < nfield; ++f)
        if (!std::isfinite(q[f]) || !std::isfinite(eta[f])) return fail(c, OV_ENAN, "non-finite q or eta");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->nfield = nfield;
    c->q.assign(q, q + nfield);
    c->eta.assign(eta, eta + nfield);
    for (auto &s : c->small) {
        dev_free(c, s.V, 16ul * 12 * c->g.Vp * s.l);
        dev_free(c, s.sgn, 8ul * s.l);
    }
    for (auto &d : c->defl) dev_free(c, d.W, 16ul * 12 * c->g.Vp * d.k);
    c->small.assign(nfield, Small());
    c->defl.assign(nfield, Defl());
    return upload_phase(c);
}

int ov_set_field_eta(ov_ctx *c, int field, double q, double eta)
{
    CHK(check_ctx(c));
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (!std::isfinite(q) || !std::isfinite(eta)) return fail(c, OV_ENAN, "non-finite q or eta");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->q[field] = q;
    c->eta[field] = eta;
    return upload_phase(c);
}

int ov_set_sign_params(ov_ctx *c, int n, double eps, double norm, const double *coeffs)
{
    CHK(check_ctx(c));
    if (n < 1 || n > 100000) return fail(c, OV_EINVAL, "polynomial degree %d outside [1, 100000]", n);
    if (!(eps > 0 && eps < 1)) return fail(c, OV_EINVAL, "eps must lie in (0, 1)");
    if (norm <= 0) norm = std::fabs(4.0 + c->mw) + 4.0;
    if (!std::isfinite(norm)) return fail(c, OV_ENAN, "non-finite norm");
    invalidate_graphs(c);
    c->npoly = n;
    c->eps = eps;
    c->norm = norm;
    if (coeffs) {
        c->coef.assign(coeffs, coeffs + n + 1);
        for (double v : c->coef)
            if (!std::isfinite(v)) return fail(c, OV_ENAN, "non-finite Chebyshev coefficient");
    } else {
        cheb_interp(n, eps, c->coef);
    }
    c->have_sign = true;
    return OV_OK;
}

int ov_upload_eigvecs(ov_ctx *c, int field, int l, const void *V_dev, const double *lambda)
{
    OV_RANGE("ov_upload_eigvecs");
    CHK(check_ctx(c));
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (l < 0 || l > 256) return fail(c, OV_EINVAL, "small-space dimension %d outside [0, 256]", l);
    if (l > 0 && (!V_dev || !lambda)) return fail(c, OV_EINVAL, "null V or lambda");
    Small &sm = c->small[field];
    HIPCHK(hipStreamSynchronize(c->stream));
    invalidate_graphs(c);
    dev_free(c, sm.V, 16ul * 12 * c->g.Vp * sm.l);
    dev_free(c, sm.sgn, 8ul * sm.l);
    sm = Small();
    if (l == 0) return OV_OK;
    int bad = 0;
    CHK(count_nonfinite(c, V_dev, 24L * c->g.V * l, &bad));
    if (bad) return fail(c, OV_ENAN, "small space holds non-finite numbers");
    double2 *Vp = nullptr;
    double *sg = nullptr;
    CHK(dev_alloc(c, (void **)&Vp, 16ul * 12 * c->g.Vp * l));
    CHK(dev_alloc(c, (void **)&sg, 8ul * l));
    std::vector<double> sgn(l);
    for (int i = 0; i < l; ++i) sgn[i] = lambda[i] >= 0 ? 1.0 : -1.0;
    HIPCHK(h2d(c, sg, sgn.data(), 8ul * l));
    HIPCHK(launch_pack_spinor<double2>((const double2 *)V_dev, Vp, (long)field_elems(c), nullptr, l, c->g.V,
                                       c->g.Vp, c->stream));
    // orthonormality check in FP64: G = V^dag V
    CHK(ws_reserve(c, align_up((size_t)l * l * 16) + small_arrays_bytes(c, 48)));
    double2 *G = ws_take<double2>(c, (size_t)l * l);
    const long K = 12L * c->g.Vp;
    const long nchunk = (K + proj_dot_chunk(K) - 1) / proj_dot_chunk(K);
    double2 *part = ws_take<double2>(c, (size_t)nchunk * 48 * 256);
    for (int j0 = 0; j0 < l; j0 += 48) {
        const int nn = std::min(48, l - j0);
        HIPCHK(launch_proj_dot<double2>(Vp, l, (long)field_elems(c), Vp + (long)j0 * field_elems(c),
                                        (long)field_elems(c), nullptr, nn, c->g.Vp, 0, part, G + (long)j0 * l,
                                        c->stream));
    }
    std::vector<double2> Gh((size_t)l * l);
    HIPCHK(hipMemcpyAsync(Gh.data(), G, 16ul * l * l, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double dev = 0;
    for (int j = 0; j < l; ++j)
        for (int i = 0; i < l; ++i) {
            const double re = Gh[(size_t)j * l + i].x - (i == j ? 1.0 : 0.0), im = Gh[(size_t)j * l + i].y;
            dev = std::max(dev, std::sqrt(re * re + im * im));
        }
    if (!(dev <= 1e-8)) {
        dev_free(c, Vp, 16ul * 12 * c->g.Vp * l);
        dev_free(c, sg, 8ul * l);
        return fail(c, OV_EINVAL, "small space is not orthonormal: max |V^dag V - 1| = %.3e", dev);
    }
    sm.l = l;
    sm.V = Vp;
    sm.sgn = sg;
    return OV_OK;
}

int ov_dslash(ov_ctx *c, int prec, int op, int nrhs, const int *field_of_rhs, const void *x, void *y)
{
    OV_RANGE("ov_dslash");
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (op != OV_OP_DW && op != OV_OP_HW) return fail(c, OV_EINVAL, "unknown operator %d", op);
    if (!x || !y) return fail(c, OV_EINVAL, "null spinor pointer");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    if (prec == OV_FP64) return api_dslash<double2>(c, op, nrhs, grp, x, y);
    if (prec == OV_FP32) return api_dslash<float2>(c, op, nrhs, grp, x, y);
    return api_dslash<uint32_t>(c, op, nrhs, grp, x, y);
}

int ov_dslash_noalloc(ov_ctx *c, int prec, int op, int nrhs, const int *field_of_rhs, const void *x, void *y)
{
    OV_RANGE("ov_dslash_noalloc");
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (op != OV_OP_DW && op != OV_OP_HW) return fail(c, OV_EINVAL, "unknown operator %d", op);
    if (!x || !y) return fail(c, OV_EINVAL, "null spinor pointer");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->scratch) return fail(c, OV_ESTATE, "no fixed scratch on device %d", c->device);
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    if (prec == OV_FP64) return api_dslash_noalloc<double2>(c, op, nrhs, grp, x, y);
    if (prec == OV_FP32) return api_dslash_noalloc<float2>(c, op, nrhs, grp, x, y);
    return api_dslash_noalloc<uint32_t>(c, op, nrhs, grp, x, y);
}

int ov_set_norm_check(ov_ctx *c, int mode)
{
    CHK(check_ctx(c));
    if (mode < 0 || mode > 2) return fail(c, OV_EINVAL, "norm check mode must be 0, 1 or 2");
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((mode == 0) != (c->norm_check == 0)) invalidate_graphs(c);   // captures hold the check kernels
    c->norm_check = mode;
    return OV_OK;
}

int ov_norm_status(ov_ctx *c)
{
    CHK(check_ctx(c));
    return take_norm_flag(c);
}

int ov_get_sign_norm(ov_ctx *c, int prec, double *norm)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (!norm) return fail(c, OV_EINVAL, "null argument");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    *norm = prec == OV_FP64 ? norm_of<double2>(c) : prec == OV_FP32 ? norm_of<float2>(c) : norm_of<uint32_t>(c);
    return OV_OK;
}

int ov_sign_apply(ov_ctx *c, int prec, int nrhs, const int *field_of_rhs, const void *x, void *y)
{
    OV_RANGE("ov_sign_apply");
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (!x || !y) return fail(c, OV_EINVAL, "null spinor pointer");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    if (prec == OV_FP64) return api_sign<double2>(c, nrhs, grp, x, y);
    if (prec == OV_FP32) return api_sign<float2>(c, nrhs, grp, x, y);
    return api_sign<uint32_t>(c, nrhs, grp, x, y);
}

int ov_dov_apply(ov_ctx *c, int prec, int nrhs, const int *field_of_rhs, const double *mass, int dagger,
                 const void *x, void *y)
{
    OV_RANGE("ov_dov_apply");
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (!x || !y || !mass) return fail(c, OV_EINVAL, "null pointer argument");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    for (int j = 0; j < nrhs; ++j)
        if (!std::isfinite(mass[j])) return fail(c, OV_ENAN, "non-finite mass");
    if (prec == OV_FP64) return api_dov<double2>(c, nrhs, grp, mass, dagger, x, y);
    if (prec == OV_FP32) return api_dov<float2>(c, nrhs, grp, mass, dagger, x, y);
    return api_dov<uint32_t>(c, nrhs, grp, mass, dagger, x, y);
}

int ov_set_graphs(ov_ctx *c, int on)
{
    CHK(check_ctx(c));
    HIPCHK(hipStreamSynchronize(c->stream));
    invalidate_graphs(c);
    c->use_graphs = on != 0;
    return OV_OK;
}

int ov_prof_enable(ov_ctx *c, int on)
{
    CHK(check_ctx(c));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->prof_on = on != 0;
    c->recs.clear();
    c->ev_used = 0;
    return OV_OK;
}

int ov_prof_query(ov_ctx *c, const char *cls, long *launches, double *total_ms, double *bytes)
{
    CHK(check_ctx(c));
    int k = -1;
    for (int i = 0; i < PC_N; ++i)
        if (cls && std::strcmp(cls, kProfNames[i]) == 0) k = i;
    if (k < 0) return fail(c, OV_EINVAL, "unknown kernel class");
    HIPCHK(hipStreamSynchronize(c->stream));
    long cnt = 0;
    double ms = 0, by = 0;
    for (auto &r : c->recs) {
        if (r.cls != k) continue;
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        ++cnt;
        ms += t;
        by += r.bytes;
    }
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
    return OV_OK;
}

int ov_set_tuning(ov_ctx *c, int prec, int rhs_per_thread, int block)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (rhs_per_thread != 1 && rhs_per_thread != 2 && rhs_per_thread != 4 && rhs_per_thread != 8)
        return fail(c, OV_EINVAL, "rhs_per_thread must be 1, 2, 4 or 8");
    if (block != 64 && block != 128 && block != 192 && block != 256 && block != 512)
        return fail(c, OV_EINVAL, "block must be 64, 128, 192, 256 or 512");
    invalidate_graphs(c);
    for (auto &tu : c->tune[prec]) {
        tu.nr = rhs_per_thread;
        tu.block = block;
        tu.wshare = 1;
        if (rhs_per_thread > 2) tu.split = 1;
    }
    return OV_OK;
}

int ov_set_site_order(ov_ctx *c, int prec, int order)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (order < 0 || order > 3) return fail(c, OV_EINVAL, "site order must be 0, 1, 2 or 3");
    invalidate_graphs(c);
    for (auto &tu : c->tune[prec]) tu.order = order;
    return OV_OK;
}

int ov_set_occupancy(ov_ctx *c, int prec, int blocks_per_cu)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (blocks_per_cu < 0 || blocks_per_cu > 32) return fail(c, OV_EINVAL, "blocks_per_cu outside [0, 32]");
    invalidate_graphs(c);
    for (auto &tu : c->tune[prec]) tu.cap = blocks_per_cu;
    return OV_OK;
}

int ov_get_launch_config(ov_ctx *c, int prec, int kind, int *cfg)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (kind != 0 && kind != 1) return fail(c, OV_EINVAL, "kind must be 0 (plain) or 1 (fused epilogue)");
    if (!cfg) return fail(c, OV_EINVAL, "cfg is NULL");
    const auto &tu = c->tune[prec][kind];
    cfg[0] = tu.nr;
    cfg[1] = tu.block;
    cfg[2] = tu.order;
    cfg[3] = tu.cap;
    cfg[4] = tu.stream_hint;
    cfg[5] = tu.split;
    cfg[6] = tu.cols;
    cfg[7] = tu.wshare;
    return OV_OK;
}

int ov_set_launch_config(ov_ctx *c, int prec, int kind, const int *cfg)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (kind != 0 && kind != 1) return fail(c, OV_EINVAL, "kind must be 0 (plain) or 1 (fused epilogue)");
    if (!cfg) return fail(c, OV_EINVAL, "cfg is NULL");
    const int nr = cfg[0], bl = cfg[1], od = cfg[2], cp = cfg[3], sh = cfg[4], sp = cfg[5], cl = cfg[6];
    const int ws = cfg[7];
    if (nr != 1 && nr != 2 && nr != 4 && nr != 8) return fail(c, OV_EINVAL, "rhs_per_thread must be 1, 2, 4 or 8");
    if (bl != 64 && bl != 128 && bl != 192 && bl != 256 && bl != 512)
        return fail(c, OV_EINVAL, "block must be 64, 128, 192, 256 or 512");
    if (od < 0 || od > 3) return fail(c, OV_EINVAL, "site order must be 0, 1, 2 or 3");
    if (cp < 0 || cp > 32) return fail(c, OV_EINVAL, "blocks_per_cu outside [0, 32]");
    if (sh != 0 && sh != 1) return fail(c, OV_EINVAL, "stream_hint must be 0 or 1");
    if (sp != 1 && sp != 2 && sp != 4 && sp != 8) return fail(c, OV_EINVAL, "rhs_split must be 1, 2, 4 or 8");
    if (sp == 8 && prec == OV_BF16) return fail(c, OV_EINVAL, "rhs_split 8 is for FP64 and FP32 storage");
    if (sp > 1 && nr > 2) return fail(c, OV_EINVAL, "rhs_split > 1 needs rhs_per_thread <= 2");
    if (cl < 1 || cl > 64 || c->g.Ly % cl != 0) return fail(c, OV_EINVAL, "cols must divide Ly (%d)", c->g.Ly);
    if (ws != 1 && ws != 2 && ws != 4 && ws != 8) return fail(c, OV_EINVAL, "wshare must be 1, 2, 4 or 8");
    if (ws > 1 && (nr > 2 || sp > 4)) return fail(c, OV_EINVAL, "wshare > 1 needs rhs_per_thread <= 2 and rhs_split <= 4");
    invalidate_graphs(c);
    auto &tu = c->tune[prec][kind];
    tu.nr = nr;
    tu.block = bl;
    tu.order = od;
    tu.cap = cp;
    tu.stream_hint = sh;
    tu.split = sp;
    tu.cols = cl;
    tu.wshare = ws;
    return OV_OK;
}

int ov_get_tuning(ov_ctx *c, int prec, int *rhs_per_thread, int *block)
{
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (rhs_per_thread) *rhs_per_thread = c->tune[prec][0].nr;
    if (block) *block = c->tune[prec][0].block;
    return OV_OK;
}

}  // extern "C"


// ======================================================================== solver
namespace {

// Per-RHS scalars of the inner CG, indexed by storage index.
struct CgScalars {
    double *rr, *rr_new, *stop, *red;
    double2 *pAp, *ap, *an, *beta, *one;
    int *active, *iters;
    double2 *dpart;
};

// Pinned host words for reading the active flags while the next iteration runs.
int pin_reserve(ov_ctx *c, size_t n)
{
    for (auto &e : c->ev_mask)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (n <= c->h_pin_n) return OV_OK;
    if (c->h_pin) HIPCHK(hipHostFree(c->h_pin));
    c->h_pin = nullptr;
    c->h_pin_n = 0;
    HIPCHK(hipHostMalloc((void **)&c->h_pin, n * sizeof(int), hipHostMallocDefault));
    c->h_pin_n = n;
    return OV_OK;
}

void key_ptrs(std::string &k, std::initializer_list<const void *> ps)
{
    for (const void *p : ps) k.append((const char *)&p, sizeof p);
    k.push_back('|');
}

// One inner CG iteration on batch bi: Ap = D^dag D p, alpha, e += alpha p,
// r -= alpha Ap (with |r|^2), beta and the active flags on the device,
// p = r + beta p.  Kernel launches only (captured as one graph per batch).
template <class S>
int cg_iteration(ov_ctx *c, const Batch &bi, const int *fg, const double2 *ca, const double2 *cb, S *E, S *r, S *p,
                 S *Ap, S *Dp, DovBufs<S> &w, CgScalars &s, int nstore)
{
    const long fe = (long)field_elems(c);
    int nb = 0;
    CHK(dov_batch<S>(c, bi, fg, ca, cb, false, p, Dp, w));
    CHK(dov_batch<S>(c, bi, fg, ca, cb, true, Dp, Ap, w));
    HIPCHK((launch_dot<S, S>(p, fe, Ap, fe, bi.slots, bi.n, c->g.Vp, 0, s.dpart, s.pAp, bi.slots, c->stream)));
    HIPCHK(launch_cg_alpha(s.rr, s.pAp, s.active, nstore, s.ap, s.an, c->stream));
    {   // e += alpha p ; r -= alpha Ap (with |r|^2)
        const S *in1[2] = {E, p};
        const double2 *cf1[2] = {s.one, s.ap};
        CHK((lincomb<S, S>(c, bi, E, 2, in1, cf1, nullptr, 0)));
        const S *in2[2] = {r, Ap};
        const double2 *cf2[2] = {s.one, s.an};
        CHK((lincomb<S, S>(c, bi, r, 2, in2, cf2, nullptr, 0, s.red, &nb)));
        HIPCHK(launch_reduce_r(s.red, nb, bi.n, s.rr_new, bi.slots, c->stream));
    }
    HIPCHK(launch_cg_beta(s.rr_new, s.rr, s.active, s.stop, nstore, s.beta, s.iters, c->stream));
    {   // p = r + beta p
        const S *in[2] = {r, p};
        const double2 *cf[2] = {s.one, s.beta};
        CHK((lincomb<S, S>(c, bi, p, 2, in, cf, nullptr, 0)));
    }
    return OV_OK;
}

template <class S>
size_t cg_inner_bytes(const ov_ctx *c, int n)
{
    return 5 * align_up(field_bytes<S>(c) * n) + dov_bufs_bytes<S>(c, n);
}

// FP64 true residual R = RHS - D^dag D X on batch b (uses the FP64 D_ov buffers).
int residual64(ov_ctx *c, const Batch &b, const int *fg, const double2 *ca, const double2 *cb, const double2 *RHS,
               const double2 *X, double2 *R, double2 *tmp, DovBufs<double2> &w)
{
    CHK(dov_batch<double2>(c, b, fg, ca, cb, false, X, tmp, w));
    CHK(dov_batch<double2>(c, b, fg, ca, cb, true, tmp, tmp, w));
    const double2 *in[2] = {RHS, tmp};
    const double2 cc[2] = {make_double2(1, 0), make_double2(-1, 0)};
    return lincomb<double2, double2>(c, b, R, 2, in, nullptr, cc, 0);
}

// squared norms of the entries of b (by storage index) into host vector
int norms2(ov_ctx *c, const Batch &b, const double2 *X, CgScalars &s, int nstore, std::vector<double> &out)
{
    HIPCHK((launch_dot<double2, double2>(X, (long)field_elems(c), X, (long)field_elems(c), b.slots, b.n, c->g.Vp, 0,
                                         s.dpart, s.pAp, b.slots, c->stream)));
    std::vector<double2> h(nstore);
    HIPCHK(hipMemcpyAsync(h.data(), s.pAp, 16ul * nstore, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    out.assign(nstore, 0.0);
    for (int j : b.slots_h) out[j] = h[j].x;
    return OV_OK;
}

// Inner CG on A e = r0 (r0 given in R64, FP64), e returned in E (precision S),
// for the RHS of batch bo.  RHS j stops when |r|^2 falls below
// max(inner_tol^2 |r0|^2, floor2[j]).  Iteration counts per storage index
// added to iters.
template <class S>
int inner_cg(ov_ctx *c, const Batch &bo, const std::vector<int> &grp, const int *fg, const double2 *ca,
             const double2 *cb, const double *mass, const double2 *R64, S *E, S *r, S *p, S *Ap, S *Dp,
             DovBufs<S> &w, CgScalars &s, int nstore, double inner_tol, const std::vector<double> &floor2,
             int budget, bool use_defl, std::vector<int> &iters, int &total)
{
    const long fe = (long)field_elems(c);
    // r = R ; e = 0 (or the deflation guess)
    CHK((copy_fields<double2, S>(c, bo, R64, r)));
    const double2 zero = make_double2(0, 0);
    {
        const S *in[1] = {r};
        CHK((lincomb<S, S>(c, bo, E, 1, in, nullptr, &zero, 0)));
    }
    bool did_defl = false;
    if (use_defl) {
        for (auto &gr : bo.groups) {
            const Defl &d = c->defl[gr.f];
            if (d.k == 0) continue;
            const int ng = (int)gr.slots_h.size();
            // C = W^dag R (FP64), E_coef = C / Lambda(m)
            double2 *C = w.sb.C, *Ec = w.sb.E;
            CHK(proj_dot<double2>(c, d.W, d.k, R64, gr, C, w.sb.part));
            std::vector<double> inv((size_t)ng * d.k);
            for (int j = 0; j < ng; ++j) {
                const double m = mass[gr.slots_h[j]];
                for (int i = 0; i < d.k; ++i) {
                    const double lam = (1 - 0.5 * m) * (1 - 0.5 * m) * d.a[i] + 2 * m * (1 - 0.5 * m) * d.b[i] + m * m;
                    inv[(size_t)j * d.k + i] = lam > 0 ? 1.0 / lam : 0.0;
                }
            }
            const double *invd = dev_doubles(c, inv);
            if (!invd) return fail(c, OV_ENOMEM, "deflation weights upload failed");
            HIPCHK(launch_mul_coef(C, invd, d.k, ng, Ec, c->stream));
            CHK((proj_expand<S, S>(c, d.W, d.k, (const S *)nullptr, 0.0, E, gr, Ec, 1.0)));
            did_defl = true;
        }
        if (did_defl) {   // r = R - A e0
            CHK(dov_batch<S>(c, bo, fg, ca, cb, false, E, Dp, w));
            CHK(dov_batch<S>(c, bo, fg, ca, cb, true, Dp, Ap, w));
            const S *in[2] = {r, Ap};
            const double2 cc[2] = {make_double2(1, 0), make_double2(-1, 0)};
            CHK((lincomb<S, S>(c, bo, r, 2, in, nullptr, cc, 0)));
        }
    }
    // p = r ; rr = |r|^2 ; stop = inner_tol^2 |R|^2
    int nb = 0;
    {
        const S *in[1] = {r};
        CHK((lincomb<S, S>(c, bo, p, 1, in, nullptr, nullptr, 0, s.red, &nb)));
        HIPCHK(launch_reduce_r(s.red, nb, bo.n, s.rr, bo.slots, c->stream));
    }
    std::vector<double> rr0(nstore, 0.0), stop(nstore, 0.0);
    {
        std::vector<double> h(nstore);
        HIPCHK(hipMemcpyAsync(h.data(), s.rr, 8ul * nstore, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int j : bo.slots_h) {
            rr0[j] = h[j];
            stop[j] = std::max(inner_tol * inner_tol * h[j], floor2[j]);
        }
    }
    std::vector<int> act(nstore, 0);
    for (int j : bo.slots_h) act[j] = rr0[j] > stop[j] ? 1 : 0;
    HIPCHK(h2d(c, s.stop, stop.data(), 8ul * nstore));
    HIPCHK(h2d(c, s.active, act.data(), 4ul * nstore));

    HIPCHK(launch_fill_int(s.iters, nstore, 0, c->stream));
    CHK(pin_reserve(c, 2ul * nstore));
    int *hb[2] = {c->h_pin, c->h_pin + nstore};

    // The convergence test runs on the device (k_cg_beta clears a RHS's
    // active flag and stops counting its iterations); the host reads the
    // flags of iteration i while iteration i + 1 is already queued and drops
    // converged RHS from the batch of iteration i + 2.  A converged RHS that
    // rides along for one more iteration has alpha = 0: its e and r stay
    // unchanged.  Each batch's iteration is captured as one graph.
    std::vector<int> cur;
    for (int j : bo.slots_h)
        if (act[j]) cur.push_back(j);
    const std::string kbase = "cgit|" + std::to_string(PrecOf<S>::p) + "|";
    int pending = -1;
    while (!cur.empty() && total < budget) {
        Batch bi;
        CHK(make_batch(c, cur, grp, bi));
        std::string key = kbase;
        key_ptrs(key, {E, r, p, Ap, Dp, s.rr, s.active, s.iters, ca, cb, fg, w.XG, w.sb.chi});
        key_add(key, cur);
        CHK(run_graph(c, key, [&]() { return cg_iteration<S>(c, bi, fg, ca, cb, E, r, p, Ap, Dp, w, s, nstore); }));
        total += 1;
        const int slot = total & 1;
        HIPCHK(hipMemcpyAsync(hb[slot], s.active, 4ul * nstore, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipEventRecord(c->ev_mask[slot], c->stream));
        if (pending >= 0) {
            HIPCHK(hipEventSynchronize(c->ev_mask[pending]));
            std::vector<int> nxt;
            for (int j : cur)
                if (hb[pending][j]) nxt.push_back(j);
            cur.swap(nxt);
        }
        pending = slot;
    }
    std::vector<int> hit(nstore, 0);
    HIPCHK(hipMemcpyAsync(hit.data(), s.iters, 4ul * nstore, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int j : bo.slots_h) iters[j] += hit[j];
    return OV_OK;
}

template <class S>
int api_cg(ov_ctx *c, int nrhs, const std::vector<int> &grp, const double *mass, const void *b_dev, void *x_dev,
           const ov_cg_opts &o, ov_cg_rhs_report *rep)
{
    const int n = nrhs;
    const size_t f64 = align_up(field_bytes<double2>(c) * n);
    const size_t regionA = std::max(dov_bufs_bytes<double2>(c, n) + f64, cg_inner_bytes<S>(c, n));
    const size_t scal = 17 * align_up(16ul * n) + 2 * align_up(16ul * (8192 + n));
    CHK(ws_reserve(c, 4 * f64 + regionA + scal));
    double2 *B64 = ws_take<double2>(c, field_elems(c) * n);
    double2 *X64 = ws_take<double2>(c, field_elems(c) * n);
    double2 *RHS = ws_take<double2>(c, field_elems(c) * n);
    double2 *R64 = ws_take<double2>(c, field_elems(c) * n);
    CgScalars s;
    s.rr = ws_take<double>(c, n);
    s.rr_new = ws_take<double>(c, n);
    s.stop = ws_take<double>(c, n);
    s.pAp = ws_take<double2>(c, n);
    s.ap = ws_take<double2>(c, n);
    s.an = ws_take<double2>(c, n);
    s.beta = ws_take<double2>(c, n);
    s.one = ws_take<double2>(c, n);
    s.active = ws_take<int>(c, n);
    s.iters = ws_take<int>(c, n);
    // partial sums: a launch over n RHS uses at most max(8192, n) blocks in total
    s.red = ws_take<double>(c, 8192 + (size_t)n);
    s.dpart = ws_take<double2>(c, 8192 + (size_t)n);
    const size_t regA_start = c->ws_top;
    {
        std::vector<double2> ones(n, make_double2(1, 0));
        HIPCHK(h2d(c, s.one, ones.data(), 16ul * n));
    }
    // FP64 view of region A
    double2 *T64 = ws_take<double2>(c, field_elems(c) * n);
    DovBufs<double2> w64;
    CHK(take_dov_bufs<double2>(c, n, w64));
    // precision-S view of region A (aliases the FP64 view)
    c->ws_top = regA_start;
    S *E = ws_take<S>(c, field_elems(c) * n), *r = ws_take<S>(c, field_elems(c) * n);
    S *p = ws_take<S>(c, field_elems(c) * n), *Ap = ws_take<S>(c, field_elems(c) * n);
    S *Dp = ws_take<S>(c, field_elems(c) * n);
    DovBufs<S> wS;
    CHK(take_dov_bufs<S>(c, n, wS));

    Batch ball;
    CHK(make_batch(c, iota_vec(n), grp, ball));
    const int *fg = dev_ints(c, grp);
    const double2 *ca, *cb;
    CHK(mass_coefs(c, n, mass, &ca, &cb));

    HIPCHK(launch_pack_spinor<double2>((const double2 *)b_dev, B64, (long)field_elems(c), nullptr, n, c->g.V,
                                       c->g.Vp, c->stream));
    HIPCHK(launch_pack_spinor<double2>((const double2 *)x_dev, X64, (long)field_elems(c), nullptr, n, c->g.V,
                                       c->g.Vp, c->stream));
    // RHS = D^dag b
    CHK(dov_batch<double2>(c, ball, fg, ca, cb, true, B64, RHS, w64));
    std::vector<double> rhs2, x2;
    CHK(norms2(c, ball, RHS, s, n, rhs2));
    CHK(norms2(c, ball, X64, s, n, x2));
    for (int j = 0; j < n; ++j)
        if (!std::isfinite(rhs2[j]) || !std::isfinite(x2[j])) return fail(c, OV_ENAN, "non-finite source or guess");
    bool xzero = true;
    for (int j = 0; j < n; ++j) xzero = xzero && x2[j] == 0.0;
    if (xzero)
        CHK((copy_fields<double2, double2>(c, ball, RHS, R64)));
    else
        CHK(residual64(c, ball, fg, ca, cb, RHS, X64, R64, T64, w64));

    std::vector<int> iters(n, 0), restarts(n, 0);
    std::vector<double> relres(n, 0.0);
    int total = 0;
    int rounds = 0;
    for (;;) {
        std::vector<double> res2;
        CHK(norms2(c, ball, R64, s, n, res2));
        if (c->norm_check) CHK(take_norm_flag(c));   // norms2 synchronised: the flag is current
        std::vector<int> todo;
        for (int j = 0; j < n; ++j) {
            if (!std::isfinite(res2[j])) return fail(c, OV_ENAN, "non-finite residual for RHS %d", j);
            relres[j] = rhs2[j] > 0 ? std::sqrt(res2[j] / rhs2[j]) : 0.0;
            if (relres[j] > o.tol) todo.push_back(j);
        }
        if (todo.empty() || rounds >= o.max_restarts || total >= o.maxiter) break;
        Batch bo;
        CHK(make_batch(c, todo, grp, bo));
        // No inner solve goes below a tenth of the outer target: the last
        // defect-correction pass only needs the digits still missing.
        std::vector<double> floor2(n, 0.0);
        for (int j : todo) floor2[j] = 0.01 * o.tol * o.tol * rhs2[j];
        CHK(inner_cg<S>(c, bo, grp, fg, ca, cb, mass, R64, E, r, p, Ap, Dp, wS, s, n, o.inner_tol, floor2,
                        o.maxiter, o.use_deflation != 0, iters, total));
        // X += e (through R64 as an FP64 staging buffer), then the new true residual
        CHK((copy_fields<S, double2>(c, bo, E, R64)));
        {
            const double2 *in[2] = {X64, R64};
            CHK((lincomb<double2, double2>(c, bo, X64, 2, in, nullptr, nullptr, 0)));
        }
        CHK(residual64(c, ball, fg, ca, cb, RHS, X64, R64, T64, w64));
        for (int j : todo) restarts[j] += 1;
        ++rounds;
    }
    HIPCHK(launch_unpack_spinor<double2>(X64, (double2 *)x_dev, (long)field_elems(c), nullptr, n, c->g.V, c->g.Vp,
                                         c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        const bool conv = relres[j] <= o.tol;
        ok = ok && conv;
        if (rep) {
            rep[j].iters = iters[j];
            rep[j].restarts = restarts[j];
            rep[j].relres = relres[j];
            rep[j].status = conv ? OV_OK : OV_ENOCONV;
        }
    }
    if (!ok) return fail(c, OV_ENOCONV, "CG did not reach tol = %.3e within the iteration budget", o.tol);
    return OV_OK;
}

// ---------------------------------------------------------------- adjoint
int api_backward(ov_ctx *c, int f, const void *x_dev, const void *g_dev, void *gU_dev, double *geta, void *gx_dev,
                 int K)
{
    using S = double2;
    const int n = c->npoly;
    const long fe = (long)field_elems(c);
    const int nseg = (n + K - 1) / K;
    const int nb_fin = (c->g.V + 255) / 256;
    // fields: X, Gv, chi, z, wbar, zbar, t1, t2, bb[3], seg[K], ckpt[2*nseg], sign bufs
    const size_t nf = 11 + (size_t)K + 2 * nseg;
    const size_t need = nf * align_up(field_bytes<S>(c)) + align_up(36ul * c->g.Vp * 16) + align_up(8ul * nb_fin) +
                        sign_bufs_bytes<S>(c, 1);
    CHK(ws_reserve(c, need));
    S *X = ws_take<S>(c, fe), *Gv = ws_take<S>(c, fe), *chi = ws_take<S>(c, fe), *z = ws_take<S>(c, fe);
    S *wbar = ws_take<S>(c, fe), *zbar = ws_take<S>(c, fe), *t1 = ws_take<S>(c, fe), *t2 = ws_take<S>(c, fe);
    S *bb[3] = {ws_take<S>(c, fe), ws_take<S>(c, fe), ws_take<S>(c, fe)};
    std::vector<S *> seg(K), ck(2 * nseg);
    for (int i = 0; i < K; ++i) seg[i] = ws_take<S>(c, fe);
    for (int i = 0; i < 2 * nseg; ++i) ck[i] = ws_take<S>(c, fe);
    double2 *G = ws_take<double2>(c, 36ul * c->g.Vp);
    double *epart = ws_take<double>(c, nb_fin);
    SignBufs<S> w;
    CHK(take_sign_bufs<S>(c, 1, w));
    if (!epart) return fail(c, OV_ENOMEM, "workspace too small (internal)");

    std::vector<int> grp = {f};
    Batch b;
    CHK(make_batch(c, {0}, grp, b));
    const int *fg = dev_ints(c, grp);
    const Small &sm = c->small[f];
    const double al = 2.0 / ((1.0 - c->eps) * c->norm * c->norm);
    const double be = (1.0 + c->eps) / (1.0 - c->eps);
    const double kap = 2.0 / (1.0 - c->eps);
    const double invN = 1.0 / c->norm;
    const double2 zero = make_double2(0, 0);

    HIPCHK(launch_pack_spinor<S>((const double2 *)x_dev, X, fe, nullptr, 1, c->g.V, c->g.Vp, c->stream));
    HIPCHK(launch_pack_spinor<S>((const double2 *)g_dev, Gv, fe, nullptr, 1, c->g.V, c->g.Vp, c->stream));
    if (gx_dev) {   // gx = s g
        CHK(sign_batch<S>(c, b, fg, Gv, t1, w));
        HIPCHK(launch_unpack_spinor<S>(t1, (double2 *)gx_dev, fe, nullptr, 1, c->g.V, c->g.Vp, c->stream));
    }
    if (!gU_dev && !geta) return OV_OK;

    // chi = Pi x
    if (sm.l > 0) {
        CHK(proj_dot<S>(c, sm.V, sm.l, X, b.groups[0], w.C, w.part));
        CHK((proj_expand<S, S>(c, sm.V, sm.l, X, 1.0, chi, b.groups[0], w.C, -1.0)));
    } else {
        CHK((copy_fields<S, S>(c, b, X, chi)));
    }
    // One Clenshaw step k: out = c_k chi + 2T b1 - b2 (b2 may be NULL); uses t1.
    auto step = [&](int k, const S *b1, const S *b2, S *out) -> int {
        if (k == n) {
            const S *in[1] = {chi};
            const double2 cc[1] = {make_double2(c->coef[n], 0)};
            return lincomb<S, S>(c, b, out, 1, in, nullptr, cc, 0);
        }
        CHK(dslash_launch<S>(c, b, fg, b1, t1, 1.0, true));
        return dslash_launch<S>(c, b, fg, t1, out, 2.0 * al, true, chi, c->coef[k], b1, -2.0 * be, b2, -1.0);
    };
    // forward pass: keep (b_{top+1}, b_{top+2}) of every segment [s*K+1, min((s+1)K, n)]
    {
        const S *b1 = nullptr, *b2 = nullptr;
        int i1 = 0;
        for (int k = n; k >= 1; --k) {
            const int sgi = (k - 1) / K;
            const int top = std::min((sgi + 1) * K, n);
            if (k == top) {   // checkpoint the inputs of this segment
                S *c1 = ck[2 * sgi], *c2 = ck[2 * sgi + 1];
                const double2 one = make_double2(1, 0);
                if (b1) { const S *in[1] = {b1}; CHK((lincomb<S, S>(c, b, c1, 1, in, nullptr, &one, 0))); }
                else { const S *in[1] = {chi}; CHK((lincomb<S, S>(c, b, c1, 1, in, nullptr, &zero, 0))); }
                if (b2) { const S *in[1] = {b2}; CHK((lincomb<S, S>(c, b, c2, 1, in, nullptr, &one, 0))); }
                else { const S *in[1] = {chi}; CHK((lincomb<S, S>(c, b, c2, 1, in, nullptr, &zero, 0))); }
            }
            S *out = bb[i1];
            if (b2 == bb[0] || b2 == bb[1] || b2 == bb[2]) out = (S *)b2;
            CHK(step(k, b1, b2, out));
            b2 = b1;
            b1 = out;
            i1 = (out == bb[0]) ? 1 : (out == bb[1] ? 2 : 0);
            if (b1 == bb[i1] || b2 == bb[i1]) i1 = (i1 + 1) % 3;
            if (b1 == bb[i1] || b2 == bb[i1]) i1 = (i1 + 1) % 3;
        }
        // z = c_0 chi + T b_1 - b_2
        CHK(dslash_launch<S>(c, b, fg, b1, t1, 1.0, true));
        CHK(dslash_launch<S>(c, b, fg, t1, z, al, true, chi, c->coef[0], b1, -be, b2, -1.0));
    }
    // wbar = Pi g ; zbar = Q wbar
    if (sm.l > 0) {
        CHK(proj_dot<S>(c, sm.V, sm.l, Gv, b.groups[0], w.C, w.part));
        CHK((proj_expand<S, S>(c, sm.V, sm.l, Gv, 1.0, wbar, b.groups[0], w.C, -1.0)));
    } else {
        CHK((copy_fields<S, S>(c, b, Gv, wbar)));
    }
    CHK(dslash_launch<S>(c, b, fg, wbar, zbar, invN, true));

    HIPCHK(hipMemsetAsync(G, 0, 36ul * c->g.Vp * 16, c->stream));
    auto force = [&](const S *u, const S *v, double coef) -> int {
        ForceArgs fa{u, v, G, coef, c->g};
        int pi = prof_begin(c);
        HIPCHK(launch_force(fa, c->stream));
        prof_end(c, pi, PC_FORCE, (double)c->g.V * (4 * 192.0 + 2 * 576.0));
        return OV_OK;
    };
    // Re<wbar, dQ z>
    CHK(force(wbar, z, invN));

    // adjoint vectors bb_k = T_k(T) zbar, upward; pairs with b_{k+1}
    // bb_0 = zbar (kept in bbv[0]), bb_1 = T zbar
    S *bbv[3] = {bb[0], bb[1], bb[2]};
    {
        const double2 one = make_double2(1, 0);
        const S *in[1] = {zbar};
        CHK((lincomb<S, S>(c, b, bbv[0], 1, in, nullptr, &one, 0)));
        CHK(dslash_launch<S>(c, b, fg, zbar, t1, 1.0, true));
        CHK(dslash_launch<S>(c, b, fg, t1, bbv[1], al, true, zbar, -be));
    }
    int cur = 1, prev = 0;   // indices into bbv of bb_k and bb_{k-1}
    for (int sgi = 0; sgi < nseg; ++sgi) {
        const int lo = sgi * K + 1, top = std::min((sgi + 1) * K, n);
        // replay b_top .. b_lo into seg[k - lo]
        {
            const S *b1 = ck[2 * sgi], *b2 = ck[2 * sgi + 1];
            const bool fresh = (top == n);
            for (int k = top; k >= lo; --k) {
                S *out = seg[k - lo];
                if (k == n) {
                    CHK(step(k, nullptr, nullptr, out));
                } else {
                    const bool b2zero = fresh && (k == n - 1);
                    CHK(step(k, b1, b2zero ? nullptr : b2, out));
                }
                b2 = b1;
                b1 = out;
            }
        }
        // b_{k+1} for k in [lo, top]: seg[k+1-lo] when k+1 <= top, else the checkpoint b_{top+1}
        for (int k = lo; k <= top; ++k) {
            if (k == n) break;               // b_{n+1} = 0
            const S *bk1 = (k + 1 <= top) ? seg[k + 1 - lo] : ck[2 * sgi];
            if (k == 1) {
                // Re<zbar, dT b_1> = kap (Re<zbar, dQ Q b_1> + Re<Q zbar, dQ b_1>)
                const S *b1v = seg[0];
                CHK(dslash_launch<S>(c, b, fg, b1v, t2, 1.0, true));   // N Q b_1
                CHK(force(zbar, t2, kap * invN * invN));
                CHK(dslash_launch<S>(c, b, fg, zbar, t2, 1.0, true));  // N Q zbar
                CHK(force(t2, b1v, kap * invN * invN));
            }
            // 2 Re<bb_k, dT b_{k+1}> = 2 kap (Re<bb_k, dQ Q b_{k+1}> + Re<Q bb_k, dQ b_{k+1}>)
            CHK(dslash_launch<S>(c, b, fg, bk1, t2, 1.0, true));
            CHK(force(bbv[cur], t2, 2.0 * kap * invN * invN));
            CHK(dslash_launch<S>(c, b, fg, bbv[cur], t1, 1.0, true));
            CHK(force(t1, bk1, 2.0 * kap * invN * invN));
            // bb_{k+1} = 2T bb_k - bb_{k-1} = 2 al H t1 - 2 be bb_k - bb_{k-1}, into bb_{k-1}'s buffer
            CHK(dslash_launch<S>(c, b, fg, t1, bbv[prev], 2.0 * al, true, bbv[cur], -2.0 * be, bbv[prev], -1.0));
            std::swap(cur, prev);
        }
    }
    // gradients w.r.t. the base links and eta
    const cx<double> *prow = c->phase + (size_t)f * c->g.Lt;
    HIPCHK(launch_force_finish(G, c->U64, prow, c->q[f], c->g, (double2 *)gU_dev, epart, nb_fin, c->stream));
    std::vector<double> eh(nb_fin);
    HIPCHK(hipMemcpyAsync(eh.data(), epart, 8ul * nb_fin, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (geta) {
        double sum = 0;
        for (double v : eh) sum += v;
        *geta = sum;
    }
    return OV_OK;
}

}  // namespace

extern "C" {

int ov_deflated_cg(ov_ctx *c, int nrhs, const int *field_of_rhs, const double *mass, const void *b_dev,
                   void *x_dev, const ov_cg_opts *opts, ov_cg_rhs_report *report)
{
    OV_RANGE("ov_deflated_cg");
    CHK(check_ctx(c));
    if (!b_dev || !x_dev || !mass || !opts) return fail(c, OV_EINVAL, "null pointer argument");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    CHK(check_prec(c, opts->inner_prec));
    if (!(opts->tol >= 0) || !(opts->inner_tol > 0 && opts->inner_tol < 1) || opts->maxiter < 0 ||
        opts->max_restarts < 0)
        return fail(c, OV_EINVAL, "bad CG options");
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    for (int j = 0; j < nrhs; ++j)
        if (!std::isfinite(mass[j])) return fail(c, OV_ENAN, "non-finite mass");
    CHK(clear_norm_flag(c));
    if (opts->inner_prec == OV_FP64)
        return with_norm_status(c, api_cg<double2>(c, nrhs, grp, mass, b_dev, x_dev, *opts, report));
    if (opts->inner_prec == OV_FP32)
        return with_norm_status(c, api_cg<float2>(c, nrhs, grp, mass, b_dev, x_dev, *opts, report));
    return with_norm_status(c, api_cg<uint32_t>(c, nrhs, grp, mass, b_dev, x_dev, *opts, report));
}

int ov_upload_deflation(ov_ctx *c, int field, int k, const void *W_dev)
{
    OV_RANGE("ov_upload_deflation");
    CHK(check_ctx(c));
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (k < 0 || k > 256) return fail(c, OV_EINVAL, "deflation dimension %d outside [0, 256]", k);
    if (!c->have_gauge || !c->have_sign) return fail(c, OV_ESTATE, "upload the gauge field and set the sign first");
    Defl &d = c->defl[field];
    HIPCHK(hipStreamSynchronize(c->stream));
    invalidate_graphs(c);
    dev_free(c, d.W, 16ul * 12 * c->g.Vp * d.k);
    d = Defl();
    if (k == 0) return OV_OK;
    if (!W_dev) return fail(c, OV_EINVAL, "null deflation basis");
    int bad = 0;
    CHK(count_nonfinite(c, W_dev, 24L * c->g.V * k, &bad));
    if (bad) return fail(c, OV_ENAN, "deflation basis holds non-finite numbers");
    double2 *W = nullptr;
    CHK(dev_alloc(c, (void **)&W, 16ul * 12 * c->g.Vp * k));
    HIPCHK(launch_pack_spinor<double2>((const double2 *)W_dev, W, (long)field_elems(c), nullptr, k, c->g.V, c->g.Vp,
                                       c->stream));
    // a_i = |D_ov w_i|^2, b_i = Re<w_i, D_ov w_i>, in batches of 16 (FP64)
    const int nbt = std::min(k, 16);
    CHK(ws_reserve(c, align_up(field_bytes<double2>(c) * nbt) + dov_bufs_bytes<double2>(c, nbt) +
                          2 * align_up(16ul * nbt) + align_up(16ul * nbt * 8192)));
    double2 *Y = ws_take<double2>(c, field_elems(c) * nbt);
    DovBufs<double2> w;
    CHK(take_dov_bufs<double2>(c, nbt, w));
    double2 *o1 = ws_take<double2>(c, nbt), *o2 = ws_take<double2>(c, nbt);
    double2 *part = ws_take<double2>(c, (size_t)nbt * 8192);
    std::vector<double> zeros(nbt, 0.0);
    const double2 *ca, *cb;
    CHK(mass_coefs(c, nbt, zeros.data(), &ca, &cb));
    d.a.assign(k, 0.0);
    d.b.assign(k, 0.0);
    for (int i0 = 0; i0 < k; i0 += nbt) {
        const int nn = std::min(nbt, k - i0);
        std::vector<int> gv(nbt, field);
        Batch b;
        CHK(make_batch(c, iota_vec(nn), gv, b));
        const int *fg = dev_ints(c, gv);
        const double2 *Wi = W + (long)i0 * field_elems(c);
        CHK(dov_batch<double2>(c, b, fg, ca, cb, false, Wi, Y, w));
        HIPCHK((launch_dot<double2, double2>(Y, (long)field_elems(c), Y, (long)field_elems(c), nullptr, nn, c->g.Vp,
                                             0, part, o1, nullptr, c->stream)));
        HIPCHK((launch_dot<double2, double2>(Wi, (long)field_elems(c), Y, (long)field_elems(c), nullptr, nn,
                                             c->g.Vp, 0, part, o2, nullptr, c->stream)));
        std::vector<double2> h1(nn), h2(nn);
        HIPCHK(hipMemcpyAsync(h1.data(), o1, 16ul * nn, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(h2.data(), o2, 16ul * nn, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int i = 0; i < nn; ++i) {
            d.a[i0 + i] = h1[i].x;
            d.b[i0 + i] = h2[i].x;
        }
    }
    d.k = k;
    d.W = W;
    return OV_OK;
}

int ov_sign_backward(ov_ctx *c, int field, const void *x_dev, const void *g_dev, void *gU_dev, double *geta,
                     void *gx_dev, int ckpt_every)
{
    OV_RANGE("ov_sign_backward");
    CHK(check_ctx(c));
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (!x_dev || !g_dev) return fail(c, OV_EINVAL, "null x or g");
    if (ckpt_every < 1) return fail(c, OV_EINVAL, "ckpt_every must be >= 1");
    if (!c->have_gauge || !c->have_sign) return fail(c, OV_ESTATE, "upload the gauge field and set the sign first");
    CHK(clear_norm_flag(c));
    return with_norm_status(c, api_backward(c, field, x_dev, g_dev, gU_dev, geta, gx_dev,
                                            std::min(ckpt_every, c->npoly)));
}

int ov_autotune(ov_ctx *c, int prec, int nrhs, const char *cache_path)
{
    OV_RANGE("ov_autotune");
    CHK(check_ctx(c));
    CHK(check_prec(c, prec));
    if (!c->have_gauge || c->nfield == 0) return fail(c, OV_ESTATE, "upload the gauge field and fields first");
    if (nrhs < 1 || nrhs > 4096) return fail(c, OV_EINVAL, "nrhs outside [1, 4096]");
    // Times every candidate launch shape on synthetic data already in the
    // workspace, separately for the plain H_w launch and the fused Clenshaw
    // launch (dslash + epilogue), and keeps the fastest of each.
    auto run = [&](auto tag) -> int {
        using S = decltype(tag);
        const size_t fb = align_up(field_bytes<S>(c) * nrhs);
        CHK(ws_reserve(c, 5 * fb));
        S *x = ws_take<S>(c, field_elems(c) * nrhs), *y = ws_take<S>(c, field_elems(c) * nrhs);
        S *e1 = ws_take<S>(c, field_elems(c) * nrhs), *e2 = ws_take<S>(c, field_elems(c) * nrhs);
        S *e3 = ws_take<S>(c, field_elems(c) * nrhs);
        std::vector<int> grp(nrhs, 0);
        for (int j = 0; j < nrhs; ++j) grp[j] = j % c->nfield;
        Batch b;
        CHK(make_batch(c, iota_vec(nrhs), grp, b));
        const int *fg = dev_ints(c, grp);
        hipEvent_t e0, e9;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e9));
        const int nrs[4] = {1, 2, 4, 8}, blks[4] = {64, 128, 256, 512};
        const int caps[3] = {0, 2, 4}, splits[4] = {1, 2, 4, 8}, colss[3] = {1, 2, 4}, wss[4] = {1, 2, 4, 8};
        const int reps = 3;
        const bool was = c->prof_on;
        c->prof_on = false;
        const bool slab_ok = c->g.Lz % 8 == 0 && c->g.V % 64 == 0;
        const bool tslab_ok = c->g.Lt % 8 == 0 && c->g.V % 64 == 0;
        float best_ms[2] = {0, 0};
        int rc = OV_OK;
        for (int kind = 0; kind < 2 && rc == OV_OK; ++kind) {
            auto &tu = c->tune[prec][kind];
            auto launch = [&]() -> int {
                if (kind == 0) return dslash_launch<S>(c, b, fg, x, y, 1.0, true);
                return dslash_launch<S>(c, b, fg, x, y, 1.0, true, e1, 0.5, e2, -0.5, e3, -1.0);
            };
            const auto keep = tu;
            auto bestc = tu;
            float best = 1e30f;
            for (int sh = 0; sh < 2 && rc == OV_OK; ++sh)
            for (int od = 0; od < 4 && rc == OV_OK; ++od)
            for (int cl : colss)
            for (int cp : caps)
            for (int sp : splits)
            for (int ws : wss)
            for (int nr : nrs) {
                if (ws > 1 && (od == 2 || nr > 2 || sp > 4 || (ws / 2) * sp * nr >= nrhs)) continue;
                if (cl > 1 && (od != 1 || c->g.Ly % cl != 0)) continue;
                if (sp > 1 && (nr > 2 || od == 2)) continue;
                if (sp > 1 && (sp / 2) * nr >= nrhs) continue;
                if (sp == 8 && prec == OV_BF16) continue;
                if (od == 1 && !slab_ok) continue;
                if (od == 3 && !tslab_ok) continue;
                if (od == 2 && (c->g.V % 64 != 0 || nr != 1 || cp != 0)) continue;   // t-marching: one shape
                if (nr > 1 && nr / 2 >= nrhs) continue;
                if (prec == OV_FP64 && nr == 8) continue;
                for (int bl : blks) {
                    if (ws > 1 && bl != (ws == 8 ? 256 : 64 * ws)) continue;   // link sharing: one pass, block unused
                    if (od != 2 && bl == 512) continue;   // 512 threads: t-marching only
                    if (od == 2 && bl < 256) continue;    // t-marching: 4 or 8 RHS per workgroup
                    if (od == 2 && bl == 512 && prec == OV_FP64) continue;   // FP64 needs > 256 VGPRs
                    tu.nr = nr;
                    tu.block = bl;
                    tu.order = od;
                    tu.cap = cp;
                    tu.stream_hint = sh;
                    tu.split = sp;
                    tu.cols = cl;
                    tu.wshare = ws;
                    if (rc == OV_OK) rc = launch();
                    if (rc == OV_OK && hipEventRecord(e0, c->stream) != hipSuccess) rc = OV_EHIP;
                    for (int rep = 0; rep < reps && rc == OV_OK; ++rep) rc = launch();
                    if (rc == OV_OK && hipEventRecord(e9, c->stream) != hipSuccess) rc = OV_EHIP;
                    if (rc == OV_OK && hipEventSynchronize(e9) != hipSuccess) rc = OV_EHIP;
                    float ms = 0;
                    if (rc == OV_OK && hipEventElapsedTime(&ms, e0, e9) != hipSuccess) rc = OV_EHIP;
                    if (rc != OV_OK) break;
                    if (ms < best) {
                        best = ms;
                        bestc = tu;
                    }
                }
            }
            tu = rc == OV_OK ? bestc : keep;
            best_ms[kind] = best / (float)reps;
        }
        c->prof_on = was;
        invalidate_graphs(c);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e9);
        if (rc != OV_OK) return rc == OV_EHIP ? fail(c, OV_EHIP, "autotune: HIP event call failed") : rc;
        if (cache_path) {
            FILE *fp = std::fopen(cache_path, "a");
            if (fp) {
                for (int kind = 0; kind < 2; ++kind) {
                    const auto &tu = c->tune[prec][kind];
                    std::fprintf(fp,
                                 "{\"arch\": \"gfx950\", \"L\": [%d, %d, %d, %d], \"prec\": %d, \"nrhs\": %d, "
                                 "\"kind\": \"%s\", \"rhs_per_thread\": %d, \"block\": %d, \"site_order\": %d, "
                                 "\"blocks_per_cu\": %d, \"stream_hint\": %d, \"rhs_split\": %d, \"cols\": %d, "
                                 "\"wshare\": %d, \"two_row_links\": %d, \"ms_per_launch\": %.6f}\n",
                                 c->L[0], c->L[1], c->L[2], c->L[3], prec, nrhs, kind ? "clenshaw" : "dslash",
                                 tu.nr, tu.block, tu.order, tu.cap, tu.stream_hint, tu.split, tu.cols, tu.wshare,
                                 c->recon ? 1 : 0, best_ms[kind]);
                }
                std::fclose(fp);
            }
        }
        return OV_OK;
    };
    if (prec == OV_FP64) return run(double2{});
    if (prec == OV_FP32) return run(float2{});
    return run(uint32_t{});
}

}  // extern "C"

// ---------------------------------------------------------------- H_w eigensolver
namespace {

using cd = std::complex<double>;

// C[j][i] = <V_i, X_j> for nx contiguous fields X (chunks of 48 per launch).
int block_gram(ov_ctx *c, const double2 *V, int lv, const double2 *X, int nx, double2 *C, double2 *part)
{
    const long fe = (long)field_elems(c);
    for (int j0 = 0; j0 < nx; j0 += 48) {
        const int nn = std::min(48, nx - j0);
        int pi = prof_begin(c);
        HIPCHK(launch_proj_dot<double2>(V, lv, fe, X + (long)j0 * fe, fe, nullptr, nn, c->g.Vp, 0, part,
                                        C + (long)j0 * lv, c->stream));
        prof_end(c, pi, PC_PROJ_DOT, (double)fe * (lv * 16.0 + nn * 16.0));
    }
    return OV_OK;
}

// Y_j = sum_i V_i E[j][i] for nx output fields (Y must not alias V).
int block_rotate(ov_ctx *c, const double2 *V, int lv, const double2 *E, int nx, double2 *Y)
{
    const long fe = (long)field_elems(c);
    for (int j0 = 0; j0 < nx; j0 += 48) {
        const int nn = std::min(48, nx - j0);
        int pi = prof_begin(c);
        HIPCHK((launch_proj_expand<double2, double2>(V, lv, fe, nullptr, fe, 0.0, Y + (long)j0 * fe, fe, nullptr, nn,
                                                     c->g.Vp, E + (long)j0 * lv, 1.0, c->stream)));
        prof_end(c, pi, PC_PROJ_EXPAND, (double)fe * (lv * 16.0 + nn * 16.0));
    }
    return OV_OK;
}

// k x k matrix C[j][i] on the device -> column-major host matrix (element (i, j)).
int fetch_square(ov_ctx *c, const double2 *C, int k, std::vector<cd> &M)
{
    std::vector<double2> h((size_t)k * k);
    HIPCHK(hipMemcpyAsync(h.data(), C, 16ul * k * k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    M.resize((size_t)k * k);
    for (size_t e = 0; e < h.size(); ++e) M[e] = cd(h[e].x, h[e].y);
    for (int j = 0; j < k; ++j)   // Hermitian part
        for (int i = 0; i < j; ++i) {
            const cd v = 0.5 * (M[i + (size_t)k * j] + std::conj(M[j + (size_t)k * i]));
            M[i + (size_t)k * j] = v;
            M[j + (size_t)k * i] = std::conj(v);
        }
    for (int i = 0; i < k; ++i) M[i + (size_t)k * i] = M[i + (size_t)k * i].real();
    return OV_OK;
}

int put_square(ov_ctx *c, const std::vector<cd> &M, double2 *E)
{
    std::vector<double2> h(M.size());
    for (size_t e = 0; e < M.size(); ++e) h[e] = make_double2(M[e].real(), M[e].imag());
    HIPCHK(h2d(c, E, h.data(), 16ul * h.size()));
    return OV_OK;
}

// Q = Y R^{-1} with R^H R = Y^dag Y + shift, R upper triangular.
int cholqr_pass(ov_ctx *c, const double2 *Y, double2 *Q, int k, bool shifted, double2 *G, double2 *E, double2 *part)
{
    CHK(block_gram(c, Y, k, Y, k, G, part));
    std::vector<cd> M;
    CHK(fetch_square(c, G, k, M));
    if (shifted) {   // shifted Cholesky QR: the factorisation exists for any numerically full-rank Y
        double tr = 0;
        for (int i = 0; i < k; ++i) tr += M[i + (size_t)k * i].real();
        const double rows = 12.0 * c->g.V;
        const double s = 11.0 * (rows * k + (double)k * (k + 1)) * 1.1102230246251565e-16 * tr;
        for (int i = 0; i < k; ++i) M[i + (size_t)k * i] += s;
    }
    const int bad = ov::potrf_upper(k, M.data());
    if (bad) return fail(c, OV_EBREAKDOWN, "eigensolver: Gram matrix not positive definite at pivot %d", bad);
    ov::trinv_upper(k, M.data());
    // E[j][i] = Rinv(i, j): the column-major layout of Rinv
    CHK(put_square(c, M, E));
    return block_rotate(c, Y, k, E, k, Q);
}

struct EigBufs {
    double2 *B[4] = {nullptr, nullptr, nullptr, nullptr};   // FP64 blocks of k fields
    double2 *G = nullptr, *E = nullptr, *part = nullptr, *coef = nullptr;
    double *red = nullptr, *r2 = nullptr;
};

// Scaled Chebyshev filter (Zhou and Saad) in H_w^2: damps the interval
// [a, bnd], amplifies below a, normalised to 1 at lref < a.  F[0] holds the
// input; returns the index in F of the output.
template <class S>
int cheb_filter(ov_ctx *c, const Batch &b, const int *fg, S *const F[3], S *T, int m, double a, double bnd,
                double lref, int &iout)
{
    const double e = 0.5 * (bnd - a), cc = 0.5 * (bnd + a);
    double sigma = e / (lref - cc);
    const double tau = 2.0 / sigma;
    // F1 = (sigma/e) (H^2 - cc) F0
    CHK(dslash_launch<S>(c, b, fg, F[0], T, 1.0, true));
    CHK(dslash_launch<S>(c, b, fg, T, F[1], sigma / e, true, F[0], -(sigma / e) * cc));
    int i0 = 0, i1 = 1;
    for (int j = 2; j <= m; ++j) {
        const double sn = 1.0 / (tau - sigma);
        const int i2 = 3 - i0 - i1;
        CHK(dslash_launch<S>(c, b, fg, F[i1], T, 1.0, true));
        CHK(dslash_launch<S>(c, b, fg, T, F[i2], 2.0 * sn / e, true, F[i1], -2.0 * sn / e * cc, F[i0], -sigma * sn));
        sigma = sn;
        i0 = i1;
        i1 = i2;
    }
    iout = (m >= 1) ? i1 : 0;
    return OV_OK;
}

int install_small(ov_ctx *c, int field, int l, const double2 *Vplanes, const double *lambda)
{
    Small &sm = c->small[field];
    HIPCHK(hipStreamSynchronize(c->stream));
    invalidate_graphs(c);
    dev_free(c, sm.V, 16ul * 12 * c->g.Vp * sm.l);
    dev_free(c, sm.sgn, 8ul * sm.l);
    sm = Small();
    double2 *Vp = nullptr;
    double *sg = nullptr;
    CHK(dev_alloc(c, (void **)&Vp, 16ul * 12 * c->g.Vp * l));
    CHK(dev_alloc(c, (void **)&sg, 8ul * l));
    std::vector<double> sgn(l);
    for (int i = 0; i < l; ++i) sgn[i] = lambda[i] >= 0 ? 1.0 : -1.0;
    HIPCHK(h2d(c, sg, sgn.data(), 8ul * l));
    HIPCHK(hipMemcpyAsync(Vp, Vplanes, 16ul * 12 * c->g.Vp * l, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    sm.l = l;
    sm.V = Vp;
    sm.sgn = sg;
    return OV_OK;
}

// FP32 filter (o.prec == OV_FP32) while the wanted residuals exceed
// kFp32Floor * norm and fall at least 3x per pass, FP64 filter afterwards.
constexpr double kFp32Floor = 1e-6;

int api_eigensolve(ov_ctx *c, int field, const ov_eig_opts &o, const void *X0, void *V_out, double *lambda,
                   double *resid, int install, ov_eig_report *rep)
{
    using S = float2;
    const int k = o.k, l = o.l;
    const long fe = (long)field_elems(c);
    const long K = 12L * c->g.Vp;
    const long nchunk = (K + proj_dot_chunk(K) - 1) / proj_dot_chunk(K);
    const bool has32 = o.prec == OV_FP32;
    size_t need = 4 * align_up(field_bytes<double2>(c) * k) + 2 * align_up(16ul * k * k) +
                  align_up((size_t)nchunk * 48 * 256 * 16) + align_up(16ul * k) + 2 * align_up(8ul * (8192 + k));
    if (has32) need += 4 * align_up(field_bytes<S>(c) * k);
    CHK(ws_reserve(c, need));
    EigBufs w;
    for (auto &p : w.B) p = ws_take<double2>(c, fe * k);
    w.G = ws_take<double2>(c, (size_t)k * k);
    w.E = ws_take<double2>(c, (size_t)k * k);
    w.part = ws_take<double2>(c, (size_t)nchunk * 48 * 256);
    w.coef = ws_take<double2>(c, k);
    w.red = ws_take<double>(c, 8192 + k);
    w.r2 = ws_take<double>(c, 8192 + k);
    S *FS[4] = {nullptr, nullptr, nullptr, nullptr};
    if (has32)
        for (auto &p : FS) p = ws_take<S>(c, fe * k);
    if (!w.r2 || (has32 && !FS[3])) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    bool use32 = has32;   // switched off once the FP32 floor is reached
    double rmax_prev = 1e300;

    std::vector<int> grp(k, field);
    Batch b;
    CHK(make_batch(c, iota_vec(k), grp, b));
    const int *fg = dev_ints(c, grp);
    const double bnd = c->norm * c->norm;
    double a = o.cutoff > 0 ? o.cutoff : bnd / 100.0;
    double lref = 0.0;
    HIPCHK(launch_pack_spinor<double2>((const double2 *)X0, w.B[0], fe, nullptr, k, c->g.V, c->g.Vp, c->stream));
    int ix = 0;   // block holding the current X
    std::vector<double> th(k), r(k), mu(k);
    int it = 0;
    long applies = 0;
    bool conv = false;
    while (it < o.max_iter) {
        ++it;
        if (a >= bnd) a = 0.5 * bnd;
        // 1. filter
        int iy;
        if (!use32) {
            double2 *F[3];
            int fi = 0, ti = -1;
            F[fi++] = w.B[ix];
            for (int q = 0; q < 4; ++q)
                if (q != ix) {
                    if (fi < 3) F[fi++] = w.B[q];
                    else ti = q;
                }
            int io;
            CHK(cheb_filter<double2>(c, b, fg, F, w.B[ti], o.cheb_order, a, bnd, lref, io));
            iy = 0;
            for (int q = 0; q < 4; ++q)
                if (w.B[q] == F[io]) iy = q;
        } else {
            S *F[3] = {FS[0], FS[1], FS[2]};
            CHK((copy_fields<double2, S>(c, b, w.B[ix], FS[0])));
            int io;
            CHK(cheb_filter<S>(c, b, fg, F, FS[3], o.cheb_order, a, bnd, lref, io));
            iy = (ix + 1) % 4;
            CHK((copy_fields<S, double2>(c, b, F[io], w.B[iy])));
        }
        applies += 2L * o.cheb_order * k;
        // 2. orthonormalise: shifted Cholesky QR, then two plain passes (ping-pong between iy and iq)
        int iq = (iy + 1) % 4;
        CHK(cholqr_pass(c, w.B[iy], w.B[iq], k, true, w.G, w.E, w.part));
        CHK(cholqr_pass(c, w.B[iq], w.B[iy], k, false, w.G, w.E, w.part));
        CHK(cholqr_pass(c, w.B[iy], w.B[iq], k, false, w.G, w.E, w.part));
        // 3. Rayleigh-Ritz on span(Q), Q in block iq.  With H_w itself the wanted
        //    values would be interior ones (a mix of +lambda and -lambda modes has a
        //    Rayleigh quotient near 0), so the block is rotated by the Ritz vectors
        //    of H_w^2 = (H_w Q)^dag (H_w Q), whose wanted values are the smallest,
        //    and only the l lowest of those are rotated once more by the Ritz
        //    vectors of H_w, which separates the signs.  Both rotations compose
        //    into one k x k matrix M: X = Q M, H_w X = (H_w Q) M.
        const int ih = (iq + 1) % 4, ixn = (iq + 2) % 4, it2 = (iq + 3) % 4;
        CHK(dslash_launch<double2>(c, b, fg, w.B[iq], w.B[ih], 1.0, true));
        applies += k;
        std::vector<cd> Hq, G2, Z((size_t)k * k);
        CHK(block_gram(c, w.B[iq], k, w.B[ih], k, w.G, w.part));
        CHK(fetch_square(c, w.G, k, Hq));
        CHK(block_gram(c, w.B[ih], k, w.B[ih], k, w.G, w.part));
        CHK(fetch_square(c, w.G, k, G2));
        ov::heev_jacobi(k, G2.data(), mu.data(), Z.data());
        // Hs = Z_l^dag Hq Z_l
        std::vector<cd> HZ((size_t)k * l), Hs((size_t)l * l), Y((size_t)l * l);
        for (int j = 0; j < l; ++j)
            for (int i = 0; i < k; ++i) {
                cd s = 0;
                for (int q = 0; q < k; ++q) s += Hq[i + (size_t)k * q] * Z[q + (size_t)k * j];
                HZ[i + (size_t)k * j] = s;
            }
        for (int j = 0; j < l; ++j)
            for (int i = 0; i < l; ++i) {
                cd s = 0;
                for (int q = 0; q < k; ++q) s += std::conj(Z[q + (size_t)k * i]) * HZ[q + (size_t)k * j];
                Hs[i + (size_t)l * j] = s;
            }
        for (int j = 0; j < l; ++j)
            for (int i = 0; i < j; ++i) {
                const cd v = 0.5 * (Hs[i + (size_t)l * j] + std::conj(Hs[j + (size_t)l * i]));
                Hs[i + (size_t)l * j] = v;
                Hs[j + (size_t)l * i] = std::conj(v);
            }
        std::vector<double> ev(l);
        ov::heev_jacobi(l, Hs.data(), ev.data(), Y.data());
        std::vector<int> ord(l);
        for (int i = 0; i < l; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int p, int q) { return std::fabs(ev[p]) < std::fabs(ev[q]); });
        std::vector<cd> M(Z);
        for (int j = 0; j < l; ++j) {
            th[j] = ev[ord[j]];
            for (int i = 0; i < k; ++i) {
                cd s = 0;
                for (int q = 0; q < l; ++q) s += Z[i + (size_t)k * q] * Y[q + (size_t)l * ord[j]];
                M[i + (size_t)k * j] = s;
            }
        }
        for (int j = l; j < k; ++j) th[j] = std::sqrt(std::max(mu[j], 0.0));
        CHK(put_square(c, M, w.E));
        CHK(block_rotate(c, w.B[iq], k, w.E, k, w.B[ixn]));   // X = Q M
        CHK(block_rotate(c, w.B[ih], k, w.E, k, w.B[it2]));   // H_w X
        // 4. residuals r_j = || H_w x_j - theta_j x_j ||
        {
            std::vector<double2> cf(k);
            for (int j = 0; j < k; ++j) cf[j] = make_double2(-th[j], 0.0);
            HIPCHK(h2d(c, w.coef, cf.data(), 16ul * k));
            const double2 *in[2] = {w.B[it2], w.B[ixn]};
            const double2 *cfs[2] = {nullptr, w.coef};
            int nb = 0;
            CHK((lincomb<double2, double2>(c, b, w.B[iq], 2, in, cfs, nullptr, 0, w.red, &nb)));
            HIPCHK(launch_reduce_r(w.red, nb, k, w.r2, nullptr, c->stream));
            HIPCHK(hipMemcpyAsync(r.data(), w.r2, 8ul * k, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (auto &v : r) v = std::sqrt(std::max(v, 0.0));
        }
        ix = ixn;
        conv = true;
        double rmax = 0;
        for (int j = 0; j < l; ++j) {
            conv = conv && std::isfinite(r[j]) && r[j] <= o.tol * c->norm;
            rmax = std::max(rmax, r[j]);
        }
        // hand over to FP64 at the FP32 floor, or as soon as FP32 stops making progress
        if (use32 && (rmax <= kFp32Floor * c->norm || rmax > 0.3 * rmax_prev)) use32 = false;
        rmax_prev = rmax;
        for (int j = 0; j < k; ++j)
            if (!std::isfinite(th[j]) || !std::isfinite(r[j])) return fail(c, OV_ENAN, "eigensolver: non-finite Ritz pair");
        if (conv) break;
        // next filter: damp everything above the block's largest Ritz value of H_w^2
        a = mu[k - 1];
        lref = std::max(mu[0], 0.0);
        if (!(a > lref)) a = lref + 1e-3 * bnd;
    }
    for (int j = 0; j < l; ++j) {
        lambda[j] = th[j];
        if (resid) resid[j] = r[j];
    }
    if (V_out)
        HIPCHK(launch_unpack_spinor<double2>(w.B[ix], (double2 *)V_out, fe, nullptr, l, c->g.V, c->g.Vp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rep) {
        rep->iters = it;
        rep->hw_applies = applies;
        double mr = 0;
        for (int j = 0; j < l; ++j) mr = std::max(mr, r[j]);
        rep->max_resid = mr;
    }
    if (install) CHK(install_small(c, field, l, w.B[ix], lambda));
    if (!conv) return fail(c, OV_ENOCONV, "eigensolver: %d lowest pairs not converged to %.2e in %d passes", l, o.tol, it);
    return OV_OK;
}

}  // namespace

extern "C" {

int ov_hw_eigensolve(ov_ctx *c, int field, const ov_eig_opts *o, const void *X0_dev, void *V_dev, double *lambda,
                     double *resid, int install, ov_eig_report *report)
{
    OV_RANGE("ov_hw_eigensolve");
    CHK(check_ctx(c));
    if (!o || !X0_dev || !lambda) return fail(c, OV_EINVAL, "null options, start block or lambda");
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters (norm bound) not set");
    if (o->k < 1 || o->k > 256 || o->l < 1 || o->l > o->k)
        return fail(c, OV_EINVAL, "need 1 <= l <= k <= 256 (l = %d, k = %d)", o->l, o->k);
    if (o->cheb_order < 1 || o->cheb_order > 100000) return fail(c, OV_EINVAL, "cheb_order outside [1, 100000]");
    if (o->max_iter < 1) return fail(c, OV_EINVAL, "max_iter must be >= 1");
    if (!(o->tol > 0)) return fail(c, OV_EINVAL, "tol must be positive");
    if (o->prec != OV_FP64 && o->prec != OV_FP32) return fail(c, OV_EINVAL, "filter precision must be FP64 or FP32");
    return api_eigensolve(c, field, *o, X0_dev, V_dev, lambda, resid, install, report);
}

}  // extern "C"

// ---------------------------------------------------------------- multi-mass CG in a chirality sector
namespace {

// Order of the adaptive polynomial: the smallest n whose error bound
// 2 * 0.41 exp(-2.1 n sqrt(eps)) (twice the law of eq. (2), which the
// interpolant stays below) is within `err`, clamped to [nmin, nmax].
int adaptive_order(double err, double eps, int nmin, int nmax)
{
    if (!(err > 0)) return nmax;
    const double n = std::log(0.82 / err) / (2.1 * std::sqrt(eps));
    const int ni = (int)std::ceil(n);
    return std::max(nmin, std::min(nmax, ni));
}

template <class S>
int api_mscg(ov_ctx *c, int nrhs, const std::vector<int> &grp, int nm, const double *mass, const void *b_dev,
             void *x_dev, const ov_mscg_opts &o, ov_mscg_report *rep, double *relres)
{
    const long fe = (long)field_elems(c);
    const int n = nrhs;
    // shifts sigma_i = m_i^2 / (1 - m_i^2 / 4); the base system is the smallest shift
    std::vector<double> sig(nm), fac(nm);
    int base = 0;
    for (int i = 0; i < nm; ++i) {
        fac[i] = 1.0 - 0.25 * mass[i] * mass[i];
        sig[i] = mass[i] * mass[i] / fac[i];
        if (sig[i] < sig[base]) base = i;
    }
    // workspace: FP64 sources and output staging; S-precision r, Ap, u, p[nm], y[nm]; sign buffers
    const size_t f64 = align_up(field_bytes<double2>(c) * n);
    const size_t fS = align_up(field_bytes<S>(c) * n);
    const size_t need = 2 * f64 + (3 + 2 * (size_t)nm) * fS +
                        std::max(sign_bufs_bytes<S>(c, n), dov_bufs_bytes<double2>(c, n) + f64) +
                        3 * align_up(16ul * n) + align_up(16ul * (8192 + n)) + 2 * align_up(8ul * (8192 + n));
    CHK(ws_reserve(c, need));
    double2 *B64 = ws_take<double2>(c, fe * n), *X64 = ws_take<double2>(c, fe * n);
    S *r = ws_take<S>(c, fe * n), *Ap = ws_take<S>(c, fe * n), *u = ws_take<S>(c, fe * n);
    std::vector<S *> p(nm), y(nm);
    for (int i = 0; i < nm; ++i) p[i] = ws_take<S>(c, fe * n);
    for (int i = 0; i < nm; ++i) y[i] = ws_take<S>(c, fe * n);
    double2 *cf0 = ws_take<double2>(c, n), *cf1 = ws_take<double2>(c, n), *dots = ws_take<double2>(c, n);
    double2 *dpart = ws_take<double2>(c, 8192 + n);
    double *red = ws_take<double>(c, 8192 + n), *rr_d = ws_take<double>(c, 8192 + n);
    const size_t mark = c->ws_top;
    SignBufs<S> sb;
    CHK(take_sign_bufs<S>(c, n, sb));
    if (!rr_d) return fail(c, OV_ENOMEM, "workspace too small (internal)");

    Batch ball;
    CHK(make_batch(c, iota_vec(n), grp, ball));
    const int *fg = dev_ints(c, grp);
    HIPCHK(launch_pack_spinor<double2>((const double2 *)b_dev, B64, fe, nullptr, n, c->g.V, c->g.Vp, c->stream));

    // chirality of each source: ||P- b||^2 = (||b||^2 - <b, g5 b>) / 2
    std::vector<double> bn2(n), chi(n);
    {
        std::vector<double2> h(n);
        HIPCHK((launch_dot<double2, double2>(B64, fe, B64, fe, nullptr, n, c->g.Vp, 0, dpart, dots, nullptr, c->stream)));
        HIPCHK(hipMemcpyAsync(h.data(), dots, 16ul * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int j = 0; j < n; ++j) bn2[j] = h[j].x;
        HIPCHK((launch_dot<double2, double2>(B64, fe, B64, fe, nullptr, n, c->g.Vp, 1, dpart, dots, nullptr, c->stream)));
        HIPCHK(hipMemcpyAsync(h.data(), dots, 16ul * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int j = 0; j < n; ++j) {
            if (!std::isfinite(bn2[j]) || !(bn2[j] > 0)) return fail(c, OV_EINVAL, "source %d is zero or non-finite", j);
            const double minus = 0.5 * (bn2[j] - h[j].x), plus = 0.5 * (bn2[j] + h[j].x);
            if (minus <= 1e-24 * bn2[j]) chi[j] = 1.0;
            else if (plus <= 1e-24 * bn2[j]) chi[j] = -1.0;
            else return fail(c, OV_EINVAL, "source %d has both chiralities (needs gamma5 b = +-b)", j);
        }
    }
    // r = b, p_i = b, y_i = 0
    CHK((copy_fields<double2, S>(c, ball, B64, r)));
    for (int i = 0; i < nm; ++i) {
        CHK((copy_fields<double2, S>(c, ball, B64, p[i])));
        const S *in[1] = {r};
        const double2 zero = make_double2(0, 0);
        CHK((lincomb<S, S>(c, ball, y[i], 1, in, nullptr, &zero, 0)));
    }
    std::vector<double> rr(bn2);   // (r, r) per RHS
    std::vector<double> zeta(nm * n, 1.0), zeta_old(nm * n, 1.0), alpha_old(n, 1.0), beta_old(n, 0.0);
    std::vector<char> done(nm * n, 0);
    // the adaptive order swaps the context's polynomial; the guard puts it back on every exit
    struct PolyGuard {
        ov_ctx *c;
        int n;
        std::vector<double> coef;
        ~PolyGuard()
        {
            c->npoly = n;
            c->coef = coef;
        }
    } guard{c, c->npoly, c->coef};
    const int n_full = guard.n;
    const std::vector<double> &coef_full = guard.coef;
    int cur_order = n_full;
    // an FP32 sector operator is accurate to ~1e-7, and a shifted CG cannot restart:
    // FP32 stops at 1e-5 and leaves the rest to the refinement
    const double inner_tol = (sizeof(S) == sizeof(double2)) ? o.tol : std::max(o.tol, 1e-5);
    double window_rho = 1e300;   // stagnation watch: the residual must halve every 200 iterations
    int window_start = 0;
    int it = 0;
    long sign_applies = 0, dslash_applies = 0;
    int rc = OV_OK;
    for (; it < o.maxiter; ++it) {
        double rho = 0;
        bool all = true;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < nm; ++i) {
                const double res = std::fabs(zeta[i * n + j]) * std::sqrt(rr[j] / bn2[j]);
                if (res <= inner_tol) done[i * n + j] = 1;
                all = all && done[i * n + j];
                if (!done[i * n + j]) rho = std::max(rho, res);
            }
        if (all) break;
        if (it - window_start >= 200) {
            if (!(rho < 0.5 * window_rho)) break;
            window_rho = rho;
            window_start = it;
        } else if (it == 0) {
            window_rho = rho;
        }
        // 1. order of this application (relaxation: the operator may be less accurate
        //    as the residual falls)
        if (o.adaptive) {
            const int ord = adaptive_order(0.01 * inner_tol / std::max(rho, 1e-300), c->eps, o.min_order, n_full);
            if (ord != cur_order) {
                cur_order = ord;
                c->npoly = ord;
                if (ord == n_full) c->coef = coef_full;
                else cheb_interp(ord, c->eps, c->coef);
            }
        }
        // 2. Ap = (A + sigma_b) p_b,  A v = 2 v + chi s v + g5 s v  (v in the sector of chi)
        rc = sign_batch<S>(c, ball, fg, p[base], u, sb);
        if (rc != OV_OK) break;
        sign_applies += n;
        dslash_applies += (long)n * (2 * cur_order + 1);
        {
            std::vector<double2> h0(n), h1(n);
            for (int j = 0; j < n; ++j) {
                h0[j] = make_double2(2.0 + sig[base], 0.0);
                h1[j] = make_double2(chi[j], 0.0);
            }
            HIPCHK(h2d(c, cf0, h0.data(), 16ul * n));
            HIPCHK(h2d(c, cf1, h1.data(), 16ul * n));
            const S *in[3] = {p[base], u, u};
            const double2 *cfs[3] = {cf0, cf1, nullptr};
            const double2 cc[3] = {make_double2(1, 0), make_double2(1, 0), make_double2(1, 0)};
            CHK((lincomb<S, S>(c, ball, Ap, 3, in, cfs, cc, 4)));
        }
        // 3. alpha = (r, r) / (p_b, Ap)
        std::vector<double2> h(n);
        HIPCHK((launch_dot<S, S>(p[base], fe, Ap, fe, nullptr, n, c->g.Vp, 0, dpart, dots, nullptr, c->stream)));
        HIPCHK(hipMemcpyAsync(h.data(), dots, 16ul * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::vector<double> alpha(n), zeta_new(nm * n), alpha_s(nm * n);
        for (int j = 0; j < n; ++j) {
            alpha[j] = h[j].x > 0 ? rr[j] / h[j].x : 0.0;
            for (int i = 0; i < nm; ++i) {
                const int q = i * n + j;
                const double ds = sig[i] - sig[base];
                const double den = alpha[j] * beta_old[j] * (zeta_old[q] - zeta[q]) +
                                   zeta_old[q] * alpha_old[j] * (1.0 + ds * alpha[j]);
                zeta_new[q] = (den != 0) ? zeta[q] * zeta_old[q] * alpha_old[j] / den : 0.0;
                alpha_s[q] = (zeta[q] != 0) ? alpha[j] * zeta_new[q] / zeta[q] : 0.0;
                if (done[q]) alpha_s[q] = 0.0;   // converged systems are frozen
            }
        }
        // 4. y_i += alpha_i p_i
        for (int i = 0; i < nm; ++i) {
            std::vector<double2> hc(n);
            bool any = false;
            for (int j = 0; j < n; ++j) {
                hc[j] = make_double2(alpha_s[i * n + j], 0.0);
                any = any || !done[i * n + j];
            }
            if (!any) continue;
            HIPCHK(h2d(c, cf0, hc.data(), 16ul * n));
            const S *in[2] = {y[i], p[i]};
            const double2 *cfs[2] = {nullptr, cf0};
            CHK((lincomb<S, S>(c, ball, y[i], 2, in, cfs, nullptr, 0)));
        }
        // 5. r -= alpha Ap, with (r, r)
        {
            std::vector<double2> hc(n);
            for (int j = 0; j < n; ++j) hc[j] = make_double2(-alpha[j], 0.0);
            HIPCHK(h2d(c, cf0, hc.data(), 16ul * n));
            const S *in[2] = {r, Ap};
            const double2 *cfs[2] = {nullptr, cf0};
            int nb = 0;
            CHK((lincomb<S, S>(c, ball, r, 2, in, cfs, nullptr, 0, red, &nb)));
            HIPCHK(launch_reduce_r(red, nb, n, rr_d, nullptr, c->stream));
        }
        std::vector<double> rr_new(n);
        HIPCHK(hipMemcpyAsync(rr_new.data(), rr_d, 8ul * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        // 6. p_i = zeta_new_i r + beta_i p_i
        std::vector<double> beta(n);
        for (int j = 0; j < n; ++j) beta[j] = rr[j] > 0 ? rr_new[j] / rr[j] : 0.0;
        for (int i = 0; i < nm; ++i) {
            std::vector<double2> ha(n), hb(n);
            bool any = false;
            for (int j = 0; j < n; ++j) {
                const int q = i * n + j;
                const double bs = (zeta[q] != 0) ? beta[j] * (zeta_new[q] / zeta[q]) * (zeta_new[q] / zeta[q]) : 0.0;
                ha[j] = make_double2(zeta_new[q], 0.0);
                hb[j] = make_double2(bs, 0.0);
                any = any || !done[q] || i == base;
            }
            if (!any) continue;
            HIPCHK(h2d(c, cf0, ha.data(), 16ul * n));
            HIPCHK(h2d(c, cf1, hb.data(), 16ul * n));
            const S *in[2] = {r, p[i]};
            const double2 *cfs[2] = {cf0, cf1};
            CHK((lincomb<S, S>(c, ball, p[i], 2, in, cfs, nullptr, 0)));
        }
        for (int j = 0; j < n; ++j) {
            if (!std::isfinite(rr_new[j])) return fail(c, OV_ENAN, "multi-mass CG: non-finite residual for RHS %d", j);
            alpha_old[j] = alpha[j];
            beta_old[j] = beta[j];
            rr[j] = rr_new[j];
        }
        for (int q = 0; q < nm * n; ++q) {
            zeta_old[q] = zeta[q];
            zeta[q] = zeta_new[q];
        }
    }
    CHK(rc);
    c->npoly = n_full;
    c->coef = coef_full;
    // x_i = D(m_i)^dag y_i / (1 - m_i^2 / 4), then the FP64 true residual of D(m_i) x_i = b
    c->ws_top = mark;
    double2 *T64 = ws_take<double2>(c, fe * n);
    DovBufs<double2> dw;
    CHK(take_dov_bufs<double2>(c, n, dw));
    std::vector<double> rel(nm * n, 0.0);
    for (int i = 0; i < nm; ++i) {
        const double2 sc = make_double2(1.0 / fac[i], 0.0);
        const S *in[1] = {y[i]};
        CHK((lincomb<S, double2>(c, ball, X64, 1, in, nullptr, &sc, 0)));
        std::vector<double> mv(n, mass[i]);
        const double2 *ca, *cb;
        CHK(mass_coefs(c, n, mv.data(), &ca, &cb));
        CHK(dov_batch<double2>(c, ball, fg, ca, cb, true, X64, T64, dw));
        HIPCHK(launch_unpack_spinor<double2>(T64, (double2 *)x_dev + (size_t)i * n * 12 * c->g.V, fe, nullptr, n,
                                             c->g.V, c->g.Vp, c->stream));
        CHK(dov_batch<double2>(c, ball, fg, ca, cb, false, T64, X64, dw));
        const double2 *in2[2] = {B64, X64};
        const double2 cc2[2] = {make_double2(1, 0), make_double2(-1, 0)};
        int nb = 0;
        CHK((lincomb<double2, double2>(c, ball, X64, 2, in2, nullptr, cc2, 0, red, &nb)));
        HIPCHK(launch_reduce_r(red, nb, n, rr_d, nullptr, c->stream));
        std::vector<double> h(n);
        HIPCHK(hipMemcpyAsync(h.data(), rr_d, 8ul * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int j = 0; j < n; ++j) rel[i * n + j] = std::sqrt(std::max(h[j], 0.0) / bn2[j]);
    }
    int refine_iters = 0;
    if (o.refine) {
        for (int i = 0; i < nm; ++i) {
            bool need_ref = false;
            for (int j = 0; j < n; ++j) need_ref = need_ref || rel[i * n + j] > o.tol;
            if (!need_ref) continue;
            ov_cg_opts co{};
            co.tol = o.tol;
            co.maxiter = o.maxiter;
            co.inner_prec = OV_FP32;
            co.inner_tol = 1e-5;
            co.max_restarts = 50;
            co.use_deflation = 1;
            std::vector<double> mv(n, mass[i]);
            std::vector<ov_cg_rhs_report> cr(n);
            const int r2 = api_cg<float2>(c, n, grp, mv.data(), b_dev, (double2 *)x_dev + (size_t)i * n * 12 * c->g.V,
                                          co, cr.data());
            for (int j = 0; j < n; ++j) {
                rel[i * n + j] = cr[j].relres;
                refine_iters += cr[j].iters;
            }
            if (r2 != OV_OK && r2 != OV_ENOCONV) return r2;
        }
    }
    if (relres)
        for (int q = 0; q < nm * n; ++q) relres[q] = rel[q];
    if (rep) {
        rep->iters = it;
        rep->sign_applies = sign_applies;
        rep->dslash_applies = dslash_applies;
        rep->refine_iters = refine_iters;
    }
    for (int q = 0; q < nm * n; ++q)
        if (!(rel[q] <= o.tol)) return fail(c, OV_ENOCONV, "multi-mass CG: pair %d at %.3e > tol %.3e", q, rel[q], o.tol);
    return OV_OK;
}

}  // namespace

extern "C" {

int ov_multishift_cg(ov_ctx *c, int nrhs, const int *field_of_rhs, int nmass, const double *mass, const void *b_dev,
                     void *x_dev, const ov_mscg_opts *o, ov_mscg_report *report, double *relres)
{
    OV_RANGE("ov_multishift_cg");
    CHK(check_ctx(c));
    if (!o || !mass || !b_dev || !x_dev) return fail(c, OV_EINVAL, "null argument");
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    if (nmass < 1 || nmass > 16) return fail(c, OV_EINVAL, "nmass outside [1, 16]");
    for (int i = 0; i < nmass; ++i)
        if (!(mass[i] >= 0 && mass[i] < 2)) return fail(c, OV_EINVAL, "mass %d outside [0, 2)", i);
    if (!(o->tol > 0) || o->maxiter < 1) return fail(c, OV_EINVAL, "need tol > 0 and maxiter >= 1");
    if (o->adaptive && (o->min_order < 1 || o->min_order > c->npoly))
        return fail(c, OV_EINVAL, "min_order outside [1, %d]", c->npoly);
    if (o->inner_prec != OV_FP64 && o->inner_prec != OV_FP32) return fail(c, OV_EINVAL, "inner_prec must be FP64 or FP32");
    std::vector<int> grp;
    CHK(check_fields(c, nrhs, field_of_rhs, grp));
    CHK(clear_norm_flag(c));
    if (o->inner_prec == OV_FP32)
        return with_norm_status(c, api_mscg<float2>(c, nrhs, grp, nmass, mass, b_dev, x_dev, *o, report, relres));
    return with_norm_status(c, api_mscg<double2>(c, nrhs, grp, nmass, mass, b_dev, x_dev, *o, report, relres));
}

}  // extern "C"

// ---------------------------------------------------------------- D_ov low modes (deflation basis)
namespace {

// Y = alpha A X + beta X + gamma Z on the chirality-chi sector, A X = 2 X + chi s X + gamma5 s X;
// U receives s X.  Y must not alias X, U or Z.
template <class S>
int sector_apply(ov_ctx *c, const Batch &b, const int *fg, double chi, const S *X, S *Y, S *U, SignBufs<S> &sb,
                 double alpha, double beta, const S *Z, double gamma)
{
    CHK(sign_batch<S>(c, b, fg, X, U, sb));
    {
        const S *in[3] = {X, U, Z};
        const double2 cc[3] = {make_double2(2.0 * alpha + beta, 0), make_double2(alpha * chi, 0), make_double2(gamma, 0)};
        CHK((lincomb<S, S>(c, b, Y, Z ? 3 : 2, in, nullptr, cc, 0)));
    }
    const S *in2[2] = {Y, U};
    const double2 cc2[2] = {make_double2(1, 0), make_double2(alpha, 0)};
    return lincomb<S, S>(c, b, Y, 2, in2, nullptr, cc2, 2);
}

int api_dov_eigensolve(ov_ctx *c, int field, int chirality, const ov_eig_opts &o, const void *X0, void *W_out,
                       double *lambda, double *resid, ov_eig_report *rep)
{
    using S = float2;
    const int k = o.k, l = o.l;
    const double chi = chirality > 0 ? 1.0 : -1.0;
    const long fe = (long)field_elems(c);
    const long K = 12L * c->g.Vp;
    const long nchunk = (K + proj_dot_chunk(K) - 1) / proj_dot_chunk(K);
    const bool has32 = o.prec == OV_FP32;
    size_t need = 5 * align_up(field_bytes<double2>(c) * k) + sign_bufs_bytes<double2>(c, k) +
                  2 * align_up(16ul * k * k) + align_up((size_t)nchunk * 48 * 256 * 16) + align_up(16ul * k) +
                  2 * align_up(8ul * (8192 + k));
    if (has32) need += 5 * align_up(field_bytes<S>(c) * k) + sign_bufs_bytes<S>(c, k);
    CHK(ws_reserve(c, need));
    EigBufs w;
    for (auto &p : w.B) p = ws_take<double2>(c, fe * k);
    double2 *U64 = ws_take<double2>(c, fe * k);
    w.G = ws_take<double2>(c, (size_t)k * k);
    w.E = ws_take<double2>(c, (size_t)k * k);
    w.part = ws_take<double2>(c, (size_t)nchunk * 48 * 256);
    w.coef = ws_take<double2>(c, k);
    w.red = ws_take<double>(c, 8192 + k);
    w.r2 = ws_take<double>(c, 8192 + k);
    SignBufs<double2> sb64;
    CHK(take_sign_bufs<double2>(c, k, sb64));
    S *FS[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    SignBufs<S> sb32;
    if (has32) {
        for (auto &p : FS) p = ws_take<S>(c, fe * k);
        CHK(take_sign_bufs<S>(c, k, sb32));
    }
    if (!w.r2 || !U64 || (has32 && !FS[4])) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    bool use32 = has32;
    double rmax_prev = 1e300;

    std::vector<int> grp(k, field);
    Batch b;
    CHK(make_batch(c, iota_vec(k), grp, b));
    const int *fg = dev_ints(c, grp);
    const double bnd = 4.0;   // spectrum of 2 + 2 P s P for |s| <= 1
    double a = o.cutoff > 0 ? o.cutoff : 0.1;
    double lref = 0.0;
    auto project = [&](double2 *Y) -> int {   // Y = (Y + chi gamma5 Y) / 2
        const double2 *in[2] = {Y, Y};
        const double2 cc[2] = {make_double2(0.5, 0), make_double2(0.5 * chi, 0)};
        return lincomb<double2, double2>(c, b, Y, 2, in, nullptr, cc, 2);
    };
    HIPCHK(launch_pack_spinor<double2>((const double2 *)X0, w.B[0], fe, nullptr, k, c->g.V, c->g.Vp, c->stream));
    CHK(project(w.B[0]));
    int ix = 0;
    std::vector<double> th(k), r(k);
    int it = 0;
    long applies = 0;
    bool conv = false;
    while (it < o.max_iter) {
        ++it;
        if (a >= bnd) a = 0.5 * bnd;
        const double e = 0.5 * (bnd - a), cc = 0.5 * (bnd + a);
        double sigma = e / (lref - cc);
        const double tau = 2.0 / sigma;
        const int m = o.cheb_order;
        int iy;
        if (!use32) {
            // F = three of the FP64 blocks (the first holds X), T-slot = U64
            int q[4], nq = 0;
            q[nq++] = ix;
            for (int t = 0; t < 4; ++t)
                if (t != ix) q[nq++] = t;
            double2 *F[3] = {w.B[q[0]], w.B[q[1]], w.B[q[2]]};
            CHK(sector_apply<double2>(c, b, fg, chi, F[0], F[1], U64, sb64, sigma / e, -(sigma / e) * cc, nullptr, 0.0));
            int i0 = 0, i1 = 1;
            for (int j = 2; j <= m; ++j) {
                const double sn = 1.0 / (tau - sigma);
                const int i2 = 3 - i0 - i1;
                CHK(sector_apply<double2>(c, b, fg, chi, F[i1], F[i2], U64, sb64, 2.0 * sn / e, -2.0 * sn / e * cc,
                                          F[i0], -sigma * sn));
                sigma = sn;
                i0 = i1;
                i1 = i2;
            }
            iy = q[m >= 1 ? i1 : 0];
        } else {
            S *F[3] = {FS[0], FS[1], FS[2]};
            CHK((copy_fields<double2, S>(c, b, w.B[ix], FS[0])));
            CHK(sector_apply<S>(c, b, fg, chi, F[0], F[1], FS[3], sb32, sigma / e, -(sigma / e) * cc, nullptr, 0.0));
            int i0 = 0, i1 = 1;
            for (int j = 2; j <= m; ++j) {
                const double sn = 1.0 / (tau - sigma);
                const int i2 = 3 - i0 - i1;
                CHK(sector_apply<S>(c, b, fg, chi, F[i1], F[i2], FS[3], sb32, 2.0 * sn / e, -2.0 * sn / e * cc, F[i0],
                                    -sigma * sn));
                sigma = sn;
                i0 = i1;
                i1 = i2;
            }
            iy = (ix + 1) % 4;
            CHK((copy_fields<S, double2>(c, b, F[m >= 1 ? i1 : 0], w.B[iy])));
        }
        applies += (long)m * k;
        CHK(project(w.B[iy]));
        // orthonormalise
        const int iq = (iy + 1) % 4;
        CHK(cholqr_pass(c, w.B[iy], w.B[iq], k, true, w.G, w.E, w.part));
        CHK(cholqr_pass(c, w.B[iq], w.B[iy], k, false, w.G, w.E, w.part));
        CHK(cholqr_pass(c, w.B[iy], w.B[iq], k, false, w.G, w.E, w.part));
        // Rayleigh-Ritz with A (its wanted values are the smallest: no interior problem)
        const int ih = (iq + 1) % 4, ixn = (iq + 2) % 4, it2 = (iq + 3) % 4;
        CHK(sector_apply<double2>(c, b, fg, chi, w.B[iq], w.B[ih], U64, sb64, 1.0, 0.0, nullptr, 0.0));
        applies += k;
        std::vector<cd> Hs, Z((size_t)k * k);
        CHK(block_gram(c, w.B[iq], k, w.B[ih], k, w.G, w.part));
        CHK(fetch_square(c, w.G, k, Hs));
        ov::heev_jacobi(k, Hs.data(), th.data(), Z.data());
        CHK(put_square(c, Z, w.E));
        CHK(block_rotate(c, w.B[iq], k, w.E, k, w.B[ixn]));
        CHK(block_rotate(c, w.B[ih], k, w.E, k, w.B[it2]));
        {
            std::vector<double2> cf(k);
            for (int j = 0; j < k; ++j) cf[j] = make_double2(-th[j], 0.0);
            HIPCHK(h2d(c, w.coef, cf.data(), 16ul * k));
            const double2 *in[2] = {w.B[it2], w.B[ixn]};
            const double2 *cfs[2] = {nullptr, w.coef};
            int nb = 0;
            CHK((lincomb<double2, double2>(c, b, w.B[iq], 2, in, cfs, nullptr, 0, w.red, &nb)));
            HIPCHK(launch_reduce_r(w.red, nb, k, w.r2, nullptr, c->stream));
            HIPCHK(hipMemcpyAsync(r.data(), w.r2, 8ul * k, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (auto &v : r) v = std::sqrt(std::max(v, 0.0));
        }
        ix = ixn;
        conv = true;
        double rmax = 0;
        for (int j = 0; j < l; ++j) {
            conv = conv && std::isfinite(r[j]) && r[j] <= o.tol * bnd;
            rmax = std::max(rmax, r[j]);
        }
        for (int j = 0; j < k; ++j)
            if (!std::isfinite(th[j]) || !std::isfinite(r[j])) return fail(c, OV_ENAN, "eigensolver: non-finite Ritz pair");
        if (use32 && (rmax <= kFp32Floor * bnd || rmax > 0.3 * rmax_prev)) use32 = false;
        rmax_prev = rmax;
        if (conv) break;
        a = th[k - 1];
        lref = std::max(th[0], 0.0);
        if (!(a > lref)) a = lref + 1e-3 * bnd;
    }
    for (int j = 0; j < l; ++j) {
        lambda[j] = th[j];
        if (resid) resid[j] = r[j];
    }
    if (W_out)
        HIPCHK(launch_unpack_spinor<double2>(w.B[ix], (double2 *)W_out, fe, nullptr, l, c->g.V, c->g.Vp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rep) {
        rep->iters = it;
        rep->hw_applies = applies;   // sign applications here
        double mr = 0;
        for (int j = 0; j < l; ++j) mr = std::max(mr, r[j]);
        rep->max_resid = mr;
    }
    if (!conv) return fail(c, OV_ENOCONV, "D_ov eigensolver: %d lowest pairs not converged to %.2e in %d passes", l,
                           o.tol, it);
    return OV_OK;
}

}  // namespace

extern "C" {

int ov_dov_eigensolve(ov_ctx *c, int field, int chirality, const ov_eig_opts *o, const void *X0_dev, void *W_dev,
                      double *lambda, double *resid, int install, ov_eig_report *report)
{
    OV_RANGE("ov_dov_eigensolve");
    CHK(check_ctx(c));
    if (!o || !X0_dev || !lambda) return fail(c, OV_EINVAL, "null options, start block or lambda");
    if (install && !W_dev) return fail(c, OV_EINVAL, "install needs the output basis W_dev");
    if (chirality != 1 && chirality != -1) return fail(c, OV_EINVAL, "chirality must be +1 or -1");
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (!c->have_gauge) return fail(c, OV_ESTATE, "no gauge field uploaded");
    if (!c->have_sign) return fail(c, OV_ESTATE, "sign parameters not set");
    if (o->k < 1 || o->k > 256 || o->l < 1 || o->l > o->k)
        return fail(c, OV_EINVAL, "need 1 <= l <= k <= 256 (l = %d, k = %d)", o->l, o->k);
    if (o->cheb_order < 1 || o->cheb_order > 10000) return fail(c, OV_EINVAL, "cheb_order outside [1, 10000]");
    if (o->max_iter < 1) return fail(c, OV_EINVAL, "max_iter must be >= 1");
    if (!(o->tol > 0)) return fail(c, OV_EINVAL, "tol must be positive");
    if (o->prec != OV_FP64 && o->prec != OV_FP32) return fail(c, OV_EINVAL, "filter precision must be FP64 or FP32");
    CHK(clear_norm_flag(c));
    const int rc = with_norm_status(c, api_dov_eigensolve(c, field, chirality, *o, X0_dev, W_dev, lambda, resid,
                                                          report));
    if (rc != OV_OK && rc != OV_ENOCONV) return rc;
    if (install) CHK(ov_upload_deflation(c, field, o->l, W_dev));
    return rc == OV_OK ? OV_OK : fail(c, OV_ENOCONV, "D_ov eigensolver did not converge (basis installed anyway)");
}

}  // extern "C"

extern "C" {

int ov_timeslice_norm2(ov_ctx *c, int nrhs, const void *x_dev, double *out)
{
    OV_RANGE("ov_timeslice_norm2");
    CHK(check_ctx(c));
    if (nrhs < 0 || nrhs > 65535) return fail(c, OV_EINVAL, "nrhs outside [0, 65535]");
    if (nrhs == 0) return OV_OK;
    if (!x_dev || !out) return fail(c, OV_EINVAL, "null argument");
    const int Lxyz = c->g.Lxyz, Lt = c->g.Lt;
    const int nb = slice_norm2_blocks(Lxyz);
    const size_t m = (size_t)nrhs * Lt;
    CHK(ws_reserve(c, align_up(8 * m * nb) + align_up(8 * m)));
    double *part = ws_take<double>(c, m * nb), *o = ws_take<double>(c, m);
    if (!o) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    HIPCHK(launch_slice_norm2((const double2 *)x_dev, nrhs, c->g.V, Lxyz, Lt, part, o, c->stream));
    HIPCHK(hipMemcpyAsync(out, o, 8 * m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return OV_OK;
}

int ov_pion_correlator(ov_ctx *c, int nsrc, const void *S_dev, double *G)
{
    OV_RANGE("ov_pion_correlator");
    CHK(check_ctx(c));
    if (nsrc < 1 || nsrc > 65535) return fail(c, OV_EINVAL, "nsrc outside [1, 65535]");
    if (!S_dev || !G) return fail(c, OV_EINVAL, "null argument");
    const int Lxyz = c->g.Lxyz, Lt = c->g.Lt;
    const int nb = slice_norm2_blocks(Lxyz);
    const size_t m = (size_t)nsrc * Lt;
    CHK(ws_reserve(c, align_up(8 * m * nb) + align_up(8 * m) + align_up(8ul * Lt)));
    double *part = ws_take<double>(c, m * nb), *o = ws_take<double>(c, m), *Gd = ws_take<double>(c, Lt);
    if (!Gd) return fail(c, OV_ENOMEM, "workspace too small (internal)");
    HIPCHK(launch_slice_norm2((const double2 *)S_dev, nsrc, c->g.V, Lxyz, Lt, part, o, c->stream));
    HIPCHK(launch_sum_rows(o, nsrc, Lt, Gd, c->stream));
    HIPCHK(hipMemcpyAsync(G, Gd, 8ul * Lt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return OV_OK;
}

int ov_ratio_R(int Lt, int nE, const double *G_E, const double *G_0, double *R)
{
    if (Lt < 1 || nE < 1 || !G_E || !G_0 || !R) return OV_EINVAL;
    for (int t = 0; t < Lt; ++t) {
        if (!(G_0[t] > 0) || !std::isfinite(G_0[t])) return OV_EINVAL;
        double s = 0.0;
        for (int e = 0; e < nE; ++e) s += G_E[(size_t)e * Lt + t];
        if (!std::isfinite(s)) return OV_ENAN;
        R[t] = (s / nE) / G_0[t];
    }
    return OV_OK;
}

}  // extern "C"

extern "C" {

// F = sum_t w_t C(t), C(t) = sum_j sum_{x in t} |S_j(x)|^2, S_j = D(m)^{-1} b_j; dF/deta through
// the solve: with mu_j = D^{-1} (gamma5 W S_j), dF/deta = -2 (1 - m/2) sum_j d/deta Re<mu_j, s S_j>
// (the sign adjoint of ov_sign_backward, small space and polynomial held fixed).
int ov_correlator_deta(ov_ctx *c, int field, double mass, int nsrc, const void *b_dev, const double *w,
                       double *C, double *dF, const ov_cg_opts *opts)
{
    OV_RANGE("ov_correlator_deta");
    CHK(check_ctx(c));
    if (field < 0 || field >= c->nfield) return fail(c, OV_EINVAL, "field %d outside [0, %d)", field, c->nfield);
    if (nsrc < 1 || nsrc > 4096) return fail(c, OV_EINVAL, "nsrc outside [1, 4096]");
    if (!b_dev || !w || !opts) return fail(c, OV_EINVAL, "null argument");
    if (!c->have_gauge || !c->have_sign) return fail(c, OV_ESTATE, "upload the gauge field and set the sign first");
    if (!(mass >= 0 && mass < 2)) return fail(c, OV_EINVAL, "mass outside [0, 2)");
    const int Lt = c->g.Lt;
    const size_t fb = 16ul * 12 * c->g.V * nsrc;
    double2 *S = nullptr, *R = nullptr, *M = nullptr;
    double *wd = nullptr;
    std::vector<double> ts((size_t)nsrc * Lt);
    auto cleanup = [&]() {
        dev_free(c, S, fb);
        dev_free(c, R, fb);
        dev_free(c, M, fb);
        dev_free(c, wd, 8ul * Lt);
    };
    int rc = dev_alloc(c, (void **)&S, fb);
    if (rc == OV_OK) rc = dev_alloc(c, (void **)&R, fb);
    if (rc == OV_OK) rc = dev_alloc(c, (void **)&M, fb);
    if (rc == OV_OK) rc = dev_alloc(c, (void **)&wd, 8ul * Lt);
    if (rc != OV_OK) {
        cleanup();
        return rc;
    }
    CHK(clear_norm_flag(c));
    std::vector<int> grp(nsrc, field);
    std::vector<double> mv(nsrc, mass);
    std::vector<ov_cg_rhs_report> rep(nsrc);
    auto solve = [&](const double2 *b, double2 *x) -> int {
        HIPCHK(hipMemsetAsync(x, 0, fb, c->stream));
        if (opts->inner_prec == OV_FP64) return api_cg<double2>(c, nsrc, grp, mv.data(), b, x, *opts, rep.data());
        if (opts->inner_prec == OV_BF16) return api_cg<uint32_t>(c, nsrc, grp, mv.data(), b, x, *opts, rep.data());
        return api_cg<float2>(c, nsrc, grp, mv.data(), b, x, *opts, rep.data());
    };
    rc = solve((const double2 *)b_dev, S);
    if (rc == OV_OK) rc = ov_timeslice_norm2(c, nsrc, S, ts.data());
    if (rc == OV_OK && h2d(c, wd, w, 8ul * Lt) != hipSuccess) rc = fail(c, OV_EHIP, "weight upload failed");
    if (rc == OV_OK && launch_weight_g5(S, wd, c->g.V, c->g.Lxyz, nsrc, R, c->stream) != hipSuccess)
        rc = fail(c, OV_EHIP, "weighting kernel failed");
    if (rc == OV_OK) rc = solve(R, M);
    double acc = 0.0;
    for (int j = 0; j < nsrc && rc == OV_OK; ++j) {
        double ge = 0.0;
        rc = api_backward(c, field, S + (size_t)j * 12 * c->g.V, M + (size_t)j * 12 * c->g.V, nullptr, &ge, nullptr,
                          std::min(32, c->npoly));
        acc += ge;
    }
    if (rc == OV_OK) {
        if (C)
            for (int t = 0; t < Lt; ++t) {
                double s = 0;
                for (int j = 0; j < nsrc; ++j) s += ts[(size_t)j * Lt + t];
                C[t] = s;
            }
        if (dF) *dF = -2.0 * (1.0 - 0.5 * mass) * acc;
    }
    cleanup();
    return with_norm_status(c, rc);
}

}  // extern "C"
