// C-ABI of libfeint: argument validation, per-device reference tables,
// forward dispatch, tile selection and autotuning.
#include "feint.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "capi_internal.h"
#include "launch.h"
#include "tables.h"

namespace feint {

namespace {
std::mutex g_mu;
std::map<int, DevTables *> g_tables;        // key: device * 64 + type * 16 + rule * 8 + p
int g_tile[2][8][4];                        // chosen variant per (rule, p, form), prisms
int g_tile_elem[3][8][4];                   // chosen variant per (type, p, form): 1 hexahedra, 2 tetrahedra
int g_tile_lap[8][2];                       // chosen variant per (p, form) of the Laplace kernels
thread_local std::string g_err;

bool valid_form(int form) { return form >= FEINT_FP64 && form <= FEINT_FP16X3; }
bool valid_rule(int rule) { return rule == FEINT_RULE_COLLAPSED || rule == FEINT_RULE_SYMMETRIC; }
}  // namespace

void set_error(const char *what, hipError_t e) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
}

void set_error_msg(const std::string &msg) { g_err = msg; }

const DevTables *find_tables(int p, int rule, int type) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(dev * 64 + type * 16 + rule * 8 + p);
    return it == g_tables.end() ? nullptr : it->second;
}

// Upload the tables of degree p on rule `rule` of element type `type`
// (0 prism, 1 hexahedron, 2 tetrahedron) to the current device (once).
feint_status prepare_tables(int p, int rule, int type) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_rule(rule) || type < 0 || type > 2 || (type != 0 && rule != 0)) return FEINT_ERR_INVALID_ARG;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_error("hipGetDevice", e); return FEINT_ERR_HIP; }
    std::lock_guard<std::mutex> lk(g_mu);
    const int key = dev * 64 + type * 16 + rule * 8 + p;
    if (g_tables.count(key)) return FEINT_OK;
    HostTables H = type == 2 ? build_tet_tables(p) : type == 1 ? build_hex_tables(p) : build_tables(p, rule);
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t s_tau = align(H.tau64.size() * 8), s_tau32 = align(H.tau32.size() * 4), s_lam = align(H.lam.size() * 8), s_lam32 = align(H.lam32.size() * 4);
    const size_t s_qw = align(H.qw.size() * 8), s_gll = align(H.gll.size() * 8), s_b64 = align(H.B64.size() * 8), s_b32 = align(H.B32.size() * 4);
    const size_t s_sp = align(H.bf_hi.size() * 2);
    const size_t s_ycf = align(H.Ycf.size() * 4);
    const size_t s_m64 = align(H.Mref.size() * 8), s_m32 = align(H.Mref32.size() * 4);
    const size_t s_tb = align(H.taub_hi.size() * 2);
    const size_t total = s_tau + s_tau32 + s_lam + s_lam32 + s_qw + s_gll + 2 * s_b64 + 3 * s_b32 + 4 * s_sp + s_ycf +
                         s_m64 + s_m32 + 4 * s_tb;
    char *base = nullptr;
    e = hipMalloc((void **)&base, total);
    if (e != hipSuccess) { set_error("hipMalloc(tables)", e); return FEINT_ERR_HIP; }
    std::vector<char> host(total, 0);
    size_t o = 0;
    auto put = [&](const void *src, size_t bytes, size_t slot) {
        if (bytes) std::memcpy(host.data() + o, src, bytes);   // empty tables (other element types)
        size_t at = o;
        o += slot;
        return base + at;
    };
    DevTables *T = new DevTables();
    T->p = p; T->rule = rule; T->n = H.n; T->npad = H.npad; T->nq = H.nq; T->nqp = H.nqp; T->nkb = H.nkb;
    T->f16_shift = H.f16_shift;
    double bmax = 0;
    for (double v : H.B64) bmax = std::fmax(bmax, std::fabs(v));
    T->bmax = (float)bmax;
    T->qw = (const double *)put(H.qw.data(), H.qw.size() * 8, s_qw);
    T->gll = (const double *)put(H.gll.data(), H.gll.size() * 8, s_gll);
    T->tau64 = (const double *)put(H.tau64.data(), H.tau64.size() * 8, s_tau);
    T->tau32 = (const float *)put(H.tau32.data(), H.tau32.size() * 4, s_tau32);
    T->lam32 = (const float *)put(H.lam32.data(), H.lam32.size() * 4, s_lam32);
    T->lam = (const double *)put(H.lam.data(), H.lam.size() * 8, s_lam);
    T->B64 = (const double *)put(H.B64.data(), H.B64.size() * 8, s_b64);
    T->B32 = (const float *)put(H.B32.data(), H.B32.size() * 4, s_b32);
    T->BT64 = (const double *)put(H.BT64.data(), H.BT64.size() * 8, s_b64);
    T->BT32 = (const float *)put(H.BT32.data(), H.BT32.size() * 4, s_b32);
    T->Bc32 = (const float *)put(H.Bc32.data(), H.Bc32.size() * 4, s_b32);
    T->bf_hi = (const uint16_t *)put(H.bf_hi.data(), H.bf_hi.size() * 2, s_sp);
    T->bf_lo = (const uint16_t *)put(H.bf_lo.data(), H.bf_lo.size() * 2, s_sp);
    T->hf_hi = (const uint16_t *)put(H.hf_hi.data(), H.hf_hi.size() * 2, s_sp);
    T->hf_lo = (const uint16_t *)put(H.hf_lo.data(), H.hf_lo.size() * 2, s_sp);
    T->Ycf = (const float *)put(H.Ycf.data(), H.Ycf.size() * 4, s_ycf);
    T->Mref64 = (const double *)put(H.Mref.data(), H.Mref.size() * 8, s_m64);
    T->Mref32 = (const float *)put(H.Mref32.data(), H.Mref32.size() * 4, s_m32);
    T->taubh = (const uint16_t *)put(H.taub_hi.data(), H.taub_hi.size() * 2, s_tb);
    T->taubl = (const uint16_t *)put(H.taub_lo.data(), H.taub_lo.size() * 2, s_tb);
    T->tauhh = (const uint16_t *)put(H.tauh_hi.data(), H.tauh_hi.size() * 2, s_tb);
    T->tauhl = (const uint16_t *)put(H.tauh_lo.data(), H.tauh_lo.size() * 2, s_tb);
    T->tau_f16_shift = H.tau_f16_shift;
    T->f16_zc = (float)H.f16_zc;
    T->f16_zb = (float)H.f16_zb;
    T->base = base;
    e = hipMemcpy(base, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("hipMemcpy(tables)", e);
        (void)hipFree(base);
        delete T;
        return FEINT_ERR_HIP;
    }
    g_tables[key] = T;
    return FEINT_OK;
}

// Tables for a launch on `stream`: prepared on demand unless the stream is
// being captured.
feint_status tables_for_launch(int p, hipStream_t stream, const DevTables **out, int rule, int type) {
    const DevTables *T = find_tables(p, rule, type);
    if (!T) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(stream, &cs);
        if (e != hipSuccess) { set_error("hipStreamIsCapturing", e); return FEINT_ERR_HIP; }
        if (cs != hipStreamCaptureStatusNone) return FEINT_ERR_NOT_PREPARED;
        feint_status s = prepare_tables(p, rule, type);
        if (s != FEINT_OK) return s;
        T = find_tables(p, rule, type);
    }
    *out = T;
    return FEINT_OK;
}

// Element inputs: ne >= 0; the five arrays must be non-null unless ne == 0.
feint_status check_elements(const feint_elements *el) {
    if (!el) return FEINT_ERR_INVALID_ARG;
    if (el->ne < 0) return FEINT_ERR_INVALID_ARG;
    if (el->ne == 0) return FEINT_OK;
    if (!el->coords || !el->D || !el->beta || !el->c || !el->f) return FEINT_ERR_INVALID_ARG;
    return FEINT_OK;
}

void fill_fwd_params(FwdParams &prm, const feint_elements *el, int form, const DevTables *T) {
    std::memset(&prm, 0, sizeof prm);
    prm.coords = el->coords; prm.D = el->D; prm.beta = el->beta; prm.c = el->c; prm.f = el->f;
    prm.ne = el->ne;
    prm.qw = T->qw; prm.gll = T->gll; prm.tau64 = T->tau64; prm.tau32 = T->tau32; prm.lam = T->lam; prm.lam32 = T->lam32;
    prm.B64 = T->B64; prm.B32 = T->B32; prm.Bc32 = T->Bc32; prm.Ycf = T->Ycf;
    prm.Mref64 = T->Mref64; prm.Mref32 = T->Mref32;
    prm.taubh = form == FEINT_FP16X3 ? T->tauhh : T->taubh;
    prm.taubl = form == FEINT_FP16X3 ? T->tauhl : T->taubl;
    prm.tau_f16_shift = T->tau_f16_shift;
    prm.f16_zc = T->f16_zc;
    prm.f16_zb = T->f16_zb;
    prm.Bhi = form == FEINT_FP16X3 ? T->hf_hi : T->bf_hi;
    prm.Blo = form == FEINT_FP16X3 ? T->hf_lo : T->bf_lo;
    prm.bmax = T->bmax;
    prm.f16_shift = T->f16_shift;
}

const FwdVariant *fwd_variants(int form, int p, int *count, int rule) {
    if (rule == FEINT_RULE_SYMMETRIC) return fwd_variants_sym(form, p, count);
    switch (form) {
    case FEINT_FP64: return fwd_variants_f64(p, count);
    case FEINT_FP32: return fwd_variants_f32(p, count);
    case FEINT_BF16X3: return fwd_variants_bf16(p, count);
    case FEINT_FP16X3: return fwd_variants_f16(p, count);
    }
    *count = 0;
    return nullptr;
}

const FwdVariant *chosen_variant(int p, int form, int rule) {
    int cnt = 0;
    const FwdVariant *v = fwd_variants(form, p, &cnt, rule);
    if (!v || cnt == 0) return nullptr;
    int t;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        t = g_tile[rule][p][form];
    }
    return &v[(t >= 0 && t < cnt) ? t : 0];
}

feint_status launch_forward(const FwdParams &prm, const FwdVariant *v, hipStream_t stream) {
    const int64_t blocks = (v->items(prm.ne) + 3) / 4;
    if (blocks > 0x7fffffffLL) return FEINT_ERR_TOO_LARGE;
    (void)hipGetLastError();
    v->launch(prm, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("forward launch", e); return FEINT_ERR_HIP; }
    return FEINT_OK;
}

}  // namespace feint

using namespace feint;

extern "C" {

int feint_nshp(int p) { return (p < 1 || p > kMaxP) ? -1 : nshp_of(p); }
int feint_nq(int p) { return (p < 1 || p > kMaxP) ? -1 : nq_of(p); }

size_t feint_elem_size(feint_form form) {
    if (!valid_form(form)) return 0;
    return form == FEINT_FP64 ? 8 : 4;
}

feint_status feint_prepare(int p) { return prepare_tables(p, FEINT_RULE_COLLAPSED); }

int feint_nq_rule(int p, feint_rule rule) {
    return (p < 1 || p > kMaxP || !valid_rule(rule)) ? -1 : nq_rule_of(p, rule);
}

feint_status feint_prepare_rule(int p, feint_rule rule) { return prepare_tables(p, rule); }

feint_status feint_rule_points(int p, feint_rule rule, double *pts, int64_t cap) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_rule(rule) || !pts || cap < nq_rule_of(p, rule)) return FEINT_ERR_INVALID_ARG;
    std::vector<double> qw;
    rule_points(p, rule, qw);
    std::memcpy(pts, qw.data(), qw.size() * sizeof(double));
    return FEINT_OK;
}

feint_status feint_integrate_rule(const feint_elements *el, const feint_fields *fl, int p, feint_form form,
                                  feint_rule rule, void *A, void *b, double *xq, uint32_t *dev_status,
                                  void *stream) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_form(form)) return FEINT_ERR_UNSUPPORTED_FORM;
    if (!valid_rule(rule) || (el == nullptr) == (fl == nullptr)) return FEINT_ERR_INVALID_ARG;
    feint_elements cel;
    if (el) {
        feint_status s = check_elements(el);
        if (s != FEINT_OK) return s;
        cel = *el;
    } else {
        if (fl->ne < 0) return FEINT_ERR_INVALID_ARG;
        if (fl->ne > 0 && (!fl->coords || !fl->D || !fl->beta || !fl->c || !fl->f)) return FEINT_ERR_INVALID_ARG;
        cel = {fl->coords, nullptr, nullptr, nullptr, nullptr, fl->ne};
    }
    if (cel.ne == 0) return FEINT_OK;
    if (!A || !b) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const DevTables *T = nullptr;
    feint_status s = tables_for_launch(p, st, &T, rule);
    if (s != FEINT_OK) return s;
    FwdParams prm;
    fill_fwd_params(prm, &cel, form, T);
    if (fl) { prm.fD = fl->D; prm.fbeta = fl->beta; prm.fc = fl->c; prm.ff = fl->f; }
    prm.A = A; prm.b = b; prm.xq = xq; prm.status = dev_status;
    const FwdVariant *v = chosen_variant(p, form, rule);
    if (!v) return FEINT_ERR_UNSUPPORTED_FORM;
    return launch_forward(prm, v, st);
}

feint_status feint_integrate_fields(const feint_fields *fl, int p, feint_form form, void *A, void *b,
                                    double *xq, uint32_t *dev_status, void *stream) {
    if (!fl) return FEINT_ERR_INVALID_ARG;
    return feint_integrate_rule(nullptr, fl, p, form, FEINT_RULE_COLLAPSED, A, b, xq, dev_status, stream);
}

feint_status feint_integrate(const feint_elements *el, int p, feint_form form, void *A, void *b,
                             double *xq, uint32_t *dev_status, void *stream) {
    if (!el) return FEINT_ERR_INVALID_ARG;
    return feint_integrate_rule(el, nullptr, p, form, FEINT_RULE_COLLAPSED, A, b, xq, dev_status, stream);
}

int feint_rule_tile_count(int p, feint_form form, feint_rule rule) {
    int cnt = 0;
    if (p < 1 || p > kMaxP || !valid_form(form) || !valid_rule(rule)) return 0;
    fwd_variants(form, p, &cnt, rule);
    return cnt;
}

int feint_rule_tile_get(int p, feint_form form, feint_rule rule) {
    if (p < 1 || p > kMaxP || !valid_form(form) || !valid_rule(rule)) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tile[rule][p][form];
}

feint_status feint_rule_tile_set(int p, feint_form form, feint_rule rule, int tile) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_form(form)) return FEINT_ERR_UNSUPPORTED_FORM;
    if (!valid_rule(rule) || tile < 0 || tile >= feint_rule_tile_count(p, form, rule)) return FEINT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tile[rule][p][form] = tile;
    return FEINT_OK;
}

// "TMxTN" plus the kernel kind (s staged, sa A operands staged, p pipelined,
// c shape functions computed per point, f contraction per triangle or plane
// point, fw the same with two waves per element sharing its point blocks, y split form with Y formed on
// the matrix cores; "vL" vector-ALU kernel with L lanes per element)
// and "o2" for a two-waves-per-SIMD register budget.
static void describe_variant(const FwdVariant &v, char *buf, size_t len) {
    if (v.staged == 3)
        std::snprintf(buf, len, "v%d%s", v.tn, v.minw > 1 ? ("o" + std::to_string(v.minw)).c_str() : "");
    else if (v.staged == 11)
        std::snprintf(buf, len, "ref%d%s%s%s", v.tm, v.tn % 4 == 2 ? "s" : "", v.tn >= 4 ? ("e" + std::to_string(v.tn / 4)).c_str() : "",
                      v.minw > 1 ? ("o" + std::to_string(v.minw)).c_str() : "");
    else if (v.staged >= 8 && v.staged <= 10)
        std::snprintf(buf, len, "sf%dw%s%s%s", v.tn, v.tm > 1 ? ("x" + std::to_string(v.tm)).c_str() : "",
                      v.staged == 9 ? "r" : v.staged == 10 ? "l" : "",
                      v.minw > 1 ? ("o" + std::to_string(v.minw)).c_str() : "");
    else
        std::snprintf(buf, len, "%dx%d%s%s", v.tm, v.tn,
                      v.staged == 1 ? "s" : v.staged == 2 ? "sa" : v.staged == 4 ? "p"
                      : v.staged == 5 ? "c" : v.staged == 6 ? "f" : v.staged == 7 ? "y" : v.staged == 13 ? "fw" : v.staged == 15 ? "fwg" : v.staged == 16 ? "fz" : "",
                      v.minw > 1 ? ("o" + std::to_string(v.minw)).c_str() : "");
}

feint_status feint_rule_tile_describe(int p, feint_form form, feint_rule rule, int tile, char *buf, size_t len) {
    int cnt = 0;
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_form(form)) return FEINT_ERR_UNSUPPORTED_FORM;
    if (!valid_rule(rule)) return FEINT_ERR_INVALID_ARG;
    const FwdVariant *v = fwd_variants(form, p, &cnt, rule);
    if (!buf || tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    describe_variant(v[tile], buf, len);
    return FEINT_OK;
}

int feint_tile_count(int p, feint_form form) { return feint_rule_tile_count(p, form, FEINT_RULE_COLLAPSED); }
int feint_tile_get(int p, feint_form form) { return feint_rule_tile_get(p, form, FEINT_RULE_COLLAPSED); }
feint_status feint_tile_set(int p, feint_form form, int tile) {
    return feint_rule_tile_set(p, form, FEINT_RULE_COLLAPSED, tile);
}
feint_status feint_tile_describe(int p, feint_form form, int tile, char *buf, size_t len) {
    return feint_rule_tile_describe(p, form, FEINT_RULE_COLLAPSED, tile, buf, len);
}

feint_status feint_autotune_rule(const feint_elements *el, const feint_fields *fl, int p, feint_form form,
                                 feint_rule rule, void *A, void *b, int reps, double *best_ms, void *stream) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_form(form)) return FEINT_ERR_UNSUPPORTED_FORM;
    if (!valid_rule(rule) || (el == nullptr) == (fl == nullptr) || reps < 1 || !A || !b) return FEINT_ERR_INVALID_ARG;
    feint_elements cel;
    if (el) {
        feint_status s = check_elements(el);
        if (s != FEINT_OK) return s;
        cel = *el;
    } else {
        if (fl->ne < 0 || (fl->ne > 0 && (!fl->coords || !fl->D || !fl->beta || !fl->c || !fl->f)))
            return FEINT_ERR_INVALID_ARG;
        cel = {fl->coords, nullptr, nullptr, nullptr, nullptr, fl->ne};
    }
    if (cel.ne == 0) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const DevTables *T = nullptr;
    feint_status s = tables_for_launch(p, st, &T, rule);
    if (s != FEINT_OK) return s;
    FwdParams prm;
    fill_fwd_params(prm, &cel, form, T);
    if (fl) { prm.fD = fl->D; prm.fbeta = fl->beta; prm.fc = fl->c; prm.ff = fl->f; }
    prm.A = A; prm.b = b;
    int cnt = 0;
    const FwdVariant *v = fwd_variants(form, p, &cnt, rule);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FEINT_ERR_HIP;
    int best = 0;
    float best_t = 1e30f;
    // one launch of every variant first, so that the first ones timed do not
    // pay for the device settling (clocks, first launches) after other work
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) s = launch_forward(prm, &v[t], st);
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {
        s = launch_forward(prm, &v[t], st);                 // warm-up
        if (s != FEINT_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == FEINT_OK; ++r) s = launch_forward(prm, &v[t], st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { s = FEINT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) { best_t = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FEINT_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tile[rule][p][form] = best;
    }
    if (best_ms) *best_ms = best_t;
    return FEINT_OK;
}

feint_status feint_autotune(const feint_elements *el, int p, feint_form form, void *A, void *b, int reps,
                            double *best_ms, void *stream) {
    if (!el) return FEINT_ERR_INVALID_ARG;
    return feint_autotune_rule(el, nullptr, p, form, FEINT_RULE_COLLAPSED, A, b, reps, best_ms, stream);
}

// ---- Hexahedra (type 1) and tetrahedra (type 2): generic helpers -------------
static const FwdVariant *elem_variants(int type, int form, int p, int *cnt) {
    *cnt = 0;
    if (p < 1 || p > kMaxP || !valid_form(form)) return nullptr;
    return type == 1 ? fwd_variants_hex(form, p, cnt) : fwd_variants_tet(form, p, cnt);
}

static int elem_tile_count(int type, int p, int form) {
    int cnt = 0;
    elem_variants(type, form, p, &cnt);
    return cnt;
}

static int elem_tile_get(int type, int p, int form) {
    if (elem_tile_count(type, p, form) == 0) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tile_elem[type][p][form];
}

static feint_status elem_tile_set(int type, int p, int form, int tile) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    const int cnt = elem_tile_count(type, p, form);
    if (cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tile_elem[type][p][form] = tile;
    return FEINT_OK;
}

static feint_status elem_tile_describe(int type, int p, int form, int tile, char *buf, size_t len) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (!valid_form(form)) return FEINT_ERR_UNSUPPORTED_FORM;
    int cnt = 0;
    const FwdVariant *v = elem_variants(type, form, p, &cnt);
    if (!buf || tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    describe_variant(v[tile], buf, len);
    return FEINT_OK;
}

// Forward parameters of a launch (host checks done by the caller); tile < 0
// takes the chosen variant.
static feint_status elem_params(int type, const feint_elements *el, int p, int form, void *A, void *b,
                                hipStream_t st, FwdParams &prm, const FwdVariant **vsel, int tile) {
    const DevTables *T = nullptr;
    feint_status s = tables_for_launch(p, st, &T, FEINT_RULE_COLLAPSED, type);
    if (s != FEINT_OK) return s;
    fill_fwd_params(prm, el, form, T);
    prm.A = A; prm.b = b;
    int cnt = 0;
    const FwdVariant *v = elem_variants(type, form, p, &cnt);
    if (!v || cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (tile < 0) {
        std::lock_guard<std::mutex> lk(g_mu);
        tile = g_tile_elem[type][p][form];
    }
    *vsel = &v[(tile >= 0 && tile < cnt) ? tile : 0];
    return FEINT_OK;
}

static feint_status elem_integrate(int type, const feint_elements *el, int p, int form, void *A, void *b,
                                   double *xq, uint32_t *dev_status, void *stream) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (elem_tile_count(type, p, form) == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne == 0) return FEINT_OK;
    if (!A || !b) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    FwdParams prm;
    const FwdVariant *v = nullptr;
    s = elem_params(type, el, p, form, A, b, st, prm, &v, -1);
    if (s != FEINT_OK) return s;
    prm.xq = xq;
    prm.status = dev_status;
    return launch_forward(prm, v, st);
}

static feint_status elem_autotune(int type, const feint_elements *el, int p, int form, void *A, void *b, int reps,
                                  double *best_ms, void *stream) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    const int cnt = elem_tile_count(type, p, form);
    if (cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (!A || !b || el->ne == 0 || reps < 1) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FEINT_ERR_HIP;
    int best = 0;
    float best_t = 1e30f;
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {   // one launch of every variant first
        FwdParams prm;
        const FwdVariant *v = nullptr;
        s = elem_params(type, el, p, form, A, b, st, prm, &v, t);
        if (s == FEINT_OK) s = launch_forward(prm, v, st);
    }
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {
        FwdParams prm;
        const FwdVariant *v = nullptr;
        s = elem_params(type, el, p, form, A, b, st, prm, &v, t);
        if (s != FEINT_OK) break;
        s = launch_forward(prm, v, st);                       // warm-up
        if (s != FEINT_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == FEINT_OK; ++r) s = launch_forward(prm, v, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { s = FEINT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) { best_t = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FEINT_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tile_elem[type][p][form] = best;
    }
    if (best_ms) *best_ms = best_t;
    return FEINT_OK;
}

int feint_hex_nshp(int p) { return (p < 1 || p > kMaxP) ? -1 : (p + 1) * (p + 1) * (p + 1); }
int feint_hex_nq(int p) { return feint_hex_nshp(p); }
feint_status feint_prepare_hex(int p) { return prepare_tables(p, FEINT_RULE_COLLAPSED, 1); }
int feint_hex_tile_count(int p, feint_form form) { return elem_tile_count(1, p, form); }
int feint_hex_tile_get(int p, feint_form form) { return elem_tile_get(1, p, form); }
feint_status feint_hex_tile_set(int p, feint_form form, int tile) { return elem_tile_set(1, p, form, tile); }
feint_status feint_hex_tile_describe(int p, feint_form form, int tile, char *buf, size_t len) {
    return elem_tile_describe(1, p, form, tile, buf, len);
}
feint_status feint_integrate_hex(const feint_elements *el, int p, feint_form form, void *A, void *b,
                                 double *xq, uint32_t *dev_status, void *stream) {
    return elem_integrate(1, el, p, form, A, b, xq, dev_status, stream);
}
feint_status feint_hex_autotune(const feint_elements *el, int p, feint_form form, void *A, void *b, int reps,
                                double *best_ms, void *stream) {
    return elem_autotune(1, el, p, form, A, b, reps, best_ms, stream);
}

int feint_tet_nshp(int p) { return (p < 1 || p > kMaxP) ? -1 : (p + 1) * (p + 2) * (p + 3) / 6; }
int feint_tet_nq(int p) { return (p < 1 || p > kMaxP) ? -1 : (p + 2) * (p + 2) * (p + 2); }
feint_status feint_prepare_tet(int p) { return prepare_tables(p, FEINT_RULE_COLLAPSED, 2); }
int feint_tet_tile_count(int p, feint_form form) { return elem_tile_count(2, p, form); }
int feint_tet_tile_get(int p, feint_form form) { return elem_tile_get(2, p, form); }
feint_status feint_tet_tile_set(int p, feint_form form, int tile) { return elem_tile_set(2, p, form, tile); }
feint_status feint_tet_tile_describe(int p, feint_form form, int tile, char *buf, size_t len) {
    return elem_tile_describe(2, p, form, tile, buf, len);
}
feint_status feint_integrate_tet(const feint_elements *el, int p, feint_form form, void *A, void *b,
                                 double *xq, uint32_t *dev_status, void *stream) {
    return elem_integrate(2, el, p, form, A, b, xq, dev_status, stream);
}
feint_status feint_tet_autotune(const feint_elements *el, int p, feint_form form, void *A, void *b, int reps,
                                double *best_ms, void *stream) {
    return elem_autotune(2, el, p, form, A, b, reps, best_ms, stream);
}

// ---- The Laplace term alone on the symmetric rule --------------------------
static int lap_tile_count(int p, int form) {
    int cnt = 0;
    if (p < 1 || p > kMaxP || (form != FEINT_FP64 && form != FEINT_FP32)) return 0;
    fwd_variants_lap(form, p, &cnt);
    return cnt;
}

// Forward parameters of a Laplace launch (host checks done by the caller); tile < 0
// takes the chosen variant.
static feint_status lap_params(const double *coords, int64_t ne, int p, int form, void *A, hipStream_t st,
                               FwdParams &prm, const FwdVariant **vsel, int tile) {
    const DevTables *T = nullptr;
    feint_status s = tables_for_launch(p, st, &T, FEINT_RULE_SYMMETRIC, 0);
    if (s != FEINT_OK) return s;
    const feint_elements el = {coords, nullptr, nullptr, nullptr, nullptr, ne};
    fill_fwd_params(prm, &el, form, T);
    prm.A = A;
    prm.b = nullptr;
    int cnt = 0;
    const FwdVariant *v = fwd_variants_lap(form, p, &cnt);
    if (!v || cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (tile < 0) {
        std::lock_guard<std::mutex> lk(g_mu);
        tile = g_tile_lap[p][form];
    }
    *vsel = &v[(tile >= 0 && tile < cnt) ? tile : 0];
    return FEINT_OK;
}

static feint_status lap_check(const double *coords, int64_t ne, int p, int form, const void *A) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    if (lap_tile_count(p, form) == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (ne < 0) return FEINT_ERR_INVALID_ARG;
    if (ne > 0 && (!coords || !A)) return FEINT_ERR_INVALID_ARG;
    return FEINT_OK;
}

feint_status feint_integrate_laplace(const double *coords, int64_t ne, int p, feint_form form, void *A, double *xq,
                                     uint32_t *dev_status, void *stream) {
    feint_status s = lap_check(coords, ne, p, form, A);
    if (s != FEINT_OK || ne == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    FwdParams prm;
    const FwdVariant *v = nullptr;
    s = lap_params(coords, ne, p, form, A, st, prm, &v, -1);
    if (s != FEINT_OK) return s;
    prm.xq = xq;
    prm.status = dev_status;
    return launch_forward(prm, v, st);
}

int feint_laplace_tile_count(int p, feint_form form) { return lap_tile_count(p, form); }

int feint_laplace_tile_get(int p, feint_form form) {
    if (lap_tile_count(p, form) == 0) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tile_lap[p][form];
}

feint_status feint_laplace_tile_set(int p, feint_form form, int tile) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    const int cnt = lap_tile_count(p, form);
    if (cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tile_lap[p][form] = tile;
    return FEINT_OK;
}

feint_status feint_laplace_tile_describe(int p, feint_form form, int tile, char *buf, size_t len) {
    if (p < 1 || p > kMaxP) return FEINT_ERR_UNSUPPORTED_DEGREE;
    const int cnt = lap_tile_count(p, form);
    if (cnt == 0) return FEINT_ERR_UNSUPPORTED_FORM;
    if (!buf || tile < 0 || tile >= cnt) return FEINT_ERR_INVALID_ARG;
    int c = 0;
    describe_variant(fwd_variants_lap(form, p, &c)[tile], buf, len);
    return FEINT_OK;
}

feint_status feint_laplace_autotune(const double *coords, int64_t ne, int p, feint_form form, void *A, int reps,
                                    double *best_ms, void *stream) {
    feint_status s = lap_check(coords, ne, p, form, A);
    if (s != FEINT_OK) return s;
    if (ne == 0 || reps < 1) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int cnt = lap_tile_count(p, form);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FEINT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FEINT_ERR_HIP; }
    int best = 0;
    float best_t = 1e30f;
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {   // one launch of every variant first
        FwdParams prm;
        const FwdVariant *v = nullptr;
        s = lap_params(coords, ne, p, form, A, st, prm, &v, t);
        if (s == FEINT_OK) s = launch_forward(prm, v, st);
    }
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {
        FwdParams prm;
        const FwdVariant *v = nullptr;
        s = lap_params(coords, ne, p, form, A, st, prm, &v, t);
        if (s != FEINT_OK) break;
        s = launch_forward(prm, v, st);                       // warm-up
        if (s != FEINT_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == FEINT_OK; ++r) s = launch_forward(prm, v, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { s = FEINT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) { best_t = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FEINT_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tile_lap[p][form] = best;
    }
    if (best_ms) *best_ms = best_t;
    return FEINT_OK;
}

const char *feint_status_string(feint_status s) {
    switch (s) {
    case FEINT_OK: return "ok";
    case FEINT_ERR_INVALID_ARG: return "invalid argument";
    case FEINT_ERR_UNSUPPORTED_DEGREE: return "unsupported degree";
    case FEINT_ERR_UNSUPPORTED_FORM: return "unsupported form";
    case FEINT_ERR_NOT_PREPARED: return "tables not prepared (stream is capturing)";
    case FEINT_ERR_HIP: return "HIP runtime error";
    case FEINT_ERR_TOO_LARGE: return "batch too large for one launch";
    }
    return "unknown status";
}

const char *feint_last_error(void) { return g_err.c_str(); }

void feint_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_tables) {
        (void)hipSetDevice(kv.first / 64);
        (void)hipFree(kv.second->base);
        delete kv.second;
    }
    (void)hipSetDevice(cur);
    g_tables.clear();
}

}  // extern "C"
