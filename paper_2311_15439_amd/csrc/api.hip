// C ABI of libspx.so (declared in include/spx.h): argument checks, the
// host-side constants (level multipliers, skew factor), and dispatch to the
// kernel translation units.  No allocation, no synchronisation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "spx.h"
#include "lookup.hpp"
#include "spx_internal.h"

namespace spx {

static thread_local spx_trace* g_trace = nullptr;
static thread_local bool g_trace_open = false;  // the last trace_begin recorded an event

void trace_begin(hipStream_t s, const char* name, double bytes) {
    spx_trace* t = g_trace;
    g_trace_open = false;
    if (!t || t->count >= t->capacity || (t->only && strcmp(t->only, name) != 0)) return;
    hipEventRecord(t->events[2 * t->count], s);
    t->names[t->count] = name;
    t->bytes[t->count] = bytes;
    g_trace_open = true;
}

void trace_end(hipStream_t s) {
    spx_trace* t = g_trace;
    if (!t || !g_trace_open) return;
    g_trace_open = false;
    hipEventRecord(t->events[2 * t->count + 1], s);
    t->count += 1;
}

// Side stream per device for work that can run beside the main stream
// (created on first use, default priority).  Callers hold the returned lock
// while they fork to it and join back, so concurrent callers do not share
// the fork/join events mid-sequence.
static std::mutex g_aux_mu;
static AuxStream g_aux[64];

AuxStream* aux_stream(std::unique_lock<std::mutex>& lock) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    lock = std::unique_lock<std::mutex>(g_aux_mu);
    AuxStream& a = g_aux[dev];
    if (!a.s) {
        hipStream_t st = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(st);
            return nullptr;
        }
        if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(fork);
            (void)hipStreamDestroy(st);
            return nullptr;
        }
        a.s = st;
        a.fork = fork;
        a.join = join;
    }
    return &a;
}

}  // namespace spx

namespace {

thread_local char g_err[512] = "";

spx_status fail(spx_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

spx_status from_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SPX_OK;
    return fail(SPX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t row_align(int F, int elem) {
    size_t b = (size_t)F * elem;
    return b > 16 ? 16 : b;
}

spx_status check_encoding(const spx_encoding* e) {
    if (!e) return fail(SPX_EINVAL, "encoding descriptor is NULL");
    if (e->n_dims < 1 || e->n_dims > SPX_MAX_DIMS) return fail(SPX_EINVAL, "n_dims=%d outside 1..%d", e->n_dims, SPX_MAX_DIMS);
    if (e->n_levels < 1 || e->n_levels > SPX_MAX_LEVELS)
        return fail(SPX_EINVAL, "n_levels=%d outside 1..%d", e->n_levels, SPX_MAX_LEVELS);
    if (e->log2_T < 1 || e->log2_T > SPX_MAX_LOG2_T)
        return fail(SPX_EINVAL, "log2_T=%d outside 1..%d", e->log2_T, SPX_MAX_LOG2_T);
    if (e->n_feat != 1 && e->n_feat != 2 && e->n_feat != 4 && e->n_feat != 8)
        return fail(SPX_EINVAL, "n_feat=%d not in {1,2,4,8}", e->n_feat);
    if (e->table_dtype != SPX_F32 && e->table_dtype != SPX_F16)
        return fail(SPX_EINVAL, "table_dtype=%d is not SPX_F32 or SPX_F16", e->table_dtype);
    if (e->cell != SPX_SIMPLEX && e->cell != SPX_GRID) return fail(SPX_EINVAL, "cell=%d unknown", e->cell);
    if (e->equal_memory != 0 && e->equal_memory != 1) return fail(SPX_EINVAL, "equal_memory must be 0 or 1");
    if (e->layout != SPX_LAYOUT_HASHED && e->layout != SPX_LAYOUT_SIZED)
        return fail(SPX_EINVAL, "layout=%d is not SPX_LAYOUT_HASHED or SPX_LAYOUT_SIZED", e->layout);
    for (int l = 0; l < e->n_levels; ++l)
        if (e->res[l] < 1) return fail(SPX_EINVAL, "res[%d]=%d < 1", l, e->res[l]);
    return SPX_OK;
}

void level_scales(const spx_encoding* e, float* sigma) {
    const int n = e->n_dims;
    const double S = sqrt((double)n + 1.0);
    const double c = (e->equal_memory && e->cell == SPX_SIMPLEX)
                         ? pow((double)n + 1.0, (double)(n - 1) / (2.0 * (double)n))
                         : 1.0;
    for (int l = 0; l < e->n_levels; ++l) {
        if (e->cell == SPX_GRID)
            sigma[l] = (float)(double)e->res[l];
        else
            sigma[l] = (float)(((double)e->res[l] * c) / S);
    }
}

// Box extent per axis at one level: the far corner (1, ..., 1) of the unit
// cube through the binary32 index path (skew, then scale) gives the largest
// scaled coordinate of any point of the closed cube, so its vertices lie in
// [0, floor(p) + 1].
int32_t box_extent(const spx_encoding* e, float sigma, float Fn) {
#pragma clang fp contract(off)
    float y = 1.0f;
    if (e->cell == SPX_SIMPLEX) {
        float s = 1.0f;
        for (int i = 1; i < e->n_dims; ++i) s = s + 1.0f;
        const float t = s * Fn;
        y = 1.0f + t;
    }
    const float p = y * sigma;
    return (int32_t)floorf(p) + 2;
}

// Rows of each level (Sec. 5.2, Hash Table Selection): SPX_LAYOUT_HASHED
// gives every level T rows; SPX_LAYOUT_SIZED stores a level densely when
// its ext^n box fits in T rows, and otherwise gives it the smallest power of
// two P >= u ext^n, u = (n+1)^(-(n-1)/2) for the simplex (1 for the grid),
// at most T; for the simplex the test is P^2 (n+1)^(n-1) >= (ext^n)^2 in
// integers.
void level_layout(const spx_encoding* e, spx::LevelArgs& lv) {
    const int n = e->n_dims;
    const uint64_t T = 1ull << e->log2_T;
    uint64_t off = 0;
    lv.dense = 0;
    for (int l = 0; l < e->n_levels; ++l) {
        const int32_t ext = box_extent(e, lv.sigma[l], lv.Fn);
        uint64_t B = 1;
        for (int i = 0; i < n && B <= (1ull << 40); ++i) B *= (uint64_t)ext;
        uint64_t rows = T;
        if (e->layout == SPX_LAYOUT_SIZED) {
            if (B <= T) {
                rows = B;
                lv.dense |= 1u << l;
            } else if (B <= (1ull << 40)) {
                unsigned __int128 k = 1;
                if (e->cell == SPX_SIMPLEX)
                    for (int i = 0; i + 1 < n; ++i) k *= (unsigned)(n + 1);
                const unsigned __int128 B2 = (unsigned __int128)B * B;
                uint64_t P = 1;
                while (P < T) {
                    const bool enough = e->cell == SPX_SIMPLEX ? (unsigned __int128)P * P * k >= B2 : P >= B;
                    if (enough) break;
                    P <<= 1;
                }
                rows = P;
            }
        }
        lv.ext[l] = ext;
        lv.rows[l] = (uint32_t)rows;
        lv.off[l] = off;
        off += rows;
    }
}

spx::LevelArgs level_args(const spx_encoding* e) {
    spx::LevelArgs lv;
    memset(&lv, 0, sizeof(lv));
    level_scales(e, lv.sigma);
    const int n = e->n_dims;
    lv.Fn = (float)((sqrt((double)n + 1.0) - 1.0) / (double)n);
    lv.mask = (uint32_t)((1ull << e->log2_T) - 1ull);
    lv.L = e->n_levels;
    level_layout(e, lv);
    return lv;
}

spx::EncodeCall base_call(const spx_encoding* e, int64_t N, const float* pts, hipStream_t s) {
    spx::EncodeCall c;
    memset(&c, 0, sizeof(c));
    c.D = e->n_dims;
    c.F = e->n_feat;
    c.table_f16 = e->table_dtype == SPX_F16;
    c.N = N;
    c.pts = pts;
    c.lv = level_args(e);
    c.stream = s;
    return c;
}

spx::BinLayout layout_for(const spx_encoding* e, int64_t N) {
    const spx::LevelArgs lv = level_args(e);
    return spx::bin_layout(e->n_dims, e->n_feat, N, e->cell == SPX_SIMPLEX, lv);
}

hipError_t run(const spx_encoding* e, const spx::EncodeCall& c) {
    return e->cell == SPX_GRID ? spx::encode_cell<true>(c) : spx::encode_cell<false>(c);
}

spx_status check_points(int64_t N, const float* pts) {
    if (N < 0) return fail(SPX_EINVAL, "N=%lld < 0", (long long)N);
    if (N > 0 && !pts) return fail(SPX_EINVAL, "pts is NULL");
    if (pts && !aligned(pts, 4)) return fail(SPX_EALIGN, "pts not 4-byte aligned");
    return SPX_OK;
}

}  // namespace

extern "C" {

int32_t spx_abi_version(void) { return SPX_ABI_VERSION; }

spx_status spx_trace_set(spx_trace* trace) {
    if (trace && (trace->capacity < 0 || (trace->capacity > 0 && (!trace->events || !trace->names || !trace->bytes))))
        return fail(SPX_EINVAL, "trace arrays missing");
    spx::g_trace = trace;
    return SPX_OK;
}

const char* spx_status_str(spx_status s) {
    switch (s) {
        case SPX_OK: return "SPX_OK";
        case SPX_EINVAL: return "SPX_EINVAL: invalid argument";
        case SPX_EALIGN: return "SPX_EALIGN: misaligned device pointer";
        case SPX_EUNSUPPORTED: return "SPX_EUNSUPPORTED: configuration not built";
        case SPX_EHIP: return "SPX_EHIP: HIP runtime error";
    }
    return "unknown spx_status";
}

const char* spx_last_error(void) { return g_err; }

spx_status spx_level_resolutions(double n_min, double growth, int32_t L, int32_t* res_out) {
    if (L < 1 || L > SPX_MAX_LEVELS) return fail(SPX_EINVAL, "L=%d outside 1..%d", L, SPX_MAX_LEVELS);
    if (!(n_min >= 1.0) || !(growth >= 1.0)) return fail(SPX_EINVAL, "n_min and growth must be >= 1");
    if (!res_out) return fail(SPX_EINVAL, "res_out is NULL");
    for (int l = 0; l < L; ++l) {
        const double v = floor(n_min * pow(growth, (double)l) + 1e-6);
        if (v > 2147483647.0) return fail(SPX_EINVAL, "level %d resolution overflows int32", l);
        res_out[l] = (int32_t)v;
    }
    return SPX_OK;
}

spx_status spx_level_scales(const spx_encoding* enc, float* sigma_out) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if (!sigma_out) return fail(SPX_EINVAL, "sigma_out is NULL");
    level_scales(enc, sigma_out);
    return SPX_OK;
}

spx_status spx_table_layout(const spx_encoding* enc, int64_t* level_rows, int32_t* box_extent_out,
                            int32_t* dense_out, int64_t* total_rows) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    const spx::LevelArgs lv = level_args(enc);
    int64_t total = 0;
    for (int l = 0; l < enc->n_levels; ++l) {
        if (level_rows) level_rows[l] = (int64_t)lv.rows[l];
        if (box_extent_out) box_extent_out[l] = lv.ext[l];
        if (dense_out) dense_out[l] = (int32_t)((lv.dense >> l) & 1u);
        total += (int64_t)lv.rows[l];
    }
    if (total_rows) *total_rows = total;
    return SPX_OK;
}

spx_status spx_hash_primes(uint32_t* primes_out) {
    if (!primes_out) return fail(SPX_EINVAL, "primes_out is NULL");
    for (int i = 0; i < SPX_MAX_DIMS; ++i) primes_out[i] = spx::hash_prime(i);
    return SPX_OK;
}

spx_status spx_encode_fwd(const spx_encoding* enc, int64_t N, const float* pts, const void* tables, void* out,
                          int32_t out_dtype, hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (out_dtype != SPX_F32 && out_dtype != SPX_F16) return fail(SPX_EINVAL, "out_dtype=%d", out_dtype);
    if (N == 0) return SPX_OK;
    if (!tables || !out) return fail(SPX_EINVAL, "tables or out is NULL");
    const int te = enc->table_dtype == SPX_F16 ? 2 : 4, oe = out_dtype == SPX_F16 ? 2 : 4;
    if (!aligned(tables, row_align(enc->n_feat, te))) return fail(SPX_EALIGN, "tables not row-aligned");
    if (!aligned(out, row_align(enc->n_feat, oe))) return fail(SPX_EALIGN, "out not row-aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::Forward;
    c.out_f16 = out_dtype == SPX_F16;
    c.tables = tables;
    c.out = out;
    return from_hip(run(enc, c), "spx_encode_fwd launch");
}

spx_status spx_encode_input_grad(const spx_encoding* enc, int64_t N, const float* pts, const void* tables,
                                 const void* d_out, int32_t d_out_dtype, float* d_pts, hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (d_out_dtype != SPX_F32 && d_out_dtype != SPX_F16) return fail(SPX_EINVAL, "d_out_dtype=%d", d_out_dtype);
    if (N == 0) return SPX_OK;
    if (!tables || !d_out || !d_pts) return fail(SPX_EINVAL, "tables, d_out or d_pts is NULL");
    const int te = enc->table_dtype == SPX_F16 ? 2 : 4, ge = d_out_dtype == SPX_F16 ? 2 : 4;
    if (!aligned(tables, row_align(enc->n_feat, te))) return fail(SPX_EALIGN, "tables not row-aligned");
    if (!aligned(d_out, row_align(enc->n_feat, ge))) return fail(SPX_EALIGN, "d_out not row-aligned");
    if (!aligned(d_pts, 4)) return fail(SPX_EALIGN, "d_pts not 4-byte aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::InputGrad;
    c.tables = tables;
    c.d_out = d_out;
    c.dout_f16 = d_out_dtype == SPX_F16;
    c.out = d_pts;
    return from_hip(run(enc, c), "spx_encode_input_grad launch");
}

spx_status spx_encode_gather_twin(const spx_encoding* enc, int64_t N, const float* pts, const void* tables,
                                  void* out, hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (enc->n_feat != 2 || enc->table_dtype != SPX_F16 || enc->layout != SPX_LAYOUT_HASHED)
        return fail(SPX_EUNSUPPORTED, "the gather twin covers hashed binary16 tables with n_feat = 2");
    if (N == 0) return SPX_OK;
    if (!tables || !out) return fail(SPX_EINVAL, "tables or out is NULL");
    if (!aligned(tables, 4) || !aligned(out, 4)) return fail(SPX_EALIGN, "tables/out not 4-byte aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::Twin;
    c.out_f16 = true;
    c.tables = tables;
    c.out = out;
    return from_hip(run(enc, c), "spx_encode_gather_twin launch");
}

spx_status spx_gather_probe(const void* table, int64_t n_words, int64_t n_threads, int32_t per_thread,
                            uint32_t seed, uint32_t* out, hipStream_t stream) {
    if (n_words < 1 || n_words > ((int64_t)1 << 32) || (n_words & (n_words - 1)) != 0)
        return fail(SPX_EINVAL, "n_words=%lld is not a power of two in 1..2^32", (long long)n_words);
    if (n_threads < 0 || n_threads > ((int64_t)1 << 30))
        return fail(SPX_EINVAL, "n_threads=%lld outside 0..2^30", (long long)n_threads);
    if (per_thread < 16 || per_thread > 4096 || per_thread % 16 != 0)
        return fail(SPX_EINVAL, "per_thread=%d is not a multiple of 16 in 16..4096", per_thread);
    if (n_threads == 0) return SPX_OK;
    if (!table || !out) return fail(SPX_EINVAL, "table or out is NULL");
    if (!aligned(table, 4) || !aligned(out, 4)) return fail(SPX_EALIGN, "table/out not 4-byte aligned");
    return from_hip(spx::gather_probe(table, n_words, n_threads, per_thread, seed, out, stream),
                    "spx_gather_probe launch");
}

spx_status spx_encode_bwd_workspace(const spx_encoding* enc, int64_t N, size_t* bytes) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if (N < 0) return fail(SPX_EINVAL, "N < 0");
    if (!bytes) return fail(SPX_EINVAL, "bytes is NULL");
    spx::BinLayout lay = layout_for(enc, N);
    if (!lay.ok) return fail(SPX_EUNSUPPORTED, "configuration too large for the binned adjoint");
    *bytes = lay.total_bytes;
    return SPX_OK;
}

// the workspace checks of every binned-adjoint call
static spx_status check_workspace(const spx_encoding* enc, int64_t N, const void* workspace, size_t workspace_bytes) {
    spx::BinLayout lay = layout_for(enc, N);
    if (!lay.ok) return fail(SPX_EUNSUPPORTED, "configuration too large for the binned adjoint");
    if (!workspace || workspace_bytes < lay.total_bytes)
        return fail(SPX_EINVAL, "workspace of %zu bytes needed, %zu given", lay.total_bytes, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(SPX_EALIGN, "workspace not 256-byte aligned");
    return SPX_OK;
}

spx_status spx_encode_bwd_prepare(const spx_encoding* enc, int64_t N, const float* pts, void* workspace,
                                  size_t workspace_bytes, hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (N == 0) return SPX_OK;
    if ((st = check_workspace(enc, N, workspace, workspace_bytes))) return st;
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::AdjointPrepare;
    c.workspace = workspace;
    return from_hip(run(enc, c), "spx_encode_bwd_prepare launch");
}

static spx_status encode_bwd_impl(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                  int32_t d_out_dtype, float* d_tables, void* workspace, size_t workspace_bytes,
                                  hipStream_t stream, bool prepared) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (d_out_dtype != SPX_F32 && d_out_dtype != SPX_F16) return fail(SPX_EINVAL, "d_out_dtype=%d", d_out_dtype);
    if (N == 0) return SPX_OK;
    if (!d_out || !d_tables) return fail(SPX_EINVAL, "d_out or d_tables is NULL");
    const int ge = d_out_dtype == SPX_F16 ? 2 : 4;
    if (!aligned(d_out, row_align(enc->n_feat, ge))) return fail(SPX_EALIGN, "d_out not row-aligned");
    if (!aligned(d_tables, 4)) return fail(SPX_EALIGN, "d_tables not 4-byte aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::Adjoint;
    if (workspace) {
        spx::BinLayout lay = layout_for(enc, N);
        if (!lay.ok) return fail(SPX_EUNSUPPORTED, "configuration too large for the binned adjoint");
        if (workspace_bytes < lay.total_bytes)
            return fail(SPX_EINVAL, "workspace of %zu bytes needed, %zu given", lay.total_bytes, workspace_bytes);
        if (!aligned(workspace, 256)) return fail(SPX_EALIGN, "workspace not 256-byte aligned");
        c.op = spx::EncodeOp::AdjointBinned;
        c.workspace = workspace;
    }
    if (prepared && !workspace) return fail(SPX_EINVAL, "a prepared adjoint needs its workspace");
    c.prepared = prepared;
    c.dout_f16 = d_out_dtype == SPX_F16;
    c.d_out = d_out;
    c.d_tables = d_tables;
    return from_hip(run(enc, c), prepared ? "spx_encode_bwd_prepared launch" : "spx_encode_bwd launch");
}

spx_status spx_encode_bwd(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                          int32_t d_out_dtype, float* d_tables, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
    return encode_bwd_impl(enc, N, pts, d_out, d_out_dtype, d_tables, workspace, workspace_bytes, stream, false);
}

spx_status spx_encode_bwd_prepared(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                   int32_t d_out_dtype, float* d_tables, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream) {
    return encode_bwd_impl(enc, N, pts, d_out, d_out_dtype, d_tables, workspace, workspace_bytes, stream, true);
}

static spx_status check_adam(const float* param, const float* m, const float* v, const uint16_t* param_f16,
                             float beta1, float beta2, float eps, int64_t step) {
    if (step < 1) return fail(SPX_EINVAL, "step=%lld < 1", (long long)step);
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return fail(SPX_EINVAL, "beta1/beta2 must lie in [0,1) and eps >= 0");
    if (!param || !m || !v) return fail(SPX_EINVAL, "param, m or v is NULL");
    if (!aligned(param, 16) || !aligned(m, 16) || !aligned(v, 16) || (param_f16 && !aligned(param_f16, 8)))
        return fail(SPX_EALIGN, "Adam state misaligned (param/m/v 16 bytes, param_f16 8 bytes)");
    return SPX_OK;
}

static spx::AdamArgs adam_args(float* param, float* m, float* v, uint16_t* param_f16, float lr, float beta1,
                               float beta2, float eps, int64_t step) {
    spx::AdamArgs a;
    memset(&a, 0, sizeof(a));
    a.param = param;
    a.m = m;
    a.v = v;
    a.param_f16 = param_f16;
    a.lr = lr;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.inv_bc1 = 1.0f / (float)(1.0 - pow((double)beta1, (double)step));
    a.inv_bc2 = 1.0f / (float)(1.0 - pow((double)beta2, (double)step));
    return a;
}

static spx_status encode_bwd_adam_impl(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                       int32_t d_out_dtype, float* param, float* m, float* v, uint16_t* param_f16,
                                       float lr, float beta1, float beta2, float eps, int64_t step, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream, bool prepared) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (d_out_dtype != SPX_F32 && d_out_dtype != SPX_F16) return fail(SPX_EINVAL, "d_out_dtype=%d", d_out_dtype);
    if ((st = check_adam(param, m, v, param_f16, beta1, beta2, eps, step))) return st;
    if (N > 0 && !d_out) return fail(SPX_EINVAL, "d_out is NULL");
    const int ge = d_out_dtype == SPX_F16 ? 2 : 4;
    if (d_out && !aligned(d_out, row_align(enc->n_feat, ge))) return fail(SPX_EALIGN, "d_out not row-aligned");
    spx::BinLayout lay = layout_for(enc, N);
    if (!lay.ok) return fail(SPX_EUNSUPPORTED, "configuration too large for the binned adjoint");
    if (!workspace || workspace_bytes < lay.total_bytes)
        return fail(SPX_EINVAL, "workspace of %zu bytes needed, %zu given", lay.total_bytes, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(SPX_EALIGN, "workspace not 256-byte aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::AdjointBinned;
    c.workspace = workspace;
    c.dout_f16 = d_out_dtype == SPX_F16;
    c.d_out = d_out;
    c.adam = adam_args(param, m, v, param_f16, lr, beta1, beta2, eps, step);
    c.prepared = prepared;
    return from_hip(run(enc, c), prepared ? "spx_encode_bwd_adam_prepared launch" : "spx_encode_bwd_adam launch");
}

spx_status spx_encode_bwd_adam(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                               int32_t d_out_dtype, float* param, float* m, float* v, uint16_t* param_f16,
                               float lr, float beta1, float beta2, float eps, int64_t step, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    return encode_bwd_adam_impl(enc, N, pts, d_out, d_out_dtype, param, m, v, param_f16, lr, beta1, beta2, eps, step,
                                workspace, workspace_bytes, stream, false);
}

spx_status spx_encode_bwd_adam_prepared(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                        int32_t d_out_dtype, float* param, float* m, float* v, uint16_t* param_f16,
                                        float lr, float beta1, float beta2, float eps, int64_t step, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream) {
    return encode_bwd_adam_impl(enc, N, pts, d_out, d_out_dtype, param, m, v, param_f16, lr, beta1, beta2, eps, step,
                                workspace, workspace_bytes, stream, true);
}

spx_status spx_encode_debug(const spx_encoding* enc, int64_t N, const float* pts, uint32_t* idx, float* w,
                            hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (N == 0 || (!idx && !w)) return SPX_OK;
    if ((idx && !aligned(idx, 4)) || (w && !aligned(w, 4))) return fail(SPX_EALIGN, "idx/w not 4-byte aligned");
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::Debug;
    c.F = 2;  // slots and weights do not depend on the feature count
    c.idx = idx;
    c.w = w;
    return from_hip(run(enc, c), "spx_encode_debug launch");
}

spx_status spx_composite_fwd(int64_t n_rays, int32_t n_samples, const float* raw, const float* delta, float* rgba,
                             hipStream_t stream) {
    if (n_rays < 0) return fail(SPX_EINVAL, "n_rays < 0");
    if (n_samples < 1 || n_samples > 1024) return fail(SPX_EUNSUPPORTED, "n_samples=%d outside 1..1024", n_samples);
    if (n_rays == 0) return SPX_OK;
    if (!raw || !delta || !rgba) return fail(SPX_EINVAL, "raw, delta or rgba is NULL");
    if (!aligned(raw, 16) || !aligned(delta, 4) || !aligned(rgba, 16))
        return fail(SPX_EALIGN, "raw/rgba must be 16-byte and delta 4-byte aligned");
    return from_hip(spx::composite_fwd(n_rays, n_samples, raw, delta, rgba, stream), "spx_composite_fwd launch");
}

spx_status spx_composite_bwd(int64_t n_rays, int32_t n_samples, const float* raw, const float* delta,
                             const float* d_rgba, float* d_raw, hipStream_t stream) {
    if (n_rays < 0) return fail(SPX_EINVAL, "n_rays < 0");
    if (n_samples < 1 || n_samples > 1024) return fail(SPX_EUNSUPPORTED, "n_samples=%d outside 1..1024", n_samples);
    if (n_rays == 0) return SPX_OK;
    if (!raw || !delta || !d_rgba || !d_raw) return fail(SPX_EINVAL, "raw, delta, d_rgba or d_raw is NULL");
    if (!aligned(raw, 16) || !aligned(delta, 4) || !aligned(d_rgba, 16) || !aligned(d_raw, 16))
        return fail(SPX_EALIGN, "raw/d_rgba/d_raw must be 16-byte and delta 4-byte aligned");
    return from_hip(spx::composite_bwd(n_rays, n_samples, raw, delta, d_rgba, d_raw, stream),
                    "spx_composite_bwd launch");
}

spx_status spx_cast_f32_f16(int64_t n, const float* src, uint16_t* dst, hipStream_t stream) {
    if (n < 0) return fail(SPX_EINVAL, "n < 0");
    if (n == 0) return SPX_OK;
    if (!src || !dst) return fail(SPX_EINVAL, "src or dst is NULL");
    if (!aligned(src, 4) || !aligned(dst, 2)) return fail(SPX_EALIGN, "src/dst misaligned");
    return from_hip(spx::cast_f32_f16(n, src, dst, stream), "spx_cast_f32_f16 launch");
}

spx_status spx_adam_step(int64_t n, float* param, float* grad, float* m, float* v, uint16_t* param_f16, float lr,
                         float beta1, float beta2, float eps, int64_t step, int32_t zero_grad, hipStream_t stream) {
    if (n < 0) return fail(SPX_EINVAL, "n < 0");
    if (step < 1) return fail(SPX_EINVAL, "step=%lld < 1", (long long)step);
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return fail(SPX_EINVAL, "beta1/beta2 must lie in [0,1) and eps >= 0");
    if (zero_grad != 0 && zero_grad != 1) return fail(SPX_EINVAL, "zero_grad must be 0 or 1");
    if (n == 0) return SPX_OK;
    if (!param || !grad || !m || !v) return fail(SPX_EINVAL, "param, grad, m or v is NULL");
    if (!aligned(param, 4) || !aligned(grad, 4) || !aligned(m, 4) || !aligned(v, 4) || (param_f16 && !aligned(param_f16, 2)))
        return fail(SPX_EALIGN, "Adam state misaligned");
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
    return from_hip(spx::adam_step(n, param, grad, m, v, param_f16, lr, beta1, beta2, eps, bc1, bc2, zero_grad, stream),
                    "spx_adam_step launch");
}

spx_status spx_mse_grad(int64_t n, const float* y, const float* target, float* d_y, float scale,
                        hipStream_t stream) {
    if (n < 0) return fail(SPX_EINVAL, "n < 0");
    if (n == 0) return SPX_OK;
    if (!y || !target || !d_y) return fail(SPX_EINVAL, "NULL pointer");
    if (!aligned(y, 4) || !aligned(target, 4) || !aligned(d_y, 4)) return fail(SPX_EALIGN, "misaligned");
    return from_hip(spx::mse_grad(n, y, target, d_y, scale, stream), "spx_mse_grad launch");
}

spx_status spx_field_init(const spx_encoding* enc, const void* tables, const uint16_t* W1, const uint16_t* W2,
                          const uint16_t* W3, int32_t d_out, spx_field* out) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if (!out) return fail(SPX_EINVAL, "out is NULL");
    if (enc->n_dims != 2 && enc->n_dims != 3) return fail(SPX_EUNSUPPORTED, "fields are 2- or 3-D (n_dims=%d)", enc->n_dims);
    if (enc->n_levels != 16 || enc->n_feat != 2 || enc->table_dtype != SPX_F16)
        return fail(SPX_EUNSUPPORTED, "fields use 16 levels of 2 binary16 features");
    if (enc->layout != SPX_LAYOUT_HASHED)
        return fail(SPX_EUNSUPPORTED, "fields use the hashed table layout");
    if (d_out < 1 || d_out > 16) return fail(SPX_EINVAL, "d_out=%d outside 1..16", d_out);
    if (!tables || !W1 || !W2 || !W3) return fail(SPX_EINVAL, "NULL table or weight pointer");
    if (!aligned(tables, 4) || !aligned(W1, 16) || !aligned(W2, 16) || !aligned(W3, 16))
        return fail(SPX_EALIGN, "tables must be 4-byte and weights 16-byte aligned");
    memset(out, 0, sizeof(*out));
    const spx::LevelArgs lv = level_args(enc);
    for (int l = 0; l < enc->n_levels; ++l) out->sigma[l] = lv.sigma[l];
    out->Fn = lv.Fn;
    out->mask = lv.mask;
    out->n_dims = enc->n_dims;
    out->n_levels = enc->n_levels;
    out->cell = enc->cell;
    out->d_out = d_out;
    out->tables = tables;
    out->W1 = W1;
    out->W2 = W2;
    out->W3 = W3;
    return SPX_OK;
}

spx_status spx_encode_mlp_fwd(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const float* pts,
                              const void* tables, const uint16_t* W1, const uint16_t* W2, const uint16_t* W3,
                              uint16_t* feats, float* out, hipStream_t stream) {
    if (!mlp) return fail(SPX_EINVAL, "mlp descriptor is NULL");
    if (mlp->d_in != 32 || mlp->hidden != 64) return fail(SPX_EUNSUPPORTED, "the fused forward is built for 32-64-64-d_out");
    spx_field f;
    spx_status st = spx_field_init(enc, tables, W1, W2, W3, mlp->d_out, &f);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if (N == 0) return SPX_OK;
    if (!out) return fail(SPX_EINVAL, "out is NULL");
    if (!aligned(out, 4) || (feats && !aligned(feats, 16))) return fail(SPX_EALIGN, "out 4-byte, feats 16-byte aligned");
    // Where the level-major forward applies (each group of levels fits an
    // XCD's L2, all levels together do not), it and the network forward as
    // two kernels beat the fused kernel, which gathers from every level at
    // once: the features make one round trip through memory, which needs
    // the caller's feature buffer.  The same bits either way.
    if (feats && spx::fwd_level_groups(level_args(enc), enc->n_dims, 4, N).n > 0) {
        if ((st = spx_encode_fwd(enc, N, pts, tables, feats, SPX_F16, stream))) return st;
        return spx_mlp_fwd(mlp, N, feats, W1, W2, W3, out, stream);
    }
    return from_hip(spx::encode_mlp_fwd(f, N, pts, out, feats, stream), "spx_encode_mlp_fwd launch");
}

spx_status spx_field_query_batched(const spx_field* fields, int32_t nfields, const spx_segment* segs, int32_t nseg,
                                   int64_t total_tiles, hipStream_t stream) {
    if (nfields < 0 || nseg < 0 || total_tiles < 0) return fail(SPX_EINVAL, "negative count");
    if (nseg == 0 || total_tiles == 0) return SPX_OK;
    if (!fields || !segs) return fail(SPX_EINVAL, "fields or segs is NULL");
    if (!aligned(fields, 8) || !aligned(segs, 8)) return fail(SPX_EALIGN, "fields/segs not 8-byte aligned");
    return from_hip(spx::field_query(fields, nfields, segs, nseg, total_tiles, stream), "spx_field_query_batched launch");
}

static spx_status check_mlp(const spx_mlp* mlp, int64_t N) {
    if (!mlp) return fail(SPX_EINVAL, "mlp descriptor is NULL");
    if (N < 0) return fail(SPX_EINVAL, "N < 0");
    if (mlp->hidden != 64) return fail(SPX_EUNSUPPORTED, "hidden=%d (built: 64)", mlp->hidden);
    if (mlp->d_in != 32) return fail(SPX_EUNSUPPORTED, "d_in=%d (built: 32)", mlp->d_in);
    if (mlp->d_out < 1 || mlp->d_out > 16) return fail(SPX_EINVAL, "d_out=%d outside 1..16", mlp->d_out);
    return SPX_OK;
}

spx_status spx_mlp_fwd(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1, const uint16_t* W2,
                       const uint16_t* W3, float* y, hipStream_t stream) {
    spx_status st = check_mlp(mlp, N);
    if (st) return st;
    if (N == 0) return SPX_OK;
    if (!x || !W1 || !W2 || !W3 || !y) return fail(SPX_EINVAL, "NULL pointer");
    if (!aligned(x, 16) || !aligned(W1, 16) || !aligned(W2, 16) || !aligned(W3, 16) || !aligned(y, 4))
        return fail(SPX_EALIGN, "x/W must be 16-byte and y 4-byte aligned");
    spx::MlpCall c;
    memset(&c, 0, sizeof(c));
    c.d_in = mlp->d_in;
    c.hidden = mlp->hidden;
    c.d_out = mlp->d_out;
    c.N = N;
    c.x = x;
    c.W1 = W1;
    c.W2 = W2;
    c.W3 = W3;
    c.y = y;
    c.stream = stream;
    return from_hip(spx::mlp_fwd(c), "spx_mlp_fwd launch");
}

spx_status spx_mlp_bwd_workspace(const spx_mlp* mlp, int64_t N, size_t* bytes) {
    spx_status st = check_mlp(mlp, N);
    if (st) return st;
    if (!bytes) return fail(SPX_EINVAL, "bytes is NULL");
    *bytes = spx::mlp_bwd_workspace_bytes(mlp->d_in, mlp->hidden, mlp->d_out, N);
    return SPX_OK;
}

static spx_status mlp_bwd_checked(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1,
                                  const uint16_t* W2, const uint16_t* W3, const float* d_y, float* d_x, float* dW1,
                                  float* dW2, float* dW3, void* workspace, size_t workspace_bytes,
                                  hipStream_t stream, const char* fn, int dx_cols = 0, int dx_stride = 0) {
    spx_status st = check_mlp(mlp, N);
    if (st) return st;
    if (!W1 || !W2 || !W3 || !dW1 || !dW2 || !dW3) return fail(SPX_EINVAL, "NULL weight pointer");
    if (N > 0 && (!x || !d_y)) return fail(SPX_EINVAL, "x or d_y is NULL");
    const size_t need = spx::mlp_bwd_workspace_bytes(mlp->d_in, mlp->hidden, mlp->d_out, N);
    if (!workspace || workspace_bytes < need)
        return fail(SPX_EINVAL, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (!aligned(x, 16) || !aligned(W1, 16) || !aligned(W2, 16) || !aligned(W3, 16) || !aligned(d_y, 4) ||
        (d_x && !aligned(d_x, 16)) || !aligned(dW1, 4) || !aligned(dW2, 4) || !aligned(dW3, 4) ||
        !aligned(workspace, 256))
        return fail(SPX_EALIGN, "misaligned MLP backward argument");
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return from_hip(he, "hipGetDevice");
    static int lds_cache[64];  // per-device limit, looked up once (benign race: same value)
    int lds_max = dev < 64 ? lds_cache[dev] : 0;
    if (lds_max == 0) {
        he = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (he != hipSuccess) return from_hip(he, "hipDeviceGetAttribute");
        if (dev < 64) lds_cache[dev] = lds_max;
    }
    if (spx::mlp_bwd_lds_bytes(mlp->d_in) > lds_max)
        return fail(SPX_EUNSUPPORTED, "MLP backward needs %d bytes of LDS, device allows %d",
                    spx::mlp_bwd_lds_bytes(mlp->d_in), lds_max);
    spx::MlpCall c;
    memset(&c, 0, sizeof(c));
    c.d_in = mlp->d_in;
    c.hidden = mlp->hidden;
    c.d_out = mlp->d_out;
    c.N = N;
    c.x = x;
    c.W1 = W1;
    c.W2 = W2;
    c.W3 = W3;
    c.d_y = d_y;
    c.d_x = d_x;
    c.dx_cols = dx_cols;
    c.dx_stride = dx_stride;
    c.dW1 = dW1;
    c.dW2 = dW2;
    c.dW3 = dW3;
    c.workspace = workspace;
    c.stream = stream;
    return from_hip(spx::mlp_bwd(c), fn);
}

spx_status spx_mlp_bwd(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1, const uint16_t* W2,
                       const uint16_t* W3, const float* d_y, float* d_x, float* dW1, float* dW2, float* dW3,
                       void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return mlp_bwd_checked(mlp, N, x, W1, W2, W3, d_y, d_x, dW1, dW2, dW3, workspace, workspace_bytes, stream,
                           "spx_mlp_bwd launch");
}

spx_status spx_mlp_bwd_noalloc(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1,
                               const uint16_t* W2, const uint16_t* W3, const float* d_y, float* d_x, float* dW1,
                               float* dW2, float* dW3, hipStream_t stream) {
    spx_status st = check_mlp(mlp, N);
    if (st) return st;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    hipError_t he = spx::mlp_bwd_scratch(&scratch, &scratch_bytes);
    if (he != hipSuccess) return from_hip(he, "scratch lookup (hipGetSymbolAddress)");
    const size_t need = spx::mlp_bwd_workspace_bytes(mlp->d_in, mlp->hidden, mlp->d_out, N);
    if (need > scratch_bytes)
        return fail(SPX_EUNSUPPORTED, "N=%lld needs %zu bytes of scratch, the library holds %zu", (long long)N, need,
                    scratch_bytes);
    return mlp_bwd_checked(mlp, N, x, W1, W2, W3, d_y, d_x, dW1, dW2, dW3, scratch, scratch_bytes, stream,
                           "spx_mlp_bwd_noalloc launch");
}

// Workspace of the fused network backward and adjoint: the binned
// adjoint's, then the network backward's weight-gradient partials, then the
// privatised coarse levels' units of the input gradient (rows of
// coarse_stride floats).
struct NetWorkspace {
    size_t mlp, coarse, total;
    int coarse_cols, coarse_stride;
};

static NetWorkspace net_workspace(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const spx::BinLayout& lay) {
    NetWorkspace w;
    w.coarse_cols = lay.P * enc->n_feat;
    w.coarse_stride = (w.coarse_cols + 3) & ~3;
    w.mlp = spx::bin_align(lay.total_bytes);
    w.coarse = w.mlp + spx::bin_align(spx::mlp_bwd_workspace_bytes(mlp->d_in, mlp->hidden, mlp->d_out, N));
    w.total = w.coarse + spx::bin_align((size_t)N * w.coarse_stride * sizeof(float));
    return w;
}

// What the fused path covers, before any launch: the network's input is the
// encoding (d_in = L * F), 2 features per level, 1 to 3 dimensions, and the
// adjoint's staged scatter fits one level group and the CU's LDS.
static spx_status net_covers(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const spx::BinLayout& lay) {
    if (mlp->d_in != enc->n_levels * enc->n_feat)
        return fail(SPX_EINVAL, "d_in=%d is not n_levels * n_feat = %d", mlp->d_in, enc->n_levels * enc->n_feat);
    if (enc->n_feat != 2 || enc->n_dims > 3)
        return fail(SPX_EUNSUPPORTED, "the fused network backward covers n_feat = 2 and n_dims <= 3");
    if (!lay.ok) return fail(SPX_EUNSUPPORTED, "configuration too large for the binned adjoint");
    spx::EncodeCall c = base_call(enc, N, nullptr, nullptr);
    c.op = spx::EncodeOp::AdjointBinned;
    c.net.check_only = 1;
    const hipError_t he = run(enc, c);
    if (he == hipErrorNotSupported)
        return fail(SPX_EUNSUPPORTED, "the fused network backward needs one level group and a staged scatter "
                                      "whose LDS (with the network's weights) fits the CU");
    return from_hip(he, "fused network backward check");
}

spx_status spx_encode_mlp_bwd_workspace(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, size_t* bytes) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_mlp(mlp, N))) return st;
    if (!bytes) return fail(SPX_EINVAL, "bytes is NULL");
    const spx::BinLayout lay = layout_for(enc, N);
    if ((st = net_covers(enc, mlp, N, lay))) return st;
    *bytes = net_workspace(enc, mlp, N, lay).total;
    return SPX_OK;
}

spx_status spx_encode_mlp_bwd_adam(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const float* pts,
                                   const uint16_t* x, const uint16_t* W1, const uint16_t* W2, const uint16_t* W3,
                                   const float* d_y, float* dW1, float* dW2, float* dW3, float* param, float* m,
                                   float* v, uint16_t* param_f16, float lr, float beta1, float beta2, float eps,
                                   int64_t step, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    spx_status st = check_encoding(enc);
    if (st) return st;
    if ((st = check_points(N, pts))) return st;
    if ((st = check_mlp(mlp, N))) return st;
    if ((st = check_adam(param, m, v, param_f16, beta1, beta2, eps, step))) return st;
    const spx::BinLayout lay = layout_for(enc, N);
    if ((st = net_covers(enc, mlp, N, lay))) return st;
    const NetWorkspace w = net_workspace(enc, mlp, N, lay);
    if (!workspace || workspace_bytes < w.total)
        return fail(SPX_EINVAL, "workspace of %zu bytes needed, %zu given", w.total, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(SPX_EALIGN, "workspace not 256-byte aligned");
    char* ws = (char*)workspace;
    float* coarse = (float*)(ws + w.coarse);
    // the network backward: weight gradients, and the input gradient's units
    // of the privatised coarse levels (the scatter computes the rest itself)
    st = mlp_bwd_checked(mlp, N, x, W1, W2, W3, d_y, w.coarse_cols > 0 ? coarse : nullptr, dW1, dW2, dW3,
                         ws + w.mlp, w.coarse - w.mlp, stream, "spx_encode_mlp_bwd_adam network backward",
                         w.coarse_cols, w.coarse_stride);
    if (st) return st;
    spx::EncodeCall c = base_call(enc, N, pts, stream);
    c.op = spx::EncodeOp::AdjointBinned;
    c.workspace = workspace;
    c.d_out = coarse;
    c.net.x = reinterpret_cast<const _Float16*>(x);
    c.net.W1 = reinterpret_cast<const _Float16*>(W1);
    c.net.W2 = reinterpret_cast<const _Float16*>(W2);
    c.net.W3 = reinterpret_cast<const _Float16*>(W3);
    c.net.d_y = d_y;
    c.net.d_out = mlp->d_out;
    c.net.coarse_stride = w.coarse_stride;
    c.adam = adam_args(param, m, v, param_f16, lr, beta1, beta2, eps, step);
    return from_hip(run(enc, c), "spx_encode_mlp_bwd_adam launch");
}

}  // extern "C"
