/*
 * CPU oracle for the multiresolution simplex hash encoding
 * (Wen & Yang, "Efficient Encoding of Graphics Primitives with
 * Simplex-based Structures", arXiv 2311.15439).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain statement of what
 * the GPU path must compute.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * constant table or helper with the HIP library: every constant below is
 * derived here from its definition.
 *
 * Precision policy
 *   - Where floating point decides an integer (which lattice cell, which of
 *     the n! simplices, which hash slot) the decision is taken in IEEE
 *     binary32, in a fixed operation order, with no contraction (build with
 *     -ffp-contract=off).  This is the kernel's precision; the paper fixes
 *     none.
 *   - Everything else (barycentric weights, interpolation, adjoint sums,
 *     the MLP) is evaluated in binary64 from the exact binary32 inputs.
 *   - A binary32 mirror of the weights (the same subtractions in float) is
 *     also produced so that the GPU's weights can be compared bit for bit.
 *
 * Parity pins (what fixes each function independently of this file) live in
 * tests/test_oracle_pins.py.  MLP and Adam rows: pinned against numpy and
 * closed-form special cases; nothing here is "parity unpinned".
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DIM 6
#define ORC_MAX_LEVELS 32
#define ORC_SIMPLEX 0
#define ORC_GRID 1
#define ORC_F32 0
#define ORC_F16 1
#define ORC_LAYOUT_HASHED 0
#define ORC_LAYOUT_SIZED 1

/* ------------------------------------------------------------------------ */
/* Constants.                                                               */
/* ------------------------------------------------------------------------ */

/* Skew factor of Eq. 2 (Sec. 3.2(a)): F_n = (sqrt(n+1) - 1) / n. */
double orc_skew_factor(int n) { return (sqrt((double)n + 1.0) - 1.0) / (double)n; }

/* Unskew factor of Eq. 3 (Sec. 3.2(d)): G_n = (1 - 1/sqrt(n+1)) / n. */
double orc_unskew_factor(int n) { return (1.0 - 1.0 / sqrt((double)n + 1.0)) / (double)n; }

/* Adjustment scale of Sec. 5.1: S_n = sqrt(n+1), the image of the unit
 * cube's far corner along each axis after the skew. */
double orc_adjust_scale(int n) { return sqrt((double)n + 1.0); }

/* Equal-memory level multiplier of Sec. 5.2: (n+1)^((n-1)/(2n)).  The paper
 * scales each level by it when it compares against the grid at a fixed table
 * size. */
double orc_equal_memory_factor(int n) {
    return pow((double)n + 1.0, (double)(n - 1) / (2.0 * (double)n));
}

/* Geometric level schedule N_l = floor(N_min * b^l + 1e-6).  Sec. 5.1 only
 * states that each level divides the cube at its own resolution; the
 * geometric progression and the 1e-6 guard (so that the top level of a
 * schedule given by its two ends lands on the integer end) are a reading. */
void orc_level_resolutions(double n_min, double growth, int L, int32_t* res_out) {
    for (int l = 0; l < L; ++l) res_out[l] = (int32_t)floor(n_min * pow(growth, (double)l) + 1e-6);
}

/* Per-level multiplier applied to the skewed coordinate (Sec. 5.1): the
 * skewed unit cube spans [0, S_n]^n, so dividing by S_n brings it back to
 * [0,1]^n before the level resolution N_l (times the optional equal-memory
 * factor) is applied.  Rounded to binary32 once.  The grid baseline uses N_l
 * directly (no skew). */
void orc_level_scales(int n, int L, const int32_t* res, int cell, int equal_memory, float* sigma_out) {
    double cn = equal_memory ? orc_equal_memory_factor(n) : 1.0;
    for (int l = 0; l < L; ++l) {
        if (cell == ORC_GRID)
            sigma_out[l] = (float)((double)res[l] * cn);
        else
            sigma_out[l] = (float)(((double)res[l] * cn) / orc_adjust_scale(n));
    }
}

/* ------------------------------------------------------------------------ */
/* Spatial hash.  The paper defers to the multiresolution hash encoding it   */
/* builds on and prints no function.  Reading: h(v) = XOR_i (u32(v_i)*P_i)  */
/* mod 2^32, masked to the table size, with P_0 = 1, P_1 = 2654435761, and  */
/* P_2..P_5 the smallest primes not below floor(2^32 * frac(sqrt(q))) for   */
/* q = 2, 3, 5, 7.  The primes are derived here at run time.                */
/* ------------------------------------------------------------------------ */

static uint64_t isqrt_u128(unsigned __int128 a) {
    /* floor(sqrt(a)) by bisection on 64-bit candidates. */
    uint64_t lo = 0, hi = UINT64_MAX;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2 + 1;
        unsigned __int128 sq = (unsigned __int128)mid * mid;
        if (sq <= a) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static int is_prime_u64(uint64_t v) {
    if (v < 2) return 0;
    if (v % 2 == 0) return v == 2;
    for (uint64_t d = 3; d * d <= v; d += 2)
        if (v % d == 0) return 0;
    return 1;
}

void orc_hash_primes(uint32_t* P /* [ORC_MAX_DIM] */) {
    static const uint32_t q[4] = {2, 3, 5, 7};
    P[0] = 1u;
    P[1] = 2654435761u;
    for (int k = 0; k < 4; ++k) {
        /* floor(sqrt(q) * 2^32) = isqrt(q * 2^64); drop the integer part. */
        unsigned __int128 a = (unsigned __int128)q[k] << 64;
        uint64_t r = isqrt_u128(a);
        uint64_t frac = r - ((uint64_t)isqrt_u128((unsigned __int128)q[k]) << 32);
        while (!is_prime_u64(frac)) ++frac;
        P[2 + k] = (uint32_t)frac;
    }
}

/* The multipliers are derived once when the library is loaded. */
static uint32_t g_primes[ORC_MAX_DIM];
__attribute__((constructor)) static void init_primes(void) { orc_hash_primes(g_primes); }

uint32_t orc_hash(const int32_t* v, int n, int log2_T) {
    uint32_t h = 0;
    for (int i = 0; i < n; ++i) h ^= (uint32_t)v[i] * g_primes[i];
    return h & ((1u << log2_T) - 1u);
}

/* ------------------------------------------------------------------------ */
/* binary16 <-> binary64, written from the IEEE 754 binary16 format          */
/* (1 sign bit, 5 exponent bits with bias 15, 10 fraction bits).             */
/* ------------------------------------------------------------------------ */

double orc_f16_to_f64(uint16_t h) {
    int s = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m + 1024), e - 25);
    return s ? -v : v;
}

/* Round to nearest, ties to even. */
uint16_t orc_f64_to_f16(double x) {
    uint16_t sign = (signbit(x) ? 0x8000u : 0u);
    double a = fabs(x);
    if (isnan(x)) return 0x7e00u;
    if (a >= 65520.0) return sign | 0x7c00u; /* beyond the last rounding boundary */
    if (a < ldexp(1.0, -14)) {
        double q = nearbyint(a * ldexp(1.0, 24)); /* subnormal: units of 2^-24 */
        return sign | (uint16_t)q;               /* q == 1024 is the smallest normal */
    }
    int E;
    frexp(a, &E);               /* a = m * 2^E, m in [0.5, 1) */
    int e = E - 1;              /* a in [2^e, 2^(e+1)) */
    double q = nearbyint(ldexp(a, 10 - e)); /* 11-bit significand in [1024, 2048] */
    if (q == 2048.0) { q = 1024.0; e += 1; }
    if (e > 15) return sign | 0x7c00u;
    return sign | (uint16_t)(((e + 15) << 10) | ((int)q - 1024));
}

/* bfloat16: 8 exponent bits, 7 fraction bits; round to nearest even. */
double orc_round_bf16(double x) {
    if (x == 0.0 || isnan(x) || isinf(x)) return x;
    int E;
    frexp(fabs(x), &E);
    int e = E - 1;
    if (e < -126) e = -126; /* subnormal range keeps a fixed quantum */
    double q = nearbyint(ldexp(x, 7 - e));
    return ldexp(q, e - 7);
}

static double table_value(const void* tables, int dtype, size_t idx) {
    if (dtype == ORC_F16) return orc_f16_to_f64(((const uint16_t*)tables)[idx]);
    return (double)((const float*)tables)[idx];
}

/* ------------------------------------------------------------------------ */
/* One level's lookup for one point.                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n_dims, n_levels, log2_T, n_feat, table_dtype, cell;
    int32_t res[ORC_MAX_LEVELS];
    int equal_memory;
    int layout; /* ORC_LAYOUT_HASHED or ORC_LAYOUT_SIZED */
} orc_encoding;

/* Skewed coordinate of Eq. 2 in binary32: the coordinate sum is formed left
 * to right, multiplied by F_n, and added to each coordinate. */
static void skew_point_f32(int n, const float* x, float* y) {
    float Fn = (float)orc_skew_factor(n);
    float s = x[0];
    for (int i = 1; i < n; ++i) s = s + x[i];
    float t = s * Fn;
    for (int i = 0; i < n; ++i) y[i] = x[i] + t;
}

/* ------------------------------------------------------------------------ */
/* Table layout per level (Sec. 5.2, Hash Table Selection).                  */
/*   HASHED: every level has T = 2^log2_T rows and every vertex is hashed    */
/*     (the paper's configurations).                                         */
/*   SIZED: the lattice box a level reaches from the closed unit cube has    */
/*     B = e^n vertices.  If B <= T the level is stored densely: B rows, the  */
/*     vertex v at row sum_i v_i e^i, a bijection on the box (no collisions;  */
/*     coordinates outside it are clamped to its faces).  Otherwise it is    */
/*     hashed into the smallest power of two of rows that holds the share of */
/*     the box a simplex level actually uses, (n+1)^(-(n-1)/2) (the          */
/*     volume ratio Sec. 5.2 derives; the whole box for the grid), at most T. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t off[ORC_MAX_LEVELS + 1]; /* first row of each level; off[L] = all rows */
    int64_t rows[ORC_MAX_LEVELS];
    int32_t extent[ORC_MAX_LEVELS];
    int dense[ORC_MAX_LEVELS];
} orc_layout;

/* Box extent per axis at one level: the far corner (1, ..., 1) of the unit
 * cube through the binary32 index path gives the largest scaled coordinate
 * p any point of the closed cube reaches (each step is monotone), so vertex
 * coordinates lie in [0, floor(p) + 1]. */
static int32_t box_extent(const orc_encoding* e, float sigma) {
    float one[ORC_MAX_DIM], y[ORC_MAX_DIM];
    for (int i = 0; i < e->n_dims; ++i) one[i] = 1.0f;
    if (e->cell == ORC_GRID) {
        for (int i = 0; i < e->n_dims; ++i) y[i] = one[i];
    } else {
        skew_point_f32(e->n_dims, one, y);
    }
    const float p = y[0] * sigma;
    return (int32_t)floorf(p) + 2;
}

static void make_layout(const orc_encoding* e, orc_layout* lay) {
    const int n = e->n_dims;
    const int64_t T = (int64_t)1 << e->log2_T;
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, e->n_levels, e->res, e->cell, e->equal_memory, sigma);
    lay->off[0] = 0;
    for (int l = 0; l < e->n_levels; ++l) {
        const int32_t ext = box_extent(e, sigma[l]);
        /* B = ext^n, saturated well above any table size */
        int64_t B = 1;
        for (int i = 0; i < n && B <= ((int64_t)1 << 40); ++i) B *= ext;
        int64_t rows = T;
        int dense = 0;
        if (e->layout == ORC_LAYOUT_SIZED) {
            if (B <= T) {
                rows = B;
                dense = 1;
            } else if (B <= ((int64_t)1 << 40)) {
                /* smallest power of two P with P >= u B, u = (n+1)^(-(n-1)/2):
                 * for the simplex P^2 (n+1)^(n-1) >= B^2, in integers */
                unsigned __int128 rhs = (unsigned __int128)B * (unsigned __int128)B;
                unsigned __int128 k = 1;
                if (e->cell != ORC_GRID)
                    for (int i = 0; i < n - 1; ++i) k *= (unsigned __int128)(n + 1);
                int64_t P = 1;
                while (P < T && (e->cell == ORC_GRID ? (P < B)
                                                      : ((unsigned __int128)P * (unsigned __int128)P * k < rhs)))
                    P <<= 1;
                rows = P;
            }
        }
        lay->extent[l] = ext;
        lay->dense[l] = dense;
        lay->rows[l] = rows;
        lay->off[l + 1] = lay->off[l] + rows;
    }
}

/* Host query: rows, box extent and dense flag of every level. */
void orc_table_layout(const orc_encoding* e, int64_t* rows, int32_t* extent, int32_t* dense) {
    orc_layout lay;
    make_layout(e, &lay);
    for (int l = 0; l < e->n_levels; ++l) {
        rows[l] = lay.rows[l];
        extent[l] = lay.extent[l];
        dense[l] = lay.dense[l];
    }
}

/* Row of vertex v within level l's table. */
static uint32_t level_slot(const orc_encoding* e, const orc_layout* lay, int l, const int32_t* v) {
    if (lay->dense[l]) {
        const int64_t ext = lay->extent[l];
        int64_t idx = 0, stride = 1;
        for (int i = 0; i < e->n_dims; ++i) {
            int64_t c = v[i];
            if (c < 0) c = 0;
            if (c > ext - 1) c = ext - 1;
            idx += c * stride;
            stride *= ext;
        }
        return (uint32_t)idx;
    }
    uint32_t h = 0;
    for (int i = 0; i < e->n_dims; ++i) h ^= (uint32_t)v[i] * g_primes[i];
    return h & (uint32_t)(lay->rows[l] - 1);
}

/* Host query: row of vertex v within level l's table. */
uint32_t orc_vertex_slot(const orc_encoding* e, int l, const int32_t* v) {
    orc_layout lay;
    make_layout(e, &lay);
    return level_slot(e, &lay, l, v);
}

/*
 * Simplex lookup at one level (Secs. 4.2, 4.3 and 5.1).
 *   p = sigma * y (binary32), cell corner c = floor(p), fractional part
 *   f = p - c.  The fractional parts are ordered largest first by a stable
 *   bubble sort (equal values keep axis order), which names the simplex of
 *   the Kuhn subdivision containing p (Remark 2).  The walk starts at c and
 *   adds one along the axis of each next-largest fraction, giving the n+1
 *   vertices; the barycentric weights are 1 - f(1), f(1) - f(2), ...,
 *   f(n-1) - f(n), f(n) over the sorted fractions (Sec. 4.3).
 */
static int simplex_lookup(int n, const float* y, float sigma, int32_t verts[][ORC_MAX_DIM],
                          double* w64, float* w32, float* p_out) {
    float p[ORC_MAX_DIM], f[ORC_MAX_DIM];
    int32_t c[ORC_MAX_DIM];
    int axis[ORC_MAX_DIM];
    for (int i = 0; i < n; ++i) {
        p[i] = y[i] * sigma;
        c[i] = (int32_t)floorf(p[i]);
        f[i] = p[i] - (float)c[i];
        axis[i] = i;
        if (p_out) p_out[i] = p[i];
    }
    /* bubble sort, descending, strict comparison => stable */
    for (int pass = 0; pass < n - 1; ++pass)
        for (int j = 0; j < n - 1 - pass; ++j)
            if (f[axis[j]] < f[axis[j + 1]]) {
                int t = axis[j]; axis[j] = axis[j + 1]; axis[j + 1] = t;
            }
    for (int i = 0; i < n; ++i) verts[0][i] = c[i];
    for (int k = 1; k <= n; ++k) {
        for (int i = 0; i < n; ++i) verts[k][i] = verts[k - 1][i];
        verts[k][axis[k - 1]] += 1;
    }
    /* weights over the sorted fractions */
    w64[0] = 1.0 - (double)f[axis[0]];
    w32[0] = 1.0f - f[axis[0]];
    for (int k = 1; k < n; ++k) {
        w64[k] = (double)f[axis[k - 1]] - (double)f[axis[k]];
        w32[k] = f[axis[k - 1]] - f[axis[k]];
    }
    w64[n] = (double)f[axis[n - 1]];
    w32[n] = f[axis[n - 1]];
    return n + 1;
}

/*
 * 2^n-corner grid lookup (the baseline of Sec. 3.1 / Alg. 1): p = N_l * x,
 * corners c + b for b in {0,1}^n enumerated in binary order (bit i is axis
 * i), n-linear weights prod_i (b_i ? f_i : 1 - f_i).
 */
static int grid_lookup(int n, const float* x, float sigma, int32_t verts[][ORC_MAX_DIM],
                       double* w64, float* w32, float* p_out) {
    float p[ORC_MAX_DIM], f[ORC_MAX_DIM];
    int32_t c[ORC_MAX_DIM];
    for (int i = 0; i < n; ++i) {
        p[i] = x[i] * sigma;
        c[i] = (int32_t)floorf(p[i]);
        f[i] = p[i] - (float)c[i];
        if (p_out) p_out[i] = p[i];
    }
    int V = 1 << n;
    for (int b = 0; b < V; ++b) {
        double w = 1.0;
        float wf = 1.0f;
        for (int i = 0; i < n; ++i) {
            int bit = (b >> i) & 1;
            verts[b][i] = c[i] + bit;
            w *= bit ? (double)f[i] : 1.0 - (double)f[i];
            wf *= bit ? f[i] : 1.0f - f[i];
        }
        w64[b] = w;
        w32[b] = wf;
    }
    return V;
}

static int lookup(const orc_encoding* e, const float* x, const float* y, float sigma,
                  int32_t verts[][ORC_MAX_DIM], double* w64, float* w32, float* p_out) {
    if (e->cell == ORC_GRID) return grid_lookup(e->n_dims, x, sigma, verts, w64, w32, p_out);
    return simplex_lookup(e->n_dims, y, sigma, verts, w64, w32, p_out);
}

static int n_vertices(const orc_encoding* e) {
    return e->cell == ORC_GRID ? (1 << e->n_dims) : e->n_dims + 1;
}

/* ------------------------------------------------------------------------ */
/* Public entry points.                                                     */
/* ------------------------------------------------------------------------ */

/*
 * Debug view of the lookup: for each point and level, the n+1 (or 2^n)
 * vertex coordinates, their hash slots, the binary64 and binary32 weights,
 * and the scaled point p.  Any output pointer may be NULL.
 * Shapes: verts [N,L,V,n] int32; idx [N,L,V] uint32; w64 [N,L,V];
 * w32 [N,L,V]; p [N,L,n] float.
 */
void orc_encode_debug(const orc_encoding* e, int64_t N, const float* pts, int32_t* verts_out,
                      uint32_t* idx_out, double* w64_out, float* w32_out, float* p_out) {
    int n = e->n_dims, L = e->n_levels, V = n_vertices(e);
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, L, e->res, e->cell, e->equal_memory, sigma);
    orc_layout lay;
    make_layout(e, &lay);
#pragma omp parallel for schedule(static)
    for (int64_t pt = 0; pt < N; ++pt) {
        const float* x = pts + pt * n;
        float y[ORC_MAX_DIM];
        skew_point_f32(n, x, y);
        for (int l = 0; l < L; ++l) {
            int32_t verts[1 << ORC_MAX_DIM][ORC_MAX_DIM];
            double w64[1 << ORC_MAX_DIM];
            float w32[1 << ORC_MAX_DIM], p[ORC_MAX_DIM];
            lookup(e, x, y, sigma[l], verts, w64, w32, p);
            size_t base = ((size_t)pt * L + l) * V;
            for (int k = 0; k < V; ++k) {
                if (verts_out)
                    for (int i = 0; i < n; ++i) verts_out[(base + k) * n + i] = verts[k][i];
                if (idx_out) idx_out[base + k] = level_slot(e, &lay, l, verts[k]);
                if (w64_out) w64_out[base + k] = w64[k];
                if (w32_out) w32_out[base + k] = w32[k];
            }
            if (p_out)
                for (int i = 0; i < n; ++i) p_out[((size_t)pt * L + l) * n + i] = p[i];
        }
    }
}

/*
 * Forward encoding (Sec. 5 steps (a)-(d)): for every level, hash the
 * vertices, look up their feature vectors in that level's table, take the
 * barycentric-weighted sum, and concatenate the levels.
 * tables: [rows of all levels, F] (level l from its layout offset; [L, 2^log2_T, F]
 * for the hashed layout) in binary32 or binary16; out: [N, L*F] binary64.
 */
void orc_encode_fwd(const orc_encoding* e, int64_t N, const float* pts, const void* tables, double* out) {
    int n = e->n_dims, L = e->n_levels, F = e->n_feat, V = n_vertices(e);
    orc_layout lay;
    make_layout(e, &lay);
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, L, e->res, e->cell, e->equal_memory, sigma);
#pragma omp parallel for schedule(static)
    for (int64_t pt = 0; pt < N; ++pt) {
        const float* x = pts + pt * n;
        float y[ORC_MAX_DIM];
        skew_point_f32(n, x, y);
        for (int l = 0; l < L; ++l) {
            int32_t verts[1 << ORC_MAX_DIM][ORC_MAX_DIM];
            double w64[1 << ORC_MAX_DIM];
            float w32[1 << ORC_MAX_DIM];
            lookup(e, x, y, sigma[l], verts, w64, w32, NULL);
            for (int j = 0; j < F; ++j) {
                double acc = 0.0;
                for (int k = 0; k < V; ++k) {
                    const size_t row = (size_t)lay.off[l] + level_slot(e, &lay, l, verts[k]);
                    acc += w64[k] * table_value(tables, e->table_dtype, row * F + j);
                }
                out[(size_t)pt * L * F + (size_t)l * F + j] = acc;
            }
        }
    }
}

/*
 * Magnitude companion of the forward pass: sum_k |w_k * t_k| per output.
 * Used to state the forward error relative to the size of the terms.
 */
void orc_encode_fwd_absmag(const orc_encoding* e, int64_t N, const float* pts, const void* tables,
                           double* out) {
    int n = e->n_dims, L = e->n_levels, F = e->n_feat, V = n_vertices(e);
    orc_layout lay;
    make_layout(e, &lay);
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, L, e->res, e->cell, e->equal_memory, sigma);
#pragma omp parallel for schedule(static)
    for (int64_t pt = 0; pt < N; ++pt) {
        const float* x = pts + pt * n;
        float y[ORC_MAX_DIM];
        skew_point_f32(n, x, y);
        for (int l = 0; l < L; ++l) {
            int32_t verts[1 << ORC_MAX_DIM][ORC_MAX_DIM];
            double w64[1 << ORC_MAX_DIM];
            float w32[1 << ORC_MAX_DIM];
            lookup(e, x, y, sigma[l], verts, w64, w32, NULL);
            for (int j = 0; j < F; ++j) {
                double acc = 0.0;
                for (int k = 0; k < V; ++k) {
                    const size_t row = (size_t)lay.off[l] + level_slot(e, &lay, l, verts[k]);
                    acc += fabs(w64[k] * table_value(tables, e->table_dtype, row * F + j));
                }
                out[(size_t)pt * L * F + (size_t)l * F + j] = acc;
            }
        }
    }
}

/*
 * Adjoint of the forward encoding (Sec. 5 step (e)): the gradient of each
 * output is accumulated into the looked-up feature vectors with the same
 * barycentric weights.  d_out: [N, L*F] binary64; d_tables: laid out as the tables
 * binary64, accumulated (+=).  Serial on purpose: the summation order is the
 * plain point order.  If absmag is non-NULL it receives sum |w * d_out| per
 * slot (same shape as d_tables, accumulated) and count the number of
 * contributions per slot.
 */
void orc_encode_bwd(const orc_encoding* e, int64_t N, const float* pts, const double* d_out,
                    double* d_tables, double* absmag, int64_t* count) {
    int n = e->n_dims, L = e->n_levels, F = e->n_feat, V = n_vertices(e);
    orc_layout lay;
    make_layout(e, &lay);
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, L, e->res, e->cell, e->equal_memory, sigma);
    for (int64_t pt = 0; pt < N; ++pt) {
        const float* x = pts + pt * n;
        float y[ORC_MAX_DIM];
        skew_point_f32(n, x, y);
        for (int l = 0; l < L; ++l) {
            int32_t verts[1 << ORC_MAX_DIM][ORC_MAX_DIM];
            double w64[1 << ORC_MAX_DIM];
            float w32[1 << ORC_MAX_DIM];
            lookup(e, x, y, sigma[l], verts, w64, w32, NULL);
            for (int k = 0; k < V; ++k) {
                const size_t row = (size_t)lay.off[l] + level_slot(e, &lay, l, verts[k]);
                for (int j = 0; j < F; ++j) {
                    size_t slot = row * F + j;
                    double g = d_out[(size_t)pt * L * F + (size_t)l * F + j];
                    d_tables[slot] += w64[k] * g;
                    if (absmag) absmag[slot] += fabs(w64[k] * g);
                    if (count) count[slot] += 1;
                }
            }
        }
    }
}

/*
 * Gradient with respect to the input point (the derivative the paper's
 * backward pass leaves out; needed when the encoded coordinates are
 * themselves optimised).  Inside a simplex the weights are affine in the
 * fractional parts: f of the k-th sorted axis enters w_k with a minus sign
 * and w_{k+1} with a plus sign (Sec. 4.3), so the output's derivative along
 * that axis is t(v_{k+1}) - t(v_k), the difference across the walk's k-th
 * step.  For the grid, d w_b / d f_i = (b_i ? 1 : -1) prod_{j != i}
 * (b_j ? f_j : 1 - f_j).  The fractional parts move with p = sigma * y, and
 * y = x + F_n (sum x) 1 (Eq. 2) for the simplex (p = sigma * x for the
 * grid), so d p_i / d x_m = sigma (delta_im + F_n) resp. sigma delta_im.
 * On a face the one-sided derivative of the simplex the tie rule picks is
 * returned.  d_out: [N, L*F] binary64; d_pts [N, n] binary64 (overwritten);
 * mag (optional) [N, n]: the same sums over absolute values of the terms
 * (a walk step's term is its row difference times d_out; a grid term is
 * c * t * d_out), chained through the skew with the same non-negative
 * factors.
 */
void orc_encode_input_grad(const orc_encoding* e, int64_t N, const float* pts, const void* tables,
                           const double* d_out, double* d_pts, double* mag) {
    int n = e->n_dims, L = e->n_levels, F = e->n_feat, V = n_vertices(e);
    orc_layout lay;
    make_layout(e, &lay);
    float sigma[ORC_MAX_LEVELS];
    orc_level_scales(n, L, e->res, e->cell, e->equal_memory, sigma);
    const double Fn = orc_skew_factor(n);
#pragma omp parallel for schedule(static)
    for (int64_t pt = 0; pt < N; ++pt) {
        const float* x = pts + pt * n;
        float y[ORC_MAX_DIM];
        skew_point_f32(n, x, y);
        double dx[ORC_MAX_DIM] = {0}, ax[ORC_MAX_DIM] = {0};
        for (int l = 0; l < L; ++l) {
            int32_t verts[1 << ORC_MAX_DIM][ORC_MAX_DIM];
            double w64[1 << ORC_MAX_DIM];
            float w32[1 << ORC_MAX_DIM], p[ORC_MAX_DIM];
            lookup(e, x, y, sigma[l], verts, w64, w32, p);
            double g[ORC_MAX_DIM] = {0}, a[ORC_MAX_DIM] = {0}; /* d L / d f_i and its magnitude */
            double t[1 << ORC_MAX_DIM][8];
            for (int k = 0; k < V; ++k) {
                const size_t row = (size_t)lay.off[l] + level_slot(e, &lay, l, verts[k]);
                for (int j = 0; j < F; ++j) t[k][j] = table_value(tables, e->table_dtype, row * F + j);
            }
            const double* d = d_out + (size_t)pt * L * F + (size_t)l * F;
            if (e->cell == ORC_GRID) {
                double f[ORC_MAX_DIM];
                for (int i = 0; i < n; ++i) f[i] = (double)p[i] - floor((double)p[i]);
                for (int b = 0; b < V; ++b)
                    for (int i = 0; i < n; ++i) {
                        double c = ((b >> i) & 1) ? 1.0 : -1.0;
                        for (int m = 0; m < n; ++m)
                            if (m != i) c *= ((b >> m) & 1) ? f[m] : 1.0 - f[m];
                        for (int j = 0; j < F; ++j) {
                            g[i] += c * t[b][j] * d[j];
                            a[i] += fabs(c * t[b][j] * d[j]);
                        }
                    }
            } else {
                for (int k = 0; k < n; ++k) {
                    int axis = 0; /* the axis stepped from vertex k to vertex k+1 */
                    for (int i = 0; i < n; ++i)
                        if (verts[k + 1][i] != verts[k][i]) axis = i;
                    for (int j = 0; j < F; ++j) {
                        g[axis] += (t[k + 1][j] - t[k][j]) * d[j];
                        a[axis] += fabs((t[k + 1][j] - t[k][j]) * d[j]);
                    }
                }
            }
            double gs = 0.0, as = 0.0;
            for (int i = 0; i < n; ++i) { gs += g[i]; as += a[i]; }
            for (int m = 0; m < n; ++m) {
                if (e->cell == ORC_GRID) {
                    dx[m] += (double)sigma[l] * g[m];
                    ax[m] += (double)sigma[l] * a[m];
                } else {
                    dx[m] += (double)sigma[l] * (g[m] + Fn * gs);
                    ax[m] += (double)sigma[l] * (a[m] + Fn * as);
                }
            }
        }
        for (int m = 0; m < n; ++m) {
            d_pts[pt * n + m] = dx[m];
            if (mag) mag[pt * n + m] = ax[m];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Tiny fully connected network (Sec. 5 step (e); about 7k parameters):     */
/* in -> H -> H -> out with ReLU on the hidden layers and a linear output.  */
/* Weights are binary16, row-major W[out][in].  The input and each hidden   */
/* activation are rounded to binary16 where the kernel stores them in that  */
/* format; every product and sum is binary64.                               */
/* ------------------------------------------------------------------------ */

static double f16r(double v) { return orc_f16_to_f64(orc_f64_to_f16(v)); }

/* out [N, d_out] binary64.  If absmag != NULL it receives the forward
 * pass's magnitude with the ReLU pattern applied: per layer the sum of
 * |w| times the previous layer's magnitude over the units that are active
 * (positive pre-activation), starting from |x|.  It bounds the size of
 * every partial sum on a path to the output through active units, which
 * is where a rounding of a stored activation can travel; with
 * non-negative weights and inputs it equals the output itself. */
void orc_mlp_fwd(int64_t N, int d_in, int H, int d_out, const uint16_t* x, const uint16_t* W1,
                 const uint16_t* W2, const uint16_t* W3, double* out, double* absmag) {
#pragma omp parallel for schedule(static)
    for (int64_t pt = 0; pt < N; ++pt) {
        double xin[256], h1[256], h2[256], a1[256], a2[256];
        for (int i = 0; i < d_in; ++i) xin[i] = orc_f16_to_f64(x[pt * d_in + i]);
        for (int o = 0; o < H; ++o) {
            double s = 0.0, sa = 0.0;
            for (int i = 0; i < d_in; ++i) {
                double w = orc_f16_to_f64(W1[o * d_in + i]);
                s += w * xin[i];
                sa += fabs(w) * fabs(xin[i]);
            }
            h1[o] = f16r(s > 0.0 ? s : 0.0);
            a1[o] = s > 0.0 ? sa : 0.0;
        }
        for (int o = 0; o < H; ++o) {
            double s = 0.0, sa = 0.0;
            for (int i = 0; i < H; ++i) {
                double w = orc_f16_to_f64(W2[o * H + i]);
                s += w * h1[i];
                sa += fabs(w) * a1[i];
            }
            h2[o] = f16r(s > 0.0 ? s : 0.0);
            a2[o] = s > 0.0 ? sa : 0.0;
        }
        for (int o = 0; o < d_out; ++o) {
            double s = 0.0, sa = 0.0;
            for (int i = 0; i < H; ++i) {
                double w = orc_f16_to_f64(W3[o * H + i]);
                s += w * h2[i];
                sa += fabs(w) * a2[i];
            }
            out[pt * d_out + o] = s;
            if (absmag) absmag[pt * d_out + o] = sa;
        }
    }
}

/*
 * Backward pass of the network.  The forward pass is recomputed as above
 * (input and hidden activations rounded to binary16 where the forward
 * stores them).  Two modes:
 *   ORC_MLP_BF16 (0): gradient operands are rounded to bfloat16 where the
 *     kernel feeds them to its matrix unit: the incoming output gradient,
 *     the weights in the transposed products, the activations in the
 *     weight-gradient products, and each masked hidden gradient.
 *   ORC_MLP_EXACT (1): the network's own derivative in binary64, with no
 *     rounding beyond the binary16 storage of the forward's activations.
 * The ReLU mask is taken on the stored (binary16) activation.
 *   d_y   [N, d_out] binary32 (gradient of the loss w.r.t. the output)
 *   d_x   [N, d_in] binary64 (written)
 *   dW1 [H, d_in], dW2 [H, H], dW3 [d_out, H] binary64 (written)
 *   margin [N] (optional): smallest |pre-activation| of the point, so a test
 *   can tell which points sit on a ReLU kink.
 *   mag_dx, mag_dW1..3 (optional, shapes as d_x, dW1..3): the same
 *   products over absolute values of the operands the mode uses, with the
 *   ReLU mask applied, the hidden gradients' magnitudes propagated
 *   unrounded; with non-negative weights, inputs and output gradient they
 *   equal the exact-mode results.
 */
enum { ORC_MLP_BF16 = 0, ORC_MLP_EXACT = 1 };

void orc_mlp_bwd(int64_t N, int d_in, int H, int d_out, const uint16_t* x, const uint16_t* W1,
                 const uint16_t* W2, const uint16_t* W3, const float* d_y, int mode, double* d_x, double* dW1,
                 double* dW2, double* dW3, double* margin, double* mag_dx, double* mag_dW1, double* mag_dW2,
                 double* mag_dW3) {
    /* an operand as the mode feeds it to a product */
#define OP(v) (mode == ORC_MLP_BF16 ? orc_round_bf16(v) : (v))
    const int with_mag = mag_dx && mag_dW1 && mag_dW2 && mag_dW3;
    memset(dW1, 0, sizeof(double) * H * d_in);
    memset(dW2, 0, sizeof(double) * H * H);
    memset(dW3, 0, sizeof(double) * d_out * H);
    if (with_mag) {
        memset(mag_dW1, 0, sizeof(double) * H * d_in);
        memset(mag_dW2, 0, sizeof(double) * H * H);
        memset(mag_dW3, 0, sizeof(double) * d_out * H);
    }
    for (int64_t pt = 0; pt < N; ++pt) {
        double xin[256], h1[256], h2[256], dy[256], dh2[256], dh1[256], mh2[256], mh1[256];
        double mg = INFINITY;
        for (int i = 0; i < d_in; ++i) xin[i] = orc_f16_to_f64(x[pt * d_in + i]);
        for (int o = 0; o < H; ++o) {
            double s = 0.0;
            for (int i = 0; i < d_in; ++i) s += orc_f16_to_f64(W1[o * d_in + i]) * xin[i];
            h1[o] = f16r(s > 0.0 ? s : 0.0);
            if (fabs(s) < mg) mg = fabs(s);
        }
        for (int o = 0; o < H; ++o) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += orc_f16_to_f64(W2[o * H + i]) * h1[i];
            h2[o] = f16r(s > 0.0 ? s : 0.0);
            if (fabs(s) < mg) mg = fabs(s);
        }
        if (margin) margin[pt] = mg;
        for (int o = 0; o < d_out; ++o) dy[o] = OP((double)d_y[pt * d_out + o]);
        /* layer 3: dW3 += dy h2^T ; dh2 = W3^T dy, masked */
        for (int o = 0; o < d_out; ++o)
            for (int i = 0; i < H; ++i) {
                dW3[o * H + i] += dy[o] * OP(h2[i]);
                if (with_mag) mag_dW3[o * H + i] += fabs(dy[o]) * fabs(OP(h2[i]));
            }
        for (int i = 0; i < H; ++i) {
            double s = 0.0, m = 0.0;
            for (int o = 0; o < d_out; ++o) {
                const double w = OP(orc_f16_to_f64(W3[o * H + i]));
                s += w * dy[o];
                m += fabs(w) * fabs(dy[o]);
            }
            dh2[i] = OP(h2[i] > 0.0 ? s : 0.0);
            mh2[i] = h2[i] > 0.0 ? m : 0.0;
        }
        /* layer 2 */
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < H; ++i) {
                dW2[o * H + i] += dh2[o] * OP(h1[i]);
                if (with_mag) mag_dW2[o * H + i] += mh2[o] * fabs(OP(h1[i]));
            }
        for (int i = 0; i < H; ++i) {
            double s = 0.0, m = 0.0;
            for (int o = 0; o < H; ++o) {
                const double w = OP(orc_f16_to_f64(W2[o * H + i]));
                s += w * dh2[o];
                m += fabs(w) * mh2[o];
            }
            dh1[i] = OP(h1[i] > 0.0 ? s : 0.0);
            mh1[i] = h1[i] > 0.0 ? m : 0.0;
        }
        /* layer 1 */
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < d_in; ++i) {
                dW1[o * d_in + i] += dh1[o] * OP(xin[i]);
                if (with_mag) mag_dW1[o * d_in + i] += mh1[o] * fabs(OP(xin[i]));
            }
        for (int i = 0; i < d_in; ++i) {
            double s = 0.0, m = 0.0;
            for (int o = 0; o < H; ++o) {
                const double w = OP(orc_f16_to_f64(W1[o * d_in + i]));
                s += w * dh1[o];
                m += fabs(w) * mh1[o];
            }
            d_x[pt * d_in + i] = s;
            if (with_mag) mag_dx[pt * d_in + i] = m;
        }
    }
#undef OP
}

/* ------------------------------------------------------------------------ */
/* Optimizer step for the tables (the paper trains by gradient descent and  */
/* states no optimizer; Adam, Kingma & Ba 2015, Algorithm 1, is the choice  */
/* made here).  Binary64 arithmetic on binary32 state; the binary16         */
/* copy is the round-to-nearest-even image of the updated parameter.        */
/* step is the 1-based iteration count t.                                  */
/* ------------------------------------------------------------------------ */
void orc_adam_step(int64_t n, float* param, const float* grad, float* m, float* v, double lr,
                   double beta1, double beta2, double eps, int64_t step, uint16_t* param_f16) {
    double bc1 = 1.0 - pow(beta1, (double)step);
    double bc2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        double g = grad[i];
        double mi = beta1 * m[i] + (1.0 - beta1) * g;
        double vi = beta2 * v[i] + (1.0 - beta2) * g * g;
        double mhat = mi / bc1, vhat = vi / bc2;
        double p = (double)param[i] - lr * mhat / (sqrt(vhat) + eps);
        m[i] = (float)mi;
        v[i] = (float)vi;
        param[i] = (float)p;
        if (param_f16) param_f16[i] = orc_f64_to_f16((double)param[i]);
    }
}

/* Gradient of the mean squared error (Sec. 6 trains with an L2 loss):
 * d_y = scale * (y - target), binary64 from binary32 inputs. */
void orc_mse_grad(int64_t n, const float* y, const float* target, double scale, double* d_y) {
    for (int64_t i = 0; i < n; ++i) d_y[i] = scale * ((double)y[i] - (double)target[i]);
}

/* Round-to-nearest-even binary32 -> binary16 copy. */
void orc_cast_f32_f16(int64_t n, const float* src, uint16_t* dst) {
    for (int64_t i = 0; i < n; ++i) dst[i] = orc_f64_to_f16((double)src[i]);
}

/* ------------------------------------------------------------------------ */
/* Volume rendering (Sec. 6, Eq. 5).  The paper states the integral over a   */
/* ray, C = int T(t) sigma(t) c(t) dt with T(t) = exp(-int sigma); it is     */
/* evaluated with the usual quadrature over the ray's samples (the radiance  */
/* field system the paper cites for volume rendering): per sample k,         */
/*   tau_k = sigma_k * delta_k,  alpha_k = 1 - exp(-tau_k) (evaluated as     */
/*   -expm1(-tau_k): the same number without cancellation for thin samples), */
/*   T_k = exp(-(tau_0 + ... + tau_{k-1})),  w_k = T_k * alpha_k,            */
/*   RGB = sum_k w_k c_k,  A = sum_k w_k  (the ray's opacity).               */
/* The network's raw outputs map to sigma = softplus(raw_0) and              */
/* c = sigmoid(raw_1..3) (the paper names no activations; these are a        */
/* reading).  raw [R*S][4], delta [R*S] (the sample's segment length),       */
/* out rgba [R][4].  Binary64 throughout.                                    */
/* ------------------------------------------------------------------------ */
static double softplus(double x) { return (x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x))); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

void orc_composite_fwd(int64_t R, int S, const float* raw, const float* delta, double* rgba) {
    for (int64_t r = 0; r < R; ++r) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double optical = 0.0; /* tau_0 + ... + tau_{k-1} */
        for (int k = 0; k < S; ++k) {
            const float* q = raw + (r * S + k) * 4;
            const double sigma = softplus(q[0]);
            const double tau = sigma * (double)delta[r * S + k];
            const double w = exp(-optical) * (-expm1(-tau));
            for (int ch = 0; ch < 3; ++ch) acc[ch] += w * sigmoid(q[1 + ch]);
            acc[3] += w;
            optical += tau;
        }
        for (int ch = 0; ch < 4; ++ch) rgba[r * 4 + ch] = acc[ch];
    }
}

/* Adjoint of orc_composite_fwd for d_rgba [R][4]: d_raw [R*S][4].  With
 * Q = sum_j w_j q_j (q_j = (c_j, 1)), T_{k+1} = T_k exp(-tau_k) and
 * Q_{<=k} the partial sum up to and including sample k,
 *   dQ/dtau_k = T_{k+1} q_k - (Q - Q_{<=k}),   dQ/dc_k = w_k,
 * then through the activations: d sigma/d raw = sigmoid(raw),
 * d c/d raw = c (1 - c).  mag [R*S][4] (optional) receives the same
 * expressions with every term replaced by its absolute value. */
void orc_composite_bwd(int64_t R, int S, const float* raw, const float* delta, const double* d_rgba,
                       double* d_raw, double* mag) {
    for (int64_t r = 0; r < R; ++r) {
        double Q[4] = {0.0, 0.0, 0.0, 0.0};
        double optical = 0.0;
        for (int k = 0; k < S; ++k) { /* totals first */
            const float* q = raw + (r * S + k) * 4;
            const double tau = softplus(q[0]) * (double)delta[r * S + k];
            const double w = exp(-optical) * (-expm1(-tau));
            for (int ch = 0; ch < 3; ++ch) Q[ch] += w * sigmoid(q[1 + ch]);
            Q[3] += w;
            optical += tau;
        }
        const double* dQ = d_rgba + r * 4;
        double part[4] = {0.0, 0.0, 0.0, 0.0};
        optical = 0.0;
        for (int k = 0; k < S; ++k) {
            const float* q = raw + (r * S + k) * 4;
            const double dl = (double)delta[r * S + k];
            const double tau = softplus(q[0]) * dl;
            const double Tk = exp(-optical), Tn = exp(-(optical + tau));
            const double w = Tk * (-expm1(-tau));
            double c[4];
            for (int ch = 0; ch < 3; ++ch) c[ch] = sigmoid(q[1 + ch]);
            c[3] = 1.0;
            for (int ch = 0; ch < 4; ++ch) part[ch] += w * c[ch];
            double dtau = 0.0, atau = 0.0;
            for (int ch = 0; ch < 4; ++ch) {
                const double rest = Q[ch] - part[ch];
                dtau += dQ[ch] * (Tn * c[ch] - rest);
                atau += fabs(dQ[ch]) * (Tn * fabs(c[ch]) + fabs(Q[ch]) + fabs(part[ch]));
            }
            const double ds = sigmoid(q[0]) * dl;
            double* o = d_raw + (r * S + k) * 4;
            o[0] = dtau * ds;
            for (int ch = 0; ch < 3; ++ch) o[1 + ch] = dQ[ch] * w * c[ch] * (1.0 - c[ch]);
            if (mag) {
                double* m = mag + (r * S + k) * 4;
                m[0] = atau * ds;
                for (int ch = 0; ch < 3; ++ch) m[1 + ch] = fabs(dQ[ch]) * w * c[ch] * (1.0 - c[ch]);
            }
            optical += tau;
        }
    }
}

/* Number of OpenMP threads the parallel loops above use (timing only). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

