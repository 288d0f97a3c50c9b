// Device kernels of the FlowRoI hot path for gfx950 (CDNA4, wave64).
//
// Steps (FlowRoI Method section; estimator: Farneback two-frame polynomial
// expansion, SCIA 2003):
//   k_pyr_down   pyramid level l -> l+1: 5x5 binomial blur at even pixels
//   k_polyexp    local quadratic fit f ~ x^T A x + b^T x + c per pixel
//   k_iter       one displacement update: prior flow (zero, given, or the
//                2x-upsampled coarser flow), bilinear warp of next's
//                coefficients, per-pixel normal equations, box pooling,
//                regularised 2x2 solve, optional |d|^2 epilogue
//   k_hist/k_pick radix select of the top-q threshold on |d|^2 bit patterns
//   k_dilate     threshold + binary dilation into the RoI mask
//
// Every kernel is a plain grid over output tiles staged through LDS; all
// arithmetic is FP32 (storage may be FP16). Border handling replicates the
// edge pixel for stencils and warps; the dilation treats outside as 0.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flowroi {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ float ld(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ double ldd(const double *p, size_t i) { return p[i]; }
__device__ __forceinline__ double ldd(const float *p, size_t i) { return (double)p[i]; }
__device__ __forceinline__ double ldd(const __half *p, size_t i) { return (double)__half2float(p[i]); }
__device__ __forceinline__ double ldd(const uint8_t *p, size_t i) { return (double)p[i]; }
__device__ __forceinline__ double ldd(const uint16_t *p, size_t i) { return (double)p[i]; }
__device__ __forceinline__ float ld(const __half *p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ float ld(const uint8_t *p, size_t i) { return (float)p[i]; }
__device__ __forceinline__ float ld(const uint16_t *p, size_t i) { return (float)p[i]; }

__device__ __forceinline__ void st(float *p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void st(__half *p, size_t i, float v) { p[i] = __float2half(v); }
__device__ __forceinline__ void std_(double *p, size_t i, double v) { p[i] = v; }
__device__ __forceinline__ void std_(float *p, size_t i, double v) { p[i] = (float)v; }
__device__ __forceinline__ void std_(__half *p, size_t i, double v) { p[i] = __float2half((float)v); }

// FP16 rounding of a value kept in an FP32 buffer (stage entry points).
__device__ __forceinline__ float round16(float v) { return __half2float(__float2half(v)); }

// ---------------------------------------------------------------- pyramid

constexpr int PYR_TW = 64, PYR_TH = 8;
constexpr int PYR_SW = 2 * PYR_TW + 3, PYR_SH = 2 * PYR_TH + 3;

struct PyrArgs {
    const void *src[2];
    int64_t src_pitch; // elements
    float dc;          // subtracted from every input value
    void *dst[2];
    int32_t dst_pitch;
    int32_t h, w, h2, w2;
    int32_t round16;   // FP32 destination rounded to FP16 precision
};

// dst(i, j) = sum_u k(u) sum_v k(v) src(2i+u, 2j+v), k = [1 4 6 4 1]/16,
// accumulated in FP64: pyramid images keep the frame's full dynamic range,
// and FP32 rounding of values far from zero feeds straight into the
// derivative filters of the expansion.
// grid: (ceil(w2/64), ceil(h2/8), frames)
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_pyr_down(PyrArgs a)
{
    __shared__ double s[PYR_SH][PYR_SW + 1];
    __shared__ double v[PYR_TH][PYR_SW + 1];
    const TIn *src = (const TIn *)a.src[blockIdx.z];
    TOut *dst = (TOut *)a.dst[blockIdx.z];
    const int ox0 = blockIdx.x * PYR_TW, oy0 = blockIdx.y * PYR_TH;
    const int sx0 = 2 * ox0 - 2, sy0 = 2 * oy0 - 2;
    for (int i = threadIdx.x; i < PYR_SH * PYR_SW; i += 256) {
        const int r = i / PYR_SW, c = i - r * PYR_SW;
        const int y = clampi(sy0 + r, 0, a.h - 1), x = clampi(sx0 + c, 0, a.w - 1);
        s[r][c] = ldd(src, (size_t)y * a.src_pitch + x) - (double)a.dc;
    }
    __syncthreads();
    const double k0 = 1.0 / 16, k1 = 4.0 / 16, k2 = 6.0 / 16;
    for (int i = threadIdx.x; i < PYR_TH * PYR_SW; i += 256) {
        const int r = i / PYR_SW, c = i - r * PYR_SW;
        const int b = 2 * r;
        v[r][c] = k0 * s[b][c] + k1 * s[b + 1][c] + k2 * s[b + 2][c] + k1 * s[b + 3][c] + k0 * s[b + 4][c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PYR_TH * PYR_TW; i += 256) {
        const int r = i / PYR_TW, c = i - r * PYR_TW;
        const int y = oy0 + r, x = ox0 + c;
        if (y >= a.h2 || x >= a.w2) continue;
        const int b = 2 * c;
        double o = k0 * v[r][b] + k1 * v[r][b + 1] + k2 * v[r][b + 2] + k1 * v[r][b + 3] + k0 * v[r][b + 4];
        if (a.round16) o = (double)round16((float)o);
        std_(dst, (size_t)y * a.dst_pitch + x, o);
    }
}

// ---------------------------------------------------------------- polynomial expansion

constexpr int PE_TW = 64, PE_TH = 16, PE_MAXN = 3;

struct PolyArgs {
    const void *src[2];
    int64_t src_pitch;
    float dc;
    void *dst[2];       // 5 planes each: b_x, b_y, A_xx, A_yy, A_xy
    int64_t dplane;     // elements between planes
    int32_t dpitch;
    int32_t h, w, n;    // n = poly_n / 2
    int32_t round16;
    // vertical kernels over the row offset t = -n..n:
    //   kv0 = a(t), kv1 = t a(t), kv2 = (t^2 - m2/m0) a(t)
    double kv0[2 * PE_MAXN + 1], kv1[2 * PE_MAXN + 1], kv2[2 * PE_MAXN + 1];
    // horizontal kernels over the column offset, normalisation folded in:
    //   b_x  = H[t a / (m0 m2)]                    (V0)
    //   b_y  = H[a / (m0 m2)]                      (V1)
    //   A_xy = H[t a / (2 m2^2)]                   (V1)
    //   A_xx = H[(t^2 - m2/m0) a / (m0 m4 - m2^2)] (V0)
    //   A_yy = H[a / (m0 m4 - m2^2)]               (V2)
    double hx[2 * PE_MAXN + 1], hy[2 * PE_MAXN + 1], hxy[2 * PE_MAXN + 1];
    double hxx[2 * PE_MAXN + 1], hyy[2 * PE_MAXN + 1];
};

// The expansion's derivative filters cancel the (large) local mean of the
// image, so the fit runs in FP64 arithmetic; only the stored coefficients
// are rounded to the storage type.
// grid: (ceil(w/64), ceil(h/16), frames)
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_polyexp(PolyArgs a)
{
    constexpr int SW = PE_TW + 2 * PE_MAXN, SH = PE_TH + 2 * PE_MAXN;
    __shared__ double s[SH][SW + 1];
    __shared__ double vr[3][PE_TH][SW + 1];
    const TIn *src = (const TIn *)a.src[blockIdx.z];
    TOut *dst = (TOut *)a.dst[blockIdx.z];
    const int n = a.n, sw = PE_TW + 2 * n, sh = PE_TH + 2 * n;
    const int ox0 = blockIdx.x * PE_TW, oy0 = blockIdx.y * PE_TH;
    for (int i = threadIdx.x; i < sh * sw; i += 256) {
        const int r = i / sw, c = i - r * sw;
        const int y = clampi(oy0 - n + r, 0, a.h - 1), x = clampi(ox0 - n + c, 0, a.w - 1);
        s[r][c] = ldd(src, (size_t)y * a.src_pitch + x) - (double)a.dc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PE_TH * sw; i += 256) {
        const int r = i / sw, c = i - r * sw;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        for (int t = 0; t <= 2 * n; ++t) {
            const double f = s[r + t][c];
            v0 += a.kv0[t] * f;
            v1 += a.kv1[t] * f;
            v2 += a.kv2[t] * f;
        }
        vr[0][r][c] = v0;
        vr[1][r][c] = v1;
        vr[2][r][c] = v2;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PE_TH * PE_TW; i += 256) {
        const int r = i / PE_TW, c = i - r * PE_TW;
        const int y = oy0 + r, x = ox0 + c;
        if (y >= a.h || x >= a.w) continue;
        double bx = 0.0, by = 0.0, axy = 0.0, axx = 0.0, ayy = 0.0;
        for (int t = 0; t <= 2 * n; ++t) {
            const double v0 = vr[0][r][c + t], v1 = vr[1][r][c + t], v2 = vr[2][r][c + t];
            bx += a.hx[t] * v0;
            axx += a.hxx[t] * v0;
            by += a.hy[t] * v1;
            axy += a.hxy[t] * v1;
            ayy += a.hyy[t] * v2;
        }
        float o[5] = {(float)bx, (float)by, (float)axx, (float)ayy, (float)axy};
        if (a.round16)
            for (int k = 0; k < 5; ++k) o[k] = round16(o[k]);
        const size_t q = (size_t)y * a.dpitch + x;
        for (int k = 0; k < 5; ++k) st(dst, q + k * a.dplane, o[k]);
    }
}

// ---------------------------------------------------------------- initial flow

struct InitArgs {
    const float2 *src; int32_t src_pitch, h, w; // full-resolution initial flow
    float2 *dst; int32_t dst_pitch, hl, wl;     // coarsest level
    int32_t stride;                             // 2^(levels-1)
};

__global__ __launch_bounds__(256) void k_init_flow(InitArgs a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.wl || y >= a.hl) return;
    const float2 v = a.src[(size_t)min(a.stride * y, a.h - 1) * a.src_pitch + min(a.stride * x, a.w - 1)];
    const float inv = 1.0f / (float)a.stride; // power of two: exact
    a.dst[(size_t)y * a.dst_pitch + x] = make_float2(v.x * inv, v.y * inv);
}

// ---------------------------------------------------------------- displacement update

constexpr int IT_TW = 64, IT_MAXR = 7;

enum { PRIOR_ZERO = 0, PRIOR_PLAIN = 1, PRIOR_UPSAMPLE = 2 };

struct IterArgs {
    const void *r1, *r2;     // expansions of prev and next (5 planes each)
    int64_t rplane;
    int32_t rpitch;
    int32_t h, w;
    int32_t prior;           // PRIOR_*
    const float2 *fin;       // prior flow (PLAIN: this level; UPSAMPLE: coarser level)
    int32_t fin_pitch, hc, wc;
    float2 *fout;
    int32_t fout_pitch;
    int32_t R;               // window half-width
    float eps;
    float *m2;               // nullable: epilogue writes |d|^2
    int32_t m2_pitch;
};

__device__ __forceinline__ float bilerp(float p00, float p01, float p10, float p11, float fx, float fy)
{
    return (1.f - fy) * ((1.f - fx) * p00 + fx * p01) + fy * ((1.f - fx) * p10 + fx * p11);
}

__device__ __forceinline__ float2 prior_at(const IterArgs &a, int y, int x)
{
    if (a.prior == PRIOR_ZERO) return make_float2(0.f, 0.f);
    if (a.prior == PRIOR_PLAIN) return a.fin[(size_t)y * a.fin_pitch + x];
    // pixel (y, x) of this level sits at (y/2, x/2) of the coarser grid
    float xs = fminf(x * 0.5f, (float)(a.wc - 1)), ys = fminf(y * 0.5f, (float)(a.hc - 1));
    const int x0 = (int)xs, y0 = (int)ys;
    const int x1 = min(x0 + 1, a.wc - 1), y1 = min(y0 + 1, a.hc - 1);
    const float fx = xs - x0, fy = ys - y0;
    const float2 p00 = a.fin[(size_t)y0 * a.fin_pitch + x0], p01 = a.fin[(size_t)y0 * a.fin_pitch + x1];
    const float2 p10 = a.fin[(size_t)y1 * a.fin_pitch + x0], p11 = a.fin[(size_t)y1 * a.fin_pitch + x1];
    return make_float2(2.f * bilerp(p00.x, p01.x, p10.x, p11.x, fx, fy),
                       2.f * bilerp(p00.y, p01.y, p10.y, p11.y, fx, fy));
}

// Per-pixel normal-equation terms G = A^T A (g11, g12, g22) and h = A^T db
// for the prior displacement d~ at (y, x):
//   A  = (A1(x) + A2(x + d~)) / 2,  db = -(b2(x + d~) - b1(x)) / 2 + A d~,
// next's coefficients sampled bilinearly at x + d~ clamped into the frame.
template <typename TS>
__device__ __forceinline__ void update_terms(const IterArgs &a, const TS *r1, const TS *r2, int y, int x,
                                             float g[5])
{
    const size_t P = (size_t)a.rplane;
    const size_t i1 = (size_t)y * a.rpitch + x;
    const float b1x = ld(r1, i1), b1y = ld(r1, i1 + P);
    const float a11 = ld(r1, i1 + 2 * P), a22 = ld(r1, i1 + 3 * P), a12 = ld(r1, i1 + 4 * P);
    const float2 d = prior_at(a, y, x);
    // Sample point x + d~ kept as integer pixel + fraction: an absolute FP32
    // coordinate near x = 2000 only resolves 1.2e-4 px, which the solve can
    // amplify past 1e-3 px at sensitive pixels. Clamping into the frame
    // follows the real-valued point (outside -> edge pixel, zero weight).
    const float dxc = fminf(fmaxf(d.x, -(float)(a.w + 1)), (float)(a.w + 1));
    const float dyc = fminf(fmaxf(d.y, -(float)(a.h + 1)), (float)(a.h + 1));
    const float flx = floorf(dxc), fly = floorf(dyc);
    float fx = dxc - flx, fy = dyc - fly;
    int x0 = x + (int)flx, y0 = y + (int)fly;
    if (x0 < 0) {
        x0 = 0;
        fx = 0.f;
    } else if (x0 > a.w - 1 || (x0 == a.w - 1 && fx > 0.f)) {
        x0 = a.w - 1;
        fx = 0.f;
    }
    if (y0 < 0) {
        y0 = 0;
        fy = 0.f;
    } else if (y0 > a.h - 1 || (y0 == a.h - 1 && fy > 0.f)) {
        y0 = a.h - 1;
        fy = 0.f;
    }
    const int x1 = min(x0 + 1, a.w - 1), y1 = min(y0 + 1, a.h - 1);
    const size_t q00 = (size_t)y0 * a.rpitch + x0, q01 = (size_t)y0 * a.rpitch + x1;
    const size_t q10 = (size_t)y1 * a.rpitch + x0, q11 = (size_t)y1 * a.rpitch + x1;
    float c[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const TS *p = r2 + k * P;
        c[k] = bilerp(ld(p, q00), ld(p, q01), ld(p, q10), ld(p, q11), fx, fy);
    }
    const float A11 = 0.5f * (a11 + c[2]), A22 = 0.5f * (a22 + c[3]), A12 = 0.5f * (a12 + c[4]);
    const float dbx = -0.5f * (c[0] - b1x) + A11 * d.x + A12 * d.y;
    const float dby = -0.5f * (c[1] - b1y) + A12 * d.x + A22 * d.y;
    g[0] = A11 * A11 + A12 * A12;
    g[1] = A12 * (A11 + A22);
    g[2] = A12 * A12 + A22 * A22;
    g[3] = A11 * dbx + A12 * dby;
    g[4] = A12 * dbx + A22 * dby;
}

// Solve of the pooled 2x2 system G d = h (g11, g12, g22, h1, h2):
// d = adj(G) h / max(det G, eps tr(G)^2), zero where tr G = 0.
__device__ __forceinline__ float2 solve2(float g11, float g12, float g22, float h1, float h2, float eps)
{
    const float tr = g11 + g22;
    if (tr == 0.f) return make_float2(0.f, 0.f);
    const float det = g11 * g22 - g12 * g12;
    const float den = fmaxf(det, eps * tr * tr);
    return make_float2((g22 * h1 - g12 * h2) / den, (g11 * h2 - g12 * h1) / den);
}

// Strip walker. A workgroup owns IT_TW output columns and a strip of rows
// [y_begin, y_end); it walks down in chunks of IT_CH rows:
//   1. per-pixel terms for IT_CH new rows over IT_TW + 2R columns -> LDS;
//   2. horizontal window sums of those rows -> a ring of IT_CH + 2R rows;
//   3. vertical window sums for the output rows whose window is complete,
//      then the solve; each thread finishes two vertically adjacent pixels.
// Replicated borders: out-of-frame rows/columns take the edge pixel's terms.
// Window sums are exact sums of 2R+1 terms in a fixed order that depends
// only on absolute pixel positions (segments of 16 columns, row pairs
// starting at even rows), so results do not depend on the strip height.
// grid: (ceil(w / IT_TW) * ceil(h / strip) remapped so that consecutive
// strips land on the same XCD), block 256.
constexpr int IT_CH = 8, IT_SEG = 16;

template <typename TS, int R>
__global__ __launch_bounds__(256) void k_iter(IterArgs a, int32_t strip, int32_t nx, int32_t ntiles)
{
    constexpr int CW = IT_TW + 2 * R;   // columns of per-pixel terms
    constexpr int RING = IT_CH + 2 * R; // rows of horizontal sums kept
    __shared__ float gh[5][IT_CH][CW];
    __shared__ float hs[5][RING][IT_TW];

    // XCD-aware tile order: hardware hands workgroup b to XCD b % 8, so give
    // each XCD a contiguous run of tiles (neighbours share halo columns in L2)
    int b = blockIdx.x;
    const int n8 = ntiles & ~7;
    if (b < n8) b = (b & 7) * (n8 >> 3) + (b >> 3);
    const int tx = b % nx, ty = b / nx;
    const int x0 = tx * IT_TW;
    const int ys = ty * strip, ye = min(ys + strip, a.h);
    const TS *r1 = (const TS *)a.r1, *r2 = (const TS *)a.r2;
    const int t = threadIdx.x;

    for (int cy = ys - R; cy < ye + R; cy += IT_CH) {
        // 1. per-pixel terms of rows [cy, cy + IT_CH)
        for (int i = t; i < IT_CH * CW; i += 256) {
            const int r = i / CW, c = i - r * CW;
            const int y = clampi(cy + r, 0, a.h - 1), x = clampi(x0 - R + c, 0, a.w - 1);
            float g[5];
            update_terms<TS>(a, r1, r2, y, x, g);
#pragma unroll
            for (int k = 0; k < 5; ++k) gh[k][r][c] = g[k];
        }
        __syncthreads();
        // 2. horizontal sums: task = (channel, row, 16-column segment)
        if (t < 5 * IT_CH * (IT_TW / IT_SEG)) {
            const int k = t / (IT_CH * (IT_TW / IT_SEG));
            const int rem = t - k * (IT_CH * (IT_TW / IT_SEG));
            const int r = rem / (IT_TW / IT_SEG), sg = rem - r * (IT_TW / IT_SEG);
            const float *src = &gh[k][r][sg * IT_SEG];
            float v[IT_SEG + 2 * R];
#pragma unroll
            for (int j = 0; j < IT_SEG + 2 * R; ++j) v[j] = src[j];
            float *dst = &hs[k][(cy + r - (ys - R)) % RING][sg * IT_SEG];
#pragma unroll
            for (int j = 0; j < IT_SEG; ++j) {
                float sum = 0.f;
#pragma unroll
                for (int u = 0; u <= 2 * R; ++u) sum += v[j + u];
                dst[j] = sum;
            }
        }
        __syncthreads();
        // 3. outputs [cy - R, cy - R + IT_CH) that lie in the strip; thread
        //    (column c, pair q) finishes rows cy - R + 2q and cy - R + 2q + 1
        {
            const int c = t & (IT_TW - 1), q = t >> 6;
            const int oy = cy - R + 2 * q, x = x0 + c;
            if (oy + 1 >= ys && oy < ye && x < a.w) {
                float S0[5], S1[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    float col[2 * R + 2];
#pragma unroll
                    for (int u = 0; u < 2 * R + 2; ++u) col[u] = hs[k][(oy - ys + u + RING) % RING][c];
                    float s0 = 0.f, s1 = 0.f;
#pragma unroll
                    for (int u = 0; u <= 2 * R; ++u) {
                        s0 += col[u];
                        s1 += col[u + 1];
                    }
                    S0[k] = s0;
                    S1[k] = s1;
                }
                if (oy >= ys) {
                    const float2 d = solve2(S0[0], S0[1], S0[2], S0[3], S0[4], a.eps);
                    a.fout[(size_t)oy * a.fout_pitch + x] = d;
                    if (a.m2) a.m2[(size_t)oy * a.m2_pitch + x] = d.x * d.x + d.y * d.y;
                }
                if (oy + 1 < ye) {
                    const float2 d = solve2(S1[0], S1[1], S1[2], S1[3], S1[4], a.eps);
                    a.fout[(size_t)(oy + 1) * a.fout_pitch + x] = d;
                    if (a.m2) a.m2[(size_t)(oy + 1) * a.m2_pitch + x] = d.x * d.x + d.y * d.y;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- top-q select

// Radix select over the bit patterns of |d|^2 (non-negative floats order
// like their unsigned bits): three passes of 11, 11 and 10 bits from the top.
// state[0] = bit prefix found so far, state[1] = rank still sought among the
// values that share it (0 = the largest), state[2] = tau^2 bits when done.
constexpr int SEL_BINS = 2048;

struct SelState { uint32_t prefix, rank, tau2_bits, pad; };

__host__ __device__ constexpr int sel_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__host__ __device__ constexpr int sel_bits(int pass) { return pass == 2 ? 10 : 11; }

__global__ __launch_bounds__(256) void k_sel_init(SelState *st, uint32_t *hist, uint32_t rank, uint32_t tau2_bits)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->prefix = 0;
        st->rank = rank;
        st->tau2_bits = tau2_bits;
        st->pad = 0;
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < SEL_BINS; i += gridDim.x * 256) hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_sel_hist(const float *m2, int32_t pitch, int32_t h, int32_t w,
                                                  const SelState *st, uint32_t *hist, int32_t pass)
{
    __shared__ uint32_t lh[SEL_BINS];
    for (int i = threadIdx.x; i < SEL_BINS; i += 256) lh[i] = 0;
    __syncthreads();
    const int shift = sel_shift(pass), nb = 1 << sel_bits(pass);
    const uint32_t prefix = st->prefix;
    const int hi = shift + sel_bits(pass);
    const size_t n = (size_t)h * w;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const size_t y = i / w, x = i - y * w;
        const uint32_t v = __float_as_uint(m2[y * pitch + x]);
        if (pass > 0 && (v >> hi) != prefix) continue;
        atomicAdd(&lh[(v >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += 256)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// one block of 256 threads; each owns 8 consecutive bins
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, uint32_t *hist, int32_t pass)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t above[256];
    const int nb = 1 << sel_bits(pass), per = nb / 256;
    const int t = threadIdx.x;
    // read the state before any thread can update it (updates follow the barriers)
    const uint32_t rank = st->rank, prefix0 = st->prefix;
    // thread t covers bins [nb - per (t+1), nb - per t): thread 0 holds the largest values
    const int b_hi = nb - per * t - 1;
    uint32_t cnt[8];
    uint32_t sum = 0;
    for (int j = 0; j < per; ++j) {
        cnt[j] = hist[b_hi - j];
        sum += cnt[j];
    }
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < 256; ++i) {
            above[i] = acc;
            acc += part[i];
        }
    }
    __syncthreads();
    uint32_t acc = above[t];
    if (rank >= acc && rank < acc + sum) {
        for (int j = 0; j < per; ++j) {
            if (rank < acc + cnt[j]) {
                const uint32_t prefix = (prefix0 << sel_bits(pass)) | (uint32_t)(b_hi - j);
                st->prefix = prefix;
                st->rank = rank - acc;
                if (pass == 2) st->tau2_bits = prefix;
                break;
            }
            acc += cnt[j];
        }
    }
    __syncthreads();
    for (int j = 0; j < per; ++j) hist[b_hi - j] = 0;
}

// ---------------------------------------------------------------- threshold + dilation

constexpr int DIL_TW = 64, DIL_TH = 16, DIL_MAXR = 32;

struct DilArgs {
    const float *m2; int32_t m2_pitch;
    const SelState *st;        // tau^2 bits live in st->tau2_bits
    uint8_t *mask; int32_t mask_pitch;
    int32_t h, w, r;
    int8_t hw[2 * DIL_MAXR + 1]; // half-width of the structuring element on row offset u
};

// pre(y, x) = [|d|^2 > tau^2]; mask(y, x) = OR_{(u,v) in SE} pre(y+u, x+v),
// outside the frame counting as 0. Row pass: distance to the nearest set
// pixel within +-r on the same row; column pass: OR_u [dist(y+u) <= hw(u)].
// grid: (ceil(w/64), ceil(h/16))
__global__ __launch_bounds__(256) void k_dilate(DilArgs a)
{
    constexpr int SW = DIL_TW + 2 * DIL_MAXR, SH = DIL_TH + 2 * DIL_MAXR;
    __shared__ uint8_t pre[SH][SW];
    __shared__ uint8_t dist[SH][DIL_TW];
    const int r = a.r, sw = DIL_TW + 2 * r, sh = DIL_TH + 2 * r;
    const int ox0 = blockIdx.x * DIL_TW, oy0 = blockIdx.y * DIL_TH;
    const uint32_t t2 = a.st->tau2_bits;
    for (int i = threadIdx.x; i < sh * sw; i += 256) {
        const int rr = i / sw, c = i - rr * sw;
        const int y = oy0 - r + rr, x = ox0 - r + c;
        uint8_t v = 0;
        if (y >= 0 && y < a.h && x >= 0 && x < a.w)
            v = __float_as_uint(a.m2[(size_t)y * a.m2_pitch + x]) > t2 ? 1 : 0;
        pre[rr][c] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < sh * DIL_TW; i += 256) {
        const int rr = i / DIL_TW, c = i - rr * DIL_TW;
        int d = r + 1;
        for (int v = -r; v <= r; ++v)
            if (pre[rr][c + r + v]) d = min(d, abs(v));
        dist[rr][c] = (uint8_t)d;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < DIL_TH * DIL_TW; i += 256) {
        const int rr = i / DIL_TW, c = i - rr * DIL_TW;
        const int y = oy0 + rr, x = ox0 + c;
        if (y >= a.h || x >= a.w) continue;
        uint8_t m = 0;
        for (int u = -r; u <= r; ++u) m |= dist[rr + r + u][c] <= a.hw[u + r] ? 1 : 0;
        a.mask[(size_t)y * a.mask_pitch + x] = m;
    }
}

} // namespace flowroi
