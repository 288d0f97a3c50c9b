// Device kernels of the FlowRoI hot path for gfx950 (CDNA4, wave64).
//
// Steps (FlowRoI Method section; estimator: Farneback two-frame polynomial
// expansion, SCIA 2003):
//   k_polyexp    local quadratic fit f ~ x^T A x + b^T x + c per pixel; with
//                poly_n >= 5 the same launch also writes the next pyramid
//                level (5x5 binomial blur at even pixels)
//   k_pyr_down   the pyramid step on its own (stage entry point, poly_n 3)
//   k_iter       one displacement update: prior flow (zero, given, or the
//                2x-upsampled coarser flow), bilinear warp of next's
//                coefficients, per-pixel normal equations, box pooling,
//                regularised 2x2 solve; the last launch also writes the
//                mask stage's input (pre-mask bytes or |d|^2)
//   k_sel_*      radix select of the top-q threshold on float bit patterns
//                (|d|^2, or the saliency)
//   k_dilate_wide, k_dilate_bits, k_dilate   binary dilation into the RoI mask
// Denoising pre-stage (k_denoise: median then bilateral), the saliency rule
// (k_sal_max, k_sal: motion saliency from |d| and its gradient; k_open_close:
// threshold, opening, closing and tile-local component labels; k_cc_border,
// k_cc_compress, k_cc_keep: components across tiles, their areas, the kept
// ones), phase-correlation stabilisation (k_ph_*, k_fft_*)
// and the adjacent-frame ensemble (k_ensemble) complete the set.
//
// Every kernel is a plain grid over output tiles staged through LDS. Pyramid
// and expansion arithmetic is FP64 (storage FP32, or FP16 for the
// expansions), the rest FP32. Border handling replicates the edge pixel for
// stencils and warps; the dilation treats outside as 0.
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

// Raw buffer descriptors (gfx9 family: dword3 = 0x00020000). Loads through
// them take a 32-bit byte offset in a VGPR against a scalar base, which keeps
// address arithmetic of the gathers off the vector ALU; out-of-range offsets
// read 0 instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
}
__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}
__device__ __forceinline__ float bload1(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ float bload1h(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0)
{
    return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0)));
}
__device__ __forceinline__ float4 bload4h(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0)
{
    const uint2 u = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    const __half2 lo = __builtin_bit_cast(__half2, u.x), hi = __builtin_bit_cast(__half2, u.y);
    return make_float4(__low2float(lo), __high2float(lo), __low2float(hi), __high2float(hi));
}

// Packed storage of one frame's expansion: P4 = (b_x, b_y, A_xx, A_yy) per
// pixel (float4, or 4 x FP16), P1 = A_xy (float or FP16). Both (h + 1) x
// pitch: columns w..pitch-1 and row h are zero.
template <typename TS> struct Packed;
template <> struct Packed<float> {
    static constexpr uint32_t B4 = 16, B1 = 4;
    __device__ static float4 load4(__amdgpu_buffer_rsrc_t r, uint32_t px) { return bload4(r, px * B4); }
    __device__ static float load1(__amdgpu_buffer_rsrc_t r, uint32_t px) { return bload1(r, px * B1); }
    // byte offset + scalar offset (row stride) forms, for the bilinear corners
    __device__ static float4 load4b(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t sb) { return bload4(r, b, sb); }
    __device__ static float load1b(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t sb) { return bload1(r, b, sb); }
    __device__ static void store(void *p4, void *p1, size_t px, const float o[5])
    {
        ((float4 *)p4)[px] = make_float4(o[0], o[1], o[2], o[3]);
        ((float *)p1)[px] = o[4];
    }
};
template <> struct Packed<__half> {
    static constexpr uint32_t B4 = 8, B1 = 2;
    __device__ static float4 load4(__amdgpu_buffer_rsrc_t r, uint32_t px) { return bload4h(r, px * B4); }
    __device__ static float load1(__amdgpu_buffer_rsrc_t r, uint32_t px) { return bload1h(r, px * B1); }
    __device__ static float4 load4b(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t sb) { return bload4h(r, b, sb); }
    __device__ static float load1b(__amdgpu_buffer_rsrc_t r, uint32_t b, uint32_t sb) { return bload1h(r, b, sb); }
    __device__ static void store(void *p4, void *p1, size_t px, const float o[5])
    {
        const __half2 lo = __floats2half2_rn(o[0], o[1]), hi = __floats2half2_rn(o[2], o[3]);
        ((uint2 *)p4)[px] = make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
        ((__half *)p1)[px] = __float2half(o[4]);
    }
};

// FP16 rounding of a value kept in an FP32 buffer (stage entry points).
__device__ __forceinline__ float round16(float v) { return __half2float(__float2half(v)); }

// Threshold state of one pair (the radix select's progress; the applied
// threshold's float bits).
struct SelState { uint32_t prefix, rank, tau2_bits, pad; };

// ---------------------------------------------------------------- pyramid

constexpr int PYR_TW = 62, PYR_TH = 16; // 2 x 62 + 3 = 127 input columns: one vertical job per thread
constexpr int PYR_SW = 2 * PYR_TW + 3, PYR_SH = 2 * PYR_TH + 3; // input columns / rows per tile

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
// Vertical pass straight from global memory: a job is one input column and
// one half of the tile's output rows (19 input rows, loaded together), its
// vertical sums go to LDS; in the horizontal pass the lanes take
// consecutive output columns, so stores write whole row segments.
// grid: (ceil(w2/62), ceil(h2/16), frames), 256 threads
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_pyr_down(PyrArgs a)
{
    constexpr int JOBS = 2 * PYR_SW, ROWS = PYR_TH / 2, IN = 2 * ROWS + 3;
    static_assert(JOBS <= 256, "one vertical job per thread");
    constexpr int NE = (PYR_SW + 1) / 2, NO = PYR_SW / 2; // even / odd input columns
    // vertical sums kept by column parity: output column c needs even
    // columns c, c+1, c+2 and odd columns c, c+1, so lanes over c read
    // consecutive doubles (the odd array starts one double later to keep
    // the two arrays' banks apart)
    __shared__ double ve[PYR_TH][NE];
    __shared__ double vo[PYR_TH][NO + 1];
    const TIn *src = (const TIn *)a.src[blockIdx.z];
    TOut *dst = (TOut *)a.dst[blockIdx.z];
    const int ox0 = blockIdx.x * PYR_TW, oy0 = blockIdx.y * PYR_TH;
    const int sx0 = 2 * ox0 - 2, sy0 = 2 * oy0 - 2;
    const double k0 = 1.0 / 16, k1 = 4.0 / 16, k2 = 6.0 / 16;
    double f[IN];
    const int j = min((int)threadIdx.x, JOBS - 1);
    const int cj = j % PYR_SW, half = j / PYR_SW;
    {
        const int x = clampi(sx0 + cj, 0, a.w - 1);
#pragma unroll
        for (int i = 0; i < IN; ++i) {
            const int y = clampi(sy0 + 2 * ROWS * half + i, 0, a.h - 1);
            f[i] = ldd(src, (size_t)y * a.src_pitch + x) - (double)a.dc;
        }
    }
    if ((int)threadIdx.x < JOBS) {
        double *col = (cj & 1) ? &vo[0][1 + (cj >> 1)] : &ve[0][cj >> 1];
        const int stride = (cj & 1) ? NO + 1 : NE;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int b = 2 * r;
            col[(ROWS * half + r) * stride] =
                k0 * f[b] + k1 * f[b + 1] + k2 * f[b + 2] + k1 * f[b + 3] + k0 * f[b + 4];
        }
    }
    __syncthreads();
    // horizontal pass: lane = output column, rows (t >> 6) + 4 i
    const int c = threadIdx.x & 63, x = ox0 + c;
    if (c >= PYR_TW || x >= a.w2) return;
#pragma unroll
    for (int i = 0; i < PYR_TH / 4; ++i) {
        const int r = (threadIdx.x >> 6) + 4 * i, y = oy0 + r;
        if (y >= a.h2) break;
        double o = k0 * ve[r][c] + k1 * vo[r][1 + c] + k2 * ve[r][c + 1] + k1 * vo[r][2 + c] + k0 * ve[r][c + 2];
        if (a.round16) o = (double)round16((float)o);
        std_(dst, (size_t)y * a.dst_pitch + x, o);
    }
}

// ---------------------------------------------------------------- denoising pre-stage

constexpr int DN_TW = 64, DN_TH = 16, DN_MAXM = 2, DN_MAXB = 3;

struct DenoiseArgs {
    const void *src[2];
    int64_t src_pitch;
    float *dst[2];
    int32_t dst_pitch;
    int32_t h, w;
    float inv2sr2;                                       // 1 / (2 sigma_range^2)
    float ws[(2 * DN_MAXB + 1) * (2 * DN_MAXB + 1)];     // spatial weights exp(-|t|^2 / (2 sigma_space^2))
};

__device__ __forceinline__ void cswap(float &a, float &b)
{
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

// exact median of 9 (compare-exchange network, Devillard's median search)
__device__ __forceinline__ float median9(float p[9])
{
    cswap(p[1], p[2]); cswap(p[4], p[5]); cswap(p[7], p[8]);
    cswap(p[0], p[1]); cswap(p[3], p[4]); cswap(p[6], p[7]);
    cswap(p[1], p[2]); cswap(p[4], p[5]); cswap(p[7], p[8]);
    cswap(p[0], p[3]); cswap(p[5], p[8]); cswap(p[4], p[7]);
    cswap(p[3], p[6]); cswap(p[1], p[4]); cswap(p[2], p[5]);
    cswap(p[4], p[7]); cswap(p[4], p[2]); cswap(p[6], p[4]);
    cswap(p[4], p[2]);
    return p[4];
}

// Median of radius MR then bilateral of radius BR, replicate borders at both
// stages (the bilateral sees the median image extended by its edge pixels,
// exactly as filtering the whole median image would). Values stay in the
// input's grey levels.
// grid: (ceil(w/64), ceil(h/16), frames)
template <typename TIn, int MR, int BR>
__global__ __launch_bounds__(256) void k_denoise(DenoiseArgs a)
{
    constexpr int HALO = MR + BR;
    constexpr int RW = DN_TW + 2 * HALO, RH = DN_TH + 2 * HALO; // raw region
    constexpr int MW = DN_TW + 2 * BR, MH = DN_TH + 2 * BR;     // median region
    __shared__ float raw[RH][RW + 1];
    __shared__ float med[MH][MW + 1];
    const TIn *src = (const TIn *)a.src[blockIdx.z];
    const int x0 = blockIdx.x * DN_TW, y0 = blockIdx.y * DN_TH;
    const int xb = x0 - HALO, yb = y0 - HALO; // image position of raw[0][0]
    for (int i = threadIdx.x; i < RH * RW; i += 256) {
        const int r = i / RW, c = i - r * RW;
        raw[r][c] = ld(src, (size_t)clampi(yb + r, 0, a.h - 1) * a.src_pitch + clampi(xb + c, 0, a.w - 1));
    }
    __syncthreads();
    // median image at the clamped positions the bilateral window reaches;
    // an in-frame row r sits at raw row r - yb
    for (int i = threadIdx.x; i < MH * MW; i += 256) {
        const int r = i / MW, c = i - r * MW;
        const int cy = clampi(y0 - BR + r, 0, a.h - 1), cx = clampi(x0 - BR + c, 0, a.w - 1);
        float m;
        if (MR == 0) {
            m = raw[cy - yb][cx - xb];
        } else if (MR == 1) {
            float p[9];
#pragma unroll
            for (int u = -1; u <= 1; ++u)
#pragma unroll
                for (int v = -1; v <= 1; ++v)
                    p[(u + 1) * 3 + v + 1] = raw[clampi(cy + u, 0, a.h - 1) - yb][clampi(cx + v, 0, a.w - 1) - xb];
            m = median9(p);
        } else {
            constexpr int N = (2 * MR + 1) * (2 * MR + 1);
            float p[N];
            int k = 0;
#pragma unroll
            for (int u = -MR; u <= MR; ++u)
#pragma unroll
                for (int v = -MR; v <= MR; ++v) p[k++] = raw[clampi(cy + u, 0, a.h - 1) - yb][clampi(cx + v, 0, a.w - 1) - xb];
            // odd-even transposition sort (exact)
#pragma unroll
            for (int pass = 0; pass < N; ++pass)
#pragma unroll
                for (int q = pass & 1; q + 1 < N; q += 2) cswap(p[q], p[q + 1]);
            m = p[N / 2];
        }
        med[r][c] = m;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < DN_TH * DN_TW; i += 256) {
        const int r = i / DN_TW, c = i - r * DN_TW;
        const int y = y0 + r, x = x0 + c;
        if (y >= a.h || x >= a.w) continue;
        float o;
        if (BR == 0) {
            o = med[r][c];
        } else {
            const float ctr = med[r + BR][c + BR];
            float num = 0.f, den = 0.f;
#pragma unroll
            for (int u = 0; u <= 2 * BR; ++u)
#pragma unroll
                for (int v = 0; v <= 2 * BR; ++v) {
                    const float q = med[r + u][c + v], e = q - ctr;
                    const float wt = a.ws[u * (2 * DN_MAXB + 1) + v] * expf(-e * e * a.inv2sr2);
                    num += wt * q;
                    den += wt;
                }
            o = num / den;
        }
        a.dst[blockIdx.z][(size_t)y * a.dst_pitch + x] = o;
    }
}

// ---------------------------------------------------------------- polynomial expansion

constexpr int PE_TW = 64, PE_TH = 16, PE_MAXN = 3;

struct PolyArgs {
    const void *src[2];
    int64_t src_pitch;
    float dc;
    void *dst[2];       // planar: 5 float planes b_x, b_y, A_xx, A_yy, A_xy; packed: P4
    void *dst1[2];      // packed: P1 (A_xy)
    int64_t dplane;     // planar: elements between planes
    int32_t dpitch;
    int32_t h, w, n;    // n = poly_n / 2
    int32_t round16;    // planar: values rounded to FP16 precision
    int32_t packed;     // 1: Packed<TOut> layout (P4, P1); 0: 5 float planes
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
    // nullable (n >= 2 only): the next pyramid level of the same input,
    // h2 x w2 FP64 with row pitch pdst_pitch, written by the same launch
    // (the tile's input rows and columns cover its 5 x 5 footprints)
    double *pdst[2];
    int32_t pdst_pitch, h2, w2;
};

// The expansion's derivative filters cancel the (large) local mean of the
// image, so the fit runs in FP64 arithmetic; only the stored coefficients
// are rounded to the storage type.
// Vertical pass straight from global memory: a job (one per thread) is one
// input column and a quarter (8 rows) of the 64 x 32 tile's output rows, its
// 8 + 2N input rows loaded together; the three vertical sums go to LDS.
// Horizontal pass: lanes over the columns of a row, 4 rows per thread. The filters are symmetric or
// antisymmetric, so they run on sums and differences of mirrored taps.
// With pdst set, the launch also writes the next pyramid level from the
// same loaded columns: binomial rows of each job, then one output per thread
// (the taps and their order are those of the pyramid kernel, so the level
// is bitwise the same).
// grid: (ceil(cols/64), ceil(rows/32), frames), 512 threads; N = poly_n / 2
constexpr int PE_TH2 = 32;

// Symmetric (even) and antisymmetric (odd) 2N+1-tap kernels on a window x
// centred at x[N]: even = e[N] x[N] + sum_j e[N+j] (x[N+j] + x[N-j]),
// odd = sum_j o[N+j] (x[N+j] - x[N-j]).
template <int N>
__device__ __forceinline__ void sym_sums(const double *x, double *s, double *d)
{
#pragma unroll
    for (int j = 1; j <= N; ++j) {
        s[j] = x[N + j] + x[N - j];
        d[j] = x[N + j] - x[N - j];
    }
}

template <int N>
__device__ __forceinline__ double even_tap(const double *e, double x0, const double *s)
{
    double r = e[N] * x0;
#pragma unroll
    for (int j = 1; j <= N; ++j) r += e[N + j] * s[j];
    return r;
}

template <int N>
__device__ __forceinline__ double odd_tap(const double *o, const double *d)
{
    double r = o[N + 1] * d[1];
#pragma unroll
    for (int j = 2; j <= N; ++j) r += o[N + j] * d[j];
    return r;
}

constexpr int PE_THREADS = 512;

template <typename TIn, typename TOut, int N>
__global__ __launch_bounds__(PE_THREADS) void k_polyexp(PolyArgs a)
{
    // SW + 1 is odd for every N: the horizontal pass's lanes read 32 rows at
    // once without bank conflicts
    constexpr int SW = PE_TW + 2 * N, JOBS = 4 * SW, ROWS = PE_TH2 / 4, IN = ROWS + 2 * N;
    __shared__ double vr[3][PE_TH2][SW + 1];
    const TIn *src = (const TIn *)a.src[blockIdx.z];
    const int ox0 = blockIdx.x * PE_TW, oy0 = blockIdx.y * PE_TH2;
    // one job per thread: 4 SW jobs <= 512 threads for N <= 3
    static_assert(JOBS <= PE_THREADS, "one vertical job per thread");
    const int j = min((int)threadIdx.x, JOBS - 1);
    const int cj = j % SW, qr = j / SW;
    double f[IN];
    {
        const int x = clampi(ox0 - N + cj, 0, a.w - 1);
#pragma unroll
        for (int i = 0; i < IN; ++i) {
            const int y = clampi(oy0 - N + ROWS * qr + i, 0, a.h - 1);
            f[i] = ldd(src, (size_t)y * a.src_pitch + x) - (double)a.dc;
        }
    }
    // kv0, kv2 even, kv1 odd
    if ((int)threadIdx.x < JOBS) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            double sm[N + 1], df[N + 1];
            sym_sums<N>(&f[r], sm, df);
            vr[0][ROWS * qr + r][cj] = even_tap<N>(a.kv0, f[r + N], sm);
            vr[1][ROWS * qr + r][cj] = odd_tap<N>(a.kv1, df);
            vr[2][ROWS * qr + r][cj] = even_tap<N>(a.kv2, f[r + N], sm);
        }
    }
    // next pyramid level: this job's column cp (relative to input column
    // ox0 - 2) and pyramid rows oy0/2 + ROWS/2 qr + r, whose input rows
    // 2Y-2 .. 2Y+2 are f[2r + N - 2 ...]; the vertical sums wait in
    // registers until the expansion's horizontal pass has released vr
    constexpr int PH = PE_TH2 / 2, PWC = PE_TW / 2 + 3;
    const bool pyr = N >= 2 && a.pdst[0] != nullptr;
    const int cp = cj - (N - 2);
    const bool pjob = pyr && (int)threadIdx.x < JOBS && cp >= 0 && cp < PE_TW + 3;
    double pv[ROWS / 2];
    if constexpr (N >= 2) {
        const double k0 = 1.0 / 16, k1 = 4.0 / 16, k2 = 6.0 / 16;
#pragma unroll
        for (int r = 0; r < ROWS / 2; ++r) {
            const int b = 2 * r + N - 2;
            pv[r] = k0 * f[b] + k1 * f[b + 1] + k2 * f[b + 2] + k1 * f[b + 3] + k0 * f[b + 4];
        }
    }
    __syncthreads();
    // horizontal pass: lane = column, so LDS reads are consecutive doubles
    // and every store instruction writes whole row segments; thread t takes
    // rows (t >> 6) + 8 i of column t & 63
    const int c = threadIdx.x & 63, x = ox0 + c;
#pragma unroll
    for (int i = 0; i < PE_TH2 / 8; ++i) {
        const int r = (threadIdx.x >> 6) + 8 * i, y = oy0 + r;
        if (y > a.h || (y == a.h && !a.packed)) break;
        double sm[N + 1], df[N + 1];
        float o[5];
        sym_sums<N>(&vr[0][r][c], sm, df);
        o[0] = (float)odd_tap<N>(a.hx, df);
        o[2] = (float)even_tap<N>(a.hxx, vr[0][r][c + N], sm);
        sym_sums<N>(&vr[1][r][c], sm, df);
        o[1] = (float)even_tap<N>(a.hy, vr[1][r][c + N], sm);
        o[4] = (float)odd_tap<N>(a.hxy, df);
        sym_sums<N>(&vr[2][r][c], sm, df);
        o[3] = (float)even_tap<N>(a.hyy, vr[2][r][c + N], sm);
        const size_t px = (size_t)y * a.dpitch + x;
        if (a.packed) {
            if (x >= a.dpitch) continue;
            if (x >= a.w || y == a.h) {
                // packed planes: zero the row padding and the extra row below
                // the frame (the iteration kernel's bilinear corners may read
                // them with zero weight)
                const float z[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
                Packed<TOut>::store(a.dst[blockIdx.z], a.dst1[blockIdx.z], px, z);
            } else {
                Packed<TOut>::store(a.dst[blockIdx.z], a.dst1[blockIdx.z], px, o);
            }
        } else if (x < a.w) {
            for (int p = 0; p < 5; ++p)
                st((float *)a.dst[blockIdx.z], px + p * a.dplane, a.round16 ? round16(o[p]) : o[p]);
        }
    }
    if constexpr (N >= 2) {
        if (!pyr) return; // (uniform)
        // vertical sums by column parity as in the pyramid kernel, in vr's space
        static_assert(2 * PH * PWC <= 3 * PE_TH2 * (SW + 1), "pyramid sums fit in vr");
        static_assert(PH * (PE_TW / 2) == PE_THREADS, "one pyramid output per thread");
        double (*pe)[PWC] = (double (*)[PWC]) & vr[0][0][0];
        double (*po)[PWC] = pe + PH;
        __syncthreads(); // every read of vr done
        if (pjob) {
            double *col = (cp & 1) ? &po[0][1 + (cp >> 1)] : &pe[0][cp >> 1];
#pragma unroll
            for (int r = 0; r < ROWS / 2; ++r) col[(ROWS / 2 * qr + r) * PWC] = pv[r];
        }
        __syncthreads();
        const double k0 = 1.0 / 16, k1 = 4.0 / 16, k2 = 6.0 / 16;
        const int c = threadIdx.x & (PE_TW / 2 - 1), r = threadIdx.x / (PE_TW / 2);
        const int X = ox0 / 2 + c, Y = oy0 / 2 + r;
        if (X < a.w2 && Y < a.h2)
            a.pdst[blockIdx.z][(size_t)Y * a.pdst_pitch + X] =
                k0 * pe[r][c] + k1 * po[r][1 + c] + k2 * pe[r][c + 1] + k1 * po[r][2 + c] + k0 * pe[r][c + 2];
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

// |d|^2 as every kernel that thresholds or weights the flow magnitude computes it
__device__ __forceinline__ float mag2(float2 d) { return __fmaf_rn(d.x, d.x, d.y * d.y); }

struct IterArgs {
    const void *p4[2], *p1[2]; // packed expansions of prev [0] and next [1]
    int32_t rpitch;            // pixels per row of the packed planes
    int32_t h, w;
    int32_t prior;           // PRIOR_* (the kernel is specialised on it)
    const float2 *fin;       // prior flow (PLAIN: this level; UPSAMPLE: coarser level)
    int32_t fin_pitch, hc, wc;
    float2 *fout;
    int32_t fout_pitch;
    int32_t R;               // window half-width
    float eps;
    float *m2;               // nullable: epilogue writes |d|^2
    int32_t m2_pitch;
    // nullable: epilogue writes the pre-mask [|d|^2 > tau^2] (bits t2bits)
    // as bytes, pitch w, instead of |d|^2 (the absolute threshold is known
    // before the flow), and block 0 records t2bits in *st
    uint8_t *pre8;
    uint32_t t2bits;
    SelState *st;
};

__device__ __forceinline__ float bilerp(float p00, float p01, float p10, float p11, float fx, float fy)
{
    return (1.f - fy) * ((1.f - fx) * p00 + fx * p01) + fy * ((1.f - fx) * p10 + fx * p11);
}

// Buffer descriptors of one launch (uniform across the grid).
struct IterRes {
    __amdgpu_buffer_rsrc_t p4a, p1a, p4b, p1b, fin, fout;
};

// Loads that need nothing but the pixel position: prev's coefficients at x
// and the raw prior-flow samples (one vector, or the four coarse-grid
// neighbours when the prior is the upsampled coarser flow; those come from
// a tile of the coarser flow staged in LDS).
struct PxIn {
    float4 q1;   // b1x, b1y, a11, a22
    float a12;
    float2 p00, p01, p10, p11;
};

// The bilinear gather of next's coefficients around x + d~.
struct PxG {
    float4 v00, v01, v10, v11;
    float w00, w01, w10, w11;
    float fx, fy;
    float2 d;
};

template <typename TS, int PRIOR>
__device__ __forceinline__ PxIn load_in(const IterArgs &a, const IterRes &rs, int y, int x)
{
    using PK = Packed<TS>;
    PxIn r;
    const uint32_t c = (uint32_t)y * a.rpitch + x;
    r.q1 = PK::load4(rs.p4a, c);
    r.a12 = PK::load1(rs.p1a, c);
    if (PRIOR == PRIOR_PLAIN) r.p00 = bload2(rs.fin, ((uint32_t)y * a.fin_pitch + x) * 8u);
    return r;
}

template <int PRIOR>
__device__ __forceinline__ float2 prior_of(const IterArgs &a, const PxIn &in, int y, int x)
{
    if (PRIOR == PRIOR_ZERO) return make_float2(0.f, 0.f);
    if (PRIOR == PRIOR_PLAIN) return in.p00;
    // 2 x bilinear(coarse, x/2, y/2), the point clamped into the coarse grid
    // (half-integer coordinates: exact in FP32)
    const float fx = (x >> 1) < a.wc - 1 ? 0.5f * (x & 1) : 0.f;
    const float fy = (y >> 1) < a.hc - 1 ? 0.5f * (y & 1) : 0.f;
    return make_float2(2.f * bilerp(in.p00.x, in.p01.x, in.p10.x, in.p11.x, fx, fy),
                       2.f * bilerp(in.p00.y, in.p01.y, in.p10.y, in.p11.y, fx, fy));
}

// Sample point x + d~ kept as integer pixel + fraction: an absolute FP32
// coordinate near x = 2000 only resolves 1.2e-4 px, which the solve can
// amplify past 1e-3 px at sensitive pixels. Clamping into the frame follows
// the real-valued point (outside -> edge pixel, zero weight). A NaN prior
// clamps to the frame's left/top edge, so every load stays in bounds.
template <typename TS, int PRIOR>
__device__ __forceinline__ PxG issue_gather(const IterArgs &a, const IterRes &rs, const PxIn &in, int y, int x,
                                            float xlo, float xhi)
{
    using PK = Packed<TS>;
    PxG g;
    g.d = prior_of<PRIOR>(a, in, y, x);
    // clamping x + d~ into [0, w-1] is clamping d~ into [-x, w-1-x] (integer
    // bounds: exact); afterwards x0 = w-1 implies a zero fraction
    const float dxc = fminf(fmaxf(g.d.x, xlo), xhi);
    const float dyc = fminf(fmaxf(g.d.y, (float)-y), (float)(a.h - 1 - y));
    const float flx = floorf(dxc), fly = floorf(dyc);
    g.fx = dxc - flx;
    g.fy = dyc - fly;
    const uint32_t c00 = (uint32_t)(y + (int)fly) * a.rpitch + (uint32_t)(x + (int)flx);
    // corners (x0+1, y0+1) at +1 pixel / +1 row; at the right or bottom edge
    // they have zero weight and read the zeroed row padding, the next row's
    // first pixel or (past the last row) the descriptor's out-of-range zero
    const uint32_t row4 = (uint32_t)a.rpitch * PK::B4, row1 = (uint32_t)a.rpitch * PK::B1;
    const uint32_t o4 = c00 * PK::B4, o1 = c00 * PK::B1;
    g.v00 = PK::load4b(rs.p4b, o4, 0);
    g.v01 = PK::load4b(rs.p4b, o4 + PK::B4, 0);
    g.v10 = PK::load4b(rs.p4b, o4, row4);
    g.v11 = PK::load4b(rs.p4b, o4 + PK::B4, row4);
    g.w00 = PK::load1b(rs.p1b, o1, 0);
    g.w01 = PK::load1b(rs.p1b, o1 + PK::B1, 0);
    g.w10 = PK::load1b(rs.p1b, o1, row1);
    g.w11 = PK::load1b(rs.p1b, o1 + PK::B1, row1);
    return g;
}

// Per-pixel normal-equation terms G = A^T A (g11, g12, g22) and h = A^T db
// for the prior displacement d~, computed as 4 G and 4 h:
//   A  = (A1(x) + A2(x + d~)) / 2,  db = -(b2(x + d~) - b1(x)) / 2 + A d~.
__device__ __forceinline__ void update_terms(const PxIn &in, const PxG &g, float o[5])
{
    // bilinear weights once, then one multiply and three FMAs per channel
    const float gx = 1.f - g.fx, gy = 1.f - g.fy;
    const float w00 = gx * gy, w01 = g.fx * gy, w10 = gx * g.fy, w11 = g.fx * g.fy;
    auto bl = [&](float p00, float p01, float p10, float p11) {
        return __fmaf_rn(w11, p11, __fmaf_rn(w10, p10, __fmaf_rn(w01, p01, w00 * p00)));
    };
    const float b2x = bl(g.v00.x, g.v01.x, g.v10.x, g.v11.x);
    const float b2y = bl(g.v00.y, g.v01.y, g.v10.y, g.v11.y);
    const float c11 = bl(g.v00.z, g.v01.z, g.v10.z, g.v11.z);
    const float c22 = bl(g.v00.w, g.v01.w, g.v10.w, g.v11.w);
    const float c12 = bl(g.w00, g.w01, g.w10, g.w11);
    // 2A and 2 db: every term below is 4x the plain one (an exact power-of-two
    // scale), which the scale-free solve leaves unchanged bit for bit
    const float S11 = in.q1.z + c11, S22 = in.q1.w + c22, S12 = in.a12 + c12;
    const float ex = -(b2x - in.q1.x) + S11 * g.d.x + S12 * g.d.y;
    const float ey = -(b2y - in.q1.y) + S12 * g.d.x + S22 * g.d.y;
    o[0] = S11 * S11 + S12 * S12;
    o[1] = S12 * (S11 + S22);
    o[2] = S12 * S12 + S22 * S22;
    o[3] = S11 * ex + S12 * ey;
    o[4] = S12 * ex + S22 * ey;
}

// Solve of the pooled 2x2 system G d = h (g11, g12, g22, h1, h2):
// d = adj(G) h / max(det G, eps tr(G)^2), zero where tr G = 0.
__device__ __forceinline__ float2 solve2(float g11, float g12, float g22, float h1, float h2, float eps)
{
    const float tr = g11 + g22;
    if (tr == 0.f) return make_float2(0.f, 0.f);
    const float det = g11 * g22 - g12 * g12;
    const float inv = __builtin_amdgcn_rcpf(fmaxf(det, eps * tr * tr)); // v_rcp_f32: 1 ulp
    return make_float2((g22 * h1 - g12 * h2) * inv, (g11 * h2 - g12 * h1) * inv);
}

// Strip walker. A workgroup of 320 threads owns IT_TW output columns and a
// strip of rows [ys, ye) (ys a multiple of 8); it walks down in chunks of
// IT_CH computed rows:
//   1. per-pixel terms of the chunk's rows over IT_TW + 2R columns -> LDS;
//   2. horizontal window sums of those rows (task = channel, row, 8-column
//      segment) -> LDS;
//   3a. thread (channel, column) appends its 8 new horizontal sums to a
//      register ring and forms the vertical sums of one aligned group of 8
//      output rows -> LDS;
//   3b. the 2x2 solves of those 512 pixels (no barrier after it: the next
//      chunk's loads start while slower waves still solve).
// Computed rows start PRE rows above ys - R so that output groups sit at
// multiples of 8; every window sum is either taken directly (first of an
// 8-column segment / 8-row group) or slid by one from its neighbour, in a
// pattern fixed by absolute positions, so results do not depend on the
// strip height. The chunk loop is unrolled over the NPH ring phases, which
// makes every register-ring index a compile-time constant.
// Replicated borders: out-of-frame rows/columns take the edge pixel's terms.
constexpr int IT_CH = 8, IT_THREADS = 320, IT_HSP = IT_TW + 1;
// step 2 tasks: (channel, row, segment of IT_SEG columns), one per thread
constexpr int IT_NSEG = IT_THREADS / (5 * IT_CH), IT_SEG = IT_TW / IT_NSEG;
static_assert(IT_THREADS % (5 * IT_CH) == 0 && IT_TW % IT_NSEG == 0 && IT_THREADS >= 5 * IT_TW, "iteration layout");

template <int R> struct IterGeom {
    static constexpr int CW = IT_TW + 2 * R;                      // columns of per-pixel terms
    static constexpr int PRE = (IT_CH - (2 * R) % IT_CH) % IT_CH; // extra rows above ys - R
    static constexpr int J0 = (2 * R + PRE) / IT_CH;              // chunks before the first output group
    static constexpr int NPH = J0 + 1;                            // ring phases
    static constexpr int RING = IT_CH * NPH;                      // ring length (>= IT_CH + 2R)
    static constexpr int NR1 = (IT_CH * CW + IT_THREADS - 1) / IT_THREADS; // step-1 pixels per thread
    static constexpr int GH = 5 * IT_CH * CW;                     // floats of step-1 terms
    static constexpr int HN = 5 * IT_CH * IT_HSP;                 // floats of new horizontal sums
    static constexpr int VS = 5 * IT_CH * IT_TW;                  // floats of vertical sums
    // upsampled prior: pixel (y, x) sits at (y/2, x/2) of the coarser grid;
    // a chunk's CW columns and IT_CH rows touch at most UC x UR coarse
    // samples (bilinear neighbours included), staged in LDS (two buffers)
    static constexpr int UC = CW / 2 + 2, UR = IT_CH / 2 + 2, UT = UC * UR;
    static_assert(UT <= IT_THREADS, "one coarse sample per thread");
};

struct IterCtx {
    int x0, ys, ye, y_first, nch;
    int xb; // first coarse column of the staged prior tile
};

// Per-thread constants: the step-1 pixel slots (row, column in the chunk,
// clamped frame column).
template <int R> struct IterSlots {
    int rr[IterGeom<R>::NR1], cc[IterGeom<R>::NR1], xs[IterGeom<R>::NR1];
    bool live[IterGeom<R>::NR1];
};

// Thread t's sample of the coarser flow for the staged tile whose first
// coarse row is yb: tile entry t = (q, u) holds coarse pixel
// (min(yb + q, hc - 1), min(xb + u, wc - 1)). Recomputed per chunk rather
// than kept: registers are the iteration kernel's scarce resource.
template <int R>
__device__ __forceinline__ float2 up_sample(const IterArgs &a, const IterRes &rs, int yb, int xb, int t)
{
    const int q = t / IterGeom<R>::UC, u = t - q * IterGeom<R>::UC;
    const int row = min(yb + q, a.hc - 1), col = min(xb + u, a.wc - 1);
    return bload2(rs.fin, ((uint32_t)row * a.fin_pitch + col) * 8u);
}

// Whether step 1 issues the gathers of all of a thread's pixels before
// using any (one memory round trip per chunk; more registers).
constexpr bool iter_gather_all(int prior) { return prior != PRIOR_UPSAMPLE; }

// One chunk j (ring phase P = j mod NPH) of computed rows [y_first + 8 j, + 8).
template <typename TS, int R, int PRIOR, int P>
__device__ __forceinline__ void iter_chunk(const IterArgs &a, const IterRes &rs, float *lds, const IterCtx &cx, int j,
                                           const IterSlots<R> &sl, float (&ring)[IterGeom<R>::RING],
                                           PxIn (&pre)[IterGeom<R>::NR1])
{
    using G = IterGeom<R>;
    float *gh = lds;                                   // [5][IT_CH][CW]
    float *hn = lds + G::GH;                           // [5][IT_CH][IT_HSP]
    float *vsb = lds + G::GH + G::HN;                  // [5][IT_CH][IT_TW]
    float2 *up = (float2 *)(lds + G::GH + G::HN + G::VS); // [2][UT] coarse tiles (upsampled prior)
    const int t = threadIdx.x;
    const int cy = cx.y_first + IT_CH * j;
    const bool more = j + 1 < cx.nch;
    // 1. per-pixel terms of rows [cy, cy + IT_CH). The position-only loads
    //    of this chunk were issued during the previous one (pre). Every
    //    gather of the chunk is issued first, then the next chunk's loads,
    //    and only then is any of them used: one memory round trip per chunk.
    float2 tile_next = make_float2(0.f, 0.f);
    if constexpr (PRIOR == PRIOR_UPSAMPLE) {
        // the four coarse neighbours of each pixel from this chunk's tile
        const float2 *T = up + (j & 1) * G::UT;
        const int yb = clampi(cy, 0, a.h - 1) >> 1;
#pragma unroll
        for (int m = 0; m < G::NR1; ++m) {
            // the pixel's coarse position and its lower/right neighbours,
            // relative to the tile: rows within [0, UR) and columns within
            // [0, UC), since the chunk's rows and xs >= max(x0 - R, 0) span
            // at most IT_CH rows and CW columns
            const int y = clampi(cy + sl.rr[m], 0, a.h - 1);
            const int yc = min(y >> 1, a.hc - 1), y1 = min(yc + 1, a.hc - 1);
            const int xc = min(sl.xs[m] >> 1, a.wc - 1), x1 = min(xc + 1, a.wc - 1);
            const int r0 = (yc - yb) * G::UC, r1 = (y1 - yb) * G::UC;
            pre[m].p00 = T[r0 + xc - cx.xb];
            pre[m].p01 = T[r0 + x1 - cx.xb];
            pre[m].p10 = T[r1 + xc - cx.xb];
            pre[m].p11 = T[r1 + x1 - cx.xb];
        }
        if (more && t < G::UT) tile_next = up_sample<R>(a, rs, clampi(cy + IT_CH, 0, a.h - 1) >> 1, cx.xb, t);
    }
    PxIn cur[G::NR1];
    PxG g[G::NR1];
    if constexpr (iter_gather_all(PRIOR)) {
#pragma unroll
        for (int m = 0; m < G::NR1; ++m) {
            cur[m] = pre[m];
            g[m] = issue_gather<TS, PRIOR>(a, rs, cur[m], clampi(cy + sl.rr[m], 0, a.h - 1), sl.xs[m],
                                           -(float)sl.xs[m], (float)(a.w - 1 - sl.xs[m]));
        }
        if (more) {
#pragma unroll
            for (int m = 0; m < G::NR1; ++m)
                pre[m] = load_in<TS, PRIOR>(a, rs, clampi(cy + IT_CH + sl.rr[m], 0, a.h - 1), sl.xs[m]);
        }
#pragma unroll
        for (int m = 0; m < G::NR1; ++m) {
            if (sl.live[m]) {
                float o[5];
                update_terms(cur[m], g[m], o);
#pragma unroll
                for (int k = 0; k < 5; ++k) gh[(k * IT_CH + sl.rr[m]) * G::CW + sl.cc[m]] = o[k];
            }
        }
    } else {
        // one pixel's gathers in flight at a time (fewer registers)
#pragma unroll
        for (int m = 0; m < G::NR1; ++m) {
            cur[m] = pre[m];
            g[m] = issue_gather<TS, PRIOR>(a, rs, cur[m], clampi(cy + sl.rr[m], 0, a.h - 1), sl.xs[m],
                                           -(float)sl.xs[m], (float)(a.w - 1 - sl.xs[m]));
            if (more) pre[m] = load_in<TS, PRIOR>(a, rs, clampi(cy + IT_CH + sl.rr[m], 0, a.h - 1), sl.xs[m]);
            if (sl.live[m]) {
                float o[5];
                update_terms(cur[m], g[m], o);
#pragma unroll
                for (int k = 0; k < 5; ++k) gh[(k * IT_CH + sl.rr[m]) * G::CW + sl.cc[m]] = o[k];
            }
        }
    }
    __syncthreads();
    // the next chunk's coarse tile goes to the other buffer (last read in
    // step 1 of the previous chunk, two barriers ago)
    if constexpr (PRIOR == PRIOR_UPSAMPLE) {
        if (more && t < G::UT) up[((j + 1) & 1) * G::UT + t] = tile_next;
    }
    // 2. horizontal sums: task = (channel, row, IT_SEG-column segment)
    {
        const int k = t / (IT_CH * IT_NSEG), r = (t / IT_NSEG) % IT_CH, sg = t % IT_NSEG;
        const float *src = gh + (k * IT_CH + r) * G::CW + sg * IT_SEG;
        float v[IT_SEG + 2 * R];
#pragma unroll
        for (int q = 0; q < IT_SEG + 2 * R; ++q) v[q] = src[q];
        float *dst = hn + (k * IT_CH + r) * IT_HSP + sg * IT_SEG;
        float sum = 0.f;
#pragma unroll
        for (int u = 0; u <= 2 * R; ++u) sum += v[u];
        dst[0] = sum;
#pragma unroll
        for (int q = 1; q < IT_SEG; ++q) {
            sum = sum - v[q - 1] + v[q + 2 * R];
            dst[q] = sum;
        }
    }
    __syncthreads();
    // 3a. thread (channel k, column c): ring update, vertical sums of the group
    const int grp = j - G::J0; // output group: rows ys + 8 grp ... + 7
    const int k = t >> 6, c = t & 63;
    // threads beyond 5 x IT_TW (if any) have no column here
    const bool vt = IT_THREADS == 5 * IT_TW || t < 5 * IT_TW;
    if (vt) {
#pragma unroll
        for (int i = 0; i < IT_CH; ++i) ring[IT_CH * P + i] = hn[(k * IT_CH + i) * IT_HSP + c];
    }
    if (grp < 0) return; // (uniform) the ring is still filling
    if (vt) {
        // ring position of row (group start - R)
        constexpr int S0 = ((IT_CH * P - IT_CH * G::J0 + G::PRE) % G::RING + G::RING) % G::RING;
        float sum = 0.f;
#pragma unroll
        for (int u = 0; u <= 2 * R; ++u) sum += ring[(S0 + u) % G::RING];
        float *vs = vsb + k * IT_CH * IT_TW + c;
        vs[0] = sum;
#pragma unroll
        for (int i = 1; i < IT_CH; ++i) {
            sum = sum - ring[(S0 + i - 1) % G::RING] + ring[(S0 + i + 2 * R) % G::RING];
            vs[i * IT_TW] = sum;
        }
    }
    __syncthreads();
    // 3b. solves of the group's 512 pixels
    for (int px = t; px < IT_CH * IT_TW; px += IT_THREADS) {
        const int i = px >> 6, cc2 = px & 63;
        const int oy = cx.ys + IT_CH * grp + i, x = cx.x0 + cc2;
        if (oy < cx.ye && x < a.w) {
            const float *vv = vsb + i * IT_TW + cc2;
            const float2 d = solve2(vv[0], vv[IT_CH * IT_TW], vv[2 * IT_CH * IT_TW], vv[3 * IT_CH * IT_TW],
                                    vv[4 * IT_CH * IT_TW], a.eps);
            bstore2(rs.fout, ((uint32_t)oy * a.fout_pitch + x) * 8u, d);
            if (a.m2) a.m2[(size_t)oy * a.m2_pitch + x] = mag2(d);
            if (a.pre8) a.pre8[(size_t)oy * a.w + x] = __float_as_uint(mag2(d)) > a.t2bits ? 1 : 0;
        }
    }
    // no barrier: vs is next written by 3a of a later chunk, two barriers away
}

template <int R, int PRIOR> struct IterLds {
    static constexpr int FLOATS = IterGeom<R>::GH + IterGeom<R>::HN + IterGeom<R>::VS +
                                  (PRIOR == PRIOR_UPSAMPLE ? 4 * IterGeom<R>::UT : 0);
};

// One workgroup's strip: tile b (in launch order) of a level of `ntiles`
// tiles, nx per row of strips.
template <typename TS, int R, int PRIOR>
__device__ __forceinline__ void iter_tile(const IterArgs &a, int32_t strip, int32_t nx, int32_t ntiles, int b,
                                          float *lds)
{
    if (a.st && b == 0 && threadIdx.x == 0) a.st->tau2_bits = a.t2bits;
    using G = IterGeom<R>;
    // XCD-aware tile order: hardware hands workgroup b to XCD b % 8, so give
    // each XCD a contiguous run of tiles (neighbours share halo columns in L2)
    const int n8 = ntiles & ~7;
    if (b < n8) b = (b & 7) * (n8 >> 3) + (b >> 3);
    const int tx = b % nx, ty = b / nx;
    IterCtx cx;
    cx.x0 = tx * IT_TW;
    cx.ys = ty * strip;
    cx.ye = min(cx.ys + strip, a.h);
    cx.y_first = cx.ys - R - G::PRE;
    cx.nch = (cx.ye - cx.ys + IT_CH - 1) / IT_CH + G::J0;
    cx.xb = max(cx.x0 - R, 0) >> 1;
    const uint32_t npx = (uint32_t)(a.h + 1) * a.rpitch; // packed planes carry one zero row below the frame
    IterRes rs;
    rs.p4a = make_rsrc(a.p4[0], npx * Packed<TS>::B4);
    rs.p1a = make_rsrc(a.p1[0], npx * Packed<TS>::B1);
    rs.p4b = make_rsrc(a.p4[1], npx * Packed<TS>::B4);
    rs.p1b = make_rsrc(a.p1[1], npx * Packed<TS>::B1);
    rs.fin = make_rsrc(a.fin, PRIOR == PRIOR_UPSAMPLE ? (uint32_t)a.hc * a.fin_pitch * 8u
                                                      : (uint32_t)a.h * a.fin_pitch * 8u);
    rs.fout = make_rsrc(a.fout, (uint32_t)a.h * a.fout_pitch * 8u);
    // step-1 pixels of this thread (the same slots in every chunk)
    IterSlots<R> sl;
#pragma unroll
    for (int m = 0; m < G::NR1; ++m) {
        const int i = (int)threadIdx.x + IT_THREADS * m;
        sl.live[m] = i < IT_CH * G::CW;
        const int ic = sl.live[m] ? i : 0;
        sl.rr[m] = ic / G::CW;
        sl.cc[m] = ic - sl.rr[m] * G::CW;
        sl.xs[m] = clampi(cx.x0 - R + sl.cc[m], 0, a.w - 1);
    }
    float ring[G::RING];
#pragma unroll
    for (int i = 0; i < G::RING; ++i) ring[i] = 0.f;
    PxIn pre[G::NR1];
#pragma unroll
    for (int m = 0; m < G::NR1; ++m)
        pre[m] = load_in<TS, PRIOR>(a, rs, clampi(cx.y_first + sl.rr[m], 0, a.h - 1), sl.xs[m]);
    if constexpr (PRIOR == PRIOR_UPSAMPLE) {
        float2 *up = (float2 *)(lds + G::GH + G::HN + G::VS);
        if ((int)threadIdx.x < G::UT)
            up[threadIdx.x] = up_sample<R>(a, rs, clampi(cx.y_first, 0, a.h - 1) >> 1, cx.xb, (int)threadIdx.x);
        __syncthreads();
    }
    for (int j = 0; j < cx.nch; j += G::NPH) {
        iter_chunk<TS, R, PRIOR, 0>(a, rs, lds, cx, j, sl, ring, pre);
        if (G::NPH > 1 && j + 1 < cx.nch) iter_chunk<TS, R, PRIOR, 1 % G::NPH>(a, rs, lds, cx, j + 1, sl, ring, pre);
        if (G::NPH > 2 && j + 2 < cx.nch) iter_chunk<TS, R, PRIOR, 2 % G::NPH>(a, rs, lds, cx, j + 2, sl, ring, pre);
    }
}

template <typename TS, int R, int PRIOR>
__global__ __launch_bounds__(IT_THREADS) void k_iter(IterArgs a, int32_t strip, int32_t nx, int32_t ntiles)
{
    __shared__ __align__(16) float lds[IterLds<R, PRIOR>::FLOATS];
    iter_tile<TS, R, PRIOR>(a, strip, nx, ntiles, blockIdx.x, lds);
}

// Several pairs' launches of one level and iteration in one grid: pair i
// owns workgroups [tile0[i], tile0[i+1]), a run rounded up to a multiple of
// 8 so that each pair keeps the XCD-aware order (workgroups past a pair's
// own tiles exit at once). All pairs share the prior mode and window.
constexpr int IT_MULTI = 16;
struct IterMulti {
    IterArgs a[IT_MULTI];
    int32_t strip[IT_MULTI], nx[IT_MULTI], ntiles[IT_MULTI];
    int32_t tile0[IT_MULTI + 1];
    int32_t n;
};

template <typename TS, int R, int PRIOR>
__global__ __launch_bounds__(IT_THREADS) void k_iter_multi(IterMulti m)
{
    __shared__ __align__(16) float lds[IterLds<R, PRIOR>::FLOATS];
    int i = 0;
    while (i + 1 < m.n && (int)blockIdx.x >= m.tile0[i + 1]) ++i; // (uniform)
    const int b = (int)blockIdx.x - m.tile0[i];
    if (b >= m.ntiles[i]) return;
    iter_tile<TS, R, PRIOR>(m.a[i], m.strip[i], m.nx[i], m.ntiles[i], b, lds);
}

// ---------------------------------------------------------------- top-q select

// Radix select over the bit patterns of |d|^2 (non-negative floats order
// like their unsigned bits): three passes of 11, 11 and 10 bits from the top.
// state[0] = bit prefix found so far, state[1] = rank still sought among the
// values that share it (0 = the largest), state[2] = tau^2 bits when done.
constexpr int SEL_BINS = 2048;


// The global histogram is kept in SEL_COPIES copies, block b adding into
// copy b mod SEL_COPIES, so that a bin's atomics from a thousand blocks
// spread over several addresses; the pick sums the copies.
constexpr int SEL_COPIES = 8;

// Frame maxima of the saliency rule (max |d|, max |grad |d||, max S): each
// is kept in MAXSLOTS counters 256 bytes apart, block b raising counter
// b mod MAXSLOTS, so that the atomics of thousands of blocks spread over
// the L2 channels instead of queueing on one address; readers reduce the
// counters with one load per lane of a wave.
constexpr int MAXSLOTS = 64, MAXSLOT_STRIDE = 64, MAXSLOT_WORDS = MAXSLOTS * MAXSLOT_STRIDE;

__host__ __device__ constexpr int sel_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__host__ __device__ constexpr int sel_bits(int pass) { return pass == 2 ? 10 : 11; }

// maxs (nullable): 3 MAXSLOT_WORDS counter groups to clear
// hist: SEL_COPIES * SEL_BINS counters
__global__ __launch_bounds__(256) void k_sel_init(SelState *st, uint32_t *hist, uint32_t rank, uint32_t tau2_bits,
                                                  uint32_t *maxs)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->prefix = 0;
        st->rank = rank;
        st->tau2_bits = tau2_bits;
        st->pad = 0;
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < SEL_COPIES * SEL_BINS; i += gridDim.x * 256) hist[i] = 0;
    if (maxs && blockIdx.x == 0 && threadIdx.x < 3 * MAXSLOTS) maxs[threadIdx.x * MAXSLOT_STRIDE] = 0;
}

// One histogram pass: the next digit of the values that share the prefix
// found so far. Thread (tx, ty) of block (bx, by) reads 16 consecutive
// values of row 4 by + ty from column 16 (64 bx + tx) with all four loads in
// flight together (rows start 64-byte aligned: the pitch is a multiple of
// 64), and merges runs of equal bins before its LDS atomic, which matters
// for smooth fields whose neighbours share the top bits.
// grid: (ceil(w/1024), ceil(h/4)), 256 threads
__global__ __launch_bounds__(256) void k_sel_hist(const float *m2, int32_t pitch, int32_t h, int32_t w,
                                                  const SelState *st, uint32_t *hist, int32_t pass)
{
    __shared__ uint32_t lh[SEL_BINS];
    for (int i = threadIdx.x; i < SEL_BINS; i += 256) lh[i] = 0;
    const int shift = sel_shift(pass), nb = 1 << sel_bits(pass);
    const uint32_t prefix = st->prefix;
    const int hi = shift + sel_bits(pass);
    const int tx = threadIdx.x & 63, y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int x0 = (blockIdx.x * 64 + tx) * 16;
    const int n = y < h ? max(0, min(16, w - x0)) : 0;
    uint32_t v[16];
    const float *row = m2 + (size_t)min(y, h - 1) * pitch;
    if (n == 16) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 q = *(const float4 *)(row + x0 + 4 * k);
            v[4 * k] = __float_as_uint(q.x);
            v[4 * k + 1] = __float_as_uint(q.y);
            v[4 * k + 2] = __float_as_uint(q.z);
            v[4 * k + 3] = __float_as_uint(q.w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = k < n ? __float_as_uint(row[x0 + k]) : 0u;
    }
    __syncthreads();
    int cur = -1;
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k >= n || (pass > 0 && (v[k] >> hi) != prefix)) continue;
        const int bin = (int)((v[k] >> shift) & (uint32_t)(nb - 1));
        if (bin == cur) {
            ++cnt;
        } else {
            if (cnt) atomicAdd(&lh[cur], cnt);
            cur = bin;
            cnt = 1;
        }
    }
    if (cnt) atomicAdd(&lh[cur], cnt);
    __syncthreads();
    uint32_t *hc = hist + (size_t)((blockIdx.y * gridDim.x + blockIdx.x) % SEL_COPIES) * SEL_BINS;
    for (int i = threadIdx.x; i < nb; i += 256)
        if (lh[i]) atomicAdd(&hc[i], lh[i]);
}

// Picks the bin holding the sought rank from the finished histogram of a
// pass: thread t (of 256) covers bins [nb - per (t+1), nb - per t), so thread
// 0 holds the largest values; an exclusive scan of the per-thread counts
// (wave scans, then the four wave totals) gives each thread the number of
// values above its bins. Clears the bins it read for the next pass.
// grid: 1 block of 256 threads
template <int PASS>
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, uint32_t *hist)
{
    constexpr int pass = PASS, nb = 1 << sel_bits(PASS), per = nb / 256;
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t rank = st->rank, prefix0 = st->prefix;
    const int b_hi = nb - per * t - 1;
    uint32_t cnt[per];
    uint32_t sum = 0;
    // all per * SEL_COPIES loads in flight together
    uint32_t raw[per][SEL_COPIES];
#pragma unroll
    for (int j = 0; j < per; ++j)
#pragma unroll
        for (int k = 0; k < SEL_COPIES; ++k) raw[j][k] = hist[k * SEL_BINS + b_hi - j];
#pragma unroll
    for (int j = 0; j < per; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < SEL_COPIES; ++k) c += raw[j][k];
        cnt[j] = c;
        sum += c;
    }
    uint32_t inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t acc = inc - sum;
    for (int k = 0; k < wv; ++k) acc += wsum[k];
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
#pragma unroll
    for (int j = 0; j < per; ++j)
#pragma unroll
        for (int k = 0; k < SEL_COPIES; ++k) hist[k * SEL_BINS + b_hi - j] = 0;
}

// ---------------------------------------------------------------- threshold + dilation

constexpr int DIL_TW = 64, DIL_TH = 16, DIL_MAXR = 32, DIL_FASTR = 4;
static_assert(DIL_TW == 64, "one wave spans a tile row");

struct DilArgs {
    const float *m2; int32_t m2_pitch;
    const SelState *st;        // tau^2 bits live in st->tau2_bits
    // alternative sources of pre (saliency rule): when lab is set, pre(p) =
    // [lab(p) >= 0 and area(lab(p)) >= min_area]; else when pre8 is set,
    // pre(p) = pre8(p); both pitch w
    const int32_t *lab; const int32_t *area; int32_t min_area;
    const uint8_t *pre8;
    uint8_t *mask; int32_t mask_pitch;
    int32_t h, w, r;
    int8_t hw[2 * DIL_MAXR + 1]; // half-width of the structuring element on row offset u
};

// pre(y, x) = [|d|^2 > tau^2]; mask(y, x) = OR_{(u,v) in SE} pre(y+u, x+v),
// outside the frame counting as 0. Row pass: distance to the nearest set
// pixel within +-r on the same row; column pass: OR_u [dist(y+u) <= hw(u)].
// grid: (ceil(w/64), ceil(h/16))
// RF >= 0: the radius is RF (a.r == RF), so the tap loops unroll; RF < 0:
// any radius up to DIL_MAXR.
template <int RF>
__global__ __launch_bounds__(256) void k_dilate(DilArgs a)
{
    constexpr int SW = DIL_TW + 2 * DIL_MAXR, SH = DIL_TH + 2 * DIL_MAXR;
    __shared__ uint8_t pre[SH][SW];
    __shared__ uint8_t dist[SH][DIL_TW];
    const int r = RF >= 0 ? RF : a.r, sw = DIL_TW + 2 * r, sh = DIL_TH + 2 * r;
    const int ox0 = blockIdx.x * DIL_TW, oy0 = blockIdx.y * DIL_TH;
    const uint32_t t2 = a.lab || a.pre8 ? 0u : a.st->tau2_bits;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    auto pre_at = [&](int rr, int c) -> uint8_t {
        const int y = oy0 - r + rr, x = ox0 - r + c;
        if (y < 0 || y >= a.h || x < 0 || x >= a.w) return 0;
        const size_t q = (size_t)y * a.w + x;
        if (a.lab) {
            const int32_t l = a.lab[q];
            return l >= 0 && a.area[l] >= a.min_area ? 1 : 0;
        }
        if (a.pre8) return a.pre8[q];
        return __float_as_uint(a.m2[(size_t)y * a.m2_pitch + x]) > t2 ? 1 : 0;
    };
    if (r <= DIL_FASTR) {
        // small radius: every load of the thread is issued before the first
        // LDS store (rows ty + 4k, columns tx and, in the right halo, tx + 64)
        constexpr int LR = (DIL_TH + 2 * DIL_FASTR) / 4;
        uint8_t v0[LR], v1[LR];
#pragma unroll
        for (int k = 0; k < LR; ++k) {
            const int rr = ty + 4 * k;
            v0[k] = rr < sh ? pre_at(rr, tx) : 0;
            v1[k] = rr < sh && tx + 64 < sw ? pre_at(rr, tx + 64) : 0;
        }
#pragma unroll
        for (int k = 0; k < LR; ++k) {
            const int rr = ty + 4 * k;
            if (rr < sh) {
                pre[rr][tx] = v0[k];
                if (tx + 64 < sw) pre[rr][tx + 64] = v1[k];
            }
        }
    } else {
        for (int rr = ty; rr < sh; rr += 4)
            for (int c = tx; c < sw; c += 64) pre[rr][c] = pre_at(rr, c);
    }
    __syncthreads();
    for (int rr = ty; rr < sh; rr += 4) {
        const int c = tx;
        int d = r + 1;
#pragma unroll
        for (int v = -r; v <= r; ++v)
            if (pre[rr][c + r + v]) d = min(d, abs(v));
        dist[rr][c] = (uint8_t)d;
    }
    __syncthreads();
    for (int rr = ty; rr < DIL_TH; rr += 4) {
        const int c = tx;
        const int y = oy0 + rr, x = ox0 + c;
        if (y >= a.h || x >= a.w) continue;
        uint8_t m = 0;
#pragma unroll
        for (int u = -r; u <= r; ++u) m |= dist[rr + r + u][c] <= a.hw[u + r] ? 1 : 0;
        a.mask[(size_t)y * a.mask_pitch + x] = m;
    }
}

// Bit-parallel dilation for radii up to DB_MAXR: a 64-column tile row with
// a halo of r columns on each side is a 128-bit word from two wave ballots
// (bit k = column ox0 - r + k; pixels outside the frame are 0); the output
// row y is the OR over row offsets u of the word of row y + u dilated
// horizontally by the SE's half-width hw(u). Tile: 64 x 32 outputs.
constexpr int DB_TH = 32, DB_MAXR = 16;
typedef unsigned __int128 u128d;

template <int MODE> // 0: |d|^2 bits above tau^2 bits; 1: pre-mask bytes; 2: component labels and areas
__global__ __launch_bounds__(256) void k_dilate_bits(DilArgs a)
{
    __shared__ uint64_t rows[DB_TH + 2 * DB_MAXR][2];
    __shared__ uint64_t out[DB_TH];
    const int r = a.r, tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ox0 = blockIdx.x * DIL_TW - r, oy0 = blockIdx.y * DB_TH - r;
    const int nrows = DB_TH + 2 * r;
    const uint32_t t2 = MODE == 0 ? a.st->tau2_bits : 0u;
    // the decision at (y, x), loaded at clamped coordinates (always a valid
    // address, no branch, so every load of the thread is in flight before
    // the first ballot) and masked by `in`
    auto pre_at = [&](int y, int x, bool in) -> bool {
        const int yc = min(max(y, 0), a.h - 1), xc = min(max(x, 0), a.w - 1);
        bool v;
        if (MODE == 0) {
            v = __float_as_uint(a.m2[(size_t)yc * a.m2_pitch + xc]) > t2;
        } else if (MODE == 1) {
            v = a.pre8[(size_t)yc * a.w + xc] != 0;
        } else {
            const int32_t l = a.lab[(size_t)yc * a.w + xc];
            v = l >= 0 && a.area[l] >= a.min_area;
        }
        return v && in && y >= 0 && y < a.h && x >= 0 && x < a.w;
    };
    // wave ty takes rows ty + 4k, lane tx columns tx and tx + 64 (the latter
    // only in the right halo); out-of-tile rows are clamped and discarded
    const int nk = (nrows - ty + 3) / 4;
    constexpr int LR = (DB_TH + 2 * DB_MAXR) / 4;
    bool d0[LR], d1[LR];
#pragma unroll
    for (int k = 0; k < LR; ++k) {
        const int ly = ty + 4 * k;
        d0[k] = pre_at(oy0 + ly, ox0 + tx, k < nk);
        d1[k] = pre_at(oy0 + ly, ox0 + 64 + tx, k < nk && tx < 2 * r);
    }
#pragma unroll
    for (int k = 0; k < LR; ++k) {
        const int ly = ty + 4 * k;
        const uint64_t lo = __ballot(d0[k]), hi = __ballot(d1[k]);
        if (k < nk && tx == 0) {
            rows[ly][0] = lo;
            rows[ly][1] = hi;
        }
    }
    __syncthreads();
    if (ty == 0 && tx < DB_TH) {
        u128d m = 0;
        for (int u = -r; u <= r; ++u) {
            const int ly = tx + r + u;
            const u128d x = ((u128d)rows[ly][1] << 64) | rows[ly][0];
            u128d e = x;
            for (int q = 1; q <= a.hw[u + r]; ++q) e |= (x << q) | (x >> q);
            m |= e;
        }
        out[tx] = (uint64_t)(m >> r); // the tile's own 64 columns
    }
    __syncthreads();
    const int x = blockIdx.x * DIL_TW + tx;
    if (x >= a.w) return;
    for (int yy = ty; yy < DB_TH; yy += 4) {
        const int y = blockIdx.y * DB_TH + yy;
        if (y >= a.h) break;
        a.mask[(size_t)y * a.mask_pitch + x] = (uint8_t)((out[yy] >> tx) & 1);
    }
}

// Pre-mask dilation with wide loads (frame width a multiple of 8): a tile
// row's pre-mask bytes are read as 8-byte words, 12 per row covering columns
// bx*64 - 16 ... bx*64 + 79, and each word becomes 8 bits with one multiply
// (bytes are 0 or 1), so bit k of the row's 128-bit word is column
// bx*64 - 16 + k. Words outside the frame are 0 (a word lies wholly inside
// or outside since the width and the word columns are multiples of 8).
// Radius up to DB_MAXR; tile 64 x 32 outputs; grid as k_dilate_bits.
__global__ __launch_bounds__(256) void k_dilate_wide(DilArgs a)
{
    constexpr int WW = 12, MAXROWS = DB_TH + 2 * DB_MAXR, KW = (MAXROWS * WW + 255) / 256;
    __shared__ uint64_t rows[MAXROWS][2];
    __shared__ uint64_t out[DB_TH];
    const int r = a.r, t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int xw0 = blockIdx.x * DIL_TW - 16, oy0 = blockIdx.y * DB_TH - r;
    const int nrows = DB_TH + 2 * r, n = nrows * WW;
    uint8_t *rb = (uint8_t *)&rows[0][0];
    uint64_t v[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        // every load at a clamped, valid address (all in flight at once)
        const int e = t + 256 * k, ly = e / WW, sgi = e - ly * WW;
        const int y = oy0 + ly, x = xw0 + 8 * sgi;
        const bool ok = e < n && y >= 0 && y < a.h && x >= 0 && x < a.w;
        const int yc = min(max(y, 0), a.h - 1), xc = min(max(x, 0), a.w - 8);
        const uint64_t w8 = *(const uint64_t *)(a.pre8 + (size_t)yc * a.w + xc);
        v[k] = ok ? w8 : 0ull;
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int e = t + 256 * k, ly = e / WW, sgi = e - ly * WW;
        if (e < n) rb[ly * 16 + sgi] = (uint8_t)((v[k] * 0x0102040810204080ull) >> 56);
    }
    if (t < nrows) *(uint32_t *)(rb + t * 16 + WW) = 0u; // bytes 12..15 of each row
    __syncthreads();
    if (ty == 0 && tx < DB_TH) {
        u128d m = 0;
        for (int u = -r; u <= r; ++u) {
            const int ly = tx + r + u;
            const u128d x = ((u128d)rows[ly][1] << 64) | rows[ly][0];
            u128d e = x;
            for (int q = 1; q <= a.hw[u + r]; ++q) e |= (x << q) | (x >> q);
            m |= e;
        }
        out[tx] = (uint64_t)(m >> 16); // the tile's own 64 columns
    }
    __syncthreads();
    // 4 mask bytes per lane: 16 lanes per row, 16 rows per pass (w is a
    // multiple of 8 and the mask rows 4-byte aligned on this path)
    const int q = t & 15, x4 = blockIdx.x * DIL_TW + 4 * q;
    if (x4 >= a.w) return;
    for (int yy = t >> 4; yy < DB_TH; yy += 16) {
        const int y = blockIdx.y * DB_TH + yy;
        if (y >= a.h) break;
        const uint32_t b = (uint32_t)(out[yy] >> (4 * q)) & 15u;
        *(uint32_t *)(a.mask + (size_t)y * a.mask_pitch + x4) =
            (b & 1u) | ((b & 2u) << 7) | ((b & 4u) << 14) | ((b & 8u) << 21);
    }
}

// ---------------------------------------------------------------- saliency rule

// |d|^2 of a flow field (pitch w, interleaved x/y) into m2 (pitch m2_pitch).
// grid: (ceil(w/64), ceil(h/4)), 256 threads
__global__ __launch_bounds__(256) void k_mag2(const float2 *flow, int32_t h, int32_t w, float *m2, int32_t m2_pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < w && y < h) m2[(size_t)y * m2_pitch + x] = mag2(flow[(size_t)y * w + x]);
}

constexpr int SAL_TW = 64, SAL_TH = 32; // one block: 64 x 32 pixels, 8 per thread

struct SalArgs {
    const float *m2; int32_t m2_pitch;
    float *sal; int32_t sal_pitch; // S before normalisation by its maximum
    float *out; int32_t out_pitch; // nullable: S / max S
    uint32_t *maxs;                // counter groups of max M, max G, max S
    int32_t h, w;
    float wt;
};

// maximum of v over the block, then one atomic max per block into the
// block's counter of the group (non-negative floats order like their bits)
__device__ __forceinline__ void block_max_to(float v, uint32_t *group, float *red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        const int slot = (int)((blockIdx.y * gridDim.x + blockIdx.x) % MAXSLOTS);
        atomicMax(group + slot * MAXSLOT_STRIDE, __float_as_uint(m));
    }
}

// the group's maximum, in every lane of the calling wave
__device__ __forceinline__ float group_max(const uint32_t *group)
{
    float v = __uint_as_float(group[(threadIdx.x & 63) * MAXSLOT_STRIDE]);
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// M = |d| over the block's tile and a one-pixel halo, edges replicated
// (coordinates clamped to the frame), into LDS; the hardware square root
// (within 1 ulp). Every load of the thread is issued before the first LDS
// store. Thread (tx, ty) of 64 x 4 fills rows ty + 4k, columns tx and 64 + tx.
constexpr int SAL_LW = SAL_TW + 2, SAL_LH = SAL_TH + 2, SAL_LR = (SAL_LH + 3) / 4;

__device__ __forceinline__ void stage_mag(const SalArgs &a, float (*Ms)[SAL_LW], int tx, int ty)
{
    const int x0 = blockIdx.x * SAL_TW - 1, y0 = blockIdx.y * SAL_TH - 1;
    float v0[SAL_LR], v1[SAL_LR];
    const int xa = min(max(x0 + tx, 0), a.w - 1), xb = min(x0 + 64 + tx, a.w - 1);
#pragma unroll
    for (int k = 0; k < SAL_LR; ++k) {
        const int ly = min(ty + 4 * k, SAL_LH - 1);
        const float *row = a.m2 + (size_t)min(max(y0 + ly, 0), a.h - 1) * a.m2_pitch;
        v0[k] = row[xa];
        v1[k] = row[xb];
    }
#pragma unroll
    for (int k = 0; k < SAL_LR; ++k) {
        const int ly = ty + 4 * k;
        if (ly < SAL_LH) {
            Ms[ly][tx] = __builtin_amdgcn_sqrtf(v0[k]);
            if (tx < SAL_LW - 64) Ms[ly][64 + tx] = __builtin_amdgcn_sqrtf(v1[k]);
        }
    }
    __syncthreads();
}

// G = |grad M| by central differences at tile pixel (ly, lx), whose LDS
// cell is (ly + 1, lx + 1)
__device__ __forceinline__ float grad_mag(const float (*Ms)[SAL_LW], int ly, int lx)
{
    const float gx = 0.5f * (Ms[ly + 1][lx + 2] - Ms[ly + 1][lx]);
    const float gy = 0.5f * (Ms[ly + 2][lx + 1] - Ms[ly][lx + 1]);
    return __builtin_amdgcn_sqrtf(__fmaf_rn(gx, gx, gy * gy));
}

// pass 1: max M and max G. grid: (ceil(w/64), ceil(h/32)), 256 threads
__global__ __launch_bounds__(256) void k_sal_max(SalArgs a)
{
    __shared__ float Ms[SAL_LH][SAL_LW];
    __shared__ float red[2][4];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    stage_mag(a, Ms, tx, ty);
    const int x = blockIdx.x * SAL_TW + tx;
    float mM = 0.0f, mG = 0.0f;
#pragma unroll
    for (int k = 0; k < SAL_TH / 4; ++k) {
        const int ly = ty + 4 * k, y = blockIdx.y * SAL_TH + ly;
        if (x < a.w && y < a.h) {
            mM = fmaxf(mM, Ms[ly + 1][tx + 1]);
            mG = fmaxf(mG, grad_mag(Ms, ly, tx));
        }
    }
    block_max_to(mM, a.maxs, red[0]);
    block_max_to(mG, a.maxs + MAXSLOT_WORDS, red[1]);
}

// pass 2: S = wt M / max M + (1 - wt) G / max G (a term with a zero maximum
// contributes 0), stored before normalisation; max S. Same grid as pass 1.
__global__ __launch_bounds__(256) void k_sal(SalArgs a)
{
    __shared__ float Ms[SAL_LH][SAL_LW];
    __shared__ float red[4];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const float mM = group_max(a.maxs), mG = group_max(a.maxs + MAXSLOT_WORDS);
    const float cM = mM > 0.0f ? a.wt / mM : 0.0f, cG = mG > 0.0f ? (1.0f - a.wt) / mG : 0.0f;
    stage_mag(a, Ms, tx, ty);
    const int x = blockIdx.x * SAL_TW + tx;
    float mS = 0.0f;
#pragma unroll
    for (int k = 0; k < SAL_TH / 4; ++k) {
        const int ly = ty + 4 * k, y = blockIdx.y * SAL_TH + ly;
        if (x < a.w && y < a.h) {
            const float S = __fmaf_rn(cM, Ms[ly + 1][tx + 1], cG * grad_mag(Ms, ly, tx));
            a.sal[(size_t)y * a.sal_pitch + x] = S;
            mS = fmaxf(mS, S);
        }
    }
    block_max_to(mS, a.maxs + 2 * MAXSLOT_WORDS, red);
}

__device__ __forceinline__ float sal_norm(float S, float mS) { return mS > 0.0f ? S / mS : 0.0f; }

// normalised saliency out. grid: (ceil(w/64), ceil(h/4)), 256 threads
__global__ __launch_bounds__(256) void k_sal_norm(SalArgs a)
{
    const float mS = group_max(a.maxs + 2 * MAXSLOT_WORDS); // whole wave, before the bounds test
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < a.w && y < a.h) a.out[(size_t)y * a.out_pitch + x] = sal_norm(a.sal[(size_t)y * a.sal_pitch + x], mS);
}

// Threshold, opening and closing with the (2r+1)^2 square, all in LDS.
// Erosion takes the minimum and dilation the maximum over the part of the
// square inside the frame (separably: rows, then columns). The four
// operations widen the support by 4r, so a 64 x 32 tile loads a 4r halo.
// With the component stage on, the kernel then labels the tile's
// 8-connected components in LDS (the first pass of the labelling below).
constexpr int MO_TW = 64, MO_TH = 32, MO_MAXR = 2, MO_HALO = 4 * MO_MAXR;
static_assert(MO_TW == 64, "one wave spans a tile row; local indices split as (i >> 6, i & 63)");

struct MorphArgs {
    const float *sal; int32_t sal_pitch;
    const SelState *st;
    const uint32_t *maxs_S;  // counter group of max S
    int32_t top;     // 1: pre = [S > tau] (tau bits in st->tau2_bits); 0: pre = [S / max S > thresh]
    float thresh;
    int32_t h, w, r;
    // component stage (lab set): lab(p) = index y w + x of the smallest
    // pixel of p's component within its tile (-1 background); at that pixel
    // (the tile root) link(p) = p and area(p) = 0. All pitch-free h w int32.
    int32_t *lab, *link, *area;
    uint8_t *pre;    // without lab: the opened and closed mask (pitch w)
};

// Union-find on label links. Every link points to a smaller or equal index
// (L[x] <= x) and links only decrease (atomic minimum), so a find walks a
// strictly decreasing chain and a union retries with a strictly smaller
// root each time it loses a race. Finds halve paths (x -> grandparent);
// only roots are ever linked by a union, and a node that is not a root
// never becomes one again, so halving never touches a root.
template <int SCOPE>
__device__ __forceinline__ int32_t uf_load(const int32_t *L, int32_t x)
{
    return __hip_atomic_load(L + x, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ int32_t uf_find(int32_t *L, int32_t x)
{
    for (;;) {
        const int32_t p = uf_load<SCOPE>(L, x);
        if (p == x) return x;
        const int32_t g = uf_load<SCOPE>(L, p);
        if (g == p) return p;
        atomicMin(L + x, g);
        x = g;
    }
}

template <int SCOPE>
__device__ __forceinline__ void uf_union(int32_t *L, int32_t a, int32_t b)
{
    for (;;) {
        a = uf_find<SCOPE>(L, a);
        b = uf_find<SCOPE>(L, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicMin(L + b, a);
        if (old == b) return;
        b = old;
    }
}

// First and last column of the run of set bits of m that holds bit x.
__device__ __forceinline__ int run_start(uint64_t m, int x)
{
    const uint64_t below = ~m & ((1ull << x) - 1); // clear bits under x
    return below ? 64 - __clzll((long long)below) : 0;
}

__device__ __forceinline__ int run_end(uint64_t m, int x)
{
    const uint64_t above = x == 63 ? 0ull : ~m & ~((2ull << x) - 1); // clear bits over x
    return above ? __ffsll((long long)above) - 2 : 63;
}

// Bit-parallel tile morphology. A tile row with its halo (64 + 8R columns
// from ox0) is a 128-bit word, bit k = column ox0 + k; one lane holds one
// row. An erosion (dilation) of radius R is the AND (OR) of the word shifted
// by -R..R, then of the rows -R..R around it (neighbouring lanes). Cells
// outside the frame are set to the operation's identity (1 for erosion, 0
// for dilation) before each pass, which is what restricting the square to
// the frame means. Shifts bring garbage only into the outer R columns and
// rows of what was valid, which is exactly where the result stops being
// valid (operation k leaves rows and columns [(k+1) R, S - (k+1) R)).
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 shfl128(u128 v, int src)
{
    const uint64_t lo = __shfl((unsigned long long)(uint64_t)v, src, 64);
    const uint64_t hi = __shfl((unsigned long long)(uint64_t)(v >> 64), src, 64);
    return ((u128)hi << 64) | lo;
}

// bits [k0, k1] of a 128-bit word (empty when k1 < k0)
__device__ __forceinline__ u128 bit_range(int k0, int k1)
{
    if (k1 < k0) return 0;
    const u128 upto = k1 >= 127 ? ~(u128)0 : (((u128)1 << (k1 + 1)) - 1);
    return upto & ~(((u128)1 << k0) - 1);
}

template <int R, bool ERODE>
__device__ __forceinline__ u128 morph_pass(u128 x, u128 valid, int lane)
{
    x = ERODE ? (x | ~valid) : (x & valid);
    u128 e = x;
#pragma unroll
    for (int q = 1; q <= R; ++q) e = ERODE ? (e & (x << q) & (x >> q)) : (e | (x << q) | (x >> q));
    e = ERODE ? (e | ~valid) : (e & valid);
    u128 f = e;
#pragma unroll
    for (int q = 1; q <= R; ++q) {
        const u128 up = shfl128(e, max(lane - q, 0)), dn = shfl128(e, min(lane + q, 63));
        f = ERODE ? (f & up & dn) : (f | up | dn);
    }
    return f;
}

// grid: (ceil(w/64), ceil(h/32)), 256 threads as 64 columns x 4 rows
template <int R>
__global__ __launch_bounds__(256) void k_open_close(MorphArgs a)
{
    constexpr int HAL = 4 * R, SW = MO_TW + 2 * HAL, SH = MO_TH + 2 * HAL;
    static_assert(SH <= 64, "one lane per tile row");
    __shared__ uint64_t rows[SH][2];
    __shared__ int32_t lbl[MO_TH * MO_TW];
    __shared__ uint64_t rowmask[MO_TH];
    const int ox0 = blockIdx.x * MO_TW - HAL, oy0 = blockIdx.y * MO_TH - HAL;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const uint32_t tb = a.st->tau2_bits;
    const float mS = group_max(a.maxs_S);
    // threshold decisions, every load of the thread in flight before the
    // first ballot: wave ty takes rows ty + 4k, lane tx columns tx and tx + 64
    constexpr int LR = (SH + 3) / 4;
    bool d0[LR], d1[LR];
    auto decide = [&](int y, int x) -> bool {
        if (y < 0 || y >= a.h || x < 0 || x >= a.w) return false;
        const float S = a.sal[(size_t)y * a.sal_pitch + x];
        return a.top ? (__float_as_uint(S) > tb) : (sal_norm(S, mS) > a.thresh);
    };
#pragma unroll
    for (int k = 0; k < LR; ++k) {
        const int ly = ty + 4 * k;
        d0[k] = ly < SH && decide(oy0 + ly, ox0 + tx);
        d1[k] = ly < SH && tx + 64 < SW && decide(oy0 + ly, ox0 + tx + 64);
    }
#pragma unroll
    for (int k = 0; k < LR; ++k) {
        const int ly = ty + 4 * k;
        const uint64_t lo = __ballot(d0[k]), hi = __ballot(d1[k]);
        if (ly < SH && tx == 0) {
            rows[ly][0] = lo;
            rows[ly][1] = hi;
        }
    }
    __syncthreads();
    const int ty0 = blockIdx.y * MO_TH, tx0 = blockIdx.x * MO_TW;
    const int th = min(MO_TH, a.h - ty0), tw = min(MO_TW, a.w - tx0);
    if (ty == 0) {
        // wave 0, lane = tile row with halo: erode, dilate (opening), dilate,
        // erode (closing)
        const int ly = min(tx, SH - 1), y = oy0 + ly;
        const u128 valid = y >= 0 && y < a.h ? bit_range(max(0, -ox0), min(SW - 1, a.w - 1 - ox0)) : 0;
        u128 x = ((u128)rows[ly][1] << 64) | rows[ly][0];
        if constexpr (R > 0) {
            x = morph_pass<R, true>(x, valid, tx);
            x = morph_pass<R, false>(x, valid, tx);
            x = morph_pass<R, false>(x, valid, tx);
            x = morph_pass<R, true>(x, valid, tx);
        }
        // the tile's own 64 columns, in-frame cells only
        const uint64_t m = (uint64_t)((x & valid) >> HAL);
        const int yt = tx - HAL;
        if (yt >= 0 && yt < MO_TH) rowmask[yt] = yt < th ? m : 0;
    }
    __syncthreads();
    if (!a.lab) {
        for (int y = ty; y < th; y += 4)
            if (tx < tw) a.pre[(size_t)(ty0 + y) * a.w + tx0 + tx] = (uint8_t)((rowmask[y] >> tx) & 1);
        return;
    }
    // Local labelling over the tile's in-frame part, by horizontal runs: a
    // wave holds one tile row, so the row's foreground is one ballot mask and
    // each pixel finds its run's first column with a bit scan. Union-find
    // nodes are runs (local index y 64 + first column); a run joins each run
    // of the row above that overlaps it or touches it diagonally, once, at
    // the leftmost column where that run begins to overlap (or at the run's
    // ends for the diagonal contacts).
    for (int y = ty; y < MO_TH; y += 4) {
        const uint64_t m = rowmask[y];
        lbl[y * MO_TW + tx] = (m >> tx) & 1 ? y * MO_TW + run_start(m, tx) : -1;
    }
    __syncthreads();
    for (int y = ty; y < th; y += 4) {
        const uint64_t m = rowmask[y];
        if (y == 0 || !((m >> tx) & 1)) continue;
        const uint64_t am = rowmask[y - 1];
        const int s = run_start(m, tx), e = run_end(m, tx);
        const int self = y * MO_TW + s, up = (y - 1) * MO_TW;
        if (((am >> tx) & 1) && (tx == s || !((am >> (tx - 1)) & 1)))
            uf_union<__HIP_MEMORY_SCOPE_WORKGROUP>(lbl, self, up + run_start(am, tx));
        if (tx == s && s > 0 && ((am >> (s - 1)) & 1))
            uf_union<__HIP_MEMORY_SCOPE_WORKGROUP>(lbl, self, up + run_start(am, s - 1));
        if (tx == e && e < MO_TW - 1 && ((am >> (e + 1)) & 1))
            uf_union<__HIP_MEMORY_SCOPE_WORKGROUP>(lbl, self, up + run_start(am, e + 1));
    }
    __syncthreads();
    if (tx >= tw) return;
    for (int y = ty; y < th; y += 4) {
        const uint64_t m = rowmask[y];
        const int32_t q = (ty0 + y) * a.w + tx0 + tx;
        int32_t out = -1;
        if ((m >> tx) & 1) {
            const int root = uf_find<__HIP_MEMORY_SCOPE_WORKGROUP>(lbl, y * MO_TW + run_start(m, tx));
            out = (ty0 + (root >> 6)) * a.w + tx0 + (root & 63);
            if (root == y * MO_TW + tx) {
                a.link[q] = q;
                a.area[q] = 0;
            }
        }
        a.lab[q] = out;
    }
}

// Second pass: joins the tile roots of 8-adjacent foreground pixels that lie
// in different tiles. Such a pair has its later pixel p on its tile's top
// row (N, NW, NE cross), left column (W, NW cross) or right column (NE
// crosses). One block per tile, thread t: t < 64 top row (0, t); t < 95
// left column (t - 63, 0); t < 126 right column (t - 94, 63). A contact is
// joined once, by the first pixel of a run of same-label pixels along the
// border that touches it: p skips a neighbour that the previous pixel of
// its border line (left on the top row, above on the left column) also
// touches when that pixel carries the same label.
// grid: (ceil(w/64), ceil(h/32)), 128 threads
__global__ __launch_bounds__(128) void k_cc_border(const int32_t *lab, int32_t *link, int32_t h, int32_t w)
{
    const int t = threadIdx.x;
    int ty, tx;
    if (t < 64) {
        ty = 0;
        tx = t;
    } else if (t < 95) {
        ty = t - 63;
        tx = 0;
    } else if (t < 126) {
        ty = t - 94;
        tx = MO_TW - 1;
    } else {
        return;
    }
    const int y = blockIdx.y * MO_TH + ty, x = blockIdx.x * MO_TW + tx;
    if (y >= h || x >= w) return;
    const int32_t p = y * w + x;
    const int32_t lp = lab[p];
    if (lp < 0) return;
    // the previous pixel along this border line, in the same tile
    int32_t prev = -1;
    if (ty == 0 && tx > 0) prev = lab[p - 1];
    else if (tx == 0 && ty > 0) prev = lab[p - w];
    const bool same_prev = prev == lp;
    // labels of the cross-tile neighbours W, NW, N, NE (-1: none)
    const int dy[4] = {0, -1, -1, -1}, dx[4] = {-1, -1, 0, 1};
    int32_t lq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int qy = y + dy[k], qx = x + dx[k];
        const bool cross = qy >= 0 && qx >= 0 && qx < w &&
                           !(qy / MO_TH == (int)blockIdx.y && qx / MO_TW == (int)blockIdx.x);
        lq[k] = cross ? lab[qy * w + qx] : -1;
    }
    if (same_prev) {
        if (ty == 0 && tx > 0) {
            // the left pixel touches NW and N of p (its N and NE), and joins
            // the label of N, so NE is new only with another label
            if (lq[3] == lq[2]) lq[3] = -1;
            lq[1] = lq[2] = -1;
        } else if (tx == 0 && ty > 0) {
            // the pixel above touches NW of p (its W)
            if (lq[0] == lq[1]) lq[0] = -1;
            lq[1] = -1;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool seen = lq[k] < 0;
#pragma unroll
        for (int j = 0; j < k; ++j) seen |= lq[j] == lq[k];
        if (!seen) uf_union<__HIP_MEMORY_SCOPE_AGENT>(link, lp, lq[k]);
    }
}

// Third pass, one block per tile: counts the tile's pixels per tile root in
// LDS (one atomic per segment of equal labels along a tile row: a wave holds
// a row, a ballot marks where segments start), adds each count at the root
// of the whole component, and relabels every pixel with that root.
// grid: (ceil(w/64), ceil(h/32)), 256 threads as 64 columns x 4 rows
__global__ __launch_bounds__(256) void k_cc_compress(int32_t *lab, int32_t *link, int32_t *area, int32_t h,
                                                     int32_t w)
{
    __shared__ int32_t cnt[MO_TH * MO_TW];
    __shared__ int32_t groot[MO_TH * MO_TW];
    constexpr int PER = MO_TH / 4;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ty0 = blockIdx.y * MO_TH, tx0 = blockIdx.x * MO_TW;
    const int th = min(MO_TH, h - ty0), tw = min(MO_TW, w - tx0);
    const int32_t base = ty0 * w + tx0;
    const float inv_w = 1.0f / (float)w;
    int32_t l[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int y = ty + 4 * k;
        l[k] = y < th && tx < tw ? lab[base + y * w + tx] : -1;
    }
    for (int i = threadIdx.x; i < MO_TH * MO_TW; i += 256) cnt[i] = 0;
    __syncthreads();
    int16_t li[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        // the tile root lies in this tile: d = ry w + rx with ry < 32 and
        // rx < min(64, w); the float quotient lands within one of ry and is
        // corrected exactly
        const int32_t d = l[k] >= 0 ? l[k] - base : 0;
        const int32_t ry = (int32_t)((float)d * inv_w);
        const int32_t ry2 = ry - (ry * w > d ? 1 : 0) + ((ry + 1) * w <= d ? 1 : 0);
        li[k] = l[k] >= 0 ? (int16_t)(ry2 * MO_TW + (d - ry2 * w)) : (int16_t)-1;
        const int32_t left = __shfl_up(l[k], 1, 64);
        const bool head = l[k] >= 0 && (tx == 0 || left != l[k]);
        const uint64_t H = __ballot(head), F = __ballot(l[k] >= 0);
        if (head) {
            // the segment runs to the next head or the next background pixel
            const uint64_t after = tx == 63 ? 0ull : ~((2ull << tx) - 1);
            const uint64_t stop = (H | ~F) & after;
            const int end = stop ? __ffsll((long long)stop) - 1 : 64;
            atomicAdd(&cnt[li[k]], end - tx);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MO_TH * MO_TW; i += 256) {
        const int c = cnt[i];
        if (!c) continue;
        const int32_t g = uf_find<__HIP_MEMORY_SCOPE_AGENT>(link, base + (i >> 6) * w + (i & 63));
        groot[i] = g;
        atomicAdd(area + g, c);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (li[k] >= 0) lab[base + (ty + 4 * k) * w + tx] = groot[li[k]];
}

// ---------------------------------------------------------------- stabilisation

// Phase correlation of two frames (the registration of a frame to its
// predecessor): both frames are cut to the centred P x P window (P a power
// of two, at most PH_MAXP), multiplied by the separable Hann window and
// packed as one complex field z = a + i b, so one 2-D FFT transforms both.
// The 2-D FFT is a row FFT, a transpose and a row FFT, so the spectrum is
// held transposed (row kx, column ky). From Z(k) and Z(-k): A = Z + conj Z(-k)
// and B = -i (Z - conj Z(-k)) (twice the spectra of a and b); the cross
// power R = (B / |B|) conj(A / |A|) (0 where either is 0); its inverse FFT
// (rows, transpose, rows: back in the frames' orientation) peaks at the
// translation of b against a. The largest value (first in row-major order
// on ties) is found with packed (value, index) keys and an atomic maximum
// over spread counters.
constexpr int PH_MAXP = 2048, PH_SLOTS = 64, PH_SLOT_STRIDE = 32; // 64-bit counters 256 bytes apart

struct PhaseState { int32_t sy, sx; float peak; uint32_t valid; };

__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// twiddles tw[m] = exp(-2 pi i m / P) (m < P) and the Hann window
// hann[i] = (1 - cos(2 pi i / (P - 1))) / 2, in double, rounded to float;
// clears the argmax counters. grid: ceil(2P/256) blocks, 256 threads
__global__ __launch_bounds__(256) void k_ph_tables(float2 *tw, float *hann, unsigned long long *keys, int32_t P)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < P) {
        double sn, cs;
        sincospi(-2.0 * (double)i / (double)P, &sn, &cs);
        tw[i] = make_float2((float)cs, (float)sn);
    } else if (i < 2 * P) {
        const int j = i - P;
        hann[j] = (float)(0.5 - 0.5 * cospi(2.0 * (double)j / (double)(P - 1)));
    }
    if (blockIdx.x == 0 && threadIdx.x < PH_SLOTS) keys[threadIdx.x * PH_SLOT_STRIDE] = 0ull;
}

struct PhArgs {
    const void *a, *b; int64_t pitch_a, pitch_b; // the two frames (reference, moving)
    int32_t y0, x0, P;                           // the window
    const float *hann;
    float2 *z;                                   // P x P
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// v * (-i) forward, v * (+i) inverse
template <bool INV> __device__ __forceinline__ float2 mul_mi(float2 v)
{
    return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
}

// In-register DFT of R = 2, 4, 8 points, natural order in and out:
// X(k) = sum_r v(r) exp(-+2 pi i r k / R).
template <bool INV, int R> __device__ __forceinline__ void dft_small(float2 *v);

template <> __device__ __forceinline__ void dft_small<false, 2>(float2 *v)
{
    const float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}
template <> __device__ __forceinline__ void dft_small<true, 2>(float2 *v) { dft_small<false, 2>(v); }

template <bool INV> __device__ __forceinline__ void dft4(float2 *v)
{
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}
template <> __device__ __forceinline__ void dft_small<false, 4>(float2 *v) { dft4<false>(v); }
template <> __device__ __forceinline__ void dft_small<true, 4>(float2 *v) { dft4<true>(v); }

template <bool INV> __device__ __forceinline__ void dft8(float2 *v)
{
    float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    constexpr float c = 0.70710678118654752f;
    // o(k) * exp(-+2 pi i k / 8)
    const float2 o1 = INV ? make_float2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                          : make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    const float2 o2 = mul_mi<INV>(o[2]);
    const float2 o3 = INV ? make_float2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                          : make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}
template <> __device__ __forceinline__ void dft_small<false, 8>(float2 *v) { dft8<false>(v); }
template <> __device__ __forceinline__ void dft_small<true, 8>(float2 *v) { dft8<true>(v); }

// One radix-R Stockham step over an N-point sequence (Ns: the size of the
// sub-transforms already done): job j takes the R values j + r N/R, turns
// them by exp(-+2 pi i r k / (Ns R)) with k = j mod Ns (table entry
// r k N / (Ns R) of the full-circle table), transforms them in registers and
// stores them at (j - k) R + k + r Ns.
// LDS buffers are indexed with one float2 of padding after every 16, so
// the strided stores of the first steps spread over the banks
__device__ __forceinline__ int fpad(int i) { return i + (i >> 4); }

template <bool INV, int R>
__device__ __forceinline__ void fft_step(const float2 *src, bool src_lds, float2 *dst, bool dst_lds, int N, int Ns,
                                         const float2 *tw, float scale)
{
    const int stride = N / (Ns * R);
    for (int j = threadIdx.x; j < N / R; j += 256) {
        const int k = j & (Ns - 1);
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = j + r * (N / R);
            v[r] = src[src_lds ? fpad(i) : i];
        }
#pragma unroll
        for (int r = 1; r < R; ++r) {
            float2 t = tw[(r * k * stride) & (N - 1)];
            if (INV) t.y = -t.y;
            v[r] = cmul(v[r], t);
        }
        dft_small<INV, R>(v);
        const int d = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = d + r * Ns;
            dst[dst_lds ? fpad(i) : i] = make_float2(v[r].x * scale, v[r].y * scale);
        }
    }
}

// Row y of the packed windowed pair z = hann(y) hann(x) (a + i b), the
// frames read in their own element types: the registration's input, made
// on the fly by the first forward pass.
template <typename TA, typename TB> struct PackSrc {
    PhArgs g;
    int y;
    __device__ float2 operator()(int x) const
    {
        const float va = (float)((const TA *)g.a)[(size_t)(g.y0 + y) * g.pitch_a + g.x0 + x];
        const float vb = (float)((const TB *)g.b)[(size_t)(g.y0 + y) * g.pitch_b + g.x0 + x];
        const float wgt = g.hann[y] * g.hann[x];
        return make_float2(wgt * va, wgt * vb);
    }
};

// Row q of the normalised cross power spectrum, made on the fly by the first
// inverse pass from the transposed spectrum zt of z = a + i b: with Z(k) and
// M = Z(-k), A = Z + conj(M) = 2 F_a, B = -i (Z - conj(M)) = 2 F_b and
// R = B conj(A) / (|A| |B|) (0 where either vanishes), so the correlation
// peak sits at the shift of b against a.
struct CrossSrc {
    const float2 *zt;
    int q, P;
    __device__ float2 operator()(int x) const
    {
        const float2 Z = zt[(size_t)q * P + x];
        const float2 M = zt[(size_t)((P - q) & (P - 1)) * P + ((P - x) & (P - 1))];
        const float2 A = make_float2(Z.x + M.x, Z.y - M.y); // Z + conj(M)
        const float2 D = make_float2(Z.x - M.x, Z.y + M.y); // Z - conj(M)
        const float2 B = make_float2(D.y, -D.x);            // -i D
        const float na = __fmaf_rn(A.x, A.x, A.y * A.y), nb = __fmaf_rn(B.x, B.x, B.y * B.y);
        float2 r = make_float2(0.0f, 0.0f);
        if (na > 0.0f && nb > 0.0f) {
            const float sc = rsqrtf(na) * rsqrtf(nb);
            r = make_float2((B.x * A.x + B.y * A.y) * sc, (B.y * A.x - B.x * A.y) * sc);
        }
        return r;
    }
};

// One Stockham FFT per row of a P x P complex field (P a power of two):
// radix-8 steps then one radix-4 or radix-2 step, each step a pass through
// LDS (two P-point buffers), the first reading its input through `in`
// (PackSrc, CrossSrc, ColSrc: element x of the row, made on the fly) and the
// last writing the row to `row`; rid is the row's index in the field.
// INV: inverse with 1/P. LAST (inverse only): instead of storing the row,
// the real parts go to `surface` (nullable) and into the argmax keys.
// grid: P blocks, 256 threads, 2 fpad(P) + P float2 of dynamic LDS (two row
// buffers and the twiddle table)
template <bool INV, bool LAST, typename Src>
__device__ __forceinline__ void fft_row(const Src &in, float2 *row, int32_t P, const float2 *tw, float *surface,
                                        unsigned long long *keys, int rid)
{
    extern __shared__ float2 fsm[];
    const int lg = __ffs(P) - 1, n8 = lg / 3, rem = lg % 3;
    const int steps = n8 + (rem ? 1 : 0);
    const float sc = INV ? 1.0f / (float)P : 1.0f;
    const int buf = fpad(P); // padded buffer length
    // the twiddle table staged once per block after the two row buffers
    float2 *tws = fsm + 2 * buf;
    const float2 *src = row;
    bool src_lds = false;
    int Ns = 1;
    int st0 = 0;
    if (n8 > 0 && P / 8 <= 256 && steps > 1) {
        // the first radix-8 step needs no twiddles (Ns = 1): its row loads and
        // the table's loads go out together, and one barrier serves both
        constexpr int TWR = PH_MAXP / 256;
        float2 twv[TWR];
#pragma unroll
        for (int k = 0; k < TWR; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            if (i < P) twv[k] = tw[i];
        }
        const int j = threadIdx.x;
        if (j < P / 8) {
            float2 v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) v[r] = in(j + r * (P / 8));
            dft_small<INV, 8>(v);
#pragma unroll
            for (int r = 0; r < 8; ++r) fsm[fpad(j * 8 + r)] = v[r];
        }
#pragma unroll
        for (int k = 0; k < TWR; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            if (i < P) tws[i] = twv[k];
        }
        __syncthreads();
        src = fsm;
        src_lds = true;
        Ns = 8;
        st0 = 1;
    } else {
        for (int i = threadIdx.x; i < P; i += 256) tws[i] = tw[i];
        // the second row buffer holds the input row; step 0 writes the first
        for (int i = threadIdx.x; i < P; i += 256) fsm[buf + fpad(i)] = in(i);
        src = fsm + buf;
        src_lds = true;
        __syncthreads();
    }
    tw = tws;
    for (int st = st0; st < steps; ++st) {
        const bool last = st == steps - 1;
        float2 *dst = fsm + (st & 1) * buf;
        bool dst_lds = true;
        if (last && !LAST) {
            dst = row;
            dst_lds = false;
        }
        const float scale = last ? sc : 1.0f;
        if (st < n8) {
            fft_step<INV, 8>(src, src_lds, dst, dst_lds, P, Ns, tw, scale);
            Ns *= 8;
        } else if (rem == 2) {
            fft_step<INV, 4>(src, src_lds, dst, dst_lds, P, Ns, tw, scale);
            Ns *= 4;
        } else {
            fft_step<INV, 2>(src, src_lds, dst, dst_lds, P, Ns, tw, scale);
            Ns *= 2;
        }
        __syncthreads();
        src = dst;
        src_lds = dst_lds;
    }
    if (!LAST) return;
    unsigned long long best = 0ull;
    for (int i = threadIdx.x; i < P; i += 256) {
        const float v = src[src_lds ? fpad(i) : i].x;
        if (surface) surface[(size_t)rid * P + i] = v;
        const uint32_t b = __float_as_uint(v);
        const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u); // orders like the float
        const uint32_t idx = (uint32_t)(rid * P + i);
        const unsigned long long key = ((unsigned long long)ord << 32) | (0xFFFFFFFFu - idx);
        best = key > best ? key : best;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(best, o, 64);
        best = other > best ? other : best;
    }
    __shared__ unsigned long long red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int k = 1; k < 4; ++k) m = red[k] > m ? red[k] : m;
        atomicMax(keys + (rid % PH_SLOTS) * PH_SLOT_STRIDE, m);
    }
}

// The first forward pass over rows, its input packed from the two frames on
// the fly (PackSrc); output rows to g.z. grid and LDS as fft_row
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_fft_rows_pack(PhArgs g, const float2 *tw)
{
    fft_row<false, false>(PackSrc<TA, TB>{g, (int)blockIdx.x}, g.z + (size_t)blockIdx.x * g.P, g.P, tw, nullptr,
                          nullptr, (int)blockIdx.x);
}

// The first inverse pass over rows, its input the cross power made on the
// fly from the transposed spectrum zt (CrossSrc); output rows to rt.
// grid and LDS as fft_row
__global__ __launch_bounds__(256) void k_fft_rows_cross(const float2 *zt, float2 *rt, int32_t P, const float2 *tw)
{
    fft_row<true, false>(CrossSrc{zt, (int)blockIdx.x, P}, rt + (size_t)blockIdx.x * P, P, tw, nullptr, nullptr,
                         (int)blockIdx.x);
}

// Column q of m, for a row pass over m^T.
struct ColSrc {
    const float2 *m;
    int q, P;
    __device__ float2 operator()(int x) const { return m[(size_t)x * P + q]; }
};

// Row q of out = the row pass over column q of in (in^T's row q): a
// transpose and a row pass in one. Columns go to XCDs in contiguous runs so
// neighbouring columns share cache lines in one L2. grid and LDS as fft_row
template <bool INV, bool LAST>
__global__ __launch_bounds__(256) void k_fft_cols(const float2 *in, float2 *out, int32_t P, const float2 *tw,
                                                  float *surface, unsigned long long *keys)
{
    const uint32_t n = gridDim.x, n8 = n & ~7u;
    uint32_t q = blockIdx.x;
    if (q < n8) q = (q & 7u) * (n8 >> 3) + (q >> 3);
    fft_row<INV, LAST>(ColSrc{in, (int)q, P}, out + (size_t)q * P, P, tw, surface, keys, (int)q);
}

struct ApplyArgs {
    const void *src; int64_t pitch;    // the frame to move (its own element type)
    float *dst; int32_t dpitch;        // the registered frame, as floats
    const void *src2; int64_t pitch2;  // nullable: a frame copied unmoved, as floats,
    float *dst2;                       //   into dst2 (row pitch dpitch)
    int32_t h, w, P;
    const unsigned long long *keys;
    PhaseState *st;                    // nullable
};

// The shift from the argmax keys (every block decodes it), then
// dst(y, x) = src(y + sy, x + sx), coordinates clamped into the frame; block
// (0, 0) records the shift. P == 0: no estimate, zero shift. A thread
// writes 4 consecutive pixels of a row.
// grid: (ceil(w/256), ceil(h/4)), 256 threads
template <typename TS, typename TS2>
__global__ __launch_bounds__(256) void k_ph_apply(ApplyArgs a)
{
    const unsigned long long *keys = a.keys;
    const int P = a.P, h = a.h, w = a.w;
    PhaseState *st = a.st;
    int sy = 0, sx = 0;
    float peak = 0.0f;
    if (P > 0) {
        unsigned long long k = keys[(threadIdx.x & 63) * PH_SLOT_STRIDE];
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long other = __shfl_xor(k, o, 64);
            k = other > k ? other : k;
        }
        const uint32_t idx = 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull);
        const uint32_t ord = (uint32_t)(k >> 32);
        peak = __uint_as_float((ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord);
        const int py = (int)(idx / (uint32_t)P), px = (int)(idx % (uint32_t)P);
        sy = py >= P / 2 ? py - P : py;
        sx = px >= P / 2 ? px - P : px;
    }
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (st && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        st->sy = sy;
        st->sx = sx;
        st->peak = peak;
        st->valid = 1;
    }
    if (y >= h) return;
    const TS *src = (const TS *)a.src + (size_t)min(max(y + sy, 0), h - 1) * a.pitch;
    const TS2 *src2 = a.src2 ? (const TS2 *)a.src2 + (size_t)y * a.pitch2 : nullptr;
    const int x0 = blockIdx.x * 256 + (threadIdx.x & 63) * 4;
    float v[4], c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int xk = min(x0 + k, w - 1);
        v[k] = (float)src[min(max(xk + sx, 0), w - 1)];
        c[k] = src2 ? (float)src2[xk] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (x0 + k >= w) break;
        a.dst[(size_t)y * a.dpitch + x0 + k] = v[k];
        if (a.src2) a.dst2[(size_t)y * a.dpitch + x0 + k] = c[k];
    }
}

// Pre-mask bytes of the kept components: [lab(p) >= 0 and area(lab(p)) >=
// min_area], 4 pixels per thread with all loads in flight.
// grid: ceil(h w / 1024) blocks, 256 threads
__global__ __launch_bounds__(256) void k_cc_keep(const int32_t *lab, const int32_t *area, int32_t min_area,
                                                 int64_t n, uint8_t *pre)
{
    const int64_t b = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    int32_t l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) l[k] = b + k < n ? lab[b + k] : -1;
    int32_t ar[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ar[k] = l[k] >= 0 ? area[l[k]] : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (b + k < n) pre[b + k] = l[k] >= 0 && ar[k] >= min_area ? 1 : 0;
}

// ---------------------------------------------------------------- adjacent-frame ensemble

constexpr int ENS_MAX = 8;

struct EnsembleArgs {
    uint8_t *mask;               // current mask in, union out (pitch w)
    uint8_t *store;              // history slot that receives the current mask
    const uint8_t *prev[ENS_MAX]; // previous masks to join (n of them)
    int32_t n;
    int64_t count;               // h * w
};

// history slot <- mask; mask <- mask | prev[0] | ... | prev[n-1]
// (history slots start on 256-byte boundaries, so they share the mask's
// 16-byte alignment test)
// grid: ceil(count / 4096) blocks of 256 threads, 16 bytes per thread
__global__ __launch_bounds__(256) void k_ensemble(EnsembleArgs a)
{
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    // every previous mask is read before the slot is written: once the ring
    // is full the slot receiving this mask holds the oldest one still joined
    if (base + 16 <= a.count && ((uintptr_t)(a.mask + base) & 15) == 0) {
        const uint4 own = *(const uint4 *)(a.mask + base);
        uint4 m = own;
        for (int k = 0; k < a.n; ++k) {
            const uint4 q = *(const uint4 *)(a.prev[k] + base);
            m.x |= q.x;
            m.y |= q.y;
            m.z |= q.z;
            m.w |= q.w;
        }
        *(uint4 *)(a.store + base) = own;
        *(uint4 *)(a.mask + base) = m;
    } else {
        for (int64_t i = base; i < base + 16 && i < a.count; ++i) {
            const uint8_t own = a.mask[i];
            uint8_t m = own;
            for (int k = 0; k < a.n; ++k) m |= a.prev[k][i];
            a.store[i] = own;
            a.mask[i] = m;
        }
    }
}

} // namespace flowroi
