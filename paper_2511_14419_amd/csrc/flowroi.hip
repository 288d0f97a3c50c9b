// Host side of libflowroi: C ABI (include/flowroi.h), workspace planning and
// the launch sequence of the hot path on the caller's HIP stream.
//
// Sequence for one frame pair (FlowRoI Method: flow between adjacent frames,
// then thresholding and morphology; estimator: Farneback's two-frame
// polynomial expansion):
//   pyramid (both frames per launch) -> expansion per level (both frames per
//   launch) -> coarse-to-fine iterations (one launch each; the first launch
//   of every finer level upsamples the coarser flow on the fly, the last one
//   at full resolution also writes |d|^2) -> [top-q radix select] ->
//   threshold + dilation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "flowroi.h"
#include "kernels.h"

using namespace flowroi;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_LEVELS = 10;
constexpr int MAX_BATCH = 256;
// per-pair state slots at the start of every workspace: the threshold state
// of each pair, then the translation found by stabilisation
constexpr size_t HDR_BYTES = (sizeof(SelState) + sizeof(PhaseState)) * MAX_BATCH;

PhaseState *phase_slot(void *ws, int index)
{
    return (PhaseState *)((uint8_t *)ws + sizeof(SelState) * MAX_BATCH) + index;
}

// side of the square window the translation is estimated on: the largest
// power of two <= min(h, w, PH_MAXP), 0 when the frame is thinner than 2
int phase_size(int h, int w)
{
    const int m = std::min(std::min(h, w), PH_MAXP);
    if (m < 2) return 0;
    int P = 1;
    while (P * 2 <= m) P *= 2;
    return P;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int level_dim(int n, int l)
{
    for (int k = 0; k < l; ++k) n = (n + 1) / 2;
    return n;
}

float dc_of(roi_dtype d) { return d == ROI_U8 ? 128.0f : (d == ROI_U16 ? 2048.0f : 0.0f); }

size_t dtype_bytes(roi_dtype d) { return d == ROI_U8 ? 1 : (d == ROI_U16 ? 2 : 4); }

// Device buffers of one frame pair, as byte offsets from the pair's base.
struct Level {
    int h, w, pitch;  // pitch in elements, a multiple of 64
    size_t img[2];    // pyramid image of each frame (levels >= 1)
    size_t r4[2];     // packed expansion of each frame: (b_x, b_y, A_xx, A_yy) per pixel
    size_t r1[2];     // and A_xy per pixel
    size_t fa, fb;    // flow ping-pong (fb unused at level 0: the caller's buffer)
};

struct Plan {
    int L;
    bool fp16;
    size_t ts;        // storage bytes per expansion value
    size_t is;        // storage bytes per pyramid image value (FP64)
    Level lv[MAX_LEVELS];
    size_t den[2];    // level-0 frames as floats (pitch lv[0].pitch): denoised, or converted for stabilisation
    size_t al[2];     // registered level-0 frames (floats, pitch lv[0].pitch), when stabilising
    int ph_P;         // stabilisation window side (0: none)
    size_t ph_z, ph_t, ph_tw, ph_hann, ph_keys;
    size_t init_off;  // coarsest-level initial flow
    size_t m2_off;    // |d|^2 at full resolution, pitch lv[0].pitch
    size_t hist_off;  // radix-select histogram
    size_t area_off;  // component areas (h w int32), saliency rule only
    size_t max_off;   // saliency maxima counters, saliency rule only
    size_t bytes;
};

Plan make_plan(int h, int w, const roi_params *p)
{
    Plan pl{};
    pl.L = p->levels;
    pl.fp16 = (p->flags & ROI_FP16_STORAGE) != 0;
    pl.ts = pl.fp16 ? 2 : 4;
    pl.is = 8; // pyramid images stay FP64 in both variants (under 2 % of the traffic)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, ALIGN);
        return o;
    };
    for (int l = 0; l < pl.L; ++l) {
        Level &v = pl.lv[l];
        v.h = level_dim(h, l);
        v.w = level_dim(w, l);
        // at least one padding column: the iteration kernel's (x0 + 1) corner
        // at the right edge reads it (zero weight, zeroed by the expansion)
        v.pitch = (int)align_up((size_t)v.w + 1, 64);
        const size_t plane = (size_t)v.h * v.pitch;
        const size_t pplane = (size_t)(v.h + 1) * v.pitch; // packed planes: one zero row below the frame
        for (int f = 0; f < 2; ++f) {
            v.img[f] = l > 0 ? take(plane * pl.is) : 0;
            v.r4[f] = take(4 * pplane * pl.ts);
            v.r1[f] = take(pplane * pl.ts);
        }
        v.fa = take(plane * sizeof(float2));
        v.fb = l > 0 ? take(plane * sizeof(float2)) : 0;
    }
    const bool stab = (p->flags & ROI_STABILIZE) != 0;
    const size_t fplane = (size_t)pl.lv[0].h * pl.lv[0].pitch * sizeof(float);
    for (int f = 0; f < 2; ++f) {
        pl.den[f] = p->denoise || stab ? take(fplane) : 0;
        pl.al[f] = stab ? take(fplane) : 0;
    }
    pl.ph_P = stab ? phase_size(h, w) : 0;
    if (pl.ph_P > 0) {
        const size_t P = (size_t)pl.ph_P;
        pl.ph_z = take(P * P * sizeof(float2));
        pl.ph_t = take(P * P * sizeof(float2));
        pl.ph_tw = take(P * sizeof(float2));
        pl.ph_hann = take(P * sizeof(float));
        pl.ph_keys = take(PH_SLOTS * PH_SLOT_STRIDE * sizeof(unsigned long long));
    }
    const Level &c = pl.lv[pl.L - 1];
    pl.init_off = take((size_t)c.h * c.pitch * sizeof(float2));
    pl.m2_off = take((size_t)pl.lv[0].h * pl.lv[0].pitch * sizeof(float));
    pl.hist_off = take(SEL_COPIES * SEL_BINS * sizeof(uint32_t));
    pl.area_off = p->rule == ROI_RULE_SALIENCY ? take((size_t)h * w * sizeof(int32_t)) : 0;
    pl.max_off = p->rule == ROI_RULE_SALIENCY ? take(3 * MAXSLOT_WORDS * sizeof(uint32_t)) : 0;
    pl.bytes = off;
    return pl;
}

// ---------------------------------------------------------------- kernel timing

struct TimedLaunch {
    hipEvent_t e0, e1;
    int64_t px;
    double bytes;
    int32_t n; // launches inside the bracket
};

// An event used only for its timestamp: no system-scope fence when it is
// recorded (nothing reads memory through it), so the record does not write
// back and invalidate the caches between the launches it brackets.
static hipEvent_t timing_event()
{
    hipEvent_t e = nullptr;
    return hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess ? e : nullptr;
}

struct Timing {
    std::mutex mu;
    int mode = 0; // 0 off, 1 per launch, 2 per call
    int every = 1;         // mode 2 brackets every `every`-th call
    int64_t calls = 0;     // mode-2 calls seen since the last reset
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
    double done_ms = 0, done_bytes = 0;
    int64_t done_n = 0, done_px = 0;
    std::vector<double> rec_ms, rec_bytes;
    std::vector<int64_t> rec_px;

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        return timing_event();
    }
} g_timing;

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// ---------------------------------------------------------------- launch helpers

#define LAUNCH_CHECK()                                                                                  \
    do {                                                                                                \
        if (hipGetLastError() != hipSuccess) return ROI_EDEVICE;                                        \
    } while (0)

struct PolyConsts {
    int n;
    double kv0[7], kv1[7], kv2[7], hx[7], hy[7], hxy[7], hxx[7], hyy[7];
};

// Separable form of the weighted least-squares quadratic fit with Gaussian
// applicability a(t) = exp(-t^2 / (2 sigma^2)) on t = -n..n. With moments
// m0 = sum a, m2 = sum a t^2, m4 = sum a t^4 the normal equations decouple:
//   b_x = <x, f> / (m0 m2), b_y = <y, f> / (m0 m2), c_xy = <xy, f> / m2^2,
//   c_xx = <x^2 - m2/m0, f> / (m0 m4 - m2^2) (and c_yy likewise),
// every inner product being a separable correlation of f.
PolyConsts poly_consts(int poly_n, double sigma)
{
    PolyConsts c{};
    const int n = poly_n / 2;
    c.n = n;
    double a[7], m0 = 0, m2 = 0, m4 = 0;
    for (int t = -n; t <= n; ++t) {
        a[t + n] = std::exp(-(double)(t * t) / (2 * sigma * sigma));
        m0 += a[t + n];
        m2 += a[t + n] * t * t;
        m4 += a[t + n] * t * t * t * t;
    }
    const double r = m2 / m0, dxx = m0 * m4 - m2 * m2;
    for (int t = -n; t <= n; ++t) {
        const double at = a[t + n];
        c.kv0[t + n] = at;
        c.kv1[t + n] = (t * at);
        c.kv2[t + n] = ((t * t - r) * at);
        c.hx[t + n] = (t * at / (m0 * m2));
        c.hy[t + n] = (at / (m0 * m2));
        c.hxy[t + n] = (t * at / (2 * m2 * m2));
        c.hxx[t + n] = ((t * t - r) * at / dxx);
        c.hyy[t + n] = (at / dxx);
    }
    return c;
}

void fill_poly(PolyArgs &pa, const PolyConsts &c)
{
    pa.n = c.n;
    std::memcpy(pa.kv0, c.kv0, sizeof c.kv0);
    std::memcpy(pa.kv1, c.kv1, sizeof c.kv1);
    std::memcpy(pa.kv2, c.kv2, sizeof c.kv2);
    std::memcpy(pa.hx, c.hx, sizeof c.hx);
    std::memcpy(pa.hy, c.hy, sizeof c.hy);
    std::memcpy(pa.hxy, c.hxy, sizeof c.hxy);
    std::memcpy(pa.hxx, c.hxx, sizeof c.hxx);
    std::memcpy(pa.hyy, c.hyy, sizeof c.hyy);
}

template <typename TIn, typename TOut>
void launch_pyr(const PyrArgs &a, int frames, hipStream_t s)
{
    dim3 g((a.w2 + PYR_TW - 1) / PYR_TW, (a.h2 + PYR_TH - 1) / PYR_TH, frames);
    hipLaunchKernelGGL((k_pyr_down<TIn, TOut>), g, dim3(256), 0, s, a);
}

template <typename TIn, typename TOut>
void launch_poly(const PolyArgs &a, int frames, hipStream_t s)
{
    // packed output also covers the zero padding columns and the zero row below the frame
    const int cols = a.packed ? a.dpitch : a.w;
    dim3 g((cols + PE_TW - 1) / PE_TW, (a.h + (a.packed ? 1 : 0) + PE_TH2 - 1) / PE_TH2, frames);
    const dim3 b(PE_THREADS);
    if (a.n == 1) hipLaunchKernelGGL((k_polyexp<TIn, TOut, 1>), g, b, 0, s, a);
    else if (a.n == 2) hipLaunchKernelGGL((k_polyexp<TIn, TOut, 2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_polyexp<TIn, TOut, 3>), g, b, 0, s, a);
}

template <typename TOut>
void launch_pyr_raw(roi_dtype dt, const PyrArgs &a, int frames, hipStream_t s)
{
    if (dt == ROI_U8) launch_pyr<uint8_t, TOut>(a, frames, s);
    else if (dt == ROI_U16) launch_pyr<uint16_t, TOut>(a, frames, s);
    else launch_pyr<float, TOut>(a, frames, s);
}

template <typename TOut>
void launch_poly_raw(roi_dtype dt, const PolyArgs &a, int frames, hipStream_t s)
{
    if (dt == ROI_U8) launch_poly<uint8_t, TOut>(a, frames, s);
    else if (dt == ROI_U16) launch_poly<uint16_t, TOut>(a, frames, s);
    else launch_poly<float, TOut>(a, frames, s);
}

template <typename TIn, int MR>
void launch_denoise_b(const DenoiseArgs &a, int br, int frames, hipStream_t s)
{
    dim3 g((a.w + DN_TW - 1) / DN_TW, (a.h + DN_TH - 1) / DN_TH, frames);
    switch (br) {
    case 0: hipLaunchKernelGGL((k_denoise<TIn, MR, 0>), g, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_denoise<TIn, MR, 1>), g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_denoise<TIn, MR, 2>), g, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_denoise<TIn, MR, 3>), g, dim3(256), 0, s, a); break;
    }
}

template <typename TIn>
void launch_denoise_t(const DenoiseArgs &a, int mr, int br, int frames, hipStream_t s)
{
    if (mr == 0) launch_denoise_b<TIn, 0>(a, br, frames, s);
    else if (mr == 1) launch_denoise_b<TIn, 1>(a, br, frames, s);
    else launch_denoise_b<TIn, 2>(a, br, frames, s);
}

void fill_denoise(DenoiseArgs &a, const roi_params *p)
{
    const int br = p->bilateral_radius;
    a.inv2sr2 = br > 0 ? (float)(1.0 / (2.0 * (double)p->sigma_range * (double)p->sigma_range)) : 0.f;
    for (int u = -br; u <= br; ++u)
        for (int v = -br; v <= br; ++v)
            a.ws[(u + br) * (2 * DN_MAXB + 1) + (v + br)] =
                (float)std::exp(-(double)(u * u + v * v) / (2.0 * (double)p->sigma_space * (double)p->sigma_space));
}

roi_status launch_denoise(roi_dtype dt, const DenoiseArgs &a, const roi_params *p, int frames, hipStream_t s)
{
    if (dt == ROI_U8) launch_denoise_t<uint8_t>(a, p->median_radius, p->bilateral_radius, frames, s);
    else if (dt == ROI_U16) launch_denoise_t<uint16_t>(a, p->median_radius, p->bilateral_radius, frames, s);
    else launch_denoise_t<float>(a, p->median_radius, p->bilateral_radius, frames, s);
    LAUNCH_CHECK();
    return ROI_OK;
}

// Pyramid and expansions of `nf` (1 or 2) frames into expansion sets `set[]`.
// Buffers of one phase correlation: P (0: no estimate, zero shift), the
// two P x P complex fields, the tables and the argmax counters.
struct PhaseBufs {
    int P;
    float2 *z, *t, *tw;
    float *hann;
    unsigned long long *keys;
};


// One registration: `mov` (element type dmov, row pitch pmov) against `ref`
// (dref, pref); `out` (floats, row pitch opitch) receives mov moved back by
// the translation; `copy` (nullable; dcopy, pcopy) is written unmoved as
// floats into `copy_out` (row pitch opitch).
struct PhaseIO {
    const void *ref; roi_dtype dref; int64_t pref;
    const void *mov; roi_dtype dmov; int64_t pmov;
    float *out; int opitch;
    const void *copy; roi_dtype dcopy; int64_t pcopy;
    float *copy_out;
};

// The first forward row pass, packing the two frames as it reads them.
template <typename TA, typename TB>
void launch_pack2(const PhArgs &g, const float2 *tw, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_fft_rows_pack<TA, TB>), dim3(g.P), dim3(256), lds, s, g, tw);
}

template <typename TA>
void launch_pack(roi_dtype db, const PhArgs &g, const float2 *tw, size_t lds, hipStream_t s)
{
    if (db == ROI_U8) launch_pack2<TA, uint8_t>(g, tw, lds, s);
    else if (db == ROI_U16) launch_pack2<TA, uint16_t>(g, tw, lds, s);
    else launch_pack2<TA, float>(g, tw, lds, s);
}

template <typename TS>
void launch_apply2(roi_dtype d2, const ApplyArgs &a, dim3 g, hipStream_t s)
{
    if (d2 == ROI_U8) hipLaunchKernelGGL((k_ph_apply<TS, uint8_t>), g, dim3(256), 0, s, a);
    else if (d2 == ROI_U16) hipLaunchKernelGGL((k_ph_apply<TS, uint16_t>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_ph_apply<TS, float>), g, dim3(256), 0, s, a);
}

// Registration by phase correlation over the centred P x P window (see
// PhaseIO); the shift goes to *ph; `surface` (nullable, P x P floats)
// receives the correlation surface.
roi_status enqueue_phase(const PhaseBufs &b, const PhaseIO &io, int h, int w, PhaseState *ph, float *surface,
                         hipStream_t s)
{
    const int P = b.P;
    if (P > 0) {
        hipLaunchKernelGGL(k_ph_tables, dim3((2 * P + 255) / 256), dim3(256), 0, s, b.tw, b.hann, b.keys, P);
        PhArgs g{};
        g.a = io.ref;
        g.b = io.mov;
        g.pitch_a = io.pref;
        g.pitch_b = io.pmov;
        g.y0 = (h - P) / 2;
        g.x0 = (w - P) / 2;
        g.P = P;
        g.hann = b.hann;
        g.z = b.z;
        const size_t lds = (2 * (size_t)(P + P / 16) + P) * sizeof(float2); // two padded row buffers + twiddles
        const float2 *tw = (const float2 *)b.tw;
        // z = window (a + i b), packed on the fly and transformed along its
        // rows; then along the columns into t = Z^T (transposed as it goes)
        if (io.dref == ROI_U8) launch_pack<uint8_t>(io.dmov, g, tw, lds, s);
        else if (io.dref == ROI_U16) launch_pack<uint16_t>(io.dmov, g, tw, lds, s);
        else launch_pack<float>(io.dmov, g, tw, lds, s);
        hipLaunchKernelGGL((k_fft_cols<false, false>), dim3(P), dim3(256), lds, s, (const float2 *)b.z, b.t, P, tw,
                           (float *)nullptr, (unsigned long long *)nullptr);
        // the cross power made on the fly from t and inverse-transformed
        // along its rows into z; then inverse along the columns, the real
        // parts to the surface and the argmax
        hipLaunchKernelGGL(k_fft_rows_cross, dim3(P), dim3(256), lds, s, (const float2 *)b.t, b.z, P, tw);
        hipLaunchKernelGGL((k_fft_cols<true, true>), dim3(P), dim3(256), lds, s, (const float2 *)b.z, b.t, P, tw,
                           surface, b.keys);
    }
    ApplyArgs a{};
    a.src = io.mov;
    a.pitch = io.pmov;
    a.dst = io.out;
    a.dpitch = io.opitch;
    a.src2 = io.copy;
    a.pitch2 = io.pcopy;
    a.dst2 = io.copy_out;
    a.h = h;
    a.w = w;
    a.P = P;
    a.keys = b.keys;
    a.st = ph;
    const roi_dtype d2 = io.copy ? io.dcopy : ROI_F32;
    const dim3 g((w + 255) / 256, (h + 3) / 4);
    if (io.dmov == ROI_U8) launch_apply2<uint8_t>(d2, a, g, s);
    else if (io.dmov == ROI_U16) launch_apply2<uint16_t>(d2, a, g, s);
    else launch_apply2<float>(d2, a, g, s);
    LAUNCH_CHECK();
    return ROI_OK;
}

PhaseBufs phase_bufs(const Plan &pl, uint8_t *base)
{
    PhaseBufs b{};
    b.P = pl.ph_P;
    if (b.P > 0) {
        b.z = (float2 *)(base + pl.ph_z);
        b.t = (float2 *)(base + pl.ph_t);
        b.tw = (float2 *)(base + pl.ph_tw);
        b.hann = (float *)(base + pl.ph_hann);
        b.keys = (unsigned long long *)(base + pl.ph_keys);
    }
    return b;
}

// Level-0 inputs of nf frames (denoised and/or registered as the flags say),
// then the pyramid and the expansions of every level into the sets set[f].
// Stabilisation registers the last frame: to the first one (nf == 2), or to
// the registered frame held in al[reg_set] (a stream; reg_set < 0 on its
// first frame, which is kept as it is). ph receives the translation.
roi_status enqueue_expand(const Plan &pl, uint8_t *base, int nf, const void *const *frames, int64_t pitch,
                          roi_dtype dt, const roi_params *p, const int *set, hipStream_t s, PhaseState *ph = nullptr,
                          int reg_set = -1)
{
    const PolyConsts pc = poly_consts(p->poly_n, p->poly_sigma);
    const void *lvl0[2] = {frames[0], nf > 1 ? frames[1] : nullptr};
    roi_dtype dt0 = dt;
    int64_t pitch0 = pitch;
    if (p->denoise) {
        DenoiseArgs da{};
        fill_denoise(da, p);
        for (int f = 0; f < nf; ++f) {
            da.src[f] = frames[f];
            da.dst[f] = (float *)(base + pl.den[set[f]]);
            lvl0[f] = da.dst[f];
        }
        da.src_pitch = pitch;
        da.dst_pitch = pl.lv[0].pitch;
        da.h = pl.lv[0].h;
        da.w = pl.lv[0].w;
        roi_status st = launch_denoise(dt, da, p, nf, s);
        if (st != ROI_OK) return st;
        dt0 = ROI_F32; // denoised frames: floats in the input's grey levels
        pitch0 = pl.lv[0].pitch;
    }
    if (p->flags & ROI_STABILIZE) {
        // the frames as they stand here (raw, or denoised floats); the
        // registered frame and, for a pair, the first frame as floats are
        // written by the alignment kernel, so both level-0 inputs are floats
        const int h = pl.lv[0].h, w = pl.lv[0].w, fp = pl.lv[0].pitch;
        const int fn = set[nf - 1];
        PhaseIO io{};
        io.mov = lvl0[nf - 1];
        io.dmov = dt0;
        io.pmov = pitch0;
        if (nf == 2) {
            io.ref = lvl0[0];
            io.dref = dt0;
            io.pref = pitch0;
            if (!p->denoise) {
                io.copy = lvl0[0];
                io.dcopy = dt0;
                io.pcopy = pitch0;
                io.copy_out = (float *)(base + pl.den[set[0]]);
            }
        } else if (reg_set >= 0) {
            io.ref = base + pl.al[reg_set];
            io.dref = ROI_F32;
            io.pref = fp;
        }
        io.out = (float *)(base + pl.al[fn]);
        io.opitch = fp;
        PhaseBufs b = phase_bufs(pl, base);
        if (!io.ref) b.P = 0; // first frame of a stream: kept as it is
        roi_status st = enqueue_phase(b, io, h, w, ph, nullptr, s);
        if (st != ROI_OK) return st;
        if (nf == 2 && !p->denoise) lvl0[0] = base + pl.den[set[0]];
        lvl0[nf - 1] = io.out;
        dt0 = ROI_F32;
        pitch0 = fp;
    }
    const float dc0 = dc_of(dt); // the frame's DC constant, also for denoised frames
    // with poly_n >= 5 each expansion launch also writes the next pyramid
    // level (its tile holds the footprints); otherwise separate launches
    const bool fused_pyr = pc.n >= 2;
    for (int l = 1; l < pl.L && !fused_pyr; ++l) {
        const Level &src = pl.lv[l - 1], &dst = pl.lv[l];
        PyrArgs a{};
        for (int f = 0; f < nf; ++f) {
            a.src[f] = l == 1 ? lvl0[f] : (const void *)(base + src.img[set[f]]);
            a.dst[f] = base + dst.img[set[f]];
        }
        a.src_pitch = l == 1 ? pitch0 : src.pitch;
        a.dc = l == 1 ? dc0 : 0.0f;
        a.dst_pitch = dst.pitch;
        a.h = src.h;
        a.w = src.w;
        a.h2 = dst.h;
        a.w2 = dst.w;
        if (l == 1) launch_pyr_raw<double>(dt0, a, nf, s);
        else launch_pyr<double, double>(a, nf, s);
        LAUNCH_CHECK();
    }
    for (int l = 0; l < pl.L; ++l) {
        const Level &v = pl.lv[l];
        PolyArgs a{};
        fill_poly(a, pc);
        for (int f = 0; f < nf; ++f) {
            a.src[f] = l == 0 ? lvl0[f] : (const void *)(base + v.img[set[f]]);
            a.dst[f] = base + v.r4[set[f]];
            a.dst1[f] = base + v.r1[set[f]];
        }
        a.packed = 1;
        if (fused_pyr && l + 1 < pl.L) {
            const Level &nx = pl.lv[l + 1];
            for (int f = 0; f < nf; ++f) a.pdst[f] = (double *)(base + nx.img[set[f]]);
            a.pdst_pitch = nx.pitch;
            a.h2 = nx.h;
            a.w2 = nx.w;
        }
        a.src_pitch = l == 0 ? pitch0 : v.pitch;
        a.dc = l == 0 ? dc0 : 0.0f;
        a.dplane = (int64_t)v.h * v.pitch;
        a.dpitch = v.pitch;
        a.h = v.h;
        a.w = v.w;
        if (pl.fp16) {
            if (l == 0) launch_poly_raw<__half>(dt0, a, nf, s);
            else launch_poly<double, __half>(a, nf, s);
        } else {
            if (l == 0) launch_poly_raw<float>(dt0, a, nf, s);
            else launch_poly<double, float>(a, nf, s);
        }
        LAUNCH_CHECK();
    }
    return ROI_OK;
}

// ---------------------------------------------------------------- iteration launch + strip autotuner

// The strip height of the iteration kernel only changes how work is split
// (results are bitwise identical for every strip), so it is tuned per
// (level size, window, storage, prior mode) by timing the candidates on the real data
// the first time a shape is seen (each candidate run rewrites the same
// output). Captured launches and disabled tuning use the heuristic.
constexpr int STRIP_CANDIDATES[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256};
constexpr int N_STRIP_CANDIDATES = sizeof(STRIP_CANDIDATES) / sizeof(STRIP_CANDIDATES[0]);

struct TuneState {
    std::mutex mu;
    int mode = 1;        // 0 heuristic only, 1 tune on first use
    int forced = 0;      // > 0: every launch uses this strip
    std::map<std::tuple<int, int, int, int, int>, int> best;
} g_tune;

int heuristic_strip(int h, int w)
{
    // aim for >= 512 workgroups (2 per CU: measured best on 2048^2 and
    // 1024^2 levels, where more resident strips thrash the L1 cache)
    const int nx = (w + IT_TW - 1) / IT_TW;
    int strip = 256;
    while (strip > 8 && (long)nx * ((h + strip - 1) / strip) < 512) strip /= 2;
    return strip;
}

template <typename TS, int PRIOR>
void launch_iter_p(const IterArgs &a, int strip, hipStream_t s)
{
    const int nx = (a.w + IT_TW - 1) / IT_TW, ny = (a.h + strip - 1) / strip;
    const int nt = nx * ny;
    dim3 g(nt), b(IT_THREADS);
    switch (a.R) {
    case 0: hipLaunchKernelGGL((k_iter<TS, 0, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 1: hipLaunchKernelGGL((k_iter<TS, 1, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 2: hipLaunchKernelGGL((k_iter<TS, 2, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 3: hipLaunchKernelGGL((k_iter<TS, 3, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 4: hipLaunchKernelGGL((k_iter<TS, 4, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 5: hipLaunchKernelGGL((k_iter<TS, 5, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    case 6: hipLaunchKernelGGL((k_iter<TS, 6, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    default: hipLaunchKernelGGL((k_iter<TS, 7, PRIOR>), g, b, 0, s, a, strip, nx, nt); break;
    }
}

template <typename TS>
void launch_iter_t(const IterArgs &a, int strip, hipStream_t s)
{
    if (a.prior == PRIOR_ZERO) launch_iter_p<TS, PRIOR_ZERO>(a, strip, s);
    else if (a.prior == PRIOR_PLAIN) launch_iter_p<TS, PRIOR_PLAIN>(a, strip, s);
    else launch_iter_p<TS, PRIOR_UPSAMPLE>(a, strip, s);
}

void launch_iter_raw(const IterArgs &a, bool fp16, int strip, hipStream_t s)
{
    if (fp16) launch_iter_t<__half>(a, strip, s);
    else launch_iter_t<float>(a, strip, s);
}

// Algorithmic bytes of one iteration launch: both frames' expansion planes,
// the prior flow (none for a zero prior, a quarter per pixel when it is the
// upsampled coarser flow), the flow written and the optional |d|^2.
double iter_bytes(const IterArgs &a, bool fp16)
{
    const double px = (double)a.h * a.w;
    double b = px * 2 * 5 * (fp16 ? 2 : 4) + px * sizeof(float2);
    if (a.prior == PRIOR_PLAIN) b += px * sizeof(float2);
    if (a.prior == PRIOR_UPSAMPLE) b += (double)a.hc * a.wc * sizeof(float2);
    if (a.m2) b += px * sizeof(float);
    if (a.pre8) b += px;
    return b;
}

int choose_strip(const IterArgs &a, bool fp16, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tune.mu);
    if (g_tune.forced > 0) return g_tune.forced;
    const auto key = std::make_tuple(a.h, a.w, a.R, fp16 ? 1 : 0, a.prior);
    auto it = g_tune.best.find(key);
    if (it != g_tune.best.end()) return it->second;
    if (g_tune.mode == 0 || capturing(s)) return heuristic_strip(a.h, a.w);
    constexpr int NE = 2 * N_STRIP_CANDIDATES;
    hipEvent_t e[NE];
    int n = 0;
    while (n < NE && (e[n] = timing_event()) != nullptr) ++n;
    int best = heuristic_strip(a.h, a.w);
    if (n == NE) {
        float best_ms = 1e30f;
        for (int c = 0; c < N_STRIP_CANDIDATES; ++c) {
            const int strip = STRIP_CANDIDATES[c];
            launch_iter_raw(a, fp16, strip, s); // warm the caches / code object
            hipEventRecord(e[2 * c], s);
            launch_iter_raw(a, fp16, strip, s);
            hipEventRecord(e[2 * c + 1], s);
        }
        if (hipEventSynchronize(e[NE - 1]) == hipSuccess) {
            for (int c = 0; c < N_STRIP_CANDIDATES; ++c) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, e[2 * c], e[2 * c + 1]) == hipSuccess && ms < best_ms) {
                    best_ms = ms;
                    best = STRIP_CANDIDATES[c];
                }
            }
        }
    }
    for (int k = 0; k < n; ++k) hipEventDestroy(e[k]);
    g_tune.best[key] = best;
    return best;
}

// An open timing bracket: events recorded on `s` at open and close when the
// timing mode is `mode` and the stream is not being captured.
struct Bracket {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    int64_t px = 0;
    double bytes = 0;
    int32_t n = 0;

    void open(int mode, hipStream_t st)
    {
        s = st;
        {
            std::lock_guard<std::mutex> lk(g_timing.mu);
            if (g_timing.mode != mode || capturing(st)) return;
            if (mode == 2 && g_timing.calls++ % g_timing.every != 0) return;
            e0 = g_timing.get();
            e1 = g_timing.get();
        }
        if (e0 && e1) hipEventRecord(e0, s);
    }
    void close()
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        if (e0 && e1 && n > 0) {
            hipEventRecord(e1, s);
            g_timing.pending.push_back({e0, e1, px, bytes, n});
        } else {
            if (e0) g_timing.pool.push_back(e0);
            if (e1) g_timing.pool.push_back(e1);
        }
        e0 = e1 = nullptr;
    }
};

roi_status launch_iter(const IterArgs &a, bool fp16, hipStream_t s, Bracket *call)
{
    const int strip = choose_strip(a, fp16, s);
    Bracket one;
    one.open(1, s);
    launch_iter_raw(a, fp16, strip, s);
    const bool ok = hipGetLastError() == hipSuccess;
    one.px = (int64_t)a.h * a.w;
    one.bytes = iter_bytes(a, fp16);
    one.n = 1;
    one.close();
    if (call) {
        call->px += (int64_t)a.h * a.w;
        call->bytes += iter_bytes(a, fp16);
        call->n += 1;
    }
    return ok ? ROI_OK : ROI_EDEVICE;
}

// Several pairs' launches of one level and update, IT_MULTI pairs per grid
// (k_iter_multi). One strip height per grid: the tallest power of two up to
// 128 rows that still gives >= 512 workgroups (2 per CU) over the group.
// Taller strips would cut the halo re-reads further, but a workgroup walks
// its strip as a chain of dependent chunks, and 256-row chains in the grid's
// last partial round left most of the chip idle (16 lens streams: 4.4 ms
// per batch with a 256-row cap, 4.25 ms with this one).
int multi_strip(const IterArgs *as, int n)
{
    auto wgs = [&](int st) {
        long t = 0;
        for (int i = 0; i < n; ++i) t += (long)((as[i].w + IT_TW - 1) / IT_TW) * ((as[i].h + st - 1) / st);
        return t;
    };
    int strip = 128;
    while (strip > 8 && wgs(strip) < 512) strip /= 2;
    return strip;
}

static_assert(sizeof(IterMulti) <= 4096, "kernel argument size");

template <typename TS, int R, int PRIOR>
void launch_multi_r(const IterMulti &m, hipStream_t s)
{
    hipLaunchKernelGGL((k_iter_multi<TS, R, PRIOR>), dim3(m.tile0[m.n]), dim3(IT_THREADS), 0, s, m);
}

template <typename TS, int PRIOR>
void launch_multi_p(const IterMulti &m, int R, hipStream_t s)
{
    switch (R) {
    case 0: launch_multi_r<TS, 0, PRIOR>(m, s); break;
    case 1: launch_multi_r<TS, 1, PRIOR>(m, s); break;
    case 2: launch_multi_r<TS, 2, PRIOR>(m, s); break;
    case 3: launch_multi_r<TS, 3, PRIOR>(m, s); break;
    case 4: launch_multi_r<TS, 4, PRIOR>(m, s); break;
    case 5: launch_multi_r<TS, 5, PRIOR>(m, s); break;
    case 6: launch_multi_r<TS, 6, PRIOR>(m, s); break;
    default: launch_multi_r<TS, 7, PRIOR>(m, s); break;
    }
}

template <typename TS>
void launch_multi_t(const IterMulti &m, int R, int prior, hipStream_t s)
{
    if (prior == PRIOR_ZERO) launch_multi_p<TS, PRIOR_ZERO>(m, R, s);
    else if (prior == PRIOR_PLAIN) launch_multi_p<TS, PRIOR_PLAIN>(m, R, s);
    else launch_multi_p<TS, PRIOR_UPSAMPLE>(m, R, s);
}

// All arguments share the level index, update, prior mode and window.
roi_status launch_iter_multi(const std::vector<IterArgs> &as, bool fp16, hipStream_t s)
{
    for (size_t g0 = 0; g0 < as.size(); g0 += IT_MULTI) {
        IterMulti m{};
        m.n = (int32_t)std::min<size_t>(IT_MULTI, as.size() - g0);
        const int strip = multi_strip(&as[g0], m.n);
        int t = 0;
        for (int i = 0; i < m.n; ++i) {
            const IterArgs &a = as[g0 + i];
            m.a[i] = a;
            m.strip[i] = strip;
            m.nx[i] = (a.w + IT_TW - 1) / IT_TW;
            m.ntiles[i] = m.nx[i] * ((a.h + strip - 1) / strip);
            m.tile0[i] = t;
            t += (m.ntiles[i] + 7) & ~7;
        }
        m.tile0[m.n] = t;
        if (fp16) launch_multi_t<__half>(m, as[g0].R, as[g0].prior, s);
        else launch_multi_t<float>(m, as[g0].R, as[g0].prior, s);
        if (hipGetLastError() != hipSuccess) return ROI_EDEVICE;
    }
    return ROI_OK;
}

// Buffers of the stage from |d|^2 to the mask. m2 (pitch m2_pitch) holds
// |d|^2; under the saliency rule sal (h rows of sal_pitch floats), lab and
// area (h w int32 each) are scratch, and the component links reuse m2.
struct MaskBufs {
    float *m2;
    int m2_pitch;
    uint32_t *hist;
    float *sal;
    int sal_pitch;
    int32_t *lab;
    int32_t *area;
    uint32_t *maxs; // 3 MAXSLOT_WORDS counters: max M, max G, max S
    bool pre8;      // m2 holds the pre-mask bytes (pitch w) of an absolute threshold, already recorded
};

void launch_select(const float *v, int pitch, int h, int w, const roi_params *p, SelState *slot, uint32_t *hist,
                   hipStream_t s)
{
    const size_t N = (size_t)h * w;
    const uint32_t rank = (uint32_t)std::floor((double)p->thresh * (double)N);
    hipLaunchKernelGGL(k_sel_init, dim3(8), dim3(256), 0, s, slot, hist, rank, 0u, (uint32_t *)nullptr);
    const dim3 g((w + 1023) / 1024, (h + 3) / 4);
    hipLaunchKernelGGL(k_sel_hist, g, dim3(256), 0, s, v, pitch, h, w, (const SelState *)slot, hist, 0);
    hipLaunchKernelGGL(k_sel_pick<0>, dim3(1), dim3(256), 0, s, slot, hist);
    hipLaunchKernelGGL(k_sel_hist, g, dim3(256), 0, s, v, pitch, h, w, (const SelState *)slot, hist, 1);
    hipLaunchKernelGGL(k_sel_pick<1>, dim3(1), dim3(256), 0, s, slot, hist);
    hipLaunchKernelGGL(k_sel_hist, g, dim3(256), 0, s, v, pitch, h, w, (const SelState *)slot, hist, 2);
    hipLaunchKernelGGL(k_sel_pick<2>, dim3(1), dim3(256), 0, s, slot, hist);
}

// Threshold (on |d| or, under the saliency rule, on the saliency after
// opening/closing and small-component removal) and dilation into mask.
// sal_out (nullable, pitch w) receives the normalised saliency.
roi_status enqueue_mask(const MaskBufs &mb, SelState *slot, int h, int w, const roi_params *p, uint8_t *mask,
                        float *sal_out, hipStream_t s)
{
    DilArgs d{};
    d.m2 = mb.m2;
    d.m2_pitch = mb.m2_pitch;
    d.st = slot;
    if (p->rule == ROI_RULE_MAGNITUDE && mb.pre8) {
        d.pre8 = (const uint8_t *)mb.m2;
    } else if (p->rule == ROI_RULE_MAGNITUDE) {
        if (p->thresh_mode == ROI_THRESH_ABS) {
            const float t2 = p->thresh * p->thresh;
            uint32_t bits;
            std::memcpy(&bits, &t2, 4);
            hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, slot, mb.hist, 0u, bits, (uint32_t *)nullptr);
        } else {
            launch_select(mb.m2, mb.m2_pitch, h, w, p, slot, mb.hist, s);
        }
        LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, slot, mb.hist, 0u, 0u, mb.maxs);
        SalArgs a{};
        a.m2 = mb.m2;
        a.m2_pitch = mb.m2_pitch;
        a.sal = mb.sal;
        a.sal_pitch = mb.sal_pitch;
        a.out = sal_out;
        a.out_pitch = w;
        a.maxs = mb.maxs;
        a.h = h;
        a.w = w;
        a.wt = p->sal_weight;
        const dim3 gs((w + SAL_TW - 1) / SAL_TW, (h + SAL_TH - 1) / SAL_TH), g4((w + 63) / 64, (h + 3) / 4);
        hipLaunchKernelGGL(k_sal_max, gs, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_sal, gs, dim3(256), 0, s, a);
        if (sal_out) hipLaunchKernelGGL(k_sal_norm, g4, dim3(256), 0, s, a);
        // the selection runs on S before normalisation: dividing by max S
        // keeps the order, so the same pixels are above the threshold
        if (p->thresh_mode == ROI_THRESH_TOP) launch_select(mb.sal, mb.sal_pitch, h, w, p, slot, mb.hist, s);
        const bool cc = p->min_area > 1;
        MorphArgs m{};
        m.sal = mb.sal;
        m.sal_pitch = mb.sal_pitch;
        m.st = slot;
        m.maxs_S = mb.maxs + 2 * MAXSLOT_WORDS;
        m.top = p->thresh_mode == ROI_THRESH_TOP;
        m.thresh = p->thresh;
        m.h = h;
        m.w = w;
        m.r = p->morph_radius;
        m.lab = cc ? mb.lab : nullptr;
        m.link = cc ? (int32_t *)mb.m2 : nullptr; // |d|^2 is no longer read
        m.area = cc ? mb.area : nullptr;
        // without the component stage the opened/closed mask goes to the lab
        // buffer's bytes (other tiles are still reading S from sal)
        m.pre = cc ? nullptr : (uint8_t *)mb.lab;
        const dim3 gt((w + MO_TW - 1) / MO_TW, (h + MO_TH - 1) / MO_TH);
        if (m.r == 0)
            hipLaunchKernelGGL(k_open_close<0>, gt, dim3(256), 0, s, m);
        else if (m.r == 1)
            hipLaunchKernelGGL(k_open_close<1>, gt, dim3(256), 0, s, m);
        else
            hipLaunchKernelGGL(k_open_close<2>, gt, dim3(256), 0, s, m);
        if (cc) {
            hipLaunchKernelGGL(k_cc_border, gt, dim3(128), 0, s, (const int32_t *)mb.lab, m.link, h, w);
            hipLaunchKernelGGL(k_cc_compress, gt, dim3(256), 0, s, mb.lab, m.link, mb.area, h, w);
            // the kept components as pre-mask bytes (into the saliency plane,
            // no longer read), so the dilation reads one byte per pixel
            const int64_t n = (int64_t)h * w;
            hipLaunchKernelGGL(k_cc_keep, dim3((unsigned)((n + 1023) / 1024)), dim3(256), 0, s,
                               (const int32_t *)mb.lab, (const int32_t *)mb.area, p->min_area, n, (uint8_t *)mb.sal);
            d.pre8 = (const uint8_t *)mb.sal;
        } else {
            d.pre8 = (const uint8_t *)mb.lab;
        }
        LAUNCH_CHECK();
    }
    d.mask = mask;
    d.mask_pitch = w;
    d.h = h;
    d.w = w;
    d.r = p->dilate_radius;
    for (int u = -d.r; u <= d.r; ++u) {
        int hw = d.r;
        if (p->se_shape == ROI_SE_DISC) {
            hw = 0;
            while ((hw + 1) * (hw + 1) + u * u <= d.r * d.r) ++hw;
        }
        d.hw[u + d.r] = (int8_t)hw;
    }
    if (d.r <= DB_MAXR) {
        const dim3 g((w + DIL_TW - 1) / DIL_TW, (h + DB_TH - 1) / DB_TH);
        if (d.lab) hipLaunchKernelGGL(k_dilate_bits<2>, g, dim3(256), 0, s, d);
        else if (d.pre8 && w % 8 == 0 && (uintptr_t)d.pre8 % 8 == 0 && (uintptr_t)d.mask % 4 == 0 &&
                 d.mask_pitch % 4 == 0)
            hipLaunchKernelGGL(k_dilate_wide, g, dim3(256), 0, s, d);
        else if (d.pre8) hipLaunchKernelGGL(k_dilate_bits<1>, g, dim3(256), 0, s, d);
        else hipLaunchKernelGGL(k_dilate_bits<0>, g, dim3(256), 0, s, d);
    } else {
        const dim3 g((w + DIL_TW - 1) / DIL_TW, (h + DIL_TH - 1) / DIL_TH);
        hipLaunchKernelGGL(k_dilate<-1>, g, dim3(256), 0, s, d);
    }
    LAUNCH_CHECK();
    return ROI_OK;
}

// The absolute threshold's |d|^2 bits (the pre-mask of the last update).
uint32_t abs_t2bits(const roi_params *p)
{
    const float t2 = p->thresh * p->thresh;
    uint32_t b = 0;
    std::memcpy(&b, &t2, 4);
    return b;
}

// An absolute threshold on |d| is known before the flow: the last update
// writes the pre-mask bytes and records the threshold itself.
bool pre8_mode_of(const roi_params *p) { return p->rule == ROI_RULE_MAGNITUDE && p->thresh_mode == ROI_THRESH_ABS; }

// Arguments of update `it` at level l, from expansion set s1 (prev) to s2
// (next). Flow buffers ping-pong between the level's fa and fb (the caller's
// flow at level 0) so that the last update of every level lands in fb / flow.
IterArgs make_iter_args(const Plan &pl, uint8_t *base, SelState *slot, int s1, int s2, int w, const roi_params *p,
                        float *flow, uint8_t *mask, int l, int it)
{
    const bool init = (p->flags & ROI_USE_INITIAL_FLOW) != 0;
    const int L = pl.L, n = p->iterations;
    const Level &v = pl.lv[l];
    float2 *X = (float2 *)(base + v.fa);
    float2 *Y = l == 0 ? (float2 *)flow : (float2 *)(base + v.fb);
    const int xp = v.pitch, yp = l == 0 ? w : v.pitch;
    auto out_of = [&](int k, int &pitch) -> float2 * {
        const bool toY = ((n - 1 - k) % 2) == 0;
        pitch = toY ? yp : xp;
        return toY ? Y : X;
    };
    IterArgs a{};
    a.p4[0] = base + v.r4[s1];
    a.p1[0] = base + v.r1[s1];
    a.p4[1] = base + v.r4[s2];
    a.p1[1] = base + v.r1[s2];
    a.rpitch = v.pitch;
    a.h = v.h;
    a.w = v.w;
    if (it > 0) {
        a.prior = PRIOR_PLAIN;
        a.fin = out_of(it - 1, a.fin_pitch);
    } else if (l < L - 1) {
        const Level &c = pl.lv[l + 1]; // its last update wrote fb
        a.prior = PRIOR_UPSAMPLE;
        a.fin = (const float2 *)(base + c.fb);
        a.fin_pitch = c.pitch;
        a.hc = c.h;
        a.wc = c.w;
    } else if (init) {
        a.prior = PRIOR_PLAIN;
        a.fin = (const float2 *)(base + pl.init_off);
        a.fin_pitch = pl.lv[L - 1].pitch;
    } else {
        a.prior = PRIOR_ZERO;
    }
    a.fout = out_of(it, a.fout_pitch);
    a.R = p->winsize / 2;
    a.eps = p->eps;
    if (l == 0 && it == n - 1 && mask) {
        if (pre8_mode_of(p)) {
            a.pre8 = base + pl.m2_off;
            a.t2bits = abs_t2bits(p);
            a.st = slot;
        } else {
            a.m2 = (float *)(base + pl.m2_off);
            a.m2_pitch = pl.lv[0].pitch;
        }
    }
    return a;
}

// The caller's initial flow, subsampled to the coarsest level.
void enqueue_init_flow(const Plan &pl, uint8_t *base, int h, int w, const roi_params *p, const float *flow,
                       hipStream_t s)
{
    if (!(p->flags & ROI_USE_INITIAL_FLOW)) return;
    const int L = pl.L;
    const Level &c = pl.lv[L - 1];
    InitArgs a{};
    a.src = (const float2 *)flow;
    a.src_pitch = w;
    a.h = h;
    a.w = w;
    a.dst = (float2 *)(base + pl.init_off);
    a.dst_pitch = c.pitch;
    a.hl = c.h;
    a.wl = c.w;
    a.stride = 1 << (L - 1);
    dim3 g((c.w + 63) / 64, (c.h + 3) / 4);
    hipLaunchKernelGGL(k_init_flow, g, dim3(256), 0, s, a);
}

// Threshold and dilation into `mask` after the last update.
roi_status enqueue_mask_stage(const Plan &pl, uint8_t *base, SelState *slot, int h, int w, const roi_params *p,
                              uint8_t *mask, hipStream_t s)
{
    MaskBufs mb{};
    mb.m2 = (float *)(base + pl.m2_off);
    mb.m2_pitch = pl.lv[0].pitch;
    mb.hist = (uint32_t *)(base + pl.hist_off);
    // the saliency rule's buffers reuse the level-0 flow scratch, free once
    // the last update has written the caller's flow
    mb.sal = (float *)(base + pl.lv[0].fa);
    mb.sal_pitch = pl.lv[0].pitch;
    mb.lab = (int32_t *)(base + pl.lv[0].fa + (size_t)pl.lv[0].h * pl.lv[0].pitch * sizeof(float));
    mb.area = (int32_t *)(base + pl.area_off);
    mb.maxs = (uint32_t *)(base + pl.max_off);
    mb.pre8 = pre8_mode_of(p);
    return enqueue_mask(mb, slot, h, w, p, mask, nullptr, s);
}

// Coarse-to-fine iterations from expansion set `s1` (prev) to `s2` (next),
// then the threshold and dilation into `mask` (skipped when mask is NULL).
roi_status enqueue_flow(const Plan &pl, uint8_t *base, SelState *slot, int s1, int s2, int h, int w,
                        const roi_params *p, float *flow, uint8_t *mask, hipStream_t s)
{
    enqueue_init_flow(pl, base, h, w, p, flow, s);
    LAUNCH_CHECK();
    Bracket call; // timing mode 2: the call's run of iteration launches
    call.open(2, s);
    for (int l = pl.L - 1; l >= 0; --l) {
        for (int it = 0; it < p->iterations; ++it) {
            const IterArgs a = make_iter_args(pl, base, slot, s1, s2, w, p, flow, mask, l, it);
            roi_status st = launch_iter(a, pl.fp16, s, &call);
            if (st != ROI_OK) {
                call.close();
                return st;
            }
        }
    }
    call.close();
    if (!mask) return ROI_OK;
    return enqueue_mask_stage(pl, base, slot, h, w, p, mask, s);
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

// ---------------------------------------------------------------- graphs for batched calls

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t tick = 0;
};

std::mutex g_graph_mu;
std::map<std::string, GraphEntry> g_graphs;
uint64_t g_tick = 0;
constexpr size_t MAX_GRAPHS = 32;

struct DeviceStreams {
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> ev;
};
std::map<int, DeviceStreams> g_dev_streams;

DeviceStreams *device_streams(int naux)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    DeviceStreams &ds = g_dev_streams[dev];
    if (!ds.cap && hipStreamCreateWithFlags(&ds.cap, hipStreamNonBlocking) != hipSuccess) return nullptr;
    while ((int)ds.aux.size() < naux) {
        hipStream_t a;
        if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) return nullptr;
        ds.aux.push_back(a);
    }
    while ((int)ds.ev.size() < 2 * naux + 2) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        ds.ev.push_back(e);
    }
    return &ds;
}

} // namespace

// ================================================================= C ABI

extern "C" {

void roi_default_params(roi_params *p)
{
    if (!p) return;
    p->levels = 3;
    p->winsize = 15;
    p->iterations = 3;
    p->poly_n = 5;
    p->poly_sigma = 1.1f;
    p->eps = 1e-3f;
    p->thresh_mode = ROI_THRESH_ABS;
    p->thresh = 1.0f;
    p->dilate_radius = 2;
    p->se_shape = ROI_SE_SQUARE;
    p->flags = 0;
    p->denoise = 0;
    p->median_radius = 1;
    p->bilateral_radius = 2;
    p->sigma_space = 1.5f;
    p->sigma_range = 20.0f;
    p->adjacent = 0;
    p->rule = ROI_RULE_MAGNITUDE;
    p->sal_weight = 0.7f;
    p->morph_radius = 1;
    p->min_area = 32;
}

// checks of the fields the mask stage reads
roi_status validate_mask_stage(const roi_params *p)
{
    if (p->rule != ROI_RULE_MAGNITUDE && p->rule != ROI_RULE_SALIENCY) return ROI_EINVAL;
    if (p->thresh_mode == ROI_THRESH_ABS) {
        if (!std::isfinite(p->thresh) || p->thresh < 0.0f) return ROI_EINVAL;
    } else if (p->thresh_mode == ROI_THRESH_TOP) {
        if (!(p->thresh > 0.0f && p->thresh < 1.0f)) return ROI_EINVAL;
    } else {
        return ROI_EINVAL;
    }
    if (p->dilate_radius < 0) return ROI_EINVAL;
    if (p->se_shape != ROI_SE_SQUARE && p->se_shape != ROI_SE_DISC) return ROI_EINVAL;
    if (p->dilate_radius > DIL_MAXR) return ROI_EUNSUPPORTED;
    if (p->rule == ROI_RULE_SALIENCY) {
        if (!(p->sal_weight >= 0.0f && p->sal_weight <= 1.0f)) return ROI_EINVAL;
        if (p->morph_radius < 0 || p->min_area < 0) return ROI_EINVAL;
        if (p->morph_radius > MO_MAXR) return ROI_EUNSUPPORTED;
    }
    return ROI_OK;
}

roi_status roi_validate(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p)
{
    if (!p || h < 0 || w < 0) return ROI_EINVAL;
    if (dtype != ROI_U8 && dtype != ROI_U16 && dtype != ROI_F32) return ROI_EINVAL;
    if (p->levels < 1 || p->levels > MAX_LEVELS) return ROI_EINVAL;
    if (p->winsize < 1 || p->winsize % 2 == 0) return ROI_EINVAL;
    if (p->iterations < 1 || p->iterations > 64) return ROI_EINVAL;
    if (p->poly_n != 3 && p->poly_n != 5 && p->poly_n != 7) return ROI_EINVAL;
    if (!finite_pos(p->poly_sigma) || !finite_pos(p->eps)) return ROI_EINVAL;
    const roi_status ms = validate_mask_stage(p);
    if (ms == ROI_EINVAL) return ms;
    if (p->flags & ~(uint32_t)(ROI_USE_INITIAL_FLOW | ROI_FP16_STORAGE | ROI_STABILIZE)) return ROI_EINVAL;
    if (p->denoise != 0 && p->denoise != 1) return ROI_EINVAL;
    if (p->adjacent < 0) return ROI_EINVAL;
    if (p->adjacent > ENS_MAX) return ROI_EUNSUPPORTED;
    if (p->denoise) {
        if (p->median_radius < 0 || p->bilateral_radius < 0) return ROI_EINVAL;
        if (p->bilateral_radius > 0 && !(finite_pos(p->sigma_space) && finite_pos(p->sigma_range))) return ROI_EINVAL;
        if (p->median_radius > DN_MAXM || p->bilateral_radius > DN_MAXB) return ROI_EUNSUPPORTED;
    }
    if (p->winsize > 2 * IT_MAXR + 1) return ROI_EUNSUPPORTED;
    if (ms != ROI_OK) return ms;
    if (h > 32768 || w > 32768) return ROI_EUNSUPPORTED;
    // the iteration kernel addresses a level's packed plane (16 B per pixel
    // of a 64-aligned row) with 32-bit byte offsets
    if ((uint64_t)(h + 1) * align_up((size_t)w + 1, 64) * 16 >= (1ull << 32)) return ROI_EUNSUPPORTED;
    return ROI_OK;
}

size_t roi_workspace_size(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p)
{
    if (roi_validate(h, w, dtype, p) != ROI_OK) return 0;
    if (h == 0 || w == 0) return HDR_BYTES;
    return HDR_BYTES + make_plan(h, w, p).bytes;
}

roi_status roi_mask(const void *prev, const void *next, int32_t h, int32_t w, int64_t pitch, roi_dtype dtype,
                    const roi_params *p, float *flow, uint8_t *mask, void *ws, size_t ws_bytes, void *stream)
{
    roi_status st = roi_validate(h, w, dtype, p);
    if (st != ROI_OK) return st;
    if (h == 0 || w == 0) return ROI_OK;
    if (!prev || !next || !flow || !ws || pitch < w) return ROI_EINVAL;
    if ((uintptr_t)ws % ALIGN) return ROI_EINVAL;
    const Plan pl = make_plan(h, w, p);
    if (ws_bytes < HDR_BYTES + pl.bytes) return ROI_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *base = (uint8_t *)ws + HDR_BYTES;
    const void *frames[2] = {prev, next};
    const int sets[2] = {0, 1};
    st = enqueue_expand(pl, base, 2, frames, pitch, dtype, p, sets, s, phase_slot(ws, 0));
    if (st != ROI_OK) return st;
    return enqueue_flow(pl, base, (SelState *)ws, 0, 1, h, w, p, flow, mask, s);
}

roi_status roi_read_tau2(const void *ws, int32_t index, float *tau2_out, void *stream)
{
    if (!ws || !tau2_out || index < 0 || index >= MAX_BATCH) return ROI_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return ROI_EDEVICE;
    SelState sst;
    if (hipMemcpy(&sst, (const SelState *)ws + index, sizeof sst, hipMemcpyDeviceToHost) != hipSuccess)
        return ROI_EDEVICE;
    std::memcpy(tau2_out, &sst.tau2_bits, 4);
    return ROI_OK;
}

roi_status roi_read_shift(const void *ws, int32_t index, int32_t *sy, int32_t *sx, float *peak, void *stream)
{
    if (!ws || !sy || !sx || index < 0 || index >= MAX_BATCH) return ROI_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return ROI_EDEVICE;
    PhaseState ph;
    if (hipMemcpy(&ph, phase_slot((void *)ws, index), sizeof ph, hipMemcpyDeviceToHost) != hipSuccess)
        return ROI_EDEVICE;
    *sy = ph.sy;
    *sx = ph.sx;
    if (peak) *peak = ph.peak;
    return ROI_OK;
}

int32_t roi_phase_size(int32_t h, int32_t w) { return h < 0 || w < 0 ? 0 : phase_size(h, w); }

// Workspace of roi_phase_correlation after the header: the registered frame
// (h rows of a 64-aligned pitch), the two complex fields, the tables and the
// argmax counters.
struct PhasePlan {
    int pitch;
    size_t al, z, t, tw, hann, keys, bytes;
};

PhasePlan phase_plan(int h, int w)
{
    PhasePlan q{};
    q.pitch = (int)align_up((size_t)w, 64);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align_up(off + b, ALIGN);
        return o;
    };
    q.al = take((size_t)h * q.pitch * sizeof(float));
    const size_t P = (size_t)phase_size(h, w);
    q.z = take(P * P * sizeof(float2));
    q.t = take(P * P * sizeof(float2));
    q.tw = take(P * sizeof(float2));
    q.hann = take(P * sizeof(float));
    q.keys = take(PH_SLOTS * PH_SLOT_STRIDE * sizeof(unsigned long long));
    q.bytes = off;
    return q;
}

size_t roi_phase_workspace_size(int32_t h, int32_t w)
{
    if (h < 0 || w < 0 || h > 32768 || w > 32768) return 0;
    if (h == 0 || w == 0) return HDR_BYTES;
    return HDR_BYTES + phase_plan(h, w).bytes;
}

roi_status roi_phase_correlation(const void *prev, const void *next, int32_t h, int32_t w, int64_t pitch,
                                 roi_dtype dtype, float *surface, float *aligned, void *ws, size_t ws_bytes,
                                 void *stream)
{
    if (h < 0 || w < 0) return ROI_EINVAL;
    if (dtype != ROI_U8 && dtype != ROI_U16 && dtype != ROI_F32) return ROI_EINVAL;
    if (h > 32768 || w > 32768) return ROI_EUNSUPPORTED;
    if (h == 0 || w == 0) return ROI_OK;
    if (!prev || !next || !ws || pitch < w || (uintptr_t)ws % ALIGN) return ROI_EINVAL;
    const PhasePlan q = phase_plan(h, w);
    if (ws_bytes < HDR_BYTES + q.bytes) return ROI_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *base = (uint8_t *)ws + HDR_BYTES;
    PhaseBufs b{};
    b.P = phase_size(h, w);
    b.z = (float2 *)(base + q.z);
    b.t = (float2 *)(base + q.t);
    b.tw = (float2 *)(base + q.tw);
    b.hann = (float *)(base + q.hann);
    b.keys = (unsigned long long *)(base + q.keys);
    PhaseIO io{};
    io.ref = prev;
    io.dref = dtype;
    io.pref = pitch;
    io.mov = next;
    io.dmov = dtype;
    io.pmov = pitch;
    io.out = aligned ? aligned : (float *)(base + q.al);
    io.opitch = aligned ? w : q.pitch;
    return enqueue_phase(b, io, h, w, phase_slot(ws, 0), b.P > 0 ? surface : nullptr, s);
}

// Workspace of roi_mask_from_flow after the header: m2 and sal (h rows of a
// 64-aligned pitch each), lab and area (h w int32 each), the select
// histogram, the saliency maxima counters.
struct FlowMaskPlan {
    int pitch;
    size_t m2, sal, lab, area, hist, maxs, bytes;
};

FlowMaskPlan flow_mask_plan(int h, int w)
{
    FlowMaskPlan f{};
    f.pitch = (int)align_up((size_t)w, 64);
    const size_t plane = align_up((size_t)h * f.pitch * sizeof(float), ALIGN);
    f.m2 = 0;
    f.sal = plane;
    f.lab = 2 * plane;
    f.area = f.lab + align_up((size_t)h * w * sizeof(int32_t), ALIGN);
    f.hist = f.area + align_up((size_t)h * w * sizeof(int32_t), ALIGN);
    f.maxs = f.hist + align_up(SEL_COPIES * SEL_BINS * sizeof(uint32_t), ALIGN);
    f.bytes = f.maxs + 3 * MAXSLOT_WORDS * sizeof(uint32_t);
    return f;
}

size_t roi_flow_mask_workspace_size(int32_t h, int32_t w, const roi_params *p)
{
    if (!p || h < 0 || w < 0 || h > 32768 || w > 32768 || validate_mask_stage(p) != ROI_OK) return 0;
    if (h == 0 || w == 0) return HDR_BYTES;
    return HDR_BYTES + flow_mask_plan(h, w).bytes;
}

roi_status roi_mask_from_flow(const float *flow, int32_t h, int32_t w, const roi_params *p, uint8_t *mask,
                              float *saliency, void *ws, size_t ws_bytes, void *stream)
{
    if (!p || h < 0 || w < 0) return ROI_EINVAL;
    roi_status st = validate_mask_stage(p);
    if (st != ROI_OK) return st;
    if (h > 32768 || w > 32768) return ROI_EUNSUPPORTED;
    if (h == 0 || w == 0) return ROI_OK;
    if (!flow || !mask || !ws || (uintptr_t)ws % ALIGN) return ROI_EINVAL;
    const FlowMaskPlan f = flow_mask_plan(h, w);
    if (ws_bytes < HDR_BYTES + f.bytes) return ROI_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *base = (uint8_t *)ws + HDR_BYTES;
    MaskBufs mb{};
    mb.m2 = (float *)(base + f.m2);
    mb.m2_pitch = f.pitch;
    mb.sal = (float *)(base + f.sal);
    mb.sal_pitch = f.pitch;
    mb.lab = (int32_t *)(base + f.lab);
    mb.area = (int32_t *)(base + f.area);
    mb.maxs = (uint32_t *)(base + f.maxs);
    mb.hist = (uint32_t *)(base + f.hist);
    hipLaunchKernelGGL(k_mag2, dim3((w + 63) / 64, (h + 3) / 4), dim3(256), 0, s, (const float2 *)flow, h, w, mb.m2,
                       f.pitch);
    LAUNCH_CHECK();
    return enqueue_mask(mb, (SelState *)ws, h, w, p, mask, p->rule == ROI_RULE_SALIENCY ? saliency : nullptr, s);
}

roi_status roi_pyr_down(const float *src, int32_t h, int32_t w, float *dst, void *stream)
{
    if (!src || !dst || h < 0 || w < 0) return ROI_EINVAL;
    if (h == 0 || w == 0) return ROI_OK;
    PyrArgs a{};
    a.src[0] = src;
    a.dst[0] = dst;
    a.src_pitch = w;
    a.dst_pitch = (w + 1) / 2;
    a.h = h;
    a.w = w;
    a.h2 = (h + 1) / 2;
    a.w2 = (w + 1) / 2;
    launch_pyr<float, float>(a, 1, (hipStream_t)stream);
    LAUNCH_CHECK();
    return ROI_OK;
}

roi_status roi_poly_expand(const void *img, int32_t h, int32_t w, int64_t pitch, roi_dtype dtype,
                           const roi_params *p, float *coef, void *stream)
{
    roi_status st = roi_validate(h, w, dtype, p);
    if (st != ROI_OK) return st;
    if (h == 0 || w == 0) return ROI_OK;
    if (!img || !coef || pitch < w) return ROI_EINVAL;
    PolyArgs a{};
    fill_poly(a, poly_consts(p->poly_n, p->poly_sigma));
    a.src[0] = img;
    a.dst[0] = coef;
    a.src_pitch = pitch;
    a.dc = dc_of(dtype);
    a.dplane = (int64_t)h * w;
    a.dpitch = w;
    a.h = h;
    a.w = w;
    a.round16 = (p->flags & ROI_FP16_STORAGE) ? 1 : 0;
    launch_poly_raw<float>(dtype, a, 1, (hipStream_t)stream);
    LAUNCH_CHECK();
    return ROI_OK;
}

roi_status roi_denoise(const void *img, int32_t h, int32_t w, int64_t pitch, roi_dtype dtype, const roi_params *p,
                       float *out, void *stream)
{
    if (!p) return ROI_EINVAL;
    roi_params q = *p;
    q.denoise = 1;
    roi_status st = roi_validate(h, w, dtype, &q);
    if (st != ROI_OK) return st;
    if (h == 0 || w == 0) return ROI_OK;
    if (!img || !out || pitch < w) return ROI_EINVAL;
    DenoiseArgs da{};
    fill_denoise(da, &q);
    da.src[0] = img;
    da.dst[0] = out;
    da.src_pitch = pitch;
    da.dst_pitch = w;
    da.h = h;
    da.w = w;
    return launch_denoise(dtype, da, &q, 1, (hipStream_t)stream);
}

// ---------------------------------------------------------------- batched

size_t roi_batched_workspace_size(int32_t n, const roi_pair *pairs, roi_dtype dtype, const roi_params *p)
{
    if (n < 1 || n > MAX_BATCH || !pairs) return 0;
    size_t total = HDR_BYTES;
    for (int i = 0; i < n; ++i) {
        if (roi_validate(pairs[i].h, pairs[i].w, dtype, p) != ROI_OK) return 0;
        if (pairs[i].h > 0 && pairs[i].w > 0) total += make_plan(pairs[i].h, pairs[i].w, p).bytes;
    }
    return total;
}

roi_status roi_mask_batched(int32_t n, const roi_pair *pairs, roi_dtype dtype, const roi_params *p, void *ws,
                            size_t ws_bytes, void *stream)
{
    if (n < 1 || n > MAX_BATCH || !pairs || !p || !ws) return ROI_EINVAL;
    if ((uintptr_t)ws % ALIGN) return ROI_EINVAL;
    for (int i = 0; i < n; ++i) {
        const roi_pair &q = pairs[i];
        roi_status st = roi_validate(q.h, q.w, dtype, p);
        if (st != ROI_OK) return st;
        if (q.h == 0 || q.w == 0) continue;
        if (!q.prev || !q.next || !q.flow || !q.mask || q.pitch < q.w) return ROI_EINVAL;
    }
    const size_t need = roi_batched_workspace_size(n, pairs, dtype, p);
    if (need == 0) return ROI_EINVAL;
    if (ws_bytes < need) return ROI_ENOMEM;
    hipStream_t us = (hipStream_t)stream;

    std::string key((const char *)pairs, sizeof(roi_pair) * n);
    key.append((const char *)p, sizeof *p);
    key.append((const char *)&dtype, sizeof dtype);
    key.append((const char *)&ws, sizeof ws);
    int dev = 0;
    hipGetDevice(&dev);
    key.append((const char *)&dev, sizeof dev);

    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        const int naux = std::min(n, 8);
        DeviceStreams *ds = device_streams(naux);
        if (!ds) return ROI_EDEVICE;
        hipStream_t cs = ds->cap;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return ROI_EDEVICE;
        roi_status st = ROI_OK;
        // event ev recorded on `from`, waited for by `to` (a graph edge)
        auto link = [&](hipEvent_t ev, hipStream_t from, hipStream_t to) {
            if (hipEventRecord(ev, from) != hipSuccess || hipStreamWaitEvent(to, ev, 0) != hipSuccess)
                st = ROI_EDEVICE;
        };
        // 1. per pair on the auxiliary streams (pairs spread over them):
        //    pyramid and expansions (with denoising / stabilisation) and the
        //    initial flow
        hipEventRecord(ds->ev[0], cs);
        for (int k = 0; k < naux; ++k)
            if (hipStreamWaitEvent(ds->aux[k], ds->ev[0], 0) != hipSuccess) st = ROI_EDEVICE;
        struct Job {
            Plan pl;
            uint8_t *base;
            int i;
        };
        std::vector<Job> jobs;
        uint8_t *base = (uint8_t *)ws + HDR_BYTES;
        for (int i = 0; i < n && st == ROI_OK; ++i) {
            const roi_pair &q = pairs[i];
            if (q.h == 0 || q.w == 0) continue;
            const Plan pl = make_plan(q.h, q.w, p);
            const void *frames[2] = {q.prev, q.next};
            const int sets[2] = {0, 1};
            hipStream_t as = ds->aux[i % naux];
            st = enqueue_expand(pl, base, 2, frames, q.pitch, dtype, p, sets, as, phase_slot(ws, i));
            if (st == ROI_OK) {
                enqueue_init_flow(pl, base, q.h, q.w, p, q.flow, as);
                if (hipGetLastError() != hipSuccess) st = ROI_EDEVICE;
            }
            jobs.push_back({pl, base, i});
            base += pl.bytes;
        }
        for (int k = 0; k < naux; ++k) link(ds->ev[k + 1], ds->aux[k], cs);
        // 2. every coarse level and update of all pairs in one grid (per
        //    IT_MULTI pairs): the coarse levels of many pairs fill the chip
        //    together
        const bool fp16 = (p->flags & ROI_FP16_STORAGE) != 0;
        for (int l = p->levels - 1; l >= 1 && st == ROI_OK && !jobs.empty(); --l) {
            for (int it = 0; it < p->iterations && st == ROI_OK; ++it) {
                std::vector<IterArgs> as;
                for (const Job &jb : jobs) {
                    const roi_pair &q = pairs[jb.i];
                    as.push_back(make_iter_args(jb.pl, jb.base, (SelState *)ws + jb.i, 0, 1, q.w, p, q.flow, q.mask,
                                                l, it));
                }
                st = launch_iter_multi(as, fp16, cs);
            }
        }
        // 3. per pair on the auxiliary streams: the full-resolution updates
        //    (each fills the chip alone), threshold and dilation
        if (hipEventRecord(ds->ev[naux + 1], cs) != hipSuccess) st = ROI_EDEVICE;
        for (int k = 0; k < naux; ++k)
            if (hipStreamWaitEvent(ds->aux[k], ds->ev[naux + 1], 0) != hipSuccess) st = ROI_EDEVICE;
        for (const Job &jb : jobs) {
            if (st != ROI_OK) break;
            const roi_pair &q = pairs[jb.i];
            hipStream_t as = ds->aux[jb.i % naux];
            for (int it = 0; it < p->iterations && st == ROI_OK; ++it)
                st = launch_iter(make_iter_args(jb.pl, jb.base, (SelState *)ws + jb.i, 0, 1, q.w, p, q.flow, q.mask, 0, it),
                                 fp16, as, nullptr);
            if (st == ROI_OK)
                st = enqueue_mask_stage(jb.pl, jb.base, (SelState *)ws + jb.i, q.h, q.w, p, q.mask, as);
        }
        for (int k = 0; k < naux; ++k) link(ds->ev[naux + 2 + k], ds->aux[k], cs);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (st != ROI_OK || ce != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return st != ROI_OK ? st : ROI_EDEVICE;
        }
        GraphEntry e;
        const hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ie != hipSuccess) return ROI_EDEVICE;
        if (g_graphs.size() >= MAX_GRAPHS) {
            auto lru = g_graphs.begin();
            for (auto j = g_graphs.begin(); j != g_graphs.end(); ++j)
                if (j->second.tick < lru->second.tick) lru = j;
            hipGraphExecDestroy(lru->second.exec);
            g_graphs.erase(lru);
        }
        it = g_graphs.emplace(key, e).first;
    }
    it->second.tick = ++g_tick;
    if (hipGraphLaunch(it->second.exec, us) != hipSuccess) return ROI_EDEVICE;
    return ROI_OK;
}

// ---------------------------------------------------------------- streaming

struct roi_stream_ctx {
    int32_t h, w;
    roi_dtype dtype;
    roi_params p;
    Plan plan;
    uint8_t *buf;   // HDR_BYTES of threshold state, then the plan
    size_t bytes;
    int primed;     // a previous frame's expansion is resident
    int cur;        // expansion set holding the previous frame
    int device;
    uint8_t *hist;  // adjacent > 0: ring of the last `adjacent` own masks (h*w bytes each)
    int hist_count; // masks stored since the last reset (capped at adjacent)
    int hist_pos;   // ring slot the next mask goes to
};

size_t roi_stream_state_bytes(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p)
{
    if (roi_validate(h, w, dtype, p) != ROI_OK || h == 0 || w == 0) return 0;
    return HDR_BYTES + make_plan(h, w, p).bytes + (size_t)p->adjacent * align_up((size_t)h * w, ALIGN);
}

roi_status roi_stream_create(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p, void **out_ctx)
{
    if (!out_ctx) return ROI_EINVAL;
    *out_ctx = nullptr;
    roi_status st = roi_validate(h, w, dtype, p);
    if (st != ROI_OK) return st;
    if (h == 0 || w == 0) return ROI_EINVAL;
    roi_stream_ctx *c = new roi_stream_ctx();
    c->h = h;
    c->w = w;
    c->dtype = dtype;
    c->p = *p;
    c->plan = make_plan(h, w, p);
    c->bytes = HDR_BYTES + c->plan.bytes;
    hipGetDevice(&c->device);
    if (hipMalloc((void **)&c->buf, c->bytes) != hipSuccess) {
        delete c;
        return ROI_ENOMEM;
    }
    c->hist = nullptr;
    c->hist_count = 0;
    c->hist_pos = 0;
    // history slots on 256-byte boundaries (the union kernel moves 16 bytes at a time)
    if (p->adjacent > 0 && hipMalloc((void **)&c->hist, (size_t)p->adjacent * align_up((size_t)h * w, ALIGN)) != hipSuccess) {
        hipFree(c->buf);
        delete c;
        return ROI_ENOMEM;
    }
    c->primed = 0;
    c->cur = 0;
    *out_ctx = c;
    return ROI_OK;
}

roi_status roi_stream_reset(void *ctx)
{
    if (!ctx) return ROI_EINVAL;
    ((roi_stream_ctx *)ctx)->primed = 0;
    ((roi_stream_ctx *)ctx)->hist_count = 0;
    return ROI_OK;
}

void roi_stream_destroy(void *ctx)
{
    if (!ctx) return;
    roi_stream_ctx *c = (roi_stream_ctx *)ctx;
    hipFree(c->buf);
    if (c->hist) hipFree(c->hist);
    delete c;
}

// Union of this mask with the stream's previous masks, then remember it.
static roi_status enqueue_ensemble(roi_stream_ctx *c, uint8_t *mask, hipStream_t s)
{
    const size_t n = (size_t)c->h * c->w, slot = align_up(n, ALIGN);
    const int K = c->p.adjacent;
    EnsembleArgs ea{};
    ea.mask = mask;
    ea.store = c->hist + (size_t)c->hist_pos * slot;
    ea.n = c->hist_count;
    for (int k = 0; k < ea.n; ++k) ea.prev[k] = c->hist + (size_t)((c->hist_pos - 1 - k + K) % K) * slot;
    ea.count = (int64_t)n;
    hipLaunchKernelGGL(k_ensemble, dim3((unsigned)((n + 4095) / 4096)), dim3(256), 0, s, ea);
    LAUNCH_CHECK();
    c->hist_pos = (c->hist_pos + 1) % K;
    if (c->hist_count < K) c->hist_count += 1;
    return ROI_OK;
}

static roi_status stream_push_one(roi_stream_ctx *c, const void *frame, int64_t pitch, float *flow, uint8_t *mask,
                                  hipStream_t s)
{
    if (!frame || pitch < c->w) return ROI_EINVAL;
    const int nxt = 1 - c->cur;
    uint8_t *base = c->buf + HDR_BYTES;
    const void *frames[1] = {frame};
    const int sets[1] = {nxt};
    roi_status st = enqueue_expand(c->plan, base, 1, frames, pitch, c->dtype, &c->p, sets, s, phase_slot(c->buf, 0),
                                   c->primed ? c->cur : -1);
    if (st != ROI_OK) return st;
    if (!c->primed) {
        c->primed = 1;
        c->cur = nxt;
        return ROI_PRIMED;
    }
    if (!flow) return ROI_EINVAL;
    st = enqueue_flow(c->plan, base, (SelState *)c->buf, c->cur, nxt, c->h, c->w, &c->p, flow, mask, s);
    if (st != ROI_OK) return st;
    c->cur = nxt;
    if (c->p.adjacent > 0 && mask) return enqueue_ensemble(c, mask, s);
    return ROI_OK;
}

// Pushes to several stream contexts (same parameters) as one batch: each
// context's expansion, full-resolution updates, mask stage and ensemble run
// on its own stream ss[i], while the coarse-level updates of all contexts
// that produce a flow share multi-pair grids on stream js (joined and forked
// with the events in evs, one per distinct stream and direction; at least
// 2 * SRV_FORK_MAX). The per-pixel arithmetic is that of stream_push_one.
constexpr int SRV_FORK_MAX = 8;
static roi_status stream_push_batch(int n, roi_stream_ctx *const *cs, const void *const *frames, const int64_t *pitches,
                                    float *const *flows, uint8_t *const *masks, int32_t *status, const hipStream_t *ss,
                                    hipStream_t js, hipEvent_t *evs)
{
    std::vector<int> jobs;
    std::vector<int> nxt(n, 0);
    for (int i = 0; i < n; ++i) {
        roi_stream_ctx *c = cs[i];
        if (!frames[i] || pitches[i] < c->w) {
            status[i] = ROI_EINVAL;
            continue;
        }
        nxt[i] = 1 - c->cur;
        uint8_t *base = c->buf + HDR_BYTES;
        const void *fr[1] = {frames[i]};
        const int sets[1] = {nxt[i]};
        roi_status st = enqueue_expand(c->plan, base, 1, fr, pitches[i], c->dtype, &c->p, sets, ss[i],
                                       phase_slot(c->buf, 0), c->primed ? c->cur : -1);
        if (st != ROI_OK) return st;
        if (!c->primed) {
            c->primed = 1;
            c->cur = nxt[i];
            status[i] = ROI_PRIMED;
            continue;
        }
        if (!flows[i]) {
            status[i] = ROI_EINVAL;
            continue;
        }
        enqueue_init_flow(c->plan, base, c->h, c->w, &c->p, flows[i], ss[i]);
        LAUNCH_CHECK();
        jobs.push_back(i);
    }
    if (!jobs.empty()) {
        // distinct streams of the jobs other than js
        std::vector<hipStream_t> us;
        for (int i : jobs)
            if (ss[i] != js && std::find(us.begin(), us.end(), ss[i]) == us.end()) us.push_back(ss[i]);
        if ((int)us.size() > SRV_FORK_MAX) return ROI_EINVAL;
        for (size_t k = 0; k < us.size(); ++k)
            if (hipEventRecord(evs[k], us[k]) != hipSuccess || hipStreamWaitEvent(js, evs[k], 0) != hipSuccess)
                return ROI_EDEVICE;
        const roi_params *p = &cs[jobs[0]]->p;
        const bool fp16 = cs[jobs[0]]->plan.fp16;
        for (int l = p->levels - 1; l >= 1; --l) {
            for (int it = 0; it < p->iterations; ++it) {
                std::vector<IterArgs> as;
                for (int i : jobs) {
                    roi_stream_ctx *c = cs[i];
                    as.push_back(make_iter_args(c->plan, c->buf + HDR_BYTES, (SelState *)c->buf, c->cur, nxt[i], c->w,
                                                &c->p, flows[i], masks[i], l, it));
                }
                roi_status st = launch_iter_multi(as, fp16, js);
                if (st != ROI_OK) return st;
            }
        }
        for (size_t k = 0; k < us.size(); ++k)
            if (hipEventRecord(evs[SRV_FORK_MAX + k], js) != hipSuccess ||
                hipStreamWaitEvent(us[k], evs[SRV_FORK_MAX + k], 0) != hipSuccess)
                return ROI_EDEVICE;
    }
    for (int i : jobs) {
        roi_stream_ctx *c = cs[i];
        uint8_t *base = c->buf + HDR_BYTES;
        for (int it = 0; it < c->p.iterations; ++it) {
            roi_status st = launch_iter(make_iter_args(c->plan, base, (SelState *)c->buf, c->cur, nxt[i], c->w, &c->p,
                                                       flows[i], masks[i], 0, it),
                                        c->plan.fp16, ss[i], nullptr);
            if (st != ROI_OK) return st;
        }
        if (masks[i]) {
            roi_status st = enqueue_mask_stage(c->plan, base, (SelState *)c->buf, c->h, c->w, &c->p, masks[i], ss[i]);
            if (st != ROI_OK) return st;
        }
        c->cur = nxt[i];
        if (c->p.adjacent > 0 && masks[i]) {
            roi_status st = enqueue_ensemble(c, masks[i], ss[i]);
            if (st != ROI_OK) return st;
        }
        status[i] = ROI_OK;
    }
    return ROI_OK;
}

roi_status roi_stream_read_shift(void *ctx, int32_t *sy, int32_t *sx, float *peak, void *stream)
{
    if (!ctx) return ROI_EINVAL;
    roi_stream_ctx *c = (roi_stream_ctx *)ctx;
    if (!(c->p.flags & ROI_STABILIZE)) return ROI_EINVAL;
    return roi_read_shift(c->buf, 0, sy, sx, peak, stream);
}

roi_status roi_stream_push(void *ctx, const void *frame, int64_t pitch, float *flow, uint8_t *mask, void *stream)
{
    if (!ctx) return ROI_EINVAL;
    roi_stream_ctx *c = (roi_stream_ctx *)ctx;
    if (c->primed && !flow) return ROI_EINVAL;
    return stream_push_one(c, frame, pitch, flow, mask, (hipStream_t)stream);
}

roi_status roi_stream_push_many(int32_t n, void *const *ctxs, const void *const *frames, const int64_t *pitches,
                                float *const *flows, uint8_t *const *masks, int32_t *status, void *stream)
{
    if (n < 1 || n > MAX_BATCH || !ctxs || !frames || !pitches || !flows || !masks || !status) return ROI_EINVAL;
    for (int i = 0; i < n; ++i) {
        roi_stream_ctx *c = (roi_stream_ctx *)ctxs[i];
        if (!c || !frames[i] || pitches[i] < c->w) return ROI_EINVAL;
        if (c->primed && !flows[i]) return ROI_EINVAL;
        if (c->dtype != ((roi_stream_ctx *)ctxs[0])->dtype ||
            std::memcmp(&c->p, &((roi_stream_ctx *)ctxs[0])->p, sizeof(roi_params)) != 0)
            return ROI_EINVAL;
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return ROI_EINVAL; // one frame per context per call
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<roi_stream_ctx *> cs(n);
    std::vector<hipStream_t> ss(n, s);
    for (int i = 0; i < n; ++i) cs[i] = (roi_stream_ctx *)ctxs[i];
    hipEvent_t evs[2 * SRV_FORK_MAX] = {}; // unused: every context runs on s
    return stream_push_batch(n, cs.data(), frames, pitches, flows, masks, status, ss.data(), s, evs);
}

// ---------------------------------------------------------------- timing

void roi_timing_enable(int32_t mode)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.mode = mode == 1 || mode == 2 ? mode : 0;
    // event creation is far slower than a record: fill the pool up front
    while (g_timing.mode && g_timing.pool.size() < ROI_TIMING_POOL) {
        hipEvent_t e = timing_event();
        if (!e) break;
        g_timing.pool.push_back(e);
    }
}

roi_status roi_timing_read(double *total_ms, int64_t *launches, int64_t *pixels, double *bytes)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    for (const TimedLaunch &t : g_timing.pending) {
        if (hipEventSynchronize(t.e1) != hipSuccess) return ROI_EDEVICE;
        float ms = 0;
        if (hipEventElapsedTime(&ms, t.e0, t.e1) != hipSuccess) return ROI_EDEVICE;
        g_timing.done_ms += ms;
        g_timing.done_n += t.n;
        g_timing.done_px += t.px;
        g_timing.done_bytes += t.bytes;
        g_timing.rec_ms.push_back(ms);
        g_timing.rec_px.push_back(t.px);
        g_timing.rec_bytes.push_back(t.bytes);
        g_timing.pool.push_back(t.e0);
        g_timing.pool.push_back(t.e1);
    }
    g_timing.pending.clear();
    if (total_ms) *total_ms = g_timing.done_ms;
    if (launches) *launches = g_timing.done_n;
    if (pixels) *pixels = g_timing.done_px;
    if (bytes) *bytes = g_timing.done_bytes;
    return ROI_OK;
}

void roi_timing_sample(int32_t every)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.every = every > 1 ? every : 1;
}

void roi_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    for (const TimedLaunch &t : g_timing.pending) {
        hipEventSynchronize(t.e1);
        g_timing.pool.push_back(t.e0);
        g_timing.pool.push_back(t.e1);
    }
    g_timing.pending.clear();
    g_timing.calls = 0;
    g_timing.done_ms = 0;
    g_timing.done_bytes = 0;
    g_timing.done_n = 0;
    g_timing.done_px = 0;
    g_timing.rec_ms.clear();
    g_timing.rec_px.clear();
    g_timing.rec_bytes.clear();
}

int32_t roi_timing_records(double *ms, int64_t *pixels, double *bytes, int32_t max)
{
    if (roi_timing_read(nullptr, nullptr, nullptr, nullptr) != ROI_OK) return -1;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    const int32_t n = (int32_t)g_timing.rec_ms.size();
    for (int32_t i = 0; i < n && i < max; ++i) {
        if (ms) ms[i] = g_timing.rec_ms[i];
        if (pixels) pixels[i] = g_timing.rec_px[i];
        if (bytes) bytes[i] = g_timing.rec_bytes[i];
    }
    return n;
}

void roi_autotune(int32_t mode)
{
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.mode = mode ? 1 : 0;
    if (mode == 2) g_tune.best.clear();
}

roi_status roi_set_strip(int32_t strip)
{
    if (strip < 0 || (strip > 0 && strip % IT_CH != 0)) return ROI_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.forced = strip;
    return ROI_OK;
}

int32_t roi_tuned_strip(int32_t h, int32_t w, int32_t winsize, int32_t fp16)
{
    std::lock_guard<std::mutex> lk(g_tune.mu);
    for (int prior : {PRIOR_PLAIN, PRIOR_UPSAMPLE, PRIOR_ZERO}) {
        auto it = g_tune.best.find(std::make_tuple(h, w, winsize / 2, fp16 ? 1 : 0, prior));
        if (it != g_tune.best.end()) return it->second;
    }
    return 0;
}

const char *roi_status_str(roi_status s)
{
    switch (s) {
    case ROI_OK: return "ok";
    case ROI_PRIMED: return "primed (first frame of a stream stored)";
    case ROI_EINVAL: return "invalid argument";
    case ROI_ENOMEM: return "workspace too small or device allocation failed";
    case ROI_EDEVICE: return "HIP launch or runtime failure";
    case ROI_EUNSUPPORTED: return "unsupported parameter value";
    }
    return "unknown status";
}

} // extern "C"

#include "server.h"
