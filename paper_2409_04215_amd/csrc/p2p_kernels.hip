// All-pairs fundamental-solution sums (the MFS representation), gfx950.
//
// Laplace (Section 2.1):  u_i = sum_j s_j / (4 pi r_ij)
// Stokes  (Section 2.2, eq. (stokeslet)):
//          u_i = sum_j (s_j + (d.s_j) d / r^2) / (8 pi mu r),  d = x_i - y_j
//
// Design (MI355X):
//  * One work item = a block of 64*TPL targets of one system x a range of
//    source bodies of the same system, run by one workgroup of four waves.
//    Every wave holds all the item's targets (TPL per lane, register blocking)
//    and takes a contiguous quarter of each source body; the four FP64
//    partial sums meet in LDS once per item and are added in wave order, so
//    results do not depend on timing.  Splitting the sources rather than the
//    targets keeps items small in targets, so a launch reaches many items
//    with few source splits (each split costs one FP64 slice of the output).
//  * Items are launched largest-first, so the hardware dispatcher hands the
//    long items out before the short ones.
//  * Stokes sources are read with wave-uniform addresses: every lane of a wave
//    walks the same source list, so the compiler turns the reads into scalar
//    loads (s_load) and the VALU instructions take the source coordinates and
//    strengths as SGPR operands.  Laplace sources (16 B, one v_rsq_f32 per 8
//    VALU instructions) are staged per run of 64 in the wave's own LDS slots
//    and read back by broadcast: 15% faster there, 1% slower for Stokes.
//  * Mixed precision: the coordinates are split into a per-body FP64 centre
//    and a small FP32 offset; per (lane, source body) the FP64 centre
//    difference is rounded to FP32 once, so the FP32 rounding of d scales
//    with |d| plus the body size.  Per pair: FP32 arithmetic with the hardware
//    v_rsq_f32; per run of at most FLUSH sources the FP32 partial is added
//    to an FP64 accumulator.
//  * FP64 variant: the same walk in FP64, 1/sqrt from v_rsq_f64 refined by
//    one third-order step (rsqrt_f64 in device_math.h).
//  * Same-body pairs: a source body equal to every active lane's own body is
//    skipped wave-uniformly; a body shared by only some lanes is evaluated
//    and its partial discarded per lane (select, not multiply), so no masking
//    sits inside the pair loop.
#include "device_math.h"
#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr int FLUSH = 64;

// Adds the FP64 accumulators of waves 1..WAVES-1 into wave 0's, in wave order.
// lds holds (WAVES-1) * NV * 64 doubles.  Every thread of the workgroup must
// call it; returns true in wave 0, which then owns the sums.
template <int NV>
__device__ __forceinline__ bool reduce_waves(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv > 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[((wv - 1) * NV + q) * 64 + lane] = v[q];
    __syncthreads();
    if (wv > 0) return false;
    for (int w = 1; w < WAVES; ++w)
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += lds[((w - 1) * NV + q) * 64 + lane];
    return true;
}

struct Src4 {
    SrcS32 s[4];
};

// One Stokes source against the lane's TPL targets, FP32 (eq. (stokeslet) without 1/(8 pi mu)).
template <int TPL>
__device__ __forceinline__ void stokes_pair(const float (&xr)[TPL][3], const float4 y, const float4 f,
                                            float (&p)[TPL][3]) {
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const float d0 = xr[t][0] - y.x, d1 = xr[t][1] - y.y, d2 = xr[t][2] - y.z;
        const float r2 = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float df = __builtin_fmaf(d2, f.z, __builtin_fmaf(d1, f.y, d0 * f.x));
        const float sc = df * (ri * ri);
        p[t][0] = __builtin_fmaf(ri, __builtin_fmaf(sc, d0, f.x), p[t][0]);
        p[t][1] = __builtin_fmaf(ri, __builtin_fmaf(sc, d1, f.y), p[t][1]);
        p[t][2] = __builtin_fmaf(ri, __builtin_fmaf(sc, d2, f.z), p[t][2]);
    }
}

// This wave's contiguous quarter [j0, j1) of the source range [b0, b1).
__device__ __forceinline__ void wave_range(int b0, int b1, int wv, int &j0, int &j1) {
    const int q = (b1 - b0 + WAVES - 1) / WAVES;
    j0 = min(b0 + wv * q, b1);
    j1 = min(j0 + q, b1);
}

struct KernelArgs {
    const P2PItem *items;
    const double *centre;      // [n_body][3]
    const int32_t *trg_body;   // [n_trg]
    const int32_t *src_ptr;    // [n_body+1]
    const int32_t *sys_active; // [n_sys] or null
    double *out;               // partial slices or final output
    const double *addend;      // added once (may be null); only when n_split == 1
    int64_t out_stride;        // elements per split slice
    double alpha;              // scale applied to the pair sum (includes 1/(4pi) or 1/(8 pi mu))
    int skip_same;
    int accumulate;
    int *queue;                // persistent mode: work-queue counter (reset to 0 before the launch), else null
    int n_items;
};

// ---------------------------------------------------------------------------
// Mixed precision, Stokes / Laplace (one kernel; item.kind is wave-uniform)
// ---------------------------------------------------------------------------
template <int TPL>
__device__ __forceinline__ void mixed_item(const KernelArgs &a, const P2PItem it, const float4 *__restrict__ trg_off,
                                           const SrcS32 *__restrict__ srcS, const SrcL32 *__restrict__ srcL,
                                           double *lds, float4 *stage) {
    // an inactive system still writes its epilogue (pair sum 0), so outputs stay finite
    const bool active = !a.sys_active || a.sys_active[it.sys];
    const bool stokes = it.kind == MFS_STOKES;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    int idx[TPL];
    bool valid[TPL];
    int body[TPL];
    double ct[TPL][3];
    float xt[TPL][3];
    double acc[TPL][3];
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        idx[t] = it.t0 + lane + t * 64;
        valid[t] = idx[t] < it.t1;
        const int i = valid[t] ? idx[t] : it.t0;
        body[t] = a.trg_body[i];
        const float4 o = trg_off[i];
        xt[t][0] = o.x;
        xt[t][1] = o.y;
        xt[t][2] = o.z;
        ct[t][0] = a.centre[3 * body[t] + 0];
        ct[t][1] = a.centre[3 * body[t] + 1];
        ct[t][2] = a.centre[3 * body[t] + 2];
        acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
    }

    for (int b = it.b0; active && b < it.b1; ++b) {
        bool use[TPL];
        bool any_use = false;
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            use[t] = valid[t] && !(a.skip_same && body[t] == b);
            any_use |= use[t];
        }
        if (!__any(any_use)) continue;
        const double cs0 = a.centre[3 * b + 0], cs1 = a.centre[3 * b + 1], cs2 = a.centre[3 * b + 2];
        float xr[TPL][3];
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            xr[t][0] = xt[t][0] + (float)(ct[t][0] - cs0);
            xr[t][1] = xt[t][1] + (float)(ct[t][1] - cs1);
            xr[t][2] = xt[t][2] + (float)(ct[t][2] - cs2);
        }
        int j0, j1;
        wave_range(a.src_ptr[b], a.src_ptr[b + 1], wv, j0, j1);
        if (stokes) {
            for (int jb = j0; jb < j1; jb += FLUSH) {
                const int je = min(jb + FLUSH, j1);
                float p[TPL][3];
#pragma unroll
                for (int t = 0; t < TPL; ++t) p[t][0] = p[t][1] = p[t][2] = 0.f;
                // four sources per 128-byte scalar load (s_load_dwordx16 pairs), then the tail
                const SrcS32 *__restrict__ ps = srcS + jb;
                const int n = je - jb;
                int k = 0;
                for (; k + 4 <= n; k += 4) {
                    const Src4 q = *reinterpret_cast<const Src4 *>(ps + k);
#pragma unroll
                    for (int u = 0; u < 4; ++u) stokes_pair<TPL>(xr, q.s[u].pos, q.s[u].str, p);
                }
                for (; k < n; ++k) stokes_pair<TPL>(xr, ps[k].pos, ps[k].str, p);
#pragma unroll
                for (int t = 0; t < TPL; ++t) {
                    acc[t][0] += use[t] ? (double)p[t][0] : 0.0;
                    acc[t][1] += use[t] ? (double)p[t][1] : 0.0;
                    acc[t][2] += use[t] ? (double)p[t][2] : 0.0;
                }
            }
        } else {
            // Laplace: each run of up to 64 sources is staged in this wave's own LDS slots by one
            // coalesced load (lane l fetches source jb + l) and read back by every lane
            // (broadcast), so the pair arithmetic takes the sources from VGPRs.  The slots belong
            // to one wave, whose LDS accesses complete in order: no workgroup barrier is needed.
            float4 *slot = stage + 64 * wv;
            for (int jb = j0; jb < j1; jb += FLUSH) {
                const int cnt = min(FLUSH, j1 - jb);
                float p[TPL];
#pragma unroll
                for (int t = 0; t < TPL; ++t) p[t] = 0.f;
                if (lane < cnt) slot[lane] = srcL[jb + lane];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 8
                for (int k = 0; k < cnt; ++k) {
                    const float4 y = slot[k];
#pragma unroll
                    for (int t = 0; t < TPL; ++t) {
                        const float d0 = xr[t][0] - y.x, d1 = xr[t][1] - y.y, d2 = xr[t][2] - y.z;
                        const float r2 = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
                        p[t] = __builtin_fmaf(y.w, __builtin_amdgcn_rsqf(r2), p[t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < TPL; ++t) acc[t][0] += use[t] ? (double)p[t] : 0.0;
                __builtin_amdgcn_wave_barrier();  // the next run's stores follow this run's reads
            }
        }
    }

    double sum[TPL * 3];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) sum[3 * t + c] = acc[t][c];
    if (!reduce_waves<TPL * 3>(sum, lds)) return;
    const int dim = stokes ? 3 : 1;
    double *out = a.out + (int64_t)it.split * a.out_stride;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        if (!valid[t]) continue;
        const int64_t o = it.out0 + (int64_t)dim * (idx[t] - it.t0);
        for (int c = 0; c < dim; ++c) {
            double v = a.alpha * it.scale * sum[3 * t + c];
            if (a.addend) v += a.addend[o + c];
            if (a.accumulate) v += out[o + c];
            out[o + c] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// FP64
// ---------------------------------------------------------------------------
template <int TPL>
__device__ __forceinline__ void f64_item(const KernelArgs &a, const P2PItem it, const double4 *__restrict__ trg_off,
                                         const SrcS64 *__restrict__ srcS, const SrcL64 *__restrict__ srcL,
                                         double *lds) {
    // an inactive system still writes its epilogue (pair sum 0), so outputs stay finite
    const bool active = !a.sys_active || a.sys_active[it.sys];
    const bool stokes = it.kind == MFS_STOKES;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    int idx[TPL];
    bool valid[TPL];
    int body[TPL];
    double ct[TPL][3];
    double xt[TPL][3];
    double acc[TPL][3];
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        idx[t] = it.t0 + lane + t * 64;
        valid[t] = idx[t] < it.t1;
        const int i = valid[t] ? idx[t] : it.t0;
        body[t] = a.trg_body[i];
        const double4 o = trg_off[i];
        xt[t][0] = o.x;
        xt[t][1] = o.y;
        xt[t][2] = o.z;
        ct[t][0] = a.centre[3 * body[t] + 0];
        ct[t][1] = a.centre[3 * body[t] + 1];
        ct[t][2] = a.centre[3 * body[t] + 2];
        acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
    }

    for (int b = it.b0; active && b < it.b1; ++b) {
        bool use[TPL];
        bool any_use = false;
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            use[t] = valid[t] && !(a.skip_same && body[t] == b);
            any_use |= use[t];
        }
        if (!__any(any_use)) continue;
        const double cs0 = a.centre[3 * b + 0], cs1 = a.centre[3 * b + 1], cs2 = a.centre[3 * b + 2];
        double xr[TPL][3];
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            xr[t][0] = xt[t][0] + (ct[t][0] - cs0);
            xr[t][1] = xt[t][1] + (ct[t][1] - cs1);
            xr[t][2] = xt[t][2] + (ct[t][2] - cs2);
        }
        int j0, j1;
        wave_range(a.src_ptr[b], a.src_ptr[b + 1], wv, j0, j1);
        double p[TPL][3];
#pragma unroll
        for (int t = 0; t < TPL; ++t) p[t][0] = p[t][1] = p[t][2] = 0.0;
        if (stokes) {
const SrcS64 *__restrict__ ps = srcS + j0;
#pragma unroll 2
            for (int k = 0; k < j1 - j0; ++k) {
                const SrcS64 &sj = ps[k];
                const double y0 = sj.pos[0], y1 = sj.pos[1], y2 = sj.pos[2];
                const double f0 = sj.str[0], f1 = sj.str[1], f2 = sj.str[2];
#pragma unroll
                for (int t = 0; t < TPL; ++t) {
                    const double d0 = xr[t][0] - y0, d1 = xr[t][1] - y1, d2 = xr[t][2] - y2;
                    const double r2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
                    const double ri = rsqrt_f64(r2);
                    const double df = __builtin_fma(d2, f2, __builtin_fma(d1, f1, d0 * f0));
                    const double s = df * (ri * ri);
                    p[t][0] = __builtin_fma(ri, __builtin_fma(s, d0, f0), p[t][0]);
                    p[t][1] = __builtin_fma(ri, __builtin_fma(s, d1, f1), p[t][1]);
                    p[t][2] = __builtin_fma(ri, __builtin_fma(s, d2, f2), p[t][2]);
                }
            }
        } else {
const SrcL64 *__restrict__ ps = srcL + j0;
#pragma unroll 4
            for (int k = 0; k < j1 - j0; ++k) {
                const SrcL64 &sj = ps[k];
                const double y0 = sj.v[0], y1 = sj.v[1], y2 = sj.v[2], q = sj.v[3];
#pragma unroll
                for (int t = 0; t < TPL; ++t) {
                    const double d0 = xr[t][0] - y0, d1 = xr[t][1] - y1, d2 = xr[t][2] - y2;
                    const double r2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
                    p[t][0] = __builtin_fma(q, rsqrt_f64(r2), p[t][0]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            acc[t][0] += use[t] ? p[t][0] : 0.0;
            acc[t][1] += use[t] ? p[t][1] : 0.0;
            acc[t][2] += use[t] ? p[t][2] : 0.0;
        }
    }

    double sum[TPL * 3];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) sum[3 * t + c] = acc[t][c];
    if (!reduce_waves<TPL * 3>(sum, lds)) return;
    const int dim = stokes ? 3 : 1;
    double *out = a.out + (int64_t)it.split * a.out_stride;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        if (!valid[t]) continue;
        const int64_t o = it.out0 + (int64_t)dim * (idx[t] - it.t0);
        for (int c = 0; c < dim; ++c) {
            double v = a.alpha * it.scale * sum[3 * t + c];
            if (a.addend) v += a.addend[o + c];
            if (a.accumulate) v += out[o + c];
            out[o + c] = v;
        }
    }
}

// One work item per workgroup, or (persistent mode) a fixed grid whose
// workgroups claim items from a counter until the list is exhausted; every
// workgroup ends with the claim that runs past the end, so the grid drains.
template <int TPL>
__global__ __launch_bounds__(BLOCK) void p2p_mixed_kernel(KernelArgs a, const float4 *__restrict__ trg_off,
                                                          const SrcS32 *__restrict__ srcS,
                                                          const SrcL32 *__restrict__ srcL) {
    __shared__ double lds[(WAVES - 1) * 3 * TPL * 64];
    __shared__ float4 stage[WAVES * 64];
    if (!a.queue) {
        mixed_item<TPL>(a, a.items[blockIdx.x], trg_off, srcS, srcL, lds, stage);
        return;
    }
    __shared__ int slot;
    for (;;) {
        __syncthreads();  // also orders the previous item's LDS reads before the next item's writes
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int k = slot;
        if (k >= a.n_items) break;
        mixed_item<TPL>(a, a.items[k], trg_off, srcS, srcL, lds, stage);
    }
}

template <int TPL>
__global__ __launch_bounds__(BLOCK) void p2p_f64_kernel(KernelArgs a, const double4 *__restrict__ trg_off,
                                                        const SrcS64 *__restrict__ srcS,
                                                        const SrcL64 *__restrict__ srcL) {
    __shared__ double lds[(WAVES - 1) * 3 * TPL * 64];
    if (!a.queue) {
        f64_item<TPL>(a, a.items[blockIdx.x], trg_off, srcS, srcL, lds);
        return;
    }
    __shared__ int slot;
    for (;;) {
        __syncthreads();  // also orders the previous item's LDS reads before the next item's writes
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int k = slot;
        if (k >= a.n_items) break;
        f64_item<TPL>(a, a.items[k], trg_off, srcS, srcL, lds);
    }
}

__global__ void reset_counter_kernel(int *c) { *c = 0; }

// Sum of split slices: out = (acc ? out : 0) + addend + sum_s partial[s]
__global__ void reduce_split_kernel(int64_t n, const double *__restrict__ partial, int64_t stride, int n_split,
                                    const double *__restrict__ addend, double *__restrict__ out, int accumulate) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += partial[k * stride + v];
    if (addend) s += addend[v];
    if (accumulate) s += out[v];
    out[v] = s;
}

// Reference point of every body for the standalone sums: its first source
// point (or first target point if it has no sources).
__global__ void body_ref_kernel(int64_t n_body, const int32_t *__restrict__ src_ptr,
                                const int32_t *__restrict__ trg_ptr, const double *__restrict__ src_xyz,
                                const double *__restrict__ trg_xyz, double *__restrict__ centre) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_body) return;
    const double *p = nullptr;
    if (src_ptr[b + 1] > src_ptr[b]) p = src_xyz + 3 * (int64_t)src_ptr[b];
    else if (trg_ptr[b + 1] > trg_ptr[b]) p = trg_xyz + 3 * (int64_t)trg_ptr[b];
    for (int c = 0; c < 3; ++c) centre[3 * b + c] = p ? p[c] : 0.0;
}

__global__ void fill_ids_kernel(int64_t n_body, const int32_t *__restrict__ ptr, int32_t *__restrict__ ids) {
    const int64_t b = blockIdx.x;
    if (b >= n_body) return;
    for (int32_t i = ptr[b] + threadIdx.x; i < ptr[b + 1]; i += blockDim.x) ids[i] = (int32_t)b;
}

__global__ void make_trg_off_kernel(int64_t n, const double *__restrict__ xyz, const int32_t *__restrict__ body,
                                    const double *__restrict__ centre, int prec, void *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = body[i];
    const double o0 = xyz[3 * i] - centre[3 * b], o1 = xyz[3 * i + 1] - centre[3 * b + 1],
                 o2 = xyz[3 * i + 2] - centre[3 * b + 2];
    if (prec == MFS_MIXED) reinterpret_cast<float4 *>(out)[i] = make_float4((float)o0, (float)o1, (float)o2, 0.f);
    else reinterpret_cast<double4 *>(out)[i] = make_double4(o0, o1, o2, 0.0);
}

__global__ void make_src_kernel(int64_t n, int kind, const double *__restrict__ xyz, const int32_t *__restrict__ body,
                                const double *__restrict__ centre, const double *__restrict__ str, int prec,
                                void *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int b = body[j];
    const double o0 = xyz[3 * j] - centre[3 * b], o1 = xyz[3 * j + 1] - centre[3 * b + 1],
                 o2 = xyz[3 * j + 2] - centre[3 * b + 2];
    if (kind == MFS_STOKES) {
        const double s0 = str ? str[3 * j] : 0.0, s1 = str ? str[3 * j + 1] : 0.0, s2 = str ? str[3 * j + 2] : 0.0;
        if (prec == MFS_MIXED) {
            SrcS32 v;
            v.pos = make_float4((float)o0, (float)o1, (float)o2, 0.f);
            v.str = make_float4((float)s0, (float)s1, (float)s2, 0.f);
            reinterpret_cast<SrcS32 *>(out)[j] = v;
        } else {
            SrcS64 v = {{o0, o1, o2, 0.0}, {s0, s1, s2, 0.0}};
            reinterpret_cast<SrcS64 *>(out)[j] = v;
        }
    } else {
        const double q = str ? str[j] : 0.0;
        if (prec == MFS_MIXED) reinterpret_cast<float4 *>(out)[j] = make_float4((float)o0, (float)o1, (float)o2, (float)q);
        else reinterpret_cast<SrcL64 *>(out)[j] = SrcL64{{o0, o1, o2, q}};
    }
}

}  // namespace

P2PItems items_of(const P2PPlan &pp) {
    P2PItems it;
    it.items = pp.d_items.as<P2PItem>();
    it.n_items = (int)pp.items.size();
    it.n_split = pp.n_split;
    it.tpl = pp.tpl;
    it.persistent = pp.persistent;
    it.persistent_grid = pp.persistent_grid;
    it.counter = pp.d_counter.as<int>();
    return it;
}

int launch_p2p(const P2PItems &pp, const P2PLaunch &L, hipStream_t s) {
    if (pp.n_items == 0) return MFS_OK;
    KernelArgs a;
    a.items = pp.items;
    a.centre = L.centre;
    a.trg_body = L.trg_body;
    a.src_ptr = L.src_ptr;
    a.sys_active = L.sys_active;
    a.alpha = L.alpha;
    a.skip_same = L.skip_same ? 1 : 0;
    const bool direct = pp.n_split == 1;
    a.out = direct ? L.out : L.partial;
    a.addend = direct ? L.addend : nullptr;
    a.accumulate = direct ? (L.accumulate ? 1 : 0) : 0;
    a.out_stride = L.n_val;
    a.n_items = pp.n_items;
    a.queue = nullptr;
    dim3 grid((unsigned)pp.n_items);
    if (pp.persistent) {
        a.queue = pp.counter;
        grid = dim3((unsigned)std::min(pp.n_items, pp.persistent_grid));
        reset_counter_kernel<<<1, 1, 0, s>>>(a.queue);
        MFS_HIP_TRY(hipGetLastError());
    }
    if (L.ev_start) MFS_HIP_TRY(hipEventRecord(L.ev_start, s));
    if (L.prec == MFS_MIXED) {
        if (pp.tpl == 2)
            p2p_mixed_kernel<2><<<grid, BLOCK, 0, s>>>(a, (const float4 *)L.trg_off, (const SrcS32 *)L.srcS,
                                                       (const SrcL32 *)L.srcL);
        else
            p2p_mixed_kernel<1><<<grid, BLOCK, 0, s>>>(a, (const float4 *)L.trg_off, (const SrcS32 *)L.srcS,
                                                       (const SrcL32 *)L.srcL);
    } else {
        if (pp.tpl == 2)
            p2p_f64_kernel<2><<<grid, BLOCK, 0, s>>>(a, (const double4 *)L.trg_off, (const SrcS64 *)L.srcS,
                                                     (const SrcL64 *)L.srcL);
        else
            p2p_f64_kernel<1><<<grid, BLOCK, 0, s>>>(a, (const double4 *)L.trg_off, (const SrcS64 *)L.srcS,
                                                     (const SrcL64 *)L.srcL);
    }
    MFS_HIP_TRY(hipGetLastError());
    if (L.ev_stop) MFS_HIP_TRY(hipEventRecord(L.ev_stop, s));
    if (!direct) {
        const int64_t n = L.n_val;
        reduce_split_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, L.partial, L.n_val, pp.n_split, L.addend,
                                                                      L.out, L.accumulate ? 1 : 0);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

int launch_body_refpoint(int64_t n_body, const int32_t *src_ptr, const int32_t *trg_ptr, const double *src_xyz,
                         const double *trg_xyz, double *centre, hipStream_t s) {
    if (n_body == 0) return MFS_OK;
    body_ref_kernel<<<(unsigned)((n_body + 127) / 128), 128, 0, s>>>(n_body, src_ptr, trg_ptr, src_xyz, trg_xyz,
                                                                     centre);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_fill_body_ids(int64_t n_body, const int32_t *ptr, int32_t *ids, hipStream_t s) {
    if (n_body == 0) return MFS_OK;
    fill_ids_kernel<<<(unsigned)n_body, 256, 0, s>>>(n_body, ptr, ids);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_make_trg_off(int64_t n, const double *xyz, const int32_t *body, const double *centre, int prec,
                        void *out, hipStream_t s) {
    if (n == 0) return MFS_OK;
    make_trg_off_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, xyz, body, centre, prec, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_make_src(int64_t n, int kind, const double *xyz, const int32_t *body, const double *centre,
                    const double *str, int prec, void *out, hipStream_t s) {
    if (n == 0) return MFS_OK;
    make_src_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, kind, xyz, body, centre, str, prec, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
