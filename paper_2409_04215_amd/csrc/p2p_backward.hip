// Position gradients of the pair sums, gfx950.
//
// For the pairing Phi = sum_i sum_j w_i . G(x_i - y_j) s_j over the pair set of
// the forward sum, with d = x - y, r = |d|:
//   Stokes:  dPhi_ij/dd = [-(w.s) d + (w.d) s + (s.d) w - 3 (w.d)(s.d) d / r^2] / (8 pi mu r^3)
//   Laplace: dPhi_ij/dd = -w s d / (4 pi r^3)
// (derived from the kernels of Sections 2.1-2.2; the paper has no gradients).
//
// One kernel computes, per lane point p carrying vector a_p,
//   g_p = sum_q dPhi/dd (d = p - q; w = a_p, s = b_q)
// over the lane's pair set.  Run on the forward orientation (lanes =
// collocation points with w, sources = proxies with s) it gives dPhi/dx_i.
// Because dPhi_ij/dd is odd in d and symmetric in (w, s), the same kernel run
// on the transposed orientation (lanes = proxies with s, sources = collocation
// points with w) gives dPhi/dy_j = -sum_i dPhi_ij/dd directly.
//
// The walk is the one of the forward sum: an item of 64 lane points, the four
// waves of the workgroup each taking a contiguous quarter of every source body
// (wave-uniform loop, scalar loads, SGPR operands), the partial gradients added
// in wave order through LDS, same-body handling and mixed FP32-pair /
// FP64-accumulation precision exactly as there.
#include "device_math.h"
#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr int FLUSH = 64;

struct GradArgs {
    const P2PItem *items;
    const double *centre;
    const int32_t *lane_body;
    const int32_t *src_ptr;
    const double *lane_vec;  // lane vectors, indexed like the forward output (out0 + dim*(i - t0))
    double *out;             // [n_lane][3] (split slices of stride out_stride)
    int64_t out_stride;
    double alpha;
    int skip_same;
    int accumulate;
};

template <class T>
struct Vec3 { T x, y, z; };

template <bool MIXED>
__global__ __launch_bounds__(BLOCK) void p2p_grad_kernel(GradArgs a, const void *__restrict__ lane_off_v,
                                                         const void *__restrict__ srcS_v,
                                                         const void *__restrict__ srcL_v) {
    typedef typename std::conditional<MIXED, float, double>::type R;
    __shared__ double lds[(WAVES - 1) * 3 * 64];
    const P2PItem it = a.items[blockIdx.x];
    const bool stokes = it.kind == MFS_STOKES;
    const int dim = stokes ? 3 : 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = it.t0 + lane;
    const bool valid = i < it.t1;
    const int ii = valid ? i : it.t0;
    const int body = a.lane_body[ii];
    double ct[3] = {a.centre[3 * body], a.centre[3 * body + 1], a.centre[3 * body + 2]};
    R xt[3];
    if (MIXED) {
        const float4 o = reinterpret_cast<const float4 *>(lane_off_v)[ii];
        xt[0] = o.x; xt[1] = o.y; xt[2] = o.z;
    } else {
        const double4 o = reinterpret_cast<const double4 *>(lane_off_v)[ii];
        xt[0] = (R)o.x; xt[1] = (R)o.y; xt[2] = (R)o.z;
    }
    const int64_t vo = it.out0 + (int64_t)dim * (ii - it.t0);
    R w[3];
    w[0] = (R)a.lane_vec[vo];
    w[1] = stokes ? (R)a.lane_vec[vo + 1] : R(0);
    w[2] = stokes ? (R)a.lane_vec[vo + 2] : R(0);
    double acc[3] = {0.0, 0.0, 0.0};

    for (int b = it.b0; b < it.b1; ++b) {
        const bool use = valid && !(a.skip_same && body == b);
        if (!__any(use)) continue;
        R xr[3];
        for (int c = 0; c < 3; ++c) xr[c] = xt[c] + (R)(ct[c] - a.centre[3 * b + c]);
        // this wave's contiguous quarter of the body's sources
        const int s0 = a.src_ptr[b], s1 = a.src_ptr[b + 1];
        const int qn = (s1 - s0 + WAVES - 1) / WAVES;
        const int j0 = min(s0 + wv * qn, s1), j1 = min(j0 + qn, s1);
        for (int jb = j0; jb < j1; jb += FLUSH) {
            const int je = min(jb + FLUSH, j1);
            R p0 = 0, p1 = 0, p2 = 0;
            if (stokes) {
#pragma unroll 2
                for (int j = jb; j < je; ++j) {
                    R y0, y1, y2, s0, s1, s2;
                    if (MIXED) {
                        const SrcS32 &sj = reinterpret_cast<const SrcS32 *>(srcS_v)[j];
                        y0 = sj.pos.x; y1 = sj.pos.y; y2 = sj.pos.z;
                        s0 = sj.str.x; s1 = sj.str.y; s2 = sj.str.z;
                    } else {
                        const SrcS64 &sj = reinterpret_cast<const SrcS64 *>(srcS_v)[j];
                        y0 = sj.pos[0]; y1 = sj.pos[1]; y2 = sj.pos[2];
                        s0 = sj.str[0]; s1 = sj.str[1]; s2 = sj.str[2];
                    }
                    const R d0 = xr[0] - y0, d1 = xr[1] - y1, d2 = xr[2] - y2;
                    const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    R ri;
                    if (MIXED) ri = __builtin_amdgcn_rsqf((float)r2);
                    else ri = (R)rsqrt_f64((double)r2);
                    const R ri2 = ri * ri;
                    const R c3 = ri * ri2;
                    const R ws = w[0] * s0 + w[1] * s1 + w[2] * s2;
                    const R wd = w[0] * d0 + w[1] * d1 + w[2] * d2;
                    const R sd = s0 * d0 + s1 * d1 + s2 * d2;
                    const R k = -ws - R(3) * wd * sd * ri2;
                    p0 += c3 * (k * d0 + wd * s0 + sd * w[0]);
                    p1 += c3 * (k * d1 + wd * s1 + sd * w[1]);
                    p2 += c3 * (k * d2 + wd * s2 + sd * w[2]);
                }
            } else {
#pragma unroll 4
                for (int j = jb; j < je; ++j) {
                    R y0, y1, y2, q;
                    if (MIXED) {
                        const float4 sj = reinterpret_cast<const float4 *>(srcL_v)[j];
                        y0 = sj.x; y1 = sj.y; y2 = sj.z; q = sj.w;
                    } else {
                        const SrcL64 &sj = reinterpret_cast<const SrcL64 *>(srcL_v)[j];
                        y0 = sj.v[0]; y1 = sj.v[1]; y2 = sj.v[2]; q = sj.v[3];
                    }
                    const R d0 = xr[0] - y0, d1 = xr[1] - y1, d2 = xr[2] - y2;
                    const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    R ri;
                    if (MIXED) ri = __builtin_amdgcn_rsqf((float)r2);
                    else ri = (R)rsqrt_f64((double)r2);
                    const R c = -w[0] * q * ri * ri * ri;
                    p0 += c * d0;
                    p1 += c * d1;
                    p2 += c * d2;
                }
            }
            acc[0] += use ? (double)p0 : 0.0;
            acc[1] += use ? (double)p1 : 0.0;
            acc[2] += use ? (double)p2 : 0.0;
        }
    }
    // waves 1..3 hand their partial gradients to wave 0, which adds them in wave order
    if (wv > 0)
        for (int c = 0; c < 3; ++c) lds[((wv - 1) * 3 + c) * 64 + lane] = acc[c];
    __syncthreads();
    if (wv > 0) return;
    for (int w = 1; w < WAVES; ++w)
        for (int c = 0; c < 3; ++c) acc[c] += lds[((w - 1) * 3 + c) * 64 + lane];
    if (!valid) return;
    double *out = a.out + (int64_t)it.split * a.out_stride + 3 * (int64_t)i;
    for (int c = 0; c < 3; ++c) {
        double v = a.alpha * it.scale * acc[c];
        if (a.accumulate) v += out[c];
        out[c] = v;
    }
}

__global__ void reduce3_kernel(int64_t n, const double *__restrict__ partial, int64_t stride, int n_split,
                               double *__restrict__ out, int accumulate) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += partial[k * stride + v];
    if (accumulate) s += out[v];
    out[v] = s;
}

}  // namespace

// lane vectors `lane_vec` indexed in the items' output layout; gradient out [n_lane][3]
int launch_p2p_grad(const P2PPlan &pp, const P2PLaunch &L, const double *lane_vec, int64_t n_lane, hipStream_t s) {
    if (pp.items.empty()) return MFS_OK;
    if (pp.tpl != 1) return fail(MFS_EINVAL, "gradient pair sums take items of one target per lane");
    GradArgs a;
    a.items = pp.d_items.as<P2PItem>();
    a.centre = L.centre;
    a.lane_body = L.trg_body;
    a.src_ptr = L.src_ptr;
    a.lane_vec = lane_vec;
    a.alpha = L.alpha;
    a.skip_same = L.skip_same ? 1 : 0;
    const bool direct = pp.n_split == 1;
    a.out = direct ? L.out : L.partial;
    a.out_stride = 3 * n_lane;
    a.accumulate = direct ? (L.accumulate ? 1 : 0) : 0;
    const dim3 grid((unsigned)pp.items.size());
    if (L.prec == MFS_MIXED) p2p_grad_kernel<true><<<grid, BLOCK, 0, s>>>(a, L.trg_off, L.srcS, L.srcL);
    else p2p_grad_kernel<false><<<grid, BLOCK, 0, s>>>(a, L.trg_off, L.srcS, L.srcL);
    MFS_HIP_TRY(hipGetLastError());
    if (!direct) {
        const int64_t n = 3 * n_lane;
        reduce3_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, L.partial, n, pp.n_split, L.out,
                                                                 L.accumulate ? 1 : 0);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

}  // namespace mfs
