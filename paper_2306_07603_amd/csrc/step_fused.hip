// step_fused.hip -- one launch per IFDLBM time step (arXiv:2306.07603,
// Section 4, Steps (2)-(6)); each wavefront reads the state of its work item
// once from HBM and writes it once.
//
// Work item: output columns [i0, i1) and rows [j0, j1) of one cavity.  The 64
// lanes of the wavefront hold columns i0 - 4 .. i0 + 59, one column per lane,
// and march up the rows.  At row t of the march:
//   A  (row t)     f-hat and lambda (prefetched one row ahead): moments,
//                  lambda (Step 2), f-bar+ (Eq. 2.16)
//   B  (row t - 2) f-bar(t + dt/2) by Eq. (3.7), walls by extrapolation, and
//                  f(t + dt/2) by Eq. (2.17)
//   C  (row t - 4) f-hat+ (Eq. 2.15) recomputed from f-hat of row t - 4
//                  (read again; it is still in L2), f-hat(t + dt) by
//                  Eq. (3.6), walls by extrapolation (Step 6), store, residual
//                  partial sums of Eq. (2.19)
// The eta-direction stencils read five-row register rings of f-bar+ and
// f(t + dt/2); the xi-direction stencils read neighbour lanes through one LDS
// row per population.  The halo costs 8 of 64 lanes across xi and 8 + 4
// recomputed rows per segment along eta.  The bottom wall row is produced with
// row 1 (its extrapolation source), the lid row from the row below it.
#include "ifdlbm_internal.h"

namespace ifd {
namespace {

constexpr int kPad = 2;
constexpr int kXcds = 8;   // MI355X: workgroups are dealt to the 8 XCDs in turn

template <typename T> __device__ __forceinline__ const T* geo_of(const StepArgs& a);
template <> __device__ __forceinline__ const double* geo_of<double>(const StepArgs& a) { return a.geo; }
template <> __device__ __forceinline__ const float* geo_of<float>(const StepArgs& a) { return a.geo32; }

// Work item of block b among nw: consecutive items (neighbouring strips and
// segments, which share halo rows and columns) go to the same XCD and L2.
__device__ __forceinline__ int xcd_order(int b, int nw)
{
    const int q = nw / kXcds, r = nw % kXcds, x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}

// Weights of Eq. (2.5) times sign(c) * 2h on the upwind-sorted points a2
// (two behind), a1 (one behind), c0 and f1 (one ahead):
// sign(c) * central = f1 - a1 (Eq. 2.6), sign(c) * upwind = 3 c0 - 4 a1 + a2
// (Eq. 2.7), so eps * central + (1 - eps) * upwind is
// eps f1 - (4 - 3 eps) a1 + 3 (1 - eps) c0 + (1 - eps) a2.
template <typename T>
struct MixedWeights {
    T wf, wa1, wc, wa2;
    __device__ __forceinline__ explicit MixedWeights(T eps)
        : wf(eps), wa1(-(T(4) - T(3) * eps)), wc(T(3) * (T(1) - eps)), wa2(T(1) - eps)
    {
    }
    __device__ __forceinline__ T apply(T a2, T a1, T c0, T f1) const { return ((wc * c0 + wa1 * a1) + wa2 * a2) + wf * f1; }
};

// c_k . grad Phi_k of Eq. (3.4) for the eight moving populations of one row,
// times the step, subtracted from `base`:
//   out[k] = base[k] - sx * |dk[k]| * D_xi - sy * D_eta
// where sx = step a_j / (2 dxi) and sy = step / (2 deta) and D are the signed
// mixed differences; the xi neighbours come from the LDS row, the eta
// neighbours from ring slots 0..4 (rows r-2..r+2).  Where the second upwind
// point would leave the grid (EDGE waves) it is replaced by the linear
// extrapolation 2 a1 - c0, which gives the first-order difference.
template <typename T, bool EDGE>
__device__ __forceinline__ void transport_row(T (*xs)[kWaveLanes + 2 * kPad], int lane, const T (&ring)[5][9],
                                              const T (&base)[9], const T (&adk)[9], const bool (&pos)[9],
                                              const bool (&edge)[9], bool lo_eta, bool hi_eta, T sx, T sy,
                                              const MixedWeights<T>& w, T (&out)[9])
{
#pragma unroll
    for (int k = 1; k < 9; ++k) xs[k - 1][lane + kPad] = ring[2][k];
    __syncthreads();
    out[0] = base[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const T* row = xs[k - 1];
        const T c0 = ring[2][k];
        const T m2 = row[lane + kPad - 2], m1 = row[lane + kPad - 1];
        const T p1 = row[lane + kPad + 1], p2 = row[lane + kPad + 2];
        const T a1 = pos[k] ? m1 : p1;
        T a2 = pos[k] ? m2 : p2;
        const T f1 = pos[k] ? p1 : m1;
        if (EDGE) a2 = edge[k] ? T(2) * a1 - c0 : a2;
        T o = base[k] - (sx * adk[k]) * w.apply(a2, a1, c0, f1);
        if (cyk(k) != 0) {
            // sign of c_k,eta = c_ky is fixed by k
            const bool up = cyk(k) > 0;
            const T e1 = up ? ring[1][k] : ring[3][k];
            T e2 = up ? ring[0][k] : ring[4][k];
            const T g1 = up ? ring[3][k] : ring[1][k];
            if ((up && lo_eta) || (!up && hi_eta)) e2 = T(2) * e1 - c0;
            o = o - sy * w.apply(e2, e1, c0, g1);
        }
        out[k] = o;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void publish(T (*w)[9], int i, int nx, const T (&x)[9])
{
    if (i == 1)
#pragma unroll
        for (int k = 0; k < 9; ++k) w[0][k] = x[k];
    if (i == nx - 2)
#pragma unroll
        for (int k = 0; k < 9; ++k) w[1][k] = x[k];
}

// Extrapolation source of a wall node: its inward neighbour at the same level,
// which is the lane's own `own` for interior columns and the published values
// of column 1 or nx - 2 for the two side columns.
template <typename T>
__device__ __forceinline__ void wall_source(T (*w)[9], int i, int nx, const T (&own)[9], T (&src)[9])
{
    const int side = i <= 0 ? 0 : 1;
    const bool interior = i >= 1 && i <= nx - 2;
#pragma unroll
    for (int k = 0; k < 9; ++k) src[k] = interior ? own[k] : w[side][k];
}

template <typename T>
__device__ __forceinline__ void half_step(const T (&fb)[9], T lam, T dt, T (&out)[9])
{
    T P, ux, uy, e[9];
    moments(fb, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const HalfStep<T> hs(lam, dt);
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = hs.a * fb[k] + hs.b * e[k];
}

template <typename T>
__device__ __forceinline__ void residual_add(const T (&gn)[9], const T (&old)[3], double (&acc)[kPartials])
{
    T P, ux, uy;
    moments(gn, P, ux, uy);
    const double du = (double)ux - (double)old[1], dv = (double)uy - (double)old[2], dp = (double)P - (double)old[0];
    acc[0] += du * du + dv * dv;
    acc[1] += (double)ux * ux + (double)uy * uy;
    acc[2] += dp * dp;
    acc[3] += (double)P * P;
    acc[4] += dp;
    acc[5] += (double)P;
    acc[6] += (isfinite((double)ux) && isfinite((double)uy) && isfinite((double)P)) ? 0.0 : 1.0;
}

// LDS of one wavefront.
template <typename T>
struct WaveLds {
    T xs[8][kWaveLanes + 2 * kPad];   // one row of each moving population, for the xi stencils
    T wb[2][9];                       // f-bar of columns 1 and nx-2 at the current half-step row
    T wc[2][9];                       // f-hat(t+dt) of columns 1 and nx-2 at the current full-step row
    T keep_b[9][kWaveLanes];          // f-bar of row ny-2, source of the lid row
    T keep_c[9][kWaveLanes];          // f-hat(t+dt) of row ny-2, source of the lid row
};

template <int PREC, bool RES, bool EDGE>
__device__ __forceinline__ void fused_item(const StepArgs& a, const StripItem& it, const CavityDesc& c,
                                           WaveLds<typename Storage<PREC>::T>& sh, double (&acc)[kPartials])
{
    using S = Storage<PREC>;
    using T = typename S::T;
    auto& xs = sh.xs;
    auto& wb = sh.wb;
    auto& wc = sh.wc;
    auto& keep_b = sh.keep_b;
    auto& keep_c = sh.keep_c;

    const int lane = threadIdx.x;
    const int nx = c.nx, ny = c.ny;
    const int i = it.i0 - kHaloCols + lane;
    // halo lanes outside the grid read the nearest column; their results are never used
    const int ic = min(max(i, 0), nx - 1);
    const bool out_col = i >= it.i0 && i < it.i1;
    const bool walls_b = it.i0 <= 2 || it.i1 >= nx - 2;
    const bool walls_c = it.i0 == 0 || it.i1 == nx;
    const PowerLaw<T> pl(c);
    const T dt = pl.dt, ulid = T(c.u_lid);
    const T sy_b = T(0.5) * dt * T(c.inv2deta), sy_c = dt * T(c.inv2deta);
    const T sx_b = T(0.5) * dt * T(c.inv2dxi), sx_c = dt * T(c.inv2dxi);
    const MixedWeights<T> mw(T(c.mix));

    // uniform base of each plane (64-bit, scalar) plus a 32-bit row offset per lane
    const auto* fin = static_cast<const typename S::F*>(a.f_in) + c.f_off;
    const auto* lin = static_cast<const typename S::L*>(a.l_in) + c.l_off;
    auto* fout = static_cast<typename S::F*>(a.f_out) + c.f_off;
    auto* lout = static_cast<typename S::L*>(a.l_out) + c.l_off;
    const int64_t plane = c.plane;
    const T* geo = geo_of<T>(a) + c.geo_off;
    const uint32_t lseed = S::kStochastic ? mix32(a.seed_ctr[0] ^ mix32(a.step)) : 0u;

    // c_kx - c_ky s_i: the contravariant xi-velocity is a_j times this (Eqs. 3.2-3.8.2)
    const T s = geo[ny + ic];
    T adk[9];
    bool pos[9], edge[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const T d = T(cxk(k)) - T(cyk(k)) * s;
        pos[k] = d >= T(0);
        adk[k] = pos[k] ? d : -d;
        edge[k] = pos[k] ? (i == 1) : (i == nx - 2);
    }

    T gbp[5][9], fh[5][9], lamr[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        lamr[r] = T(1);
#pragma unroll
        for (int k = 0; k < 9; ++k) gbp[r][k] = fh[r][k] = T(0);
    }
    T mom0[3] = {0, 0, 0};

    const int j0 = it.j0, j1 = it.j1;
    const int qlo = max(j0 - 2, 0), qhi = min(j1 + 1, ny - 1);
    const int t_begin = max(j0 - 4, 0), t_end = j1 + 3, t_last = min(t_end, ny - 1);

    // row t_begin, fetched ahead of the loop
    T gn_[9], ln_;
    {
        const uint32_t o = (uint32_t)(t_begin * c.pitch + ic);
#pragma unroll
        for (int k = 0; k < 9; ++k) gn_[k] = S::load(fin + k * plane, o, k);
        ln_ = T(lin[o]);
    }

#pragma unroll 1
    for (int t = t_begin; t <= t_end; ++t) {
        T g[9], lam_old = ln_;
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = gn_[k];
        // fetch row t + 1 now; it is consumed in the next iteration
        if (t + 1 <= t_last) {
            const uint32_t o = (uint32_t)((t + 1) * c.pitch + ic);
#pragma unroll
            for (int k = 0; k < 9; ++k) gn_[k] = S::load(fin + k * plane, o, k);
            ln_ = T(lin[o]);
        }
        // f-hat of row t - 4 for stage C (read 4 rows ago, now an L2 hit)
        const int p = t - 4;
        const bool do_c = p >= j0 && p < j1;
        T gc[9];
        if (do_c) {
            const uint32_t o = (uint32_t)(p * c.pitch + ic);
#pragma unroll
            for (int k = 0; k < 9; ++k) gc[k] = S::load(fin + k * plane, o, k);
        }

        // ---------------------------------------------------------- A: row t
        if (t <= ny - 1) {
            T P, ux, uy, e[9];
            moments(g, P, ux, uy);
            equilibrium(P, ux, uy, e);
            const T lam = relaxation_time(g, e, lam_old, pl);
            const Collision<T> coll(lam, dt);
#pragma unroll
            for (int k = 0; k < 9; ++k) gbp[4][k] = coll.a_bar * g[k] + coll.b_bar * e[k];
            lamr[4] = lam;
        }

        // ---------------------------------------------------------- B: row t - 2
        const int q = t - 2;
        if (q >= qlo && q <= qhi) {
            T fb[9];
            if (q >= 1 && q <= ny - 2) {
                transport_row<T, EDGE>(xs, lane, gbp, gbp[2], adk, pos, edge, q == 1, q == ny - 2, sx_b * geo[q], sy_b,
                                       mw, fb);
                if (walls_b) {
                    publish(wb, i, nx, fb);
                    __syncthreads();
                    if (i == 0 || i == nx - 1) {
                        T src[9];
                        wall_source(wb, i, nx, fb, src);
                        extrapolate(src, T(0), fb);
                    }
                }
                if (q == 1) {   // bottom wall row from row 1 (Eq. 1.5: at rest)
                    T src[9], fb0[9], out0[9];
                    wall_source(wb, i, nx, fb, src);
                    extrapolate(src, T(0), fb0);
                    half_step(fb0, lamr[1], dt, out0);
#pragma unroll
                    for (int k = 0; k < 9; ++k) fh[3][k] = out0[k];
                }
                if (q == ny - 2)
#pragma unroll
                    for (int k = 0; k < 9; ++k) keep_b[k][lane] = fb[k];
            } else if (q == ny - 1) {   // lid row from row ny - 2
                T own[9], src[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) own[k] = keep_b[k][lane];
                wall_source(wb, i, nx, own, src);
                extrapolate(src, ulid, fb);
            }
            if (q >= 1) {
                T out[9];
                half_step(fb, lamr[2], dt, out);
#pragma unroll
                for (int k = 0; k < 9; ++k) fh[4][k] = out[k];
            }
        }

        // ---------------------------------------------------------- C: row t - 4
        if (do_c) {
            const uint32_t node = (uint32_t)(p * c.pitch + ic);
            if (out_col) lout[node] = (typename S::L)lamr[0];
            T old[3];
            moments(gc, old[0], old[1], old[2]);
            if (p >= 1 && p <= ny - 2) {
                // f-hat+ of row p (Eq. 2.15) from its f-hat and the lambda of stage A
                T e[9], hp[9], gn[9];
                equilibrium(old[0], old[1], old[2], e);
                const Collision<T> coll(lamr[0], dt);
#pragma unroll
                for (int k = 0; k < 9; ++k) hp[k] = coll.a_hat * gc[k] + coll.b_hat * e[k];
                transport_row<T, EDGE>(xs, lane, fh, hp, adk, pos, edge, p == 1, p == ny - 2, sx_c * geo[p], sy_c, mw, gn);
                if (walls_c) {
                    publish(wc, i, nx, gn);
                    __syncthreads();
                    if (i == 0 || i == nx - 1) {
                        T src[9];
                        wall_source(wc, i, nx, gn, src);
                        extrapolate(src, T(0), gn);
                    }
                }
                if (out_col) {
                    const uint32_t ns = S::kStochastic ? node_seed(lseed, it.cav, p, i) : 0u;
#pragma unroll
                    for (int k = 0; k < 9; ++k) store_state<S>(fout + k * plane, node, k, gn[k], ns);
                    if (RES) residual_add(gn, old, acc);
                }
                if (p == 1 && j0 == 0) {   // bottom wall row from row 1
                    T src[9], g0[9];
                    wall_source(wc, i, nx, gn, src);
                    extrapolate(src, T(0), g0);
                    if (out_col) {
                        const uint32_t ns = S::kStochastic ? node_seed(lseed, it.cav, 0, i) : 0u;
#pragma unroll
                        for (int k = 0; k < 9; ++k) store_state<S>(fout + k * plane, (uint32_t)ic, k, g0[k], ns);
                        if (RES) residual_add(g0, mom0, acc);
                    }
                }
                if (p == ny - 2)
#pragma unroll
                    for (int k = 0; k < 9; ++k) keep_c[k][lane] = gn[k];
            } else if (p == ny - 1) {   // lid row from row ny - 2
                T own[9], src[9], gn[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) own[k] = keep_c[k][lane];
                wall_source(wc, i, nx, own, src);
                extrapolate(src, ulid, gn);
                if (out_col) {
                    const uint32_t ns = S::kStochastic ? node_seed(lseed, it.cav, p, i) : 0u;
#pragma unroll
                    for (int k = 0; k < 9; ++k) store_state<S>(fout + k * plane, node, k, gn[k], ns);
                    if (RES) residual_add(gn, old, acc);
                }
            } else {   // p == 0: stored with row 1; keep its old moments
#pragma unroll
                for (int m = 0; m < 3; ++m) mom0[m] = old[m];
            }
        }

        // ---------------------------------------------------------- rings
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lamr[r] = lamr[r + 1];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                gbp[r][k] = gbp[r + 1][k];
                fh[r][k] = fh[r + 1][k];
            }
        }
    }
}

template <int PREC, bool RES>
__global__ __launch_bounds__(kWaveLanes) void k_fused(StepArgs a, const StripItem* items, int w0, int nw)
{
    const int w = w0 + xcd_order(blockIdx.x, nw);
    const StripItem it = items[w];
    const CavityDesc c = a.desc[it.cav];
    __shared__ WaveLds<typename Storage<PREC>::T> sh;
    double acc[kPartials] = {0, 0, 0, 0, 0, 0, 0};
    // waves that hold column 1 or nx-2 take the first-order one-sided points (Eq. 2.7 at walls)
    if (it.i0 <= 5 || it.i1 >= c.nx - 5)
        fused_item<PREC, RES, true>(a, it, c, sh, acc);
    else
        fused_item<PREC, RES, false>(a, it, c, sh, acc);
    if (RES) {
        // wavefront sum in a fixed order
#pragma unroll
        for (int q5 = 0; q5 < kPartials; ++q5) {
            double v = acc[q5];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWaveLanes);
            if (threadIdx.x == 0) a.partial[(int64_t)w * kPartials + q5] = v;
        }
    }
}

template <int PREC>
hipError_t fused(const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    if (nw <= 0) return hipSuccess;
    if (residual)
        hipLaunchKernelGGL((k_fused<PREC, true>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0, nw);
    else
        hipLaunchKernelGGL((k_fused<PREC, false>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0, nw);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_step(int prec, const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    switch (prec) {
    case P_FP64: return fused<P_FP64>(a, items, w0, nw, residual, s);
    case P_FP32: return fused<P_FP32>(a, items, w0, nw, residual, s);
    case P_FP16DEV: return fused<P_FP16DEV>(a, items, w0, nw, residual, s);
    case P_FP32X: return fused<P_FP32X>(a, items, w0, nw, residual, s);
    case P_FP32SR: return fused<P_FP32SR>(a, items, w0, nw, residual, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace ifd
