// step_fused.hip -- one launch per IFDLBM time step (arXiv:2306.07603,
// Section 4, Steps (2)-(6)); each wavefront reads the state of its work item
// once and writes it once.
//
// Work item: output columns [i0, i1) and rows [j0, j1) of one cavity.  The 64
// lanes of the wavefront hold columns i0 - 4 .. i0 + 59, one column per lane,
// and march up the rows.  At row t of the march:
//   A  (row t)     load f-hat and lambda, moments, lambda (Step 2), f-hat+
//                  and f-bar+ (Eqs. 2.15-2.16)
//   B  (row t - 2) f-bar(t + dt/2) by Eq. (3.7), walls by extrapolation, and
//                  f(t + dt/2) by Eq. (2.17)
//   C  (row t - 4) f-hat(t + dt) by Eq. (3.6), walls by extrapolation (Step 6),
//                  store, residual partial sums of Eq. (2.19)
// The eta-direction stencils read five-row register rings; the xi-direction
// stencils read neighbour lanes through a 64-entry LDS row per population.
// The halo costs 8 of 64 lanes across xi and 8 + 4 recomputed rows per
// segment along eta.  The bottom wall row is produced together with row 1 (its
// extrapolation source), the top wall row from the row below it.
#include "ifdlbm_internal.h"

namespace ifd {
namespace {

constexpr int kPad = 2;

template <typename T> __device__ __forceinline__ const T* geo_of(const StepArgs& a);
template <> __device__ __forceinline__ const double* geo_of<double>(const StepArgs& a) { return a.geo; }
template <> __device__ __forceinline__ const float* geo_of<float>(const StepArgs& a) { return a.geo32; }

// Second-order upwind or first-order one-sided part and central part of
// Eq. (2.5) along xi for one population, from the LDS row of the wavefront;
// returns eps * central + (1 - eps) * upwind, times 2 dxi.
template <typename T>
__device__ __forceinline__ T xi_diff(const T* row, int lane, T c0, bool pos, bool lo, bool hi, T eps)
{
    const T m2 = row[lane + kPad - 2], m1 = row[lane + kPad - 1];
    const T p1 = row[lane + kPad + 1], p2 = row[lane + kPad + 2];
    return mixed_diff_2h(m2, m1, c0, p1, p2, pos, lo, hi, eps);
}

// The same along eta for population k, from the ring slots of rows q-2..q+2;
// the sign of c_k,eta = c_ky is fixed by k.
template <typename T, int K>
__device__ __forceinline__ T eta_diff(const T (&ring)[5][9], bool lo, bool hi, T eps)
{
    return mixed_diff_2h(ring[0][K], ring[1][K], ring[2][K], ring[3][K], ring[4][K], cyk(K) > 0, lo, hi, eps);
}

// c_k . grad Phi_k (Eq. 3.4) times 2 dxi resp. 2 deta folded into the scales:
// out[k] = base[k] - step * (sx * dk[k] * D_xi + cy_k * sy * D_eta).
template <typename T>
__device__ __forceinline__ void transport_row(T (*xs)[kWaveLanes + 2 * kPad], int lane, const T (&ring)[5][9],
                                              const T (&base)[9], const T (&dk)[9], const bool (&pos)[9], bool lo, bool hi,
                                              bool lo_eta, bool hi_eta, T sx, T sy, T step, T eps, T (&out)[9])
{
#pragma unroll
    for (int k = 1; k < 9; ++k) xs[k - 1][lane + kPad] = ring[2][k];
    __syncthreads();
    out[0] = base[0];
#define IFD_K(K)                                                                                   \
    {                                                                                              \
        const T dx = xi_diff(xs[K - 1], lane, ring[2][K], pos[K], lo, hi, eps);                    \
        T term = sx * dk[K] * dx;                                                                  \
        if (cyk(K) != 0) term += T(cyk(K)) * sy * eta_diff<T, K>(ring, lo_eta, hi_eta, eps);       \
        out[K] = base[K] - step * term;                                                            \
    }
    IFD_K(1) IFD_K(2) IFD_K(3) IFD_K(4) IFD_K(5) IFD_K(6) IFD_K(7) IFD_K(8)
#undef IFD_K
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

// Extrapolation source of a wall node at the same level: its own inward
// neighbour's values (same lane, `own`) for interior columns, the published
// values of column 1 or nx - 2 for the two side columns.
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

template <int PREC, bool RES>
__global__ __launch_bounds__(kWaveLanes) void k_fused(StepArgs a, const StripItem* items, int w0)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    __shared__ T xs[8][kWaveLanes + 2 * kPad];
    __shared__ T wb[2][9];   // f-bar of columns 1 and nx-2 at the current half-step row
    __shared__ T wc[2][9];   // f-hat(t+dt) of columns 1 and nx-2 at the current full-step row

    const StripItem it = items[w0 + blockIdx.x];
    const CavityDesc c = a.desc[it.cav];
    const int lane = threadIdx.x;
    const int nx = c.nx, ny = c.ny;
    const int i = it.i0 - kHaloCols + lane;
    const bool in_grid = i >= 0 && i < nx;
    const bool out_col = i >= it.i0 && i < it.i1;
    const bool lo = i == 1, hi = i == nx - 2;
    const bool walls_b = it.i0 <= 2 || it.i1 >= nx - 2;
    const bool walls_c = it.i0 == 0 || it.i1 == nx;
    const T dt = T(c.dt), half_dt = T(0.5) * dt, eps = T(c.mix), ulid = T(c.u_lid);
    const T inv2dxi = T(c.inv2dxi), inv2deta = T(c.inv2deta);

    const auto* fin = static_cast<const typename S::F*>(a.f_in);
    const auto* lin = static_cast<const typename S::L*>(a.l_in);
    auto* fout = static_cast<typename S::F*>(a.f_out);
    auto* lout = static_cast<typename S::L*>(a.l_out);
    const T* geo = geo_of<T>(a);

    // c_kx - c_ky s_i: the contravariant xi-velocity is a_j times this (Eqs. 3.2-3.8.2)
    const T s = in_grid ? geo[c.geo_off + ny + i] : T(0);
    T dk[9];
    bool pos[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        dk[k] = in_grid ? T(cxk(k)) - T(cyk(k)) * s : T(0);
        pos[k] = dk[k] >= T(0);
    }

    T gbp[5][9], ghp[5][9], fh[5][9], lamr[5], mom[5][3];
    T fbprev[9], gprev[9], mom0[3] = {0, 0, 0};
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        lamr[r] = T(1);
#pragma unroll
        for (int k = 0; k < 9; ++k) gbp[r][k] = ghp[r][k] = fh[r][k] = T(0);
#pragma unroll
        for (int q = 0; q < 3; ++q) mom[r][q] = T(0);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) fbprev[k] = gprev[k] = T(0);
    double acc[kPartials] = {0, 0, 0, 0, 0, 0, 0};

    const int j0 = it.j0, j1 = it.j1;
    const int qlo = max(j0 - 2, 0), qhi = min(j1 + 1, ny - 1);
    const int t_begin = max(j0 - 4, 0), t_end = j1 + 3;

#pragma unroll 1
    for (int t = t_begin; t <= t_end; ++t) {
        // ---------------------------------------------------------- A: row t
        if (t <= ny - 1) {
            T g[9], lo_lam = T(1);
            const int64_t node = (int64_t)t * c.pitch + i;
#pragma unroll
            for (int k = 0; k < 9; ++k) g[k] = in_grid ? S::load(fin, c.f_off + k * c.plane + node, k) : T(0);
            if (in_grid) lo_lam = T(lin[c.l_off + node]);
            T P, ux, uy, e[9];
            moments(g, P, ux, uy);
            equilibrium(P, ux, uy, e);
            const T lam = relaxation_time(g, e, lo_lam, c);
            const Collision<T> col(lam, dt);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                gbp[4][k] = col.a_bar * g[k] + col.b_bar * e[k];
                ghp[4][k] = col.a_hat * g[k] + col.b_hat * e[k];
            }
            lamr[4] = lam;
            mom[4][0] = P;
            mom[4][1] = ux;
            mom[4][2] = uy;
        }

        // ---------------------------------------------------------- B: row t - 2
        const int q = t - 2;
        if (q >= qlo && q <= qhi) {
            T fb[9];
            if (q >= 1 && q <= ny - 2) {
                const T sx = geo[c.geo_off + q] * inv2dxi;
                transport_row(xs, lane, gbp, gbp[2], dk, pos, lo, hi, q == 1, q == ny - 2, sx, inv2deta, half_dt, eps, fb);
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
                    for (int k = 0; k < 9; ++k) fbprev[k] = fb[k];
            } else if (q == ny - 1) {   // lid row from row ny - 2
                T src[9];
                wall_source(wb, i, nx, fbprev, src);
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
        const int p = t - 4;
        if (p >= j0 && p < j1) {
            const int64_t node = (int64_t)p * c.pitch + i;
            if (out_col) lout[c.l_off + node] = (typename S::L)lamr[0];
            if (p >= 1 && p <= ny - 2) {
                T gn[9];
                const T sx = geo[c.geo_off + p] * inv2dxi;
                transport_row(xs, lane, fh, ghp[0], dk, pos, lo, hi, p == 1, p == ny - 2, sx, inv2deta, dt, eps, gn);
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
#pragma unroll
                    for (int k = 0; k < 9; ++k) S::store(fout, c.f_off + k * c.plane + node, k, gn[k]);
                    if (RES) residual_add(gn, mom[0], acc);
                }
                if (p == 1 && j0 == 0) {   // bottom wall row from row 1
                    T src[9], g0[9];
                    wall_source(wc, i, nx, gn, src);
                    extrapolate(src, T(0), g0);
                    if (out_col) {
#pragma unroll
                        for (int k = 0; k < 9; ++k) S::store(fout, c.f_off + k * c.plane + i, k, g0[k]);
                        if (RES) residual_add(g0, mom0, acc);
                    }
                }
                if (p == ny - 2)
#pragma unroll
                    for (int k = 0; k < 9; ++k) gprev[k] = gn[k];
            } else if (p == ny - 1) {   // lid row from row ny - 2
                T src[9], gn[9];
                wall_source(wc, i, nx, gprev, src);
                extrapolate(src, ulid, gn);
                if (out_col) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) S::store(fout, c.f_off + k * c.plane + node, k, gn[k]);
                    if (RES) residual_add(gn, mom[0], acc);
                }
            } else {   // p == 0: stored with row 1; keep its old moments
#pragma unroll
                for (int q3 = 0; q3 < 3; ++q3) mom0[q3] = mom[0][q3];
            }
        }

        // ---------------------------------------------------------- rings
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lamr[r] = lamr[r + 1];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                gbp[r][k] = gbp[r + 1][k];
                ghp[r][k] = ghp[r + 1][k];
                fh[r][k] = fh[r + 1][k];
            }
#pragma unroll
            for (int q3 = 0; q3 < 3; ++q3) mom[r][q3] = mom[r + 1][q3];
        }
    }

    if (RES) {
        // wavefront sum in a fixed order
#pragma unroll
        for (int q5 = 0; q5 < kPartials; ++q5) {
            double v = acc[q5];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWaveLanes);
            if (lane == 0) a.partial[(int64_t)(w0 + blockIdx.x) * kPartials + q5] = v;
        }
    }
}

template <int PREC>
hipError_t fused(const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    if (nw <= 0) return hipSuccess;
    if (residual)
        hipLaunchKernelGGL((k_fused<PREC, true>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0);
    else
        hipLaunchKernelGGL((k_fused<PREC, false>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_step(int prec, const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    switch (prec) {
    case P_FP64: return fused<P_FP64>(a, items, w0, nw, residual, s);
    case P_FP32: return fused<P_FP32>(a, items, w0, nw, residual, s);
    case P_FP16DEV: return fused<P_FP16DEV>(a, items, w0, nw, residual, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace ifd
