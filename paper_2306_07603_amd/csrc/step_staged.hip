// step_staged.hip -- the IFDLBM time step as five per-node launches through
// HBM temporaries, one launch per stage of the calculational process of
// Section 4 (arXiv:2306.07603):
//   A   Steps (2)-(3) and the collision of Step (4): lambda, f-hat+, f-bar+
//   B   Eq. (3.7) at interior nodes: f-bar(t + dt/2)
//   BH  walls by extrapolation, then f(t + dt/2) by Eq. (2.17) at every node
//   C   Eq. (3.6) at interior nodes: f-hat(t + dt), and lambda at every node
//   CB  Step (6): walls of f-hat(t + dt) by extrapolation
// This schedule moves about five times the state per step; it is the simple
// counterpart of the fused kernel and serves as its cross-check.
#include "ifdlbm_internal.h"

namespace ifd {
namespace {

template <typename T> __device__ __forceinline__ const T* geo_table(const StepArgs& a);
template <> __device__ __forceinline__ const double* geo_table<double>(const StepArgs& a) { return a.geo; }
template <> __device__ __forceinline__ const float* geo_table<float>(const StepArgs& a) { return a.geo32; }

struct NodeRef {
    int i, j;
    int64_t id;   // j * pitch + i
};

__device__ __forceinline__ bool locate(const NodeBlock* blocks, int b, const CavityDesc* desc, CavityDesc& c, NodeRef& r)
{
    const NodeBlock nb = blocks[b];
    c = desc[nb.cav];
    const int n = nb.first + (int)threadIdx.x;
    if (n >= c.nx * c.ny) return false;
    r.j = n / c.nx;
    r.i = n - r.j * c.nx;
    r.id = (int64_t)r.j * c.pitch + r.i;
    return true;
}

// c_k . grad Phi_k at interior node (i, j) by Eqs. (3.4), (2.5)-(2.7):
// c_k,xi = a_j (c_kx - c_ky s_i), c_k,eta = c_ky.
template <typename T>
__device__ T transport(const T* plane, const CavityDesc& c, const T* geo, int i, int j, int k)
{
    const int cx = cxk(k), cy = cyk(k);
    const T eps = T(c.mix);
    T term = T(0);
    const T a = geo[c.geo_off + j], s = geo[c.geo_off + c.ny + i];
    const T cxi = a * (T(cx) - T(cy) * s);
    if (cxi != T(0)) {
        const T* row = plane + (int64_t)j * c.pitch;
        const bool pos = cxi >= T(0);
        const T m2 = (pos && i >= 2) ? row[i - 2] : T(0);
        const T p2 = (!pos && i <= c.nx - 3) ? row[i + 2] : T(0);
        const T d = mixed_diff_2h(m2, row[i - 1], row[i], row[i + 1], p2, pos, i == 1, i == c.nx - 2, eps);
        term += cxi * (d * T(c.inv2dxi));
    }
    if (cy != 0) {
        const T* col = plane + i;
        const int64_t p = c.pitch;
        const bool pos = cy > 0;
        const T m2 = (pos && j >= 2) ? col[(j - 2) * p] : T(0);
        const T p2 = (!pos && j <= c.ny - 3) ? col[(j + 2) * p] : T(0);
        const T d = mixed_diff_2h(m2, col[(j - 1) * p], col[j * p], col[(j + 1) * p], p2, pos, j == 1, j == c.ny - 2, eps);
        term += T(cy) * (d * T(c.inv2deta));
    }
    return term;
}

template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_stage_a(StepArgs a, const NodeBlock* blocks, int b0)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    CavityDesc c;
    NodeRef r;
    if (!locate(blocks, b0 + blockIdx.x, a.desc, c, r)) return;
    const auto* f = static_cast<const typename S::F*>(a.f_in);
    const auto* l = static_cast<const typename S::L*>(a.l_in);
    using V = typename S::V;
    T g[9], e[9], d[9], P, ux, uy;
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = S::load(f, c.f_off + k * c.plane + r.id, k);
    const PowerLaw<V> pl(c);
    V lam;
    if constexpr (S::kExactFinal) {
        // e - g in FP64 from the exact stored g (the non-equilibrium part at low shear is below an FP32 ulp)
        double gd[9], dd[9], Pd, uxd, uyd;
#pragma unroll
        for (int k = 0; k < 9; ++k) gd[k] = (double)g[k];
        moments(gd, Pd, uxd, uyd);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            dd[k] = equilibrium_k(Pd, uxd, uyd, k) - gd[k];
            d[k] = T(dd[k]);
        }
        lam = pl.implicit ? relaxation_time_d<true>(dd, V(l[c.l_off + r.id]), pl)
                          : relaxation_time_d<false>(dd, V(l[c.l_off + r.id]), pl);
    } else {
        moments(g, P, ux, uy);
        equilibrium(P, ux, uy, e);
#pragma unroll
        for (int k = 0; k < 9; ++k) d[k] = e[k] - g[k];
        lam = pl.implicit ? relaxation_time_d<true>(d, V(l[c.l_off + r.id]), pl)
                          : relaxation_time_d<false>(d, V(l[c.l_off + r.id]), pl);
    }
    const Relax<V> rx(lam, V(c.dt));
    const T b_hat = T(rx.b_hat), b_bar = T(rx.b_bar);
    T* hp = static_cast<T*>(a.hat_plus);
    T* bp = static_cast<T*>(a.bar_plus);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        hp[c.f_off + k * c.plane + r.id] = g[k] + b_hat * d[k];
        bp[c.f_off + k * c.plane + r.id] = g[k] + b_bar * d[k];
    }
    static_cast<T*>(a.lam_new)[c.l_off + r.id] = T(lam);
}

template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_stage_b(StepArgs a, const NodeBlock* blocks, int b0)
{
    using T = typename Storage<PREC>::T;
    CavityDesc c;
    NodeRef r;
    if (!locate(blocks, b0 + blockIdx.x, a.desc, c, r)) return;
    if (is_boundary(r.i, r.j, c.nx, c.ny)) return;
    const T* bp = static_cast<const T*>(a.bar_plus);
    T* fb = static_cast<T*>(a.bar_half);
    const T* geo = geo_table<T>(a);
    const T half_dt = T(0.5) * T(c.dt);
    fb[c.f_off + r.id] = bp[c.f_off + r.id];
#pragma unroll 1
    for (int k = 1; k < 9; ++k) {
        const T* plane = bp + c.f_off + k * c.plane;
        fb[c.f_off + k * c.plane + r.id] = plane[r.id] - half_dt * transport(plane, c, geo, r.i, r.j, k);
    }
}

template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_stage_bh(StepArgs a, const NodeBlock* blocks, int b0)
{
    using T = typename Storage<PREC>::T;
    CavityDesc c;
    NodeRef r;
    if (!locate(blocks, b0 + blockIdx.x, a.desc, c, r)) return;
    const T* fbar = static_cast<const T*>(a.bar_half);
    T x[9];
    if (is_boundary(r.i, r.j, c.nx, c.ny)) {
        int ni, nj;
        inward(r.i, r.j, c.nx, c.ny, ni, nj);
        const int64_t nid = (int64_t)nj * c.pitch + ni;
        T xnb[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) xnb[k] = fbar[c.f_off + k * c.plane + nid];
        extrapolate(xnb, r.j == c.ny - 1 ? T(c.u_lid) : T(0), x);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) x[k] = fbar[c.f_off + k * c.plane + r.id];
    }
    using V = typename Storage<PREC>::V;
    T P, ux, uy, e[9];
    moments(x, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const T b = T(half_coef(V(static_cast<const T*>(a.lam_new)[c.l_off + r.id]), V(c.dt)));
    T* fh = static_cast<T*>(a.bar_plus);   // f-bar+ is dead after stage B
#pragma unroll
    for (int k = 0; k < 9; ++k) fh[c.f_off + k * c.plane + r.id] = x[k] + b * (e[k] - x[k]);
}

template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_stage_c(StepArgs a, const NodeBlock* blocks, int b0)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    CavityDesc c;
    NodeRef r;
    if (!locate(blocks, b0 + blockIdx.x, a.desc, c, r)) return;
    static_cast<typename S::L*>(a.l_out)[c.l_off + r.id] = static_cast<const T*>(a.lam_new)[c.l_off + r.id];
    if (is_boundary(r.i, r.j, c.nx, c.ny)) return;
    const T* fh = static_cast<const T*>(a.bar_plus);
    // f-hat+ is read at its own node only: its slot takes the new f-hat in the
    // arithmetic type, the source of the wall extrapolation of stage CB
    T* hp = static_cast<T*>(a.hat_plus);
    auto* out = static_cast<typename S::F*>(a.f_out);
    const T* geo = geo_table<T>(a);
    const T dt = T(c.dt);
    const NodeWords nw(step_key(a.seed_ctr[0], a.step), cavity_key(c.index), (uint32_t)r.id);
    if constexpr (S::kExactFinal) {
        // f-hat+ rebuilt in FP64 from the stored f-hat (Eq. 2.15), the FP32 increment added in FP64
        using V = typename S::V;
        const auto* fin = static_cast<const typename S::F*>(a.f_in);
        double gd[9], e[9], P, ux, uy;
#pragma unroll
        for (int k = 0; k < 9; ++k) gd[k] = (double)S::load(fin, c.f_off + k * c.plane + r.id, k);
        moments(gd, P, ux, uy);
        equilibrium(P, ux, uy, e);
        const double bh = (double)Relax<V>(V(static_cast<const T*>(a.lam_new)[c.l_off + r.id]), V(c.dt)).b_hat;
#pragma unroll 1
        for (int k = 0; k < 9; ++k) {
            const int64_t o = c.f_off + k * c.plane;
            const T inc = k == 0 ? T(0) : -(dt * transport(fh + o, c, geo, r.i, r.j, k));
            const double v = (gd[k] + bh * (e[k] - gd[k])) + (double)inc;
            hp[o + r.id] = T(v);
            out[o + r.id] = encode_state<S>(v, k, &nw);
        }
        return;
    }
    out[c.f_off + r.id] = encode_state<S>(hp[c.f_off + r.id], 0, &nw);
#pragma unroll 1
    for (int k = 1; k < 9; ++k) {
        const int64_t o = c.f_off + k * c.plane;
        const T v = hp[o + r.id] - dt * transport(fh + o, c, geo, r.i, r.j, k);
        hp[o + r.id] = v;
        out[o + r.id] = encode_state<S>(v, k, &nw);
    }
}

template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_stage_cb(StepArgs a, const NodeBlock* blocks, int b0)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    CavityDesc c;
    NodeRef r;
    if (!locate(blocks, b0 + blockIdx.x, a.desc, c, r)) return;
    if (!is_boundary(r.i, r.j, c.nx, c.ny)) return;
    auto* out = static_cast<typename S::F*>(a.f_out);
    const T* fnew = static_cast<const T*>(a.hat_plus);   // new f-hat of the interior, before rounding to storage
    int ni, nj;
    inward(r.i, r.j, c.nx, c.ny, ni, nj);
    const int64_t nid = (int64_t)nj * c.pitch + ni;
    T xnb[9], x[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) xnb[k] = fnew[c.f_off + k * c.plane + nid];
    extrapolate(xnb, r.j == c.ny - 1 ? T(c.u_lid) : T(0), x);
    const NodeWords nw(step_key(a.seed_ctr[0], a.step), cavity_key(c.index), (uint32_t)r.id);
#pragma unroll
    for (int k = 0; k < 9; ++k) out[c.f_off + k * c.plane + r.id] = encode_state<S>(x[k], k, &nw);
}

// Eq. (2.19) partial sums over one node block, from the moments of f-hat
// before (f_in) and after (f_out) the step.
template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_residual(StepArgs a, const NodeBlock* blocks, int b0)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    __shared__ double sh[kPartials][kNodeBlock];
    CavityDesc c;
    NodeRef r;
    double v[kPartials];
#pragma unroll
    for (int q = 0; q < kPartials; ++q) v[q] = 0.0;
    if (locate(blocks, b0 + blockIdx.x, a.desc, c, r)) {
        const auto* fi = static_cast<const typename S::F*>(a.f_in);
        const auto* fo = static_cast<const typename S::F*>(a.f_out);
        T g0[9], g1[9], P0, u0, v0, P1, u1, v1;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            g0[k] = S::load(fi, c.f_off + k * c.plane + r.id, k);
            g1[k] = S::load(fo, c.f_off + k * c.plane + r.id, k);
        }
        moments(g0, P0, u0, v0);
        moments(g1, P1, u1, v1);
        const double du = (double)u1 - (double)u0, dv = (double)v1 - (double)v0, dp = (double)P1 - (double)P0;
        v[0] = du * du + dv * dv;
        v[1] = (double)u1 * u1 + (double)v1 * v1;
        v[2] = dp * dp;
        v[3] = (double)P1 * P1;
        const double sd = dp - a.res_ref[2 * c.index], sp = (double)P1 - a.res_ref[2 * c.index + 1];
        v[4] = sd;
        v[5] = sp;
        v[6] = (isfinite((double)u1) && isfinite((double)v1) && isfinite((double)P1)) ? 0.0 : 1.0;
        v[7] = sd * sd;
        v[8] = sp * sp;
    }
#pragma unroll
    for (int q = 0; q < kPartials; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kNodeBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < kPartials; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kPartials) a.partial[(int64_t)(b0 + blockIdx.x) * kPartials + threadIdx.x] = sh[threadIdx.x][0];
}

template <int PREC>
hipError_t staged(const StepArgs& a, const NodeBlock* blocks, int b0, int nb, bool residual, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    const dim3 grid(nb), block(kNodeBlock);
    hipLaunchKernelGGL(k_stage_a<PREC>, grid, block, 0, s, a, blocks, b0);
    hipLaunchKernelGGL(k_stage_b<PREC>, grid, block, 0, s, a, blocks, b0);
    hipLaunchKernelGGL(k_stage_bh<PREC>, grid, block, 0, s, a, blocks, b0);
    hipLaunchKernelGGL(k_stage_c<PREC>, grid, block, 0, s, a, blocks, b0);
    hipLaunchKernelGGL(k_stage_cb<PREC>, grid, block, 0, s, a, blocks, b0);
    if (residual) hipLaunchKernelGGL(k_residual<PREC>, grid, block, 0, s, a, blocks, b0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_staged_step(int prec, const StepArgs& a, const NodeBlock* blocks, int b0, int nb, bool residual,
                              hipStream_t s)
{
    switch (prec) {
    case P_FP64: return staged<P_FP64>(a, blocks, b0, nb, residual, s);
    case P_FP32: return staged<P_FP32>(a, blocks, b0, nb, residual, s);
    case P_FP16DEV: return staged<P_FP16DEV>(a, blocks, b0, nb, residual, s);
    case P_FP32X: return staged<P_FP32X>(a, blocks, b0, nb, residual, s);
    case P_FP32SR: return staged<P_FP32SR>(a, blocks, b0, nb, residual, s);
    case P_FP32SRF: return staged<P_FP32SRF>(a, blocks, b0, nb, residual, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace ifd
