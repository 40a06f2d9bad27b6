// adjoint.hip -- reverse (discrete adjoint) sweep of the IFDLBM step: the
// gradient of a cavity objective with respect to the top angle theta, the
// power-law index n and the lid speed U.
//
// One time step maps the state (f-hat, Lambda) at t to the state at t + dt
// through Steps (2)-(6) of Section 4:
//   A  every node:     moments (Eqs. 2.10-2.11), equilibrium (Eq. 2.8), the
//                      lagged power-law lambda (Eqs. 2.12-2.14, 1.4), f-hat+
//                      and f-bar+ (Eqs. 2.15-2.16);
//   B  interior:       f-bar = f-bar+ - dt/2 S[f-bar+] (Eq. 3.7);
//   BH every node:     f(t + dt/2) = f-bar + dt/(4 lambda + dt) (f_eq - f-bar)
//                      (Eq. 2.17), wall nodes first taking f-bar by
//                      non-equilibrium extrapolation from the inward node;
//   C  interior:       f-hat(t + dt) = f-hat+ - dt S[f(t + dt/2)] (Eq. 3.6);
//   CB wall nodes:     extrapolation of the new f-hat from the inward node.
// S_k[phi] = c_k,xi M_xi(phi_k) + c_k,eta M_eta(phi_k) with the mixed difference
// of Eqs. (2.5)-(2.7) and the contravariant velocity of Eq. (3.6).
//
// The adjoint step takes the adjoint of the state at t + dt and returns that
// of the state at t, walking the stages backwards: CB, C, BH, B, A.  Each
// stage's transpose is written out by hand.  Stencil stages are transposed
// as gathers: node m collects, from every interior node x whose stencil reads
// m, the weight x gives to m (which depends on the upwind side chosen at x)
// times x's adjoint; the wall extrapolation is transposed the same way, the
// inward node collecting from the wall nodes that copy it.  The forward
// quantities a step needs (f-bar+, lambda, f-bar, f(t + dt/2)) are recomputed
// from the stored state at t, in FP64.
//
// Parameter adjoints are accumulated as those of the primitive quantities:
// cot(theta) through the metric terms a_j = 1/(1 + 2 eta_j cot), s_i = cot
// (2 xi_i - 1) (Eqs. 3.2-3.8.2) and the Jacobian of the objective; the time
// step (whose CFL rule may involve cot); 3K (Eq. 2.15.1); the exponent
// (n - 1)/2 of Eq. (1.4); the lid velocity (Eq. 1.5); and, at the initial
// state of Step (1), the initial lambda and the lid row's equilibrium.  Each
// kernel reduces them per block into its own slot of a running FP64 sum, so
// the result does not depend on scheduling.
#include <cmath>
#include <vector>

#include "ifdlbm_internal.h"

namespace ifd {

namespace {

constexpr int kB = 256;   // threads per block

// accumulators of the primitive parameter adjoints
enum Acc { A_COT = 0, A_DT, A_K3, A_EXPO, A_ULID, A_LAM0, A_N };
// one slot of block sums per kernel that contributes
enum Slot { S_OBJ = 0, S_CB, S_C, S_BH, S_BH2, S_B, S_A, S_INIT, S_N };

struct AdjParams {
    int nx, ny;
    double dt, K3, expo, g2min, mix, ulid, inv2dxi, inv2deta, dxi, deta;
    const double* geo;   // a_j [ny], s_i [nx], d a_j / d cot [ny], d s_i / d cot [nx]
    double* acc;         // [S_N][blocks][A_N]
    int blocks;
};

__device__ __forceinline__ bool node_of(const AdjParams& p, int& i, int& j)
{
    const int n = blockIdx.x * kB + threadIdx.x;
    if (n >= p.nx * p.ny) return false;
    j = n / p.nx;
    i = n - j * p.nx;
    return true;
}

__device__ __forceinline__ bool interior(const AdjParams& p, int i, int j)
{
    return i >= 1 && j >= 1 && i <= p.nx - 2 && j <= p.ny - 2;
}

__device__ __forceinline__ int64_t at(const AdjParams& p, int i, int j) { return (int64_t)j * p.nx + i; }

// Block sum of up to A_N accumulators, added by thread 0 into slot `slot`
// of this block (each (slot, block) pair has one writer per launch and
// launches are stream-ordered).
__device__ void accumulate(const AdjParams& p, int slot, const double (&v)[A_N])
{
    __shared__ double sh[A_N][kB];
#pragma unroll
    for (int q = 0; q < A_N; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < A_N; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* a = p.acc + ((int64_t)slot * p.blocks + blockIdx.x) * A_N;
#pragma unroll
        for (int q = 0; q < A_N; ++q) a[q] += sh[q][0];
    }
}

// ------------------------------------------------ local transposes (FP64)

// Transpose of moments(): (P-bar, ux-bar, uy-bar) at u -> g-bar.
// P = 0.6 sum_{k>0} g_k - 0.4 |u|^2, u = sum c_k g_k.
__device__ __forceinline__ void moments_t(double ux, double uy, double Pb, double uxb, double uyb, double gb[9])
{
    const double ax = uxb - 0.8 * ux * Pb, ay = uyb - 0.8 * uy * Pb, s = 0.6 * Pb;
    gb[0] = 0.0;
#pragma unroll
    for (int k = 1; k < 9; ++k) gb[k] = cxk(k) * ax + cyk(k) * ay + s;
}

// Transpose of equilibrium(): e-bar -> (P-bar, ux-bar, uy-bar), added.
// e_0 = -5/3 P - 2/3 |u|^2; e_k = w_k (3 P - 1.5 |u|^2 + 3 c.u + 4.5 (c.u)^2).
__device__ __forceinline__ void equilibrium_t(double ux, double uy, const double eb[9], double& Pb, double& uxb,
                                              double& uyb)
{
    Pb += -5.0 / 3.0 * eb[0];
    uxb += -4.0 / 3.0 * ux * eb[0];
    uyb += -4.0 / 3.0 * uy * eb[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const double w = k < 5 ? 1.0 / 9.0 : 1.0 / 36.0, cx = cxk(k), cy = cyk(k);
        const double cu = cx * ux + cy * uy, we = w * eb[k], dq = 3.0 + 9.0 * cu;
        Pb += 3.0 * we;
        uxb += we * (-3.0 * ux + dq * cx);
        uyb += we * (-3.0 * uy + dq * cy);
    }
}

// Transpose of extrapolate(x_nb, uwall): x_b-bar -> x_nb-bar (added) and
// uwall-bar (returned).  x_b = e(P, uwall, 0) + x_nb - e(P, u_nb), (P, u_nb) =
// moments(x_nb).
__device__ __forceinline__ double extrapolate_t(const double xnb[9], double uwall, const double xbb[9], double xnbb[9])
{
    double P, ux, uy;
    moments(xnb, P, ux, uy);
    double Pb = 0.0, uwb = 0.0, uwyb = 0.0, uxb = 0.0, uyb = 0.0;
    equilibrium_t(uwall, 0.0, xbb, Pb, uwb, uwyb);
    double m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = -xbb[k];
    equilibrium_t(ux, uy, m, Pb, uxb, uyb);
    double gb[9];
    moments_t(ux, uy, Pb, uxb, uyb, gb);
#pragma unroll
    for (int k = 0; k < 9; ++k) xnbb[k] += xbb[k] + gb[k];
    return uwb;
}

// Weight of phi(i + o) in 2h M(phi)(i) (Eqs. 2.5-2.7) for the upwind side
// `pos` (contravariant velocity >= 0) and the first-order fallbacks at
// i = 1 (lo) and i = N - 2 (hi); the forward form is mixed_diff_2h.
__device__ __forceinline__ double stencil_weight(int o, bool pos, bool lo, bool hi, double eps)
{
    const double u = 1.0 - eps;
    switch (o) {
    case -2: return pos && !lo ? u : 0.0;
    case -1: return -eps + (pos ? (lo ? -2.0 * u : -4.0 * u) : 0.0);
    case 0: return pos ? (lo ? 2.0 * u : 3.0 * u) : (hi ? -2.0 * u : -3.0 * u);
    case 1: return eps + (!pos ? (hi ? 2.0 * u : 4.0 * u) : 0.0);
    default: return !pos && !hi ? -u : 0.0;
    }
}

__device__ __forceinline__ double c_xi(const AdjParams& p, int i, int j, int k)
{
    return p.geo[j] * ((double)cxk(k) - (double)cyk(k) * p.geo[p.ny + i]);
}

// d c_k,xi / d cot at (i, j).
__device__ __forceinline__ double c_xi_dcot(const AdjParams& p, int i, int j, int k)
{
    return p.geo[p.ny + p.nx + j] * ((double)cxk(k) - (double)cyk(k) * p.geo[p.ny + i]) -
           p.geo[j] * (double)cyk(k) * p.geo[2 * p.ny + p.nx + i];
}

// Forward pieces of S_k[phi](x) at interior x: M_xi * inv2dxi and M_eta * inv2deta.
__device__ __forceinline__ void stencil_parts(const AdjParams& p, const double* plane, int i, int j, int k, double& mxi,
                                              double& meta)
{
    const bool pos = c_xi(p, i, j, k) >= 0.0;
    mxi = 0.0;
    for (int o = -2; o <= 2; ++o) {
        const double w = stencil_weight(o, pos, i == 1, i == p.nx - 2, p.mix);
        if (w != 0.0) mxi += w * plane[at(p, i + o, j)];
    }
    mxi *= p.inv2dxi;
    meta = 0.0;
    const int cy = cyk(k);
    if (cy != 0)
        for (int o = -2; o <= 2; ++o) {
            const double w = stencil_weight(o, cy > 0, j == 1, j == p.ny - 2, p.mix);
            if (w != 0.0) meta += w * plane[at(p, i, j + o)];
        }
    meta *= p.inv2deta;
}

// Transposed stencil at m = (i, j): sum over interior x reading m of
// ybar(x) * (weight x gives to m in S_k).
__device__ __forceinline__ double stencil_t(const AdjParams& p, const double* ybar_plane, int i, int j, int k)
{
    double acc = 0.0;
    if (j >= 1 && j <= p.ny - 2)
        for (int o = -2; o <= 2; ++o) {
            const int ix = i - o;
            if (ix < 1 || ix > p.nx - 2) continue;
            const double c = c_xi(p, ix, j, k);
            const double w = stencil_weight(o, c >= 0.0, ix == 1, ix == p.nx - 2, p.mix);
            if (w != 0.0) acc += ybar_plane[at(p, ix, j)] * c * w * p.inv2dxi;
        }
    const int cy = cyk(k);
    if (cy != 0 && i >= 1 && i <= p.nx - 2)
        for (int o = -2; o <= 2; ++o) {
            const int jx = j - o;
            if (jx < 1 || jx > p.ny - 2) continue;
            const double w = stencil_weight(o, cy > 0, jx == 1, jx == p.ny - 2, p.mix);
            if (w != 0.0) acc += ybar_plane[at(p, i, jx)] * (double)cy * w * p.inv2deta;
        }
    return acc;
}

// Wall nodes whose inward neighbour is the interior node (i, j): at most three
// (an edge node on each adjacent wall and the diagonal corner).
__device__ __forceinline__ int walls_of(const AdjParams& p, int i, int j, int (&wi)[3], int (&wj)[3])
{
    int n = 0;
    const int di = i == 1 ? -1 : (i == p.nx - 2 ? 1 : 0);
    const int dj = j == 1 ? -1 : (j == p.ny - 2 ? 1 : 0);
    if (di) { wi[n] = i + di; wj[n] = j; ++n; }
    if (dj) { wi[n] = i; wj[n] = j + dj; ++n; }
    if (di && dj) { wi[n] = i + di; wj[n] = j + dj; ++n; }
    return n;
}

// ---------------------------------------------- forward recomputation (FP64)

// Stage A: f-bar+ (9 planes) and lambda of the step from the state at t.
__global__ __launch_bounds__(kB) void r_stage_a(AdjParams p, const double* st, double* bp, double* ln)
{
    int i, j;
    if (!node_of(p, i, j)) return;
    const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
    double g[9], e[9], P, ux, uy;
    for (int k = 0; k < 9; ++k) g[k] = st[k * pl + id];
    moments(g, P, ux, uy);
    equilibrium(P, ux, uy, e);
    double n[9];
    for (int k = 0; k < 9; ++k) n[k] = g[k] - e[k];
    const double s58 = (n[5] + n[6]) + (n[7] + n[8]);
    const double pxx = (n[1] + n[3]) + s58, pyy = (n[2] + n[4]) + s58, pxy = (n[5] - n[6]) + (n[7] - n[8]);
    const double r = 1.0 / (2.0 * st[9 * pl + id] + p.dt);
    const double gamma2 = 18.0 * (pxx * pxx + 2.0 * pxy * pxy + pyy * pyy) * r * r;
    const double lam = p.K3 * pow(gamma2 > p.g2min ? gamma2 : p.g2min, p.expo);
    const double bb = 1.5 * p.dt / (2.0 * lam + p.dt);
    for (int k = 0; k < 9; ++k) bp[k * pl + id] = g[k] + bb * (e[k] - g[k]);
    ln[id] = lam;
}

// Stage B: f-bar at interior nodes.
__global__ __launch_bounds__(kB) void r_stage_b(AdjParams p, const double* bp, double* fb)
{
    int i, j;
    if (!node_of(p, i, j) || !interior(p, i, j)) return;
    const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
    fb[id] = bp[id];
    for (int k = 1; k < 9; ++k) {
        double mxi, meta;
        stencil_parts(p, bp + k * pl, i, j, k, mxi, meta);
        fb[k * pl + id] = bp[k * pl + id] - 0.5 * p.dt * (c_xi(p, i, j, k) * mxi + (double)cyk(k) * meta);
    }
}

__device__ __forceinline__ void half_input(const AdjParams& p, const double* fb, int i, int j, double x[9])
{
    const int64_t pl = (int64_t)p.nx * p.ny;
    if (interior(p, i, j)) {
        for (int k = 0; k < 9; ++k) x[k] = fb[k * pl + at(p, i, j)];
        return;
    }
    int ni = i == 0 ? 1 : (i == p.nx - 1 ? p.nx - 2 : i);
    int nj = j == 0 ? 1 : (j == p.ny - 1 ? p.ny - 2 : j);
    double xnb[9];
    for (int k = 0; k < 9; ++k) xnb[k] = fb[k * pl + at(p, ni, nj)];
    extrapolate(xnb, j == p.ny - 1 ? p.ulid : 0.0, x);
}

// Stage BH: f(t + dt/2) at every node.
__global__ __launch_bounds__(kB) void r_stage_bh(AdjParams p, const double* fb, const double* ln, double* fh)
{
    int i, j;
    if (!node_of(p, i, j)) return;
    const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
    double x[9], e[9], P, ux, uy;
    half_input(p, fb, i, j, x);
    moments(x, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const double hc = p.dt / (4.0 * ln[id] + p.dt);
    for (int k = 0; k < 9; ++k) fh[k * pl + id] = x[k] + hc * (e[k] - x[k]);
}

// ------------------------------------------------------- adjoint stages

// Objective, Eq. (5.1): J = sum 1/2 w_i w_j dxi deta J_j |u|^2, J_j = 1 + 2
// eta_j cot.  Writes the block sums of J (slot S_OBJ, accumulator A_N - 1 is
// not used: J goes to `jpart`) and the state adjoint at the final step.
__global__ __launch_bounds__(kB) void a_objective(AdjParams p, double cot, const double* st, double* fbar,
                                                  double* lbar, double* jpart)
{
    __shared__ double sj[kB];
    double v[A_N] = {};
    double jl = 0.0;
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        double g[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) g[k] = st[k * pl + id];
        moments(g, P, ux, uy);
        const double wi = (i == 0 || i == p.nx - 1) ? 0.5 : 1.0, wj = (j == 0 || j == p.ny - 1) ? 0.5 : 1.0;
        const double w = wi * wj * p.dxi * p.deta, eta = j * p.deta, Jj = 1.0 + 2.0 * eta * cot;
        const double uu = ux * ux + uy * uy;
        jl = 0.5 * w * Jj * uu;
        v[A_COT] = w * eta * uu;
        double gb[9];
        moments_t(ux, uy, 0.0, w * Jj * ux, w * Jj * uy, gb);
        for (int k = 0; k < 9; ++k) fbar[k * pl + id] = gb[k];
        lbar[id] = 0.0;
    }
    sj[threadIdx.x] = jl;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sj[threadIdx.x] += sj[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) jpart[blockIdx.x] = sj[0];
    accumulate(p, S_OBJ, v);
}

// CB^T: the adjoint G of the interior values of the new state, f-hat(t + dt)
// before its walls are set: the state adjoint itself plus what the wall
// nodes extrapolated from this node hand back.  st1 is the state at t + dt.
__global__ __launch_bounds__(kB) void a_stage_cb(AdjParams p, const double* st1, const double* fbar, double* G)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j) && interior(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        double gb[9], x[9];
        for (int k = 0; k < 9; ++k) {
            gb[k] = fbar[k * pl + id];
            x[k] = st1[k * pl + id];
        }
        int wi[3], wj[3];
        const int nw = walls_of(p, i, j, wi, wj);
        for (int q = 0; q < nw; ++q) {
            double xb[9];
            for (int k = 0; k < 9; ++k) xb[k] = fbar[k * pl + at(p, wi[q], wj[q])];
            const double uwb = extrapolate_t(x, wj[q] == p.ny - 1 ? p.ulid : 0.0, xb, gb);
            if (wj[q] == p.ny - 1) v[A_ULID] += uwb;
        }
        for (int k = 0; k < 9; ++k) G[k * pl + id] = gb[k];
    } else if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        for (int k = 0; k < 9; ++k) G[k * pl + id] = 0.0;   // wall f-hat+ is not used
    }
    accumulate(p, S_CB, v);
}

// C^T: adjoint of f(t + dt/2) at every node (k = 0 carries no stream term)
// and the cot / dt terms of Eq. (3.6) at interior nodes.
__global__ __launch_bounds__(kB) void a_stage_c(AdjParams p, const double* G, const double* fh, double* fhb)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        fhb[id] = 0.0;
        for (int k = 1; k < 9; ++k) fhb[k * pl + id] = -p.dt * stencil_t(p, G + k * pl, i, j, k);
        if (interior(p, i, j))
            for (int k = 1; k < 9; ++k) {
                const double gk = G[k * pl + id];
                double mxi, meta;
                stencil_parts(p, fh + k * pl, i, j, k, mxi, meta);
                v[A_DT] -= gk * (c_xi(p, i, j, k) * mxi + (double)cyk(k) * meta);
                v[A_COT] -= p.dt * gk * c_xi_dcot(p, i, j, k) * mxi;
            }
    }
    accumulate(p, S_C, v);
}

// BH^T at every node: adjoint of the node's half-step input x (f-bar, or the
// extrapolated wall value), written over fhb, and lambda-bar of this stage.
__global__ __launch_bounds__(kB) void a_stage_bh(AdjParams p, const double* fb, const double* ln, double* fhb, double* lb)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        double x[9], e[9], P, ux, uy;
        half_input(p, fb, i, j, x);
        moments(x, P, ux, uy);
        equilibrium(P, ux, uy, e);
        const double lam = ln[id], den = 4.0 * lam + p.dt, hc = p.dt / den;
        double xb[9], eb[9], hcb = 0.0;
        for (int k = 0; k < 9; ++k) {
            const double y = fhb[k * pl + id];
            xb[k] = (1.0 - hc) * y;
            eb[k] = hc * y;
            hcb += y * (e[k] - x[k]);
        }
        double Pb = 0.0, uxb = 0.0, uyb = 0.0, gb[9];
        equilibrium_t(ux, uy, eb, Pb, uxb, uyb);
        moments_t(ux, uy, Pb, uxb, uyb, gb);
        for (int k = 0; k < 9; ++k) fhb[k * pl + id] = xb[k] + gb[k];
        lb[id] = hcb * (-4.0 * p.dt / (den * den));
        v[A_DT] = hcb * (4.0 * lam / (den * den));
    }
    accumulate(p, S_BH, v);
}

// Wall transpose of BH: adjoint of f-bar at interior nodes.
__global__ __launch_bounds__(kB) void a_stage_bh2(AdjParams p, const double* fb, const double* xb, double* fbb)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j) && interior(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        double gb[9], x[9];
        for (int k = 0; k < 9; ++k) {
            gb[k] = xb[k * pl + id];
            x[k] = fb[k * pl + id];
        }
        int wi[3], wj[3];
        const int nw = walls_of(p, i, j, wi, wj);
        for (int q = 0; q < nw; ++q) {
            double y[9];
            for (int k = 0; k < 9; ++k) y[k] = xb[k * pl + at(p, wi[q], wj[q])];
            const double uwb = extrapolate_t(x, wj[q] == p.ny - 1 ? p.ulid : 0.0, y, gb);
            if (wj[q] == p.ny - 1) v[A_ULID] += uwb;
        }
        for (int k = 0; k < 9; ++k) fbb[k * pl + id] = gb[k];
    }
    accumulate(p, S_BH2, v);
}

// B^T: adjoint of f-bar+ at every node, and the cot / dt terms of Eq. (3.7).
__global__ __launch_bounds__(kB) void a_stage_b(AdjParams p, const double* fbb, const double* bp, double* bpb)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        const bool in = interior(p, i, j);
        bpb[id] = in ? fbb[id] : 0.0;
        for (int k = 1; k < 9; ++k)
            bpb[k * pl + id] = (in ? fbb[k * pl + id] : 0.0) - 0.5 * p.dt * stencil_t(p, fbb + k * pl, i, j, k);
        if (in)
            for (int k = 1; k < 9; ++k) {
                const double yk = fbb[k * pl + id];
                double mxi, meta;
                stencil_parts(p, bp + k * pl, i, j, k, mxi, meta);
                v[A_DT] -= 0.5 * yk * (c_xi(p, i, j, k) * mxi + (double)cyk(k) * meta);
                v[A_COT] -= 0.5 * p.dt * yk * c_xi_dcot(p, i, j, k) * mxi;
            }
    }
    accumulate(p, S_B, v);
}

// A^T at every node: from the adjoints of f-hat+ (G, zero on walls), f-bar+
// (bpb) and lambda (lb from BH plus lbar, the adjoint of the stored Lambda of
// t + dt) to the adjoint of the state at t, written over fbar / lbar.
__global__ __launch_bounds__(kB) void a_stage_a(AdjParams p, const double* st, const double* G, const double* bpb,
                                                const double* lb, double* fbar, double* lbar)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        double g[9], e[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) g[k] = st[k * pl + id];
        const double lam_old = st[9 * pl + id];
        moments(g, P, ux, uy);
        equilibrium(P, ux, uy, e);
        double n[9];
        for (int k = 0; k < 9; ++k) n[k] = g[k] - e[k];
        const double s58 = (n[5] + n[6]) + (n[7] + n[8]);
        const double pxx = (n[1] + n[3]) + s58, pyy = (n[2] + n[4]) + s58, pxy = (n[5] - n[6]) + (n[7] - n[8]);
        const double Q = pxx * pxx + 2.0 * pxy * pxy + pyy * pyy;
        const double r = 1.0 / (2.0 * lam_old + p.dt);
        const double gamma2 = 18.0 * Q * r * r;
        const bool floor = !(gamma2 > p.g2min);
        const double m = floor ? p.g2min : gamma2;
        const double pw = pow(m, p.expo), lam = p.K3 * pw;
        const double R = 1.0 / (2.0 * lam + p.dt), bh = 2.0 * p.dt * R, bb = 1.5 * p.dt * R;
        // f-hat+ = g + bh (e - g), f-bar+ = g + bb (e - g)
        double gb[9], eb[9], bhb = 0.0, bbb = 0.0;
        for (int k = 0; k < 9; ++k) {
            const double yh = G[k * pl + id], yb = bpb[k * pl + id];
            gb[k] = (1.0 - bh) * yh + (1.0 - bb) * yb;
            eb[k] = bh * yh + bb * yb;
            bhb += yh * (e[k] - g[k]);
            bbb += yb * (e[k] - g[k]);
        }
        const double Rb = 2.0 * p.dt * bhb + 1.5 * p.dt * bbb;
        v[A_DT] += 2.0 * R * bhb + 1.5 * R * bbb - Rb * R * R;
        const double lamb = lb[id] + lbar[id] - 2.0 * Rb * R * R;
        // lambda = K3 m^expo
        v[A_K3] = lamb * pw;
        v[A_EXPO] = lamb * lam * log(m);
        double lam_old_b = 0.0;
        if (!floor) {
            const double gb2 = lamb * lam * p.expo / m;
            const double Qb = gb2 * 18.0 * r * r, rb = gb2 * 36.0 * Q * r;
            lam_old_b = -2.0 * rb * r * r;
            v[A_DT] -= rb * r * r;
            const double pxxb = 2.0 * pxx * Qb, pyyb = 2.0 * pyy * Qb, pxyb = 4.0 * pxy * Qb;
            for (int k = 1; k < 9; ++k) {
                const double cx = cxk(k), cy = cyk(k);
                const double nb = cx * cx * pxxb + cx * cy * pxyb + cy * cy * pyyb;
                gb[k] += nb;
                eb[k] -= nb;
            }
        }
        double Pb = 0.0, uxb = 0.0, uyb = 0.0, mb[9];
        equilibrium_t(ux, uy, eb, Pb, uxb, uyb);
        moments_t(ux, uy, Pb, uxb, uyb, mb);
        for (int k = 0; k < 9; ++k) fbar[k * pl + id] = gb[k] + mb[k];
        lbar[id] = lam_old_b;
    }
    accumulate(p, S_A, v);
}

// Step (1)^T: f-hat = e(0, u) with u = (U, 0) on the lid row, Lambda = lam0.
__global__ __launch_bounds__(kB) void a_initial(AdjParams p, const double* fbar, const double* lbar)
{
    double v[A_N] = {};
    int i, j;
    if (node_of(p, i, j)) {
        const int64_t id = at(p, i, j), pl = (int64_t)p.nx * p.ny;
        v[A_LAM0] = lbar[id];
        if (j == p.ny - 1) {
            double eb[9], Pb = 0.0, uxb = 0.0, uyb = 0.0;
            for (int k = 0; k < 9; ++k) eb[k] = fbar[k * pl + id];
            equilibrium_t(p.ulid, 0.0, eb, Pb, uxb, uyb);
            v[A_ULID] = uxb;
        }
    }
    accumulate(p, S_INIT, v);
}

}  // namespace

// --------------------------------------------------------------- host side

struct AdjointSweep::Impl {
    AdjParams p{};
    double cot = 0.0;
    size_t nn = 0, nb = 0;
    double *geo = nullptr, *acc = nullptr, *jpart = nullptr;
    double *bp = nullptr, *fb = nullptr, *fh = nullptr, *ln = nullptr;
    double *fbar = nullptr, *lbar = nullptr, *G = nullptr, *w1 = nullptr, *lb = nullptr, *fbb = nullptr;
};

AdjointSweep::AdjointSweep() : d(new Impl) {}

AdjointSweep::~AdjointSweep()
{
    double* ptrs[] = {d->geo, d->acc, d->jpart, d->bp, d->fb, d->fh, d->ln, d->fbar, d->lbar, d->G, d->w1, d->lb, d->fbb};
    for (double* q : ptrs)
        if (q) (void)hipFree(q);
    delete d;
}

hipError_t AdjointSweep::init(const CavityDesc& c, hipStream_t s)
{
    Impl& m = *d;
    m.cot = c.cot;
    m.nn = (size_t)c.nx * c.ny;
    m.nb = (m.nn + kB - 1) / kB;
    std::vector<double> geo(2 * (c.nx + c.ny));
    for (int j = 0; j < c.ny; ++j) {
        const double eta = j * c.deta, a = 1.0 / (1.0 + 2.0 * c.cot * eta);
        geo[j] = a;
        geo[c.ny + c.nx + j] = -2.0 * eta * a * a;
    }
    for (int i = 0; i < c.nx; ++i) {
        const double w = (double)(2 * i - (c.nx - 1)) / (double)(c.nx - 1);
        geo[c.ny + i] = c.cot * w;
        geo[2 * c.ny + c.nx + i] = w;
    }
    struct {
        double** ptr;
        size_t n;
    } bufs[] = {{&m.geo, geo.size()}, {&m.acc, (size_t)S_N * m.nb * A_N}, {&m.jpart, m.nb}, {&m.bp, 9 * m.nn},
                {&m.fb, 9 * m.nn}, {&m.fh, 9 * m.nn}, {&m.ln, m.nn}, {&m.fbar, 9 * m.nn}, {&m.lbar, m.nn},
                {&m.G, 9 * m.nn}, {&m.w1, 9 * m.nn}, {&m.lb, m.nn}, {&m.fbb, 9 * m.nn}};
    for (auto& b : bufs) {
        hipError_t e = hipMalloc(reinterpret_cast<void**>(b.ptr), b.n * sizeof(double));
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(m.geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(m.acc, 0, (size_t)S_N * m.nb * A_N * sizeof(double), s);
    // a_stage_b reads f-bar only at interior nodes; clear the walls once
    if (e == hipSuccess) e = hipMemsetAsync(m.fb, 0, 9 * m.nn * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(m.fbb, 0, 9 * m.nn * sizeof(double), s);
    AdjParams& p = m.p;
    p.nx = c.nx;
    p.ny = c.ny;
    p.dt = c.dt;
    p.K3 = 3.0 * c.K;
    p.expo = c.expo;
    p.g2min = c.g2min;
    p.mix = c.mix;
    p.ulid = c.u_lid;
    p.inv2dxi = c.inv2dxi;
    p.inv2deta = c.inv2deta;
    p.dxi = c.dxi;
    p.deta = c.deta;
    p.geo = m.geo;
    p.acc = m.acc;
    p.blocks = (int)m.nb;
    return e;
}

hipError_t AdjointSweep::objective(const double* state, hipStream_t s)
{
    Impl& m = *d;
    hipLaunchKernelGGL(a_objective, dim3(m.nb), dim3(kB), 0, s, m.p, m.cot, state, m.fbar, m.lbar, m.jpart);
    return hipGetLastError();
}

hipError_t AdjointSweep::step_back(const double* st, const double* st1, hipStream_t s)
{
    Impl& m = *d;
    const dim3 g(m.nb), b(kB);
    hipLaunchKernelGGL(r_stage_a, g, b, 0, s, m.p, st, m.bp, m.ln);
    hipLaunchKernelGGL(r_stage_b, g, b, 0, s, m.p, m.bp, m.fb);
    hipLaunchKernelGGL(r_stage_bh, g, b, 0, s, m.p, m.fb, m.ln, m.fh);
    hipLaunchKernelGGL(a_stage_cb, g, b, 0, s, m.p, st1, m.fbar, m.G);
    hipLaunchKernelGGL(a_stage_c, g, b, 0, s, m.p, m.G, m.fh, m.w1);
    hipLaunchKernelGGL(a_stage_bh, g, b, 0, s, m.p, m.fb, m.ln, m.w1, m.lb);
    hipLaunchKernelGGL(a_stage_bh2, g, b, 0, s, m.p, m.fb, m.w1, m.fbb);
    hipLaunchKernelGGL(a_stage_b, g, b, 0, s, m.p, m.fbb, m.bp, m.w1);
    hipLaunchKernelGGL(a_stage_a, g, b, 0, s, m.p, st, m.G, m.w1, m.lb, m.fbar, m.lbar);
    return hipGetLastError();
}

hipError_t AdjointSweep::finish(const CavityDesc& c, double dt_dcot, double lam0_dU, double K_dn, double K_dU,
                                hipStream_t s, double* J, double grad[3])
{
    Impl& m = *d;
    hipLaunchKernelGGL(a_initial, dim3(m.nb), dim3(kB), 0, s, m.p, m.fbar, m.lbar);
    hipError_t e = hipGetLastError();
    std::vector<double> acc((size_t)S_N * m.nb * A_N), jp(m.nb);
    if (e == hipSuccess) e = hipMemcpyAsync(acc.data(), m.acc, acc.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(jp.data(), m.jpart, jp.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    double t[A_N] = {};
    for (size_t q = 0; q < (size_t)S_N * m.nb; ++q)
        for (int a = 0; a < A_N; ++a) t[a] += acc[q * A_N + a];
    double j = 0.0;
    for (double x : jp) j += x;
    *J = j;
    const double dcot_dtheta = -(1.0 + c.cot * c.cot);
    grad[0] = (t[A_COT] + t[A_DT] * dt_dcot) * dcot_dtheta;
    grad[1] = 3.0 * t[A_K3] * K_dn + 0.5 * t[A_EXPO];
    grad[2] = 3.0 * t[A_K3] * K_dU + t[A_ULID] + t[A_LAM0] * lam0_dU;
    return hipSuccess;
}

}  // namespace ifd
