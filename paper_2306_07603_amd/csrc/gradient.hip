// gradient.hip -- derivative of a cavity objective with respect to the top
// angle theta (radians), the power-law index n and the lid speed U, by
// forward (tangent-linear) differentiation of the discrete IFDLBM step.
//
// Every quantity of the staged step carries its value and its three partial
// derivatives (Dual<3>, FP64).  The parameters enter through the metric terms
// a_j = 1/(1 + 2 eta_j cot theta), s_i = cot theta (2 xi_i - 1) (Eqs. 3.2-3.8.2),
// the time step (CFL rule on the contravariant speed 1 + cot theta), the
// consistency K = U^(2-n) / Re (Eq. 2.15.1), the exponent (n - 1)/2 of
// Eq. (1.4), the lid velocity (Eq. 1.5) and the initial lambda U / (Re c_s^2).
// The objective is the kinetic energy of Eq. (5.1) after n_steps steps.  With
// three parameters the tangent sweep costs about four forward runs and needs
// no stored trajectory; the derivative is that of the discrete objective, the
// same one a reverse sweep would return.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "dual.h"
#include "ifdlbm_internal.h"

namespace ifd {

using D3 = Dual<3>;

template <> __device__ __forceinline__ D3 recip<D3>(D3 x) { return D3(1.0) / x; }
template <> __host__ __device__ __forceinline__ D3 pow_pos<D3>(D3 x, D3 y) { return dual_pow(x, y); }

namespace {

struct TParams {
    int nx, ny;
    D3 dt, K, expo, g2min, mix, ulid, inv2dxi, inv2deta, cot, lam0;
    double dxi, deta;
};

// Step (2), Eqs. (2.12)-(2.14) and (1.4), as relaxation_time but with every
// parameter differentiated (no Newtonian shortcut: d mu / d n != 0 at n = 1).
__device__ D3 relax_t(const D3 g[9], const D3 e[9], D3 lam_old, const TParams& c)
{
    D3 n[9];
    for (int k = 0; k < 9; ++k) n[k] = g[k] - e[k];
    const D3 s58 = (n[5] + n[6]) + (n[7] + n[8]);
    const D3 pxx = (n[1] + n[3]) + s58;
    const D3 pyy = (n[2] + n[4]) + s58;
    const D3 pxy = (n[5] - n[6]) + (n[7] - n[8]);
    const D3 r = D3(1.0) / (D3(2.0) * lam_old + c.dt);
    D3 gamma2 = D3(18.0) * (pxx * pxx + D3(2.0) * pxy * pxy + pyy * pyy) * r * r;
    if (!(gamma2 > c.g2min)) gamma2 = c.g2min;
    return D3(3.0) * c.K * dual_pow(gamma2, c.expo);
}

__device__ D3 transport_t(const D3* plane, const TParams& c, const D3* geo, int i, int j, int k)
{
    const int cx = cxk(k), cy = cyk(k);
    D3 term(0.0);
    // the xi term is kept where c_xi is zero: its theta derivative need not be
    // (the upwind side is then the c >= 0 one, as in the forward step)
    const D3 cxi = geo[j] * (D3((double)cx) - D3((double)cy) * geo[c.ny + i]);
    {
        const D3* row = plane + (int64_t)j * c.nx;
        const bool pos = cxi.v >= 0.0;
        const D3 m2 = (pos && i >= 2) ? row[i - 2] : D3(0.0);
        const D3 p2 = (!pos && i <= c.nx - 3) ? row[i + 2] : D3(0.0);
        term += cxi * (mixed_diff_2h(m2, row[i - 1], row[i], row[i + 1], p2, pos, i == 1, i == c.nx - 2, c.mix) * c.inv2dxi);
    }
    if (cy != 0) {
        const D3* col = plane + i;
        const int p = c.nx;
        const bool pos = cy > 0;
        const D3 m2 = (pos && j >= 2) ? col[(j - 2) * p] : D3(0.0);
        const D3 p2 = (!pos && j <= c.ny - 3) ? col[(j + 2) * p] : D3(0.0);
        term += D3((double)cy) * (mixed_diff_2h(m2, col[(j - 1) * p], col[j * p], col[(j + 1) * p], p2, pos, j == 1,
                                                j == c.ny - 2, c.mix) * c.inv2deta);
    }
    return term;
}

// Arrays of one cavity, packed [k][j][i] (plane = nx * ny).
struct TBuf {
    D3 *f[2], *l[2], *hp, *bp, *fb, *ln, *geo, *part;
};

__device__ inline bool node(const TParams& c, int& i, int& j)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= c.nx * c.ny) return false;
    j = n / c.nx;
    i = n - j * c.nx;
    return true;
}

__global__ __launch_bounds__(256) void t_init(TParams c, D3* f, D3* l)
{
    int i, j;
    if (!node(c, i, j)) return;
    const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
    D3 e[9];
    equilibrium(D3(0.0), j == c.ny - 1 ? c.ulid : D3(0.0), D3(0.0), e);
    for (int k = 0; k < 9; ++k) f[k * pl + id] = e[k];
    l[id] = c.lam0;
}

__global__ __launch_bounds__(256) void t_stage_a(TParams c, const D3* fin, const D3* lin, D3* hp, D3* bp, D3* ln)
{
    int i, j;
    if (!node(c, i, j)) return;
    const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
    D3 g[9], e[9], P, ux, uy;
    for (int k = 0; k < 9; ++k) g[k] = fin[k * pl + id];
    moments(g, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const D3 lam = relax_t(g, e, lin[id], c);
    const Collision<D3> col(lam, c.dt);
    for (int k = 0; k < 9; ++k) {
        hp[k * pl + id] = col.a_hat * g[k] + col.b_hat * e[k];
        bp[k * pl + id] = col.a_bar * g[k] + col.b_bar * e[k];
    }
    ln[id] = lam;
}

__global__ __launch_bounds__(256) void t_stage_b(TParams c, const D3* bp, D3* fb, const D3* geo)
{
    int i, j;
    if (!node(c, i, j) || is_boundary(i, j, c.nx, c.ny)) return;
    const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
    const D3 half_dt = D3(0.5) * c.dt;
    fb[id] = bp[id];
    for (int k = 1; k < 9; ++k) fb[k * pl + id] = bp[k * pl + id] - half_dt * transport_t(bp + k * pl, c, geo, i, j, k);
}

__global__ __launch_bounds__(256) void t_stage_bh(TParams c, const D3* fbar, const D3* ln, D3* fh)
{
    int i, j;
    if (!node(c, i, j)) return;
    const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
    D3 x[9];
    if (is_boundary(i, j, c.nx, c.ny)) {
        int ni, nj;
        inward(i, j, c.nx, c.ny, ni, nj);
        D3 xnb[9];
        for (int k = 0; k < 9; ++k) xnb[k] = fbar[k * pl + (int64_t)nj * c.nx + ni];
        extrapolate(xnb, j == c.ny - 1 ? c.ulid : D3(0.0), x);
    } else {
        for (int k = 0; k < 9; ++k) x[k] = fbar[k * pl + id];
    }
    D3 P, ux, uy, e[9];
    moments(x, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const HalfStep<D3> hs(ln[id], c.dt);
    for (int k = 0; k < 9; ++k) fh[k * pl + id] = hs.a * x[k] + hs.b * e[k];
}

__global__ __launch_bounds__(256) void t_stage_c(TParams c, const D3* fh, const D3* hp, const D3* ln, D3* out, D3* lout,
                                                 const D3* geo)
{
    int i, j;
    if (!node(c, i, j)) return;
    const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
    lout[id] = ln[id];
    if (is_boundary(i, j, c.nx, c.ny)) return;
    out[id] = hp[id];
    for (int k = 1; k < 9; ++k) out[k * pl + id] = hp[k * pl + id] - c.dt * transport_t(fh + k * pl, c, geo, i, j, k);
}

__global__ __launch_bounds__(256) void t_stage_cb(TParams c, D3* out)
{
    int i, j;
    if (!node(c, i, j) || !is_boundary(i, j, c.nx, c.ny)) return;
    const int64_t pl = (int64_t)c.nx * c.ny;
    int ni, nj;
    inward(i, j, c.nx, c.ny, ni, nj);
    D3 xnb[9], x[9];
    for (int k = 0; k < 9; ++k) xnb[k] = out[k * pl + (int64_t)nj * c.nx + ni];
    extrapolate(xnb, j == c.ny - 1 ? c.ulid : D3(0.0), x);
    for (int k = 0; k < 9; ++k) out[k * pl + (int64_t)j * c.nx + i] = x[k];
}

// Eq. (5.1) per block: 1/2 |u|^2 w_i w_j J_j dxi deta with J_j = 1 + 2 eta_j cot(theta).
__global__ __launch_bounds__(256) void t_energy(TParams c, const D3* f, D3* part)
{
    __shared__ double sh[4][256];
    int i, j;
    D3 e(0.0);
    if (node(c, i, j)) {
        const int64_t id = (int64_t)j * c.nx + i, pl = (int64_t)c.nx * c.ny;
        D3 g[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) g[k] = f[k * pl + id];
        moments(g, P, ux, uy);
        const double wi = (i == 0 || i == c.nx - 1) ? 0.5 : 1.0;
        const double wj = (j == 0 || j == c.ny - 1) ? 0.5 : 1.0;
        const D3 J = D3(1.0) + D3(2.0 * j * c.deta) * c.cot;
        e = D3(0.5 * wi * wj * c.dxi * c.deta) * J * (ux * ux + uy * uy);
    }
    sh[0][threadIdx.x] = e.v;
    for (int q = 0; q < 3; ++q) sh[q + 1][threadIdx.x] = e.d[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        D3 s(sh[0][0]);
        for (int q = 0; q < 3; ++q) s.d[q] = sh[q + 1][0];
        part[blockIdx.x] = s;
    }
}

}  // namespace

namespace {

// Parameters of the step and the metric tables a_j, s_i, each with its derivatives with respect to
// (theta [rad], n, U).
void tangent_params(int nx, int ny, double re, double n, double theta_deg, double u_lid, double cfl, double mix,
                    double gamma_min, int dt_rule, TParams& P, std::vector<D3>& geo)
{
    const double th = theta_deg * (M_PI / 180.0);
    const double C = theta_deg == 90.0 ? 0.0 : 1.0 / std::tan(th);
    const double dC = -(1.0 + C * C);   // d cot / d theta
    const double U = std::fabs(u_lid), sgnU = u_lid < 0 ? -1.0 : 1.0;
    const double dxi = 1.0 / (nx - 1), deta = 1.0 / (ny - 1);
    P.nx = nx;
    P.ny = ny;
    P.dxi = dxi;
    P.deta = deta;
    {
        double d[3] = {dC, 0, 0};
        P.cot = D3::make(C, d);
    }
    if (dt_rule == 1 || 1.0 / deta > (1.0 + C) / dxi) {
        P.dt = D3(dt_rule == 1 ? cfl * std::min(dxi, deta) : cfl * deta);
    } else {
        const double dt = cfl * dxi / (1.0 + C);
        double d[3] = {-dt / (1.0 + C) * dC, 0, 0};
        P.dt = D3::make(dt, d);
    }
    const double K = std::pow(U, 2.0 - n) / re;
    {
        double d[3] = {0, -K * std::log(U), (2.0 - n) * K / U * sgnU};
        P.K = D3::make(K, d);
    }
    {
        double d[3] = {0, 0.5, 0};
        P.expo = D3::make(0.5 * (n - 1.0), d);
    }
    P.g2min = D3(gamma_min * gamma_min);
    P.mix = D3(mix);
    {
        double d[3] = {0, 0, 1.0};
        P.ulid = D3::make(u_lid, d);
    }
    P.inv2dxi = D3(0.5 / dxi);
    P.inv2deta = D3(0.5 / deta);
    {
        double d[3] = {0, 0, 3.0 / re * sgnU};
        P.lam0 = D3::make(3.0 * U / re, d);
    }
    geo.resize(ny + nx);
    for (int j = 0; j < ny; ++j) {
        const double eta = j * deta, a = 1.0 / (1.0 + 2.0 * C * eta);
        double d[3] = {-2.0 * eta * a * a * dC, 0, 0};
        geo[j] = D3::make(a, d);
    }
    for (int i = 0; i < nx; ++i) {
        const double w = (double)(2 * i - (nx - 1)) / (double)(nx - 1);
        double d[3] = {w * dC, 0, 0};
        geo[ny + i] = D3::make(C * w, d);
    }
}

// Sizes (in three-component duals) of the ten work arrays, in the order carve lays them out: the state twice
// (nine planes and lambda each), f-hat+, f-bar+ then f(t + dt/2), f-bar, lambda of the step, the metric tables,
// the energy partial sums.
void workspace_sizes(size_t nn, size_t ngeo, size_t (&sizes)[10])
{
    const size_t s[10] = {9 * nn, 9 * nn, nn, nn, 9 * nn, 9 * nn, 9 * nn, nn, ngeo, (nn + 255) / 256};
    for (int q = 0; q < 10; ++q) sizes[q] = s[q];
}

// The ten work arrays carved from one workspace of tangent_workspace_elems(nx, ny) values.
TBuf carve(D3* w, size_t nn, size_t ngeo)
{
    TBuf b{};
    D3** ptrs[] = {&b.f[0], &b.f[1], &b.l[0], &b.l[1], &b.hp, &b.bp, &b.fb, &b.ln, &b.geo, &b.part};
    size_t sizes[10];
    workspace_sizes(nn, ngeo, sizes);
    for (int q = 0; q < 10; ++q) {
        *ptrs[q] = w;
        w += sizes[q];
    }
    return b;
}

// The sweep in a given workspace: Step (1), n_steps staged steps with their derivatives, Eq. (5.1).  Every
// work array is written before it is read, so the workspace needs no clearing.
hipError_t tangent_run(const TParams& P, const std::vector<D3>& geo, D3* work, int64_t n_steps, hipStream_t s,
                       double* J, double* grad, std::string& err)
{
    const size_t nn = (size_t)P.nx * P.ny, nb = (nn + 255) / 256;
    const TBuf b = carve(work, nn, geo.size());
    auto failed = [&](hipError_t e, const char* what) {
        err = std::string("gradient: ") + what + ": " + hipGetErrorString(e);
        return e;
    };
    hipError_t e = hipMemcpyAsync(b.geo, geo.data(), geo.size() * sizeof(D3), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return failed(e, "metric tables to the device");
    const dim3 g(nb), blk(256);
    hipLaunchKernelGGL(t_init, g, blk, 0, s, P, b.f[0], b.l[0]);
    if ((e = hipGetLastError()) != hipSuccess) return failed(e, "Step (1) launch");
    int cur = 0;
    for (int64_t t = 0; t < n_steps; ++t) {
        hipLaunchKernelGGL(t_stage_a, g, blk, 0, s, P, b.f[cur], b.l[cur], b.hp, b.bp, b.ln);
        hipLaunchKernelGGL(t_stage_b, g, blk, 0, s, P, b.bp, b.fb, b.geo);
        hipLaunchKernelGGL(t_stage_bh, g, blk, 0, s, P, b.fb, b.ln, b.bp);
        hipLaunchKernelGGL(t_stage_c, g, blk, 0, s, P, b.bp, b.hp, b.ln, b.f[cur ^ 1], b.l[cur ^ 1], b.geo);
        hipLaunchKernelGGL(t_stage_cb, g, blk, 0, s, P, b.f[cur ^ 1]);
        cur ^= 1;
        if ((t & 1023) == 1023 && (e = hipGetLastError()) != hipSuccess) return failed(e, "step launch");
    }
    hipLaunchKernelGGL(t_energy, g, blk, 0, s, P, b.f[cur], b.part);
    if ((e = hipGetLastError()) != hipSuccess) return failed(e, "step or energy launch");
    std::vector<D3> part(nb);
    e = hipMemcpyAsync(part.data(), b.part, nb * sizeof(D3), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return failed(e, "energy partial sums to the host");
    D3 sum(0.0);
    for (const D3& x : part) sum += x;
    *J = sum.v;
    for (int q = 0; q < 3; ++q) grad[q] = sum.d[q];
    return hipSuccess;
}

// Work arrays of ifdlbm_gradient_noalloc: one array per GPU, held until the process ends.  Host code must not
// use this name as a device address: the address of each GPU's copy comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the first call on each device).
hipError_t scratch_of_current_device(void** out, std::string& err)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return e;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device index beyond the library's table of scratch arrays";
        return hipErrorInvalidDevice;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

size_t tangent_workspace_elems(int nx, int ny)
{
    size_t sizes[10], total = 0;
    workspace_sizes((size_t)nx * ny, (size_t)nx + (size_t)ny, sizes);
    for (size_t x : sizes) total += x;
    return total;   // 48 nn + nx + ny + ceil(nn / 256)
}

size_t tangent_scratch_capacity_elems() { return kScratchBytes / sizeof(D3); }

// Host driver; returns a HIP error or hipSuccess and fills J and grad[3].  The work arrays live in one
// allocation made and freed here, or, with use_scratch, in the current device's scratch array.
hipError_t tangent_kinetic_energy(int nx, int ny, double re, double n, double theta_deg, double u_lid, double cfl,
                                  double mix, double gamma_min, int dt_rule, int64_t n_steps, hipStream_t s, double* J,
                                  double* grad, std::string& err, bool use_scratch)
{
    TParams P;
    std::vector<D3> geo;
    tangent_params(nx, ny, re, n, theta_deg, u_lid, cfl, mix, gamma_min, dt_rule, P, geo);
    const size_t elems = tangent_workspace_elems(nx, ny);
    D3* work = nullptr;
    hipError_t e = hipSuccess;
    if (use_scratch) {
        if (elems > tangent_scratch_capacity_elems()) {
            err = "grid too large for the scratch array";
            return hipErrorInvalidValue;
        }
        void* p = nullptr;
        e = scratch_of_current_device(&p, err);
        if (e != hipSuccess) return e;
        work = static_cast<D3*>(p);
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&work), elems * sizeof(D3));
        if (e != hipSuccess) {
            err = std::string("gradient: ") + hipGetErrorString(e);
            return e;
        }
    }
    e = tangent_run(P, geo, work, n_steps, s, J, grad, err);
    if (!use_scratch) (void)hipFree(work);
    return e;
}

}  // namespace ifd
