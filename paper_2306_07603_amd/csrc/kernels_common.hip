// kernels_common.hip -- per-node kernels around the time step: Step (1)
// initialisation, the residual reduction of Eq. (2.19), macroscopic output
// (Eqs. 2.10-2.11), checkpoint conversion and the kinetic energy of Eq. (5.1).
#include "ifdlbm_internal.h"

namespace ifd {
namespace {

// Step (1): u = 0 and P = 0, except u = (u_lid, 0) on the top row (lid corners
// included), f-hat = f_eq(P, u), lambda = lambda_0.
template <int PREC>
__global__ __launch_bounds__(kNodeBlock) void k_init(void* fv, void* lv, const CavityDesc* desc, const NodeBlock* blocks)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    const NodeBlock nb = blocks[blockIdx.x];
    const CavityDesc c = desc[nb.cav];
    const int n = nb.first + (int)threadIdx.x;
    if (n >= c.nx * c.ny) return;
    const int j = n / c.nx, i = n - j * c.nx;
    const int64_t id = (int64_t)j * c.pitch + i;
    T e[9];
    equilibrium(T(0), j == c.ny - 1 ? T(c.u_lid) : T(0), T(0), e);
    auto* f = static_cast<typename S::F*>(fv);
#pragma unroll
    for (int k = 0; k < 9; ++k) S::store(f, c.f_off + k * c.plane + id, k, e[k]);
    static_cast<typename S::L*>(lv)[c.l_off + id] = T(c.lam0);
}

// out[c][q] = sum of partial[u][q] over the units of cavity c, in a fixed
// order, then the shifts the sums were taken with; the shifts move to the
// means of dP and P just found, for the next evaluation.
__global__ __launch_bounds__(256) void k_reduce(const double* partial, const int32_t* first, const int32_t* count,
                                                const CavityDesc* desc, double* ref, double* out)
{
    __shared__ double sh[kPartials][256];
    const int c = blockIdx.x;
    double v[kPartials];
#pragma unroll
    for (int q = 0; q < kPartials; ++q) v[q] = 0.0;
    for (int u = threadIdx.x; u < count[c]; u += 256)
#pragma unroll
        for (int q = 0; q < kPartials; ++q) v[q] += partial[(int64_t)(first[c] + u) * kPartials + q];
#pragma unroll
    for (int q = 0; q < kPartials; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < kPartials; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    double* o = out + (int64_t)c * kResult;
    if (threadIdx.x < kPartials) o[threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 0) {
        const double rd = ref[2 * c], rp = ref[2 * c + 1];
        o[kPartials] = rd;
        o[kPartials + 1] = rp;
        if (count[c] == 0) return;   // a stopped cavity keeps its shifts
        const double nn = (double)desc[c].nx * (double)desc[c].ny;
        const double md = rd + sh[4][0] / nn, mp = rp + sh[5][0] / nn;
        if (isfinite(md) && isfinite(mp)) {
            ref[2 * c] = md;
            ref[2 * c + 1] = mp;
        }
    }
}

template <int PREC, typename O>
__global__ __launch_bounds__(256) void k_fields(const void* fv, CavityDesc c, O* u, O* v, O* p)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= c.nx * c.ny) return;
    const int j = n / c.nx, i = n - j * c.nx;
    const int64_t id = (int64_t)j * c.pitch + i;
    const auto* f = static_cast<const typename S::F*>(fv);
    T g[9], P, ux, uy;
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = S::load(f, c.f_off + k * c.plane + id, k);
    moments(g, P, ux, uy);
    if (u) u[n] = (O)ux;
    if (v) v[n] = (O)uy;
    if (p) p[n] = (O)P;
}

__host__ __device__ constexpr double weight(int k) { return k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

template <int PREC>
__global__ __launch_bounds__(256) void k_state_out(const void* fv, const void* lv, CavityDesc c, double rho0, double* fhat,
                                                   double* lam)
{
    using S = Storage<PREC>;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int nn = c.nx * c.ny;
    if (n >= nn) return;
    const int j = n / c.nx, i = n - j * c.nx;
    const int64_t id = (int64_t)j * c.pitch + i;
    const auto* f = static_cast<const typename S::F*>(fv);
#pragma unroll
    for (int k = 0; k < 9; ++k) fhat[(int64_t)k * nn + n] = (double)S::load(f, c.f_off + k * c.plane + id, k) + weight(k) * rho0;
    lam[n] = (double)static_cast<const typename S::L*>(lv)[c.l_off + id];
}

template <int PREC>
__global__ __launch_bounds__(256) void k_state_in(void* fv, void* lv, CavityDesc c, double rho0, const double* fhat,
                                                  const double* lam)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int nn = c.nx * c.ny;
    if (n >= nn) return;
    const int j = n / c.nx, i = n - j * c.nx;
    const int64_t id = (int64_t)j * c.pitch + i;
    auto* f = static_cast<typename S::F*>(fv);
#pragma unroll
    for (int k = 0; k < 9; ++k) S::store(f, c.f_off + k * c.plane + id, k, (T)(fhat[(int64_t)k * nn + n] - weight(k) * rho0));
    static_cast<typename S::L*>(lv)[c.l_off + id] = (typename S::L)lam[n];
}

// Eq. (5.1) per block of 256 nodes: 1/2 |u|^2 w_i w_j J_j dxi deta, trapezoid
// weights w (1/2 on the walls) and J = 1 + 2 eta cot(theta).
template <int PREC>
__global__ __launch_bounds__(256) void k_energy(const void* fv, CavityDesc c, double* partial)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    __shared__ double sh[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (n < c.nx * c.ny) {
        const int j = n / c.nx, i = n - j * c.nx;
        const int64_t id = (int64_t)j * c.pitch + i;
        const auto* f = static_cast<const typename S::F*>(fv);
        T g[9], P, ux, uy;
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = S::load(f, c.f_off + k * c.plane + id, k);
        moments(g, P, ux, uy);
        const double wi = (i == 0 || i == c.nx - 1) ? 0.5 : 1.0;
        const double wj = (j == 0 || j == c.ny - 1) ? 0.5 : 1.0;
        const double J = 1.0 + 2.0 * c.cot * (j * c.deta);
        e = 0.5 * wi * wj * J * c.dxi * c.deta * ((double)ux * ux + (double)uy * uy);
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Probe record, part 1: Eq. (5.1) partial sums per node block of every cavity.
template <int PREC>
__global__ __launch_bounds__(256) void k_probe_energy(const void* fv, const CavityDesc* desc, const NodeBlock* blocks,
                                                      double* partial)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    __shared__ double sh[256];
    const NodeBlock nb = blocks[blockIdx.x];
    const CavityDesc c = desc[nb.cav];
    const int n = nb.first + (int)threadIdx.x;
    double e = 0.0;
    if (n < c.nx * c.ny) {
        const int j = n / c.nx, i = n - j * c.nx;
        const int64_t id = (int64_t)j * c.pitch + i;
        const auto* f = static_cast<const typename S::F*>(fv);
        T g[9], P, ux, uy;
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = S::load(f, c.f_off + k * c.plane + id, k);
        moments(g, P, ux, uy);
        const double wi = (i == 0 || i == c.nx - 1) ? 0.5 : 1.0;
        const double wj = (j == 0 || j == c.ny - 1) ? 0.5 : 1.0;
        const double J = 1.0 + 2.0 * c.cot * (j * c.deta);
        e = 0.5 * wi * wj * J * c.dxi * c.deta * ((double)ux * ux + (double)uy * uy);
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Probe record, part 2 (one workgroup): per cavity the kinetic energy (block
// partials summed in order) and the velocity at the centre of the
// computational square (xi = eta = 1/2: one node, or the mean of the two or
// four nearest nodes for an even count) into slot count % capacity of its
// record, then count + 1.
template <int PREC>
__global__ __launch_bounds__(256) void k_probe_finish(const void* fv, const CavityDesc* desc, int n_cav,
                                                      const double* partial, const int32_t* first,
                                                      const int32_t* count, double* rec, uint32_t* rec_count,
                                                      int capacity)
{
    using S = Storage<PREC>;
    using T = typename S::T;
    const uint32_t nrec = rec_count[0];
    const int slot = (int)(nrec % (uint32_t)capacity);
    const auto* f = static_cast<const typename S::F*>(fv);
    for (int cav = threadIdx.x; cav < n_cav; cav += blockDim.x) {
        const CavityDesc c = desc[cav];
        double ke = 0.0;
        for (int b = first[cav]; b < first[cav] + count[cav]; ++b) ke += partial[b];
        const int ia = (c.nx - 1) / 2, ib = c.nx / 2, ja = (c.ny - 1) / 2, jb = c.ny / 2;
        double su = 0.0, sv = 0.0;
        for (int j = ja; j <= jb; ++j)
            for (int i = ia; i <= ib; ++i) {
                const int64_t id = (int64_t)j * c.pitch + i;
                T g[9], P, ux, uy;
#pragma unroll
                for (int k = 0; k < 9; ++k) g[k] = S::load(f, c.f_off + k * c.plane + id, k);
                moments(g, P, ux, uy);
                su += (double)ux;
                sv += (double)uy;
            }
        const double inv = 1.0 / ((jb - ja + 1) * (ib - ia + 1));
        double* r = rec + ((int64_t)cav * capacity + slot) * 3;
        r[0] = su * inv;
        r[1] = sv * inv;
        r[2] = ke;
    }
    __syncthreads();
    if (threadIdx.x == 0) rec_count[0] = nrec + 1u;
}

__global__ void k_seed_bump(uint32_t* ctr) { ctr[0] += 1u; }

inline unsigned blocks_of(const CavityDesc& c) { return (unsigned)((c.nx * c.ny + 255) / 256); }

}  // namespace

hipError_t launch_init(int prec, void* f, void* l, const CavityDesc* desc, const NodeBlock* blocks, int nb, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    switch (prec) {
    case P_FP64: hipLaunchKernelGGL(k_init<P_FP64>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    case P_FP32: hipLaunchKernelGGL(k_init<P_FP32>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    case P_FP16DEV: hipLaunchKernelGGL(k_init<P_FP16DEV>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    case P_FP32X: hipLaunchKernelGGL(k_init<P_FP32X>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    case P_FP32SR: hipLaunchKernelGGL(k_init<P_FP32SR>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    case P_FP32SRF: hipLaunchKernelGGL(k_init<P_FP32SRF>, dim3(nb), dim3(kNodeBlock), 0, s, f, l, desc, blocks); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_seed_bump(uint32_t* ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_seed_bump, dim3(1), dim3(1), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, const int32_t* first, const int32_t* count,
                                  const CavityDesc* desc, int n_cav, double* ref, double* out, hipStream_t s)
{
    if (n_cav <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_cav), dim3(256), 0, s, partial, first, count, desc, ref, out);
    return hipGetLastError();
}

hipError_t launch_fields(int prec, const void* f, const CavityDesc*, int, const CavityDesc& hd, void* u, void* v, void* p,
                         int dtype, hipStream_t s)
{
    const dim3 g(blocks_of(hd)), b(256);
#define IFD_FIELDS(P)                                                                                              \
    if (dtype == 0)                                                                                                \
        hipLaunchKernelGGL((k_fields<P, double>), g, b, 0, s, f, hd, (double*)u, (double*)v, (double*)p);      \
    else                                                                                                           \
        hipLaunchKernelGGL((k_fields<P, float>), g, b, 0, s, f, hd, (float*)u, (float*)v, (float*)p);
    switch (prec) {
    case P_FP64: IFD_FIELDS(P_FP64) break;
    case P_FP32: IFD_FIELDS(P_FP32) break;
    case P_FP16DEV: IFD_FIELDS(P_FP16DEV) break;
    case P_FP32X: IFD_FIELDS(P_FP32X) break;
    case P_FP32SR: IFD_FIELDS(P_FP32SR) break;
    case P_FP32SRF: IFD_FIELDS(P_FP32SRF) break;
    default: return hipErrorInvalidValue;
    }
#undef IFD_FIELDS
    return hipGetLastError();
}

hipError_t launch_state_out(int prec, const void* f, const void* l, const CavityDesc& hd, double rho0, double* fhat,
                            double* lam, hipStream_t s)
{
    const dim3 g(blocks_of(hd)), b(256);
    switch (prec) {
    case P_FP64: hipLaunchKernelGGL(k_state_out<P_FP64>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32: hipLaunchKernelGGL(k_state_out<P_FP32>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP16DEV: hipLaunchKernelGGL(k_state_out<P_FP16DEV>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32X: hipLaunchKernelGGL(k_state_out<P_FP32X>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32SR: hipLaunchKernelGGL(k_state_out<P_FP32SR>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32SRF: hipLaunchKernelGGL(k_state_out<P_FP32SRF>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_state_in(int prec, void* f, void* l, const CavityDesc& hd, double rho0, const double* fhat,
                           const double* lam, hipStream_t s)
{
    const dim3 g(blocks_of(hd)), b(256);
    switch (prec) {
    case P_FP64: hipLaunchKernelGGL(k_state_in<P_FP64>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32: hipLaunchKernelGGL(k_state_in<P_FP32>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP16DEV: hipLaunchKernelGGL(k_state_in<P_FP16DEV>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32X: hipLaunchKernelGGL(k_state_in<P_FP32X>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32SR: hipLaunchKernelGGL(k_state_in<P_FP32SR>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    case P_FP32SRF: hipLaunchKernelGGL(k_state_in<P_FP32SRF>, g, b, 0, s, f, l, hd, rho0, fhat, lam); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_probe(int prec, const void* f, const CavityDesc* desc, int n_cav, const NodeBlock* blocks, int nb,
                        double* partial, const int32_t* first, const int32_t* count, double* rec, uint32_t* rec_count,
                        int capacity, hipStream_t s)
{
    if (nb <= 0 || n_cav <= 0) return hipSuccess;
#define IFD_PROBE(P)                                                                                            \
    hipLaunchKernelGGL(k_probe_energy<P>, dim3(nb), dim3(256), 0, s, f, desc, blocks, partial);                \
    hipLaunchKernelGGL(k_probe_finish<P>, dim3(1), dim3(256), 0, s, f, desc, n_cav, partial, first, count, rec, \
                       rec_count, capacity);
    switch (prec) {
    case P_FP64: IFD_PROBE(P_FP64) break;
    case P_FP32: IFD_PROBE(P_FP32) break;
    case P_FP16DEV: IFD_PROBE(P_FP16DEV) break;
    case P_FP32X: IFD_PROBE(P_FP32X) break;
    case P_FP32SR: IFD_PROBE(P_FP32SR) break;
    case P_FP32SRF: IFD_PROBE(P_FP32SRF) break;
    default: return hipErrorInvalidValue;
    }
#undef IFD_PROBE
    return hipGetLastError();
}

// The stochastic rounding of the FP32SR / FP32SRF encode on given values and
// random numbers (the low 16 bits of r16).
__global__ void k_round_stochastic(const double* v, const uint32_t* r16, float* out, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = round_stochastic(v[q], r16[q] & 0xFFFFu);
}

hipError_t launch_round_stochastic(const double* v, const uint32_t* r16, float* out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_round_stochastic, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, v, r16,
                       out, n);
    return hipGetLastError();
}

// The FP64 power of Step (2) (Eq. 1.4 on gamma^2) on given values: out[i] =
// x[i]^y as the FP64 arithmetic of the step computes it.
__global__ void k_power_law(const double* x, double y, double* out, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = pow_pos<double>(x[q], y);
}

hipError_t launch_power_law(const double* x, double y, double* out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_power_law, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, x, y, out, n);
    return hipGetLastError();
}

hipError_t launch_energy(int prec, const void* f, const CavityDesc*, const double*, int, const CavityDesc& hd,
                         double* partial, hipStream_t s)
{
    const dim3 g(blocks_of(hd)), b(256);
    switch (prec) {
    case P_FP64: hipLaunchKernelGGL(k_energy<P_FP64>, g, b, 0, s, f, hd, partial); break;
    case P_FP32: hipLaunchKernelGGL(k_energy<P_FP32>, g, b, 0, s, f, hd, partial); break;
    case P_FP16DEV: hipLaunchKernelGGL(k_energy<P_FP16DEV>, g, b, 0, s, f, hd, partial); break;
    case P_FP32X: hipLaunchKernelGGL(k_energy<P_FP32X>, g, b, 0, s, f, hd, partial); break;
    case P_FP32SR: hipLaunchKernelGGL(k_energy<P_FP32SR>, g, b, 0, s, f, hd, partial); break;
    case P_FP32SRF: hipLaunchKernelGGL(k_energy<P_FP32SRF>, g, b, 0, s, f, hd, partial); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ifd
