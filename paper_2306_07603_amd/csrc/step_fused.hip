// step_fused.hip -- one launch per IFDLBM time step (arXiv:2306.07603,
// Section 4, Steps (2)-(6)); each wavefront reads the state of its work item
// once from HBM and writes it once.
//
// Work item: output columns [i0, i1) and rows [j0, j1) of one cavity.  The 64
// lanes of the wavefront hold columns i0 - 4 .. i0 + 59, one column per lane,
// and march up the rows.  At row t of the march:
//   A  (row t)     f-hat and lambda (fetched one row ahead): moments, lambda
//                  (Step 2, stored), f-bar+ (Eq. 2.16) into a register ring
//                  and f-hat+ (Eq. 2.15) into a lane-private LDS ring
//   B  (row t - 2) f-bar(t + dt/2) by Eq. (3.7), walls by extrapolation, and
//                  f(t + dt/2) by Eq. (2.17) into a second register ring
//   C  (row t - 4) f-hat(t + dt) by Eq. (3.6) from the f-hat+ of the LDS
//                  ring, walls by extrapolation (Step 6), store, residual
//                  partial sums of Eq. (2.19)
// The eta-direction stencils read the register rings (five rows each); the
// xi-direction stencils read neighbour lanes through one LDS row per
// population, at per-lane addresses that already point at the upwind side
// (the sign of the contravariant velocity of Eq. (3.2) is fixed per column
// and population), so no operand is selected after the read.  With FP32
// arithmetic the LDS row holds backward differences of the values, each
// lane's taken across the wavefront from its left neighbour, and both
// directions apply Eq. (2.5) to differences.  The stored f-hat that the
// exact final update of FP32SRF adds at stage C comes from a lane-private
// LDS ring (populations 0-5) and from a second read of the row copied into
// LDS by the buffer unit (populations 6-8).  The rows of the march are
// unrolled five times so that ring slots are renamed, not moved.  The halo
// costs 8 of 64 lanes across xi and 8 + 4 recomputed rows per segment along
// eta.  The bottom wall row is produced with row 1 (its
// extrapolation source), the lid row of f-hat(t + dt) with row ny - 2, the
// lid row of f(t + dt/2) from row ny - 2 kept for one row in the LDS ring.
//
// Global memory is addressed through raw buffer resources: one 4-dword
// resource per array and cavity, the plane of population k as a scalar
// offset, the row and column as one 32-bit vector offset.
#include "ifdlbm_internal.h"

namespace ifd {
namespace {

constexpr int kPad = 2;                          // LDS columns beyond the wave on each side
constexpr int kRowLds = kWaveLanes + 2 * kPad;   // elements of one LDS exchange row
constexpr int kRing = 5;                         // ring slots: rows t - 4 .. t
// Exact final update: stage C needs the stored f-hat of its row again.  Stage A
// keeps populations 0 .. kGxRing - 1 of it in a lane-private LDS ring; the
// buffer unit copies the others back from memory (by then the row has left L2).
// Six ring populations fill the LDS of two waves per SIMD (20 384 bytes per
// wave, 8 waves in the 160 KiB of a CU) once the xi exchange of FP32SRF passes
// one population at a time through a single LDS row.
constexpr int kGxRing = 6;
// populations per pass of the xi exchange through LDS
constexpr int xs_rows(bool exact_final) { return exact_final ? 1 : 8; }

// Waves per SIMD the register allocation must allow: two with FP32 arithmetic (256 VGPRs each), one with
// FP64 arithmetic (its rings and stage temporaries take about 430 registers).
template <int PREC>
struct Tuning {
    static constexpr bool kWide = sizeof(typename Storage<PREC>::T) == 8;
    static constexpr int kWaves = kWide ? 1 : 2;
};

// Dword 3 of a raw buffer resource on the gfx9 family (CDNA): 32-bit data
// format, no swizzle, no index stride.
constexpr int kRawBufferWord3 = 0x00020000;
// A buffer offset beyond any buffer of the step (ifdlbm_create keeps the state
// of one cavity below 1.2 GiB, and offset plus plane offset below 2^32): loads
// from it return 0 and stores to it are dropped by the range check of raw
// buffers.
constexpr uint32_t kDroppedOffset = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRawBufferWord3);
}

template <typename F> struct Buf;
template <> struct Buf<double> {
    __device__ static double ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static void st(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        using W = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), r, vo, so, 0);
    }
};
template <> struct Buf<float> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static void st(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, 0);
    }
};
template <> struct Buf<__half> {
    __device__ static __half ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    __device__ static void st(__half v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, vo, so, 0);
    }
};

template <typename T> __device__ __forceinline__ const T* geo_of(const StepArgs& a);
template <> __device__ __forceinline__ const double* geo_of<double>(const StepArgs& a) { return a.geo; }
template <> __device__ __forceinline__ const float* geo_of<float>(const StepArgs& a) { return a.geo32; }

// Weights of Eq. (2.5) times sign(c) * 2h on the upwind-sorted points a2
// (two behind), a1 (one behind), c0 and f1 (one ahead):
// sign(c) * central = f1 - a1 (Eq. 2.6), sign(c) * upwind = 3 c0 - 4 a1 + a2
// (Eq. 2.7), so eps * central + (1 - eps) * upwind is
// eps f1 - (4 - 3 eps) a1 + 3 (1 - eps) c0 + (1 - eps) a2.
template <typename T>
struct MixedWeights {
    T wf, wa1, wc, wa2;
    __device__ __forceinline__ MixedWeights(T eps, T scale)
        : wf(scale * eps), wa1(-scale * (T(4) - T(3) * eps)), wc(scale * T(3) * (T(1) - eps)),
          wa2(scale * (T(1) - eps))
    {
    }
    __device__ __forceinline__ T apply(T a2, T a1, T c0, T f1) const { return ((wc * c0 + wa1 * a1) + wa2 * a2) + wf * f1; }
    // The same on differences, which FP32 arithmetic needs: neighbouring
    // values agree to many digits, so the weighted sum of the values above
    // loses to cancellation what differences keep (an error of order one ulp
    // of f per step that does not average out over a steady run).  With the
    // backward differences B(m) = x(m) - x(m - 1) along the upwind direction,
    // n = B at the point (c0 - a1), f = B one further upwind (a1 - a2) and
    // o = B one downwind (f1 - a1 = n + o), it is
    // (eps + 3 (1 - eps)) n - (1 - eps) f + eps o.
    __device__ __forceinline__ T apply_back(T n, T f, T o) const { return ((wc + wf) * n - wa2 * f) + wf * o; }
    // r minus the same, as three multiply-adds into r
    __device__ __forceinline__ T sub_back(T r, T n, T f, T o) const
    {
        return __builtin_fmaf(-(wc + wf), n, __builtin_fmaf(wa2, f, __builtin_fmaf(-wf, o, r)));
    }
};

// x of lane l - 1 in lane l (lane 0 reads 0): a wavefront shift of the data-parallel primitives, folded by the
// compiler into the instruction that uses it.
__device__ __forceinline__ float lane_below(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138 /* wave_shr:1 */,
                                                                0xF, 0xF, true));
}

// Mixed differences from differences first where the distributions are FP32.
template <typename T> constexpr bool kDiffForm = sizeof(T) == 4;

// Population k of the eta direction moves up (c_ky > 0: 2, 5, 6), down
// (c_ky < 0: 4, 7, 8) or not at all (0, 1, 3).
constexpr bool moves_up(int k) { return cyk(k) > 0; }
constexpr bool moves_down(int k) { return cyk(k) < 0; }

// The xi-stencil view of one lane, fixed for the work item.  The
// contravariant xi-velocity is a_j d_k(i) with d_k = c_kx - c_ky s_i
// (Eqs. 3.2-3.8.2): d = 1 for k = 1, -1 for k = 3, and for the pairs
// (2, 4), (5, 7), (6, 8) the second member has minus the first's d.  The
// upwind side follows sign(d) (ties: the c >= 0 side; there |d| = 0 and the
// term vanishes).  Byte offsets into an LDS row.
// FP64 arithmetic (rows of values): a1/a2/f1 of the first member of each
// pair, a2m the far point of the mirrored member (whose a1 and f1 are the
// pair's f1 and a1); ad = |d|.
// FP32 arithmetic (rows of backward differences B(m) = x(m) - x(m - 1)): the
// member with d >= 0 reads near B(l), far B(l - 1) and other B(l + 1), the
// member with d < 0 near B(l + 1), far B(l + 2) and other B(l).  a1 is the
// first member's near (the second's other), f1 the first's other (the
// second's near), a2 and a2m the two far points, which at a wall-adjacent
// column are the near ones (the first-order point of Eq. 2.7); ad = d,
// signed.
template <typename T>
struct XiLane {
    uint32_t own;           // this lane's column
    uint32_t a1[3], a2[3], f1[3], a2m[3];
    T ad[3];                // |d| of the pairs
    bool edge1, edge3;      // second upwind point outside the grid (first-order point, Eq. 2.7 at walls)
    bool edge_p[3], edge_m[3];

    __device__ __forceinline__ XiLane(int lane, int i, int nx, T s)
    {
        constexpr uint32_t E = sizeof(T);
        own = (uint32_t)(lane + kPad) * E;
        const T d[3] = {-s, T(1) - s, T(-1) - s};   // d of k = 2, 5, 6
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool pos = d[c] >= T(0);
            edge_p[c] = pos ? i == 1 : i == nx - 2;
            edge_m[c] = pos ? i == nx - 2 : i == 1;
            if constexpr (kDiffForm<T>) {
                const uint32_t far_p = i == 1 ? own : own - E, far_m = i == nx - 2 ? own + E : own + 2 * E;
                ad[c] = d[c];
                a1[c] = pos ? own : own + E;
                f1[c] = pos ? own + E : own;
                a2[c] = pos ? far_p : far_m;
                a2m[c] = pos ? far_m : far_p;
            } else {
                ad[c] = pos ? d[c] : -d[c];
                a1[c] = pos ? own - E : own + E;
                f1[c] = pos ? own + E : own - E;
                a2[c] = pos ? own - 2 * E : own + 2 * E;
                a2m[c] = pos ? own + 2 * E : own - 2 * E;
            }
        }
        edge1 = i == 1;
        edge3 = i == nx - 2;
    }
};

// The workgroup is one wavefront, whose LDS instructions execute in program
// order: a lane's read after another lane's write in the same wavefront sees
// the write.  Ordering them needs only a compiler-level fence at wavefront
// scope, which emits no s_barrier and no wait for outstanding memory
// operations (a workgroup barrier would also drain the loads that fetch the
// next row ahead of its use).
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

template <typename T>
__device__ __forceinline__ T lds_at(const T* row, uint32_t byte_offset)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + byte_offset);
}

// LDS of one wavefront.  NG is 9 where stage C reads the stored row again
// (exact final update), else 0.
template <typename T, int NG>
struct WaveLds {
    T xs[xs_rows(NG != 0)][kRowLds];  // one row of each moving population of a pass, for the xi stencils
    T hp[kRing][9][kWaveLanes];       // f-hat+ of rows t-4 .. t (lane-private); the slot of row ny keeps
                                      // f-bar of row ny-2 for the lid row of the half step
    T wb[2][9];                       // f-bar of columns 1 and nx-2 at the current half-step row
    T wc[2][9];                       // f-hat(t+dt) of columns 1 and nx-2 at the current full-step row
    T gr[NG ? kRing : 0][kGxRing][kWaveLanes];   // stored f-hat of populations 0 .. kGxRing - 1, rows t-4 .. t
    T gx[NG ? 9 - kGxRing : 0][kWaveLanes];      // stored f-hat of the other populations of the stage-C row,
                                                 // written by the buffer unit
};

// Compiler-level memory barrier: no memory operation is moved across it, and
// it emits no instruction.
__device__ __forceinline__ void mem_order() { asm volatile("" ::: "memory"); }

// Waits until at most N vector-memory operations of this wave are outstanding.
// The counter completes in issue order, so an operation followed by at least
// N others has then finished.
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
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

template <typename T, typename V>
__device__ __forceinline__ void half_step(const T (&fb)[9], V lam, V dt, T (&out)[9])
{
    T P, ux, uy, e[9];
    moments(fb, P, ux, uy);
    equilibrium(P, ux, uy, e);
    const T b = T(half_coef(lam, dt));
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = fb[k] + b * (e[k] - fb[k]);
}

// Eq. (2.19) sums of one node (the layout of kPartials); ref holds the
// cavity's shifts r_d, r_p.
template <typename T>
__device__ __forceinline__ void residual_add(const T (&gn)[9], const T (&old)[3], const double (&ref)[2],
                                             double (&acc)[kPartials])
{
    T P, ux, uy;
    moments(gn, P, ux, uy);
    const double du = (double)ux - (double)old[1], dv = (double)uy - (double)old[2], dp = (double)P - (double)old[0];
    const double sd = dp - ref[0], sp = (double)P - ref[1];
    acc[0] += du * du + dv * dv;
    acc[1] += (double)ux * ux + (double)uy * uy;
    acc[2] += dp * dp;
    acc[3] += (double)P * P;
    acc[4] += sd;
    acc[5] += sp;
    acc[6] += (isfinite((double)ux) && isfinite((double)uy) && isfinite((double)P)) ? 0.0 : 1.0;
    acc[7] += sd * sd;
    acc[8] += sp * sp;
}

// One work item.  Register ring slot of row t - d at unrolled phase R:
// (R + 5 - d) % 5 for f-bar+ and lambda (d = 0..4), (R + 10 - d) % 5 for
// f(t + dt/2) (d = 2..6); with one row per trip R is 0 and the rings move.
template <int PREC, bool RES, bool IMPL>
struct March {
    using S = Storage<PREC>;
    using T = typename S::T;
    using V = typename S::V;
    using F = typename S::F;
    using L = typename S::L;

    static constexpr int sg(int R, int d) { return (R + 2 * kRing - d) % kRing; }
    static constexpr int sf(int R, int d) { return (R + 3 * kRing - d) % kRing; }

    const StepArgs& a;
    const StripItem& it;
    const CavityDesc& c;
    WaveLds<T, S::kExactFinal ? 9 : 0>& sh;
    double (&acc)[kPartials];
    double ref[2];         // shifts of the residual sums (RES)

    int lane, nx, ny, i, ic, j0, j1, qlo, qhi, t_begin, t_last;
    bool out_col, walls_b, walls_c;
    PowerLaw<V> pl;
    V dtv;
    T ulid, sx_b, sy_b, sx_c, sy_c;
    T eps;
    // the row metric a_j, read-only while a step runs: through the constant address space a row's value
    // (uniform over the wave) comes by a scalar load, on the scalar counter, so that waiting for it does not
    // also wait for the vector loads of the next row in flight
    const __attribute__((address_space(4))) T* geo;
    XiLane<T> xl;
    __amdgpu_buffer_rsrc_t rf_in, rf_out, rl_in, rl_out;
    uint32_t fpb;          // bytes per distribution plane
    uint32_t skey, ckey;   // stochastic rounding keys
    int pitch;

    T gbp[kRing][9];       // f-bar+ (Eq. 2.16) of rows t-4 .. t
    T fh[kRing][9];        // f(t + dt/2) of rows t-6 .. t-2
    V lam[kRing];          // lambda of rows t-4 .. t
    // FP32SRF reads the metric a_j one row ahead into this ring (rows t-5 .. t-1, uniform): measured 1 % faster
    // there, with identical results; 0.5 % slower in FP32, and in FP64 it moves one FMA grouping (1-ulp changes),
    // so the other modes read a_j where they use it
    static constexpr bool kMetricRing = S::kExactFinal;
    T am[kRing];
    F gn_[9];              // f-hat of row t + 1, in flight
    L ln_;

    __device__ __forceinline__ March(const StepArgs& a_, const StripItem& it_, const CavityDesc& c_,
                                     WaveLds<T, S::kExactFinal ? 9 : 0>& sh_,
                                     double (&acc_)[kPartials])
        : a(a_), it(it_), c(c_), sh(sh_), acc(acc_), ref{0.0, 0.0}, pl(c_),
          xl(threadIdx.x, it_.i0 - kHaloCols + (int)threadIdx.x, c_.nx,
             geo_of<T>(a_)[c_.geo_off + c_.ny + min(max(it_.i0 - kHaloCols + (int)threadIdx.x, 0), c_.nx - 1)])
    {
        lane = threadIdx.x;
        nx = c.nx;
        ny = c.ny;
        pitch = c.pitch;
        i = it.i0 - kHaloCols + lane;
        // halo lanes outside the grid read the nearest column; their results are never used
        ic = min(max(i, 0), nx - 1);
        out_col = i >= it.i0 && i < it.i1;
        walls_b = it.i0 <= 2 || it.i1 >= nx - 2;
        walls_c = it.i0 == 0 || it.i1 == nx;
        j0 = it.j0;
        j1 = it.j1;
        qlo = max(j0 - 2, 0);
        qhi = min(j1 + 1, ny - 1);
        dtv = V(c.dt);
        const T dt = T(c.dt);
        ulid = T(c.u_lid);
        sy_b = T(0.5) * dt * T(c.inv2deta);
        sy_c = dt * T(c.inv2deta);
        sx_b = T(0.5) * dt * T(c.inv2dxi);
        sx_c = dt * T(c.inv2dxi);
        eps = T(c.mix);
        geo = (const __attribute__((address_space(4))) T*)(geo_of<T>(a) + c.geo_off);
        fpb = (uint32_t)c.plane * (uint32_t)sizeof(F);
        rf_in = buffer_of(static_cast<const F*>(a.f_in) + c.f_off, 9u * fpb);
        rf_out = buffer_of(static_cast<F*>(a.f_out) + c.f_off, 9u * fpb);
        rl_in = buffer_of(static_cast<const L*>(a.l_in) + c.l_off, (uint32_t)c.plane * (uint32_t)sizeof(L));
        rl_out = buffer_of(static_cast<L*>(a.l_out) + c.l_off, (uint32_t)c.plane * (uint32_t)sizeof(L));
        if (RES) {
            ref[0] = a.res_ref[2 * it.cav];
            ref[1] = a.res_ref[2 * it.cav + 1];
        }
        skey = S::kStochastic ? step_key(a.seed_ctr[0], a.step) : 0u;
        ckey = S::kStochastic ? cavity_key(it.cav) : 0u;
#pragma unroll
        for (int r = 0; r < kRing; ++r) {
            lam[r] = V(1);
#pragma unroll
            for (int k = 0; k < 9; ++k) gbp[r][k] = fh[r][k] = T(0);
        }
        t_begin = max(j0 - 4, 0);
        // rows up to ny - 1 are read; the lid row of the output is made with row ny - 2
        const int t_end = j1 == ny ? ny + 2 : j1 + 3;
        t_last = min(t_end, ny - 1);
        fetch(t_begin);
        march(t_begin, t_end);
    }

    // LDS ring slot of row r (a run-time index: the LDS ring is not moved when
    // the register rings are)
    __device__ __forceinline__ int hslot(int r) const { return (r - t_begin + 2 * kRing) % kRing; }

    __device__ __forceinline__ uint32_t foff(int row) const { return (uint32_t)(row * pitch + ic) * (uint32_t)sizeof(F); }
    __device__ __forceinline__ uint32_t loff(int row) const { return (uint32_t)(row * pitch + ic) * (uint32_t)sizeof(L); }

    __device__ __forceinline__ void fetch(int row)
    {
        const uint32_t vo = foff(row);
#pragma unroll
        for (int k = 0; k < 9; ++k) gn_[k] = Buf<F>::ld(rf_in, vo, (uint32_t)k * fpb);
        ln_ = Buf<L>::ld(rl_in, loff(row), 0u);
    }

    // Exact final update: populations kGxRing .. 8 of the stored f-hat of `row`
    // copied by the buffer unit straight into sh.gx, so that no registers are
    // held while they are in flight.  The compiler does not track these copies:
    // the reader waits on the vector-memory counter itself (wait_vm).
    __device__ __forceinline__ void reload_lds(int row)
    {
        static_assert(sizeof(F) == 4, "the LDS copy moves one dword per lane");
        const uint32_t vo = foff(row);
#pragma unroll
        for (int k = kGxRing; k < 9; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rf_in, (__attribute__((address_space(3))) void*)&sh.gx[k - kGxRing][0],
                                                    4u, vo, (uint32_t)k * fpb, 0, 0);
    }

    // old moments of row `row` (residual only)
    __device__ __forceinline__ void old_moments(int row, T (&m)[3]) const
    {
        const uint32_t vo = foff(row);
        T g[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] = S::cvt(Buf<F>::ld(rf_in, vo, (uint32_t)k * fpb), k);
        moments(g, m[0], m[1], m[2]);
    }

    template <typename X>
    __device__ __forceinline__ void store_row(int row, const X (&x)[9]) const
    {
        const uint32_t vo = foff(row);
        const NodeWords nw(skey, ckey, (uint32_t)(row * pitch + i));
#pragma unroll
        for (int k = 0; k < 9; ++k) Buf<F>::st(encode_state<S>(x[k], k, &nw), rf_out, vo, (uint32_t)k * fpb);
    }

    template <typename X>
    __device__ __forceinline__ void encode_row(int row, const X (&x)[9], F (&e)[9]) const
    {
        const NodeWords nw(skey, ckey, (uint32_t)(row * pitch + i));
#pragma unroll
        for (int k = 0; k < 9; ++k) e[k] = encode_state<S>(x[k], k, &nw);
    }

    // A store that every path of the row issues: lanes (or rows) with `on` false
    // take an offset past the end of the buffer, and the buffer unit drops such
    // stores.  The compiler's wait for the row fetched ahead then counts these
    // stores as issued after it instead of draining them.
    __device__ __forceinline__ void store_encoded(int row, const F (&e)[9], bool on) const
    {
        const uint32_t vo = on ? foff(row) : kDroppedOffset;
#pragma unroll
        for (int k = 0; k < 9; ++k) Buf<F>::st(e[k], rf_out, vo, (uint32_t)k * fpb);
    }

    // out[k] = base[k] - sx * a_j d_k * D_xi - sy * D_eta for the moving
    // populations of one row, where D are the signed mixed differences: xi
    // neighbours from the LDS row, eta neighbours from ring slots s[0..4]
    // (rows r-2 .. r+2).  mx carries sx * a_j, my carries sy.
    // elo / ehi: the row is 1 / ny - 2, where the eta difference of the
    // populations moving up / down falls back to first order.
    template <int S0, int S1, int S2, int S3, int S4>
    __device__ __forceinline__ void transport(const T (&ring)[kRing][9], const T (&base)[9], const MixedWeights<T>& mx,
                                              const MixedWeights<T>& my, bool elo, bool ehi, T (&out)[9])
    {
        auto& xs = sh.xs;
        out[0] = base[0];
        // the eight moving populations in passes of kXsRows through the exchange rows
        constexpr int kXsRows = xs_rows(S::kExactFinal);
        static_assert(8 % kXsRows == 0, "whole passes");
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            const int x = (k - 1) % kXsRows;
            if (x == 0) {
                if (k > 1) wave_sync();   // the previous pass has read the rows
                if constexpr (kDiffForm<T>) {
                    // the backward difference of each lane's value, its left neighbour's taken across the wavefront
#pragma unroll
                    for (int m = k; m < k + kXsRows; ++m)
                        xs[m - k][lane + kPad] = ring[S2][m] - lane_below(ring[S2][m]);
                } else {
#pragma unroll
                    for (int m = k; m < k + kXsRows; ++m) xs[m - k][lane + kPad] = ring[S2][m];
                }
                wave_sync();
            }
            const T* row = xs[x];
            const T c0 = ring[S2][k];
            constexpr uint32_t E = sizeof(T);
            if constexpr (kDiffForm<T>) {
                // xi term from the backward differences: near, far and other point of this population's upwind
                // side (XiLane), signed by d
                T n, f, o, w;
                bool minus;   // out = base - w t (d >= 0 member of a pair, k = 1) or base + w t
                if (k == 1 || k == 3) {
                    const bool pos = k == 1;
                    n = lds_at(row, pos ? xl.own : xl.own + E);
                    f = (pos ? xl.edge1 : xl.edge3) ? n : lds_at(row, pos ? xl.own - E : xl.own + 2 * E);
                    o = lds_at(row, pos ? xl.own + E : xl.own);
                    w = T(1);
                    minus = pos;
                } else {
                    const int pr = (k == 2 || k == 4) ? 0 : ((k == 5 || k == 7) ? 1 : 2);
                    const bool first = k == 2 || k == 5 || k == 6;
                    n = lds_at(row, first ? xl.a1[pr] : xl.f1[pr]);
                    f = lds_at(row, first ? xl.a2[pr] : xl.a2m[pr]);
                    o = lds_at(row, first ? xl.f1[pr] : xl.a1[pr]);
                    w = xl.ad[pr];
                    minus = first;
                }
                const T t = mx.apply_back(n, f, o);
                T r = minus ? base[k] - w * t : base[k] + w * t;
                // eta term: the backward differences along the upwind direction from the ring (the row below for
                // populations moving up, the row above for those moving down); at rows 1 and ny - 2 the far one is
                // the near one
                if (moves_up(k)) {
                    const T nb = c0 - ring[S1][k];
                    r = my.sub_back(r, nb, elo ? nb : ring[S1][k] - ring[S0][k], ring[S3][k] - c0);
                }
                if (moves_down(k)) {
                    const T nb = c0 - ring[S3][k];
                    r = my.sub_back(r, nb, ehi ? nb : ring[S3][k] - ring[S4][k], ring[S1][k] - c0);
                }
                out[k] = r;
                continue;
            }
            T a1, a2, f1, w;
            bool edge = false;
            if (k == 1 || k == 3) {
                const bool pos = k == 1;
                a1 = lds_at(row, pos ? xl.own - E : xl.own + E);
                a2 = lds_at(row, pos ? xl.own - 2 * E : xl.own + 2 * E);
                f1 = lds_at(row, pos ? xl.own + E : xl.own - E);
                w = T(1);
                edge = pos ? xl.edge1 : xl.edge3;
            } else {
                const int pr = (k == 2 || k == 4) ? 0 : ((k == 5 || k == 7) ? 1 : 2);
                const bool first = k == 2 || k == 5 || k == 6;
                a1 = lds_at(row, first ? xl.a1[pr] : xl.f1[pr]);
                a2 = lds_at(row, first ? xl.a2[pr] : xl.a2m[pr]);
                f1 = lds_at(row, first ? xl.f1[pr] : xl.a1[pr]);
                w = xl.ad[pr];
                edge = first ? xl.edge_p[pr] : xl.edge_m[pr];
            }
            a2 = edge ? T(2) * a1 - c0 : a2;
            T o = base[k] - w * mx.apply(a2, a1, c0, f1);
            if (moves_up(k)) o = o - my.apply(ring[S0][k], ring[S1][k], c0, ring[S3][k]);
            if (moves_down(k)) o = o - my.apply(ring[S4][k], ring[S3][k], c0, ring[S1][k]);
            out[k] = o;
        }
        wave_sync();
    }

    // Rows outside [1, ny-2] of a ring take the linear extrapolation 2 a1 - c0,
    // which turns the second-order one-sided difference into the first-order
    // one (the eta counterpart of the wall columns of XiLane).
    template <int S0, int S1, int S2, int S3, int S4>
    __device__ __forceinline__ void eta_ghosts(T (&ring)[kRing][9], bool lo, bool hi)
    {
        if (lo) {
#pragma unroll
            for (int k = 1; k < 9; ++k)
                if (moves_up(k)) ring[S0][k] = T(2) * ring[S1][k] - ring[S2][k];
        }
        if (hi) {
#pragma unroll
            for (int k = 1; k < 9; ++k)
                if (moves_down(k)) ring[S4][k] = T(2) * ring[S3][k] - ring[S2][k];
        }
    }

    template <int R>
    __device__ __forceinline__ void row(int t)
    {
        const int p = t - 4;
        const bool do_c = p >= j0 && p < j1 && p >= 1 && p <= ny - 2;
        // exact final update: the copies of row p go to LDS first, ahead of the fetch of row t + 1, so that
        // stage C's wait for them leaves that fetch in flight
        const bool fetch_next = t <= ny - 1 && t + 1 <= t_last;

        // ------------------------------------------------------------ A: row t
        if (t <= ny - 1) {
            const int hs = hslot(t);
            T g[9], e[9], d[9], P, ux, uy;
#pragma unroll
            for (int k = 0; k < 9; ++k) g[k] = S::cvt(gn_[k], k);
            const V lam_old = V(ln_);
            if constexpr (S::kExactFinal) {
                // the fetched row is waited for here, before the LDS copy is issued, so that the wait does not
                // cover the copy as well
#pragma unroll
                for (int k = 0; k < 9; ++k) asm volatile("" ::"v"(g[k]));
                asm volatile("" ::"v"(lam_old));
                mem_order();
                if (do_c) reload_lds(p);
                mem_order();
            }
            if (fetch_next) fetch(t + 1);   // consumed by the next row (ten vector-memory loads)
            V l;
            if constexpr (S::kExactFinal) {
                // e - g in FP64 from the exact stored g: at low shear the non-equilibrium part is far below
                // an FP32 ulp of g, and Step (2) raises it to the power (n - 1) / 2
                double gd[9], dd[9], Pd, uxd, uyd;
#pragma unroll
                for (int k = 0; k < 9; ++k) gd[k] = (double)g[k];
                moments(gd, Pd, uxd, uyd);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    dd[k] = equilibrium_k(Pd, uxd, uyd, k) - gd[k];
                    d[k] = T(dd[k]);
                }
                // the second moments of Step (2) from the FP32 values of e - g: their sums need FP32 accuracy
                // only, as the power law and the relaxation coefficients are FP32 in this mode
                l = relaxation_time_d<IMPL>(d, lam_old, pl);
            } else {
                moments(g, P, ux, uy);
                equilibrium(P, ux, uy, e);
#pragma unroll
                for (int k = 0; k < 9; ++k) d[k] = e[k] - g[k];
                l = relaxation_time_d<IMPL>(d, lam_old, pl);
            }
            const Relax<V> rx(l, dtv);
            const T b_hat = T(rx.b_hat), b_bar = T(rx.b_bar);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                gbp[sg(R, 0)][k] = g[k] + b_bar * d[k];
                // exact final update: only the collision increment of f-hat+ (Eq. 2.15); the stored g is added
                // in FP64 at stage C
                sh.hp[hs][k][lane] = S::kExactFinal ? b_hat * d[k] : g[k] + b_hat * d[k];
                if constexpr (S::kExactFinal) {
                    if (k < kGxRing) sh.gr[hs][k][lane] = g[k];
                }
            }
            lam[sg(R, 0)] = l;
            Buf<L>::st(L(l), rl_out, out_col && t >= j0 && t < j1 ? loff(t) : kDroppedOffset, 0u);
        } else if constexpr (S::kExactFinal) {
            mem_order();
            if (do_c) reload_lds(p);
            mem_order();
        }

        // ------------------------------------------------------------ B: row t - 2
        const int q = t - 2;
        if (q >= qlo && q <= qhi) {
            T fb[9];
            if (q >= 1 && q <= ny - 2) {
                eta_ghosts<sg(R, 4), sg(R, 3), sg(R, 2), sg(R, 1), sg(R, 0)>(gbp, q == 1, q == ny - 2);
                const MixedWeights<T> mx(eps, sx_b * (kMetricRing ? am[sg(R, 1)] : geo[q])), my(eps, sy_b);
                transport<sg(R, 4), sg(R, 3), sg(R, 2), sg(R, 1), sg(R, 0)>(gbp, gbp[sg(R, 2)], mx, my, q == 1, q == ny - 2, fb);
                if (walls_b) {
                    publish(sh.wb, i, nx, fb);
                    wave_sync();
                    if (i == 0 || i == nx - 1) {
                        T src[9];
                        wall_source(sh.wb, i, nx, fb, src);
                        extrapolate(src, T(0), fb);
                    }
                }
                if (q == 1) {   // bottom wall row (row t - 3) from row 1 (Eq. 1.5: at rest)
                    T src[9], fb0[9], out0[9];
                    wall_source(sh.wb, i, nx, fb, src);
                    extrapolate(src, T(0), fb0);
                    half_step(fb0, lam[sg(R, 3)], dtv, out0);
#pragma unroll
                    for (int k = 0; k < 9; ++k) fh[sf(R, 3)][k] = out0[k];
                }
                if (q == ny - 2) {   // source of the lid row, kept in the free f-hat+ slot of row t = ny
                    const int hs = hslot(t);
#pragma unroll
                    for (int k = 0; k < 9; ++k) sh.hp[hs][k][lane] = fb[k];
                }
            } else if (q == ny - 1) {   // lid row from row ny - 2 (kept one row ago)
                T own[9], src[9];
                const int hs = hslot(t - 1);
#pragma unroll
                for (int k = 0; k < 9; ++k) own[k] = sh.hp[hs][k][lane];
                wall_source(sh.wb, i, nx, own, src);
                extrapolate(src, ulid, fb);
            }
            if (q >= 1) {
                T out[9];
                half_step(fb, lam[sg(R, 2)], dtv, out);
#pragma unroll
                for (int k = 0; k < 9; ++k) fh[sf(R, 2)][k] = out[k];
            }
        }

        // ------------------------------------------------------------ C: row t - 4
        F enc[9];   // the encoded row p, stored after the branch
        if (do_c) {
            T hp[9], gn[9];
            double fin[S::kExactFinal ? 9 : 1];   // exact final update (FP32SRF): the FP64 sum of each population
            eta_ghosts<sf(R, 6), sf(R, 5), sf(R, 4), sf(R, 3), sf(R, 2)>(fh, p == 1, p == ny - 2);
            const MixedWeights<T> mx(eps, sx_c * (kMetricRing ? am[sg(R, 3)] : geo[p])), my(eps, sy_c);
            if constexpr (S::kExactFinal) {
                // f-hat(t + dt) = g + (collision increment + streaming increment): the two increments in FP32
                // (each accurate relative to itself), their sum added to the stored g in FP64
                const int hs = hslot(p);
#pragma unroll
                for (int k = 0; k < 9; ++k) hp[k] = sh.hp[hs][k][lane];
                transport<sf(R, 6), sf(R, 5), sf(R, 4), sf(R, 3), sf(R, 2)>(fh, hp, mx, my, p == 1, p == ny - 2, gn);
                if (fetch_next)
                    wait_vm<10>();   // the LDS copies of row p were followed by the ten loads of row t + 1
                else
                    wait_vm<0>();
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const T g = k < kGxRing ? sh.gr[hs][k][lane] : sh.gx[k - kGxRing][lane];
                    fin[k] = (double)S::cvt(g, k) + (double)gn[k];
                }
                if (RES || walls_c || (p == 1 && j0 == 0) || (p == ny - 2 && j1 == ny)) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) gn[k] = T(fin[k]);
                }
            } else {
                const int hs = hslot(p);
#pragma unroll
                for (int k = 0; k < 9; ++k) hp[k] = sh.hp[hs][k][lane];
                transport<sf(R, 6), sf(R, 5), sf(R, 4), sf(R, 3), sf(R, 2)>(fh, hp, mx, my, p == 1, p == ny - 2, gn);
            }
            const bool wall_lane = i == 0 || i == nx - 1;
            if (walls_c) {
                publish(sh.wc, i, nx, gn);
                wave_sync();
                if (wall_lane) {
                    T src[9];
                    wall_source(sh.wc, i, nx, gn, src);
                    extrapolate(src, T(0), gn);
                    if constexpr (S::kExactFinal) {
#pragma unroll
                        for (int k = 0; k < 9; ++k) fin[k] = (double)gn[k];   // the wall value replaces the sum
                    }
                }
            }
            // (a lane at column 0 or nx - 1 of a wave without walls_c is a halo lane: nothing of it is stored)
            if constexpr (S::kExactFinal)
                encode_row(p, fin, enc);
            else
                encode_row(p, gn, enc);
            if (RES && out_col) {
                T old[3];
                old_moments(p, old);
                residual_add(gn, old, ref, acc);
            }
            if (p == 1 && j0 == 0) {   // bottom wall row from row 1
                T src[9], g0[9];
                wall_source(sh.wc, i, nx, gn, src);
                extrapolate(src, T(0), g0);
                if (out_col) {
                    store_row(0, g0);
                    if (RES) {
                        T old[3];
                        old_moments(0, old);
                        residual_add(g0, old, ref, acc);
                    }
                }
            }
            if (p == ny - 2 && j1 == ny) {   // lid row from row ny - 2
                T src[9], gl[9];
                wall_source(sh.wc, i, nx, gn, src);
                extrapolate(src, ulid, gl);
                if (out_col) {
                    store_row(ny - 1, gl);
                    if (RES) {
                        T old[3];
                        old_moments(ny - 1, old);
                        residual_add(gl, old, ref, acc);
                    }
                }
            }
        }
        store_encoded(p, enc, do_c && out_col);
        // a_j of row t - 1, for stage B of the next row and stage C three rows on.  Scalar loads share a counter
        // with the LDS operations and may return out of order, so the first LDS wait after one waits for it too:
        // issued after the last LDS wait of the row, it has the next row's stage A (no LDS reads) to arrive.
        if constexpr (kMetricRing) am[sg(R, 0)] = geo[min(max(t - 1, 0), ny - 1)];
    }

    // Rows are unrolled over a full turn of the rings, so that slots are renamed, not moved.
    __device__ __forceinline__ void march(int t_begin, int t_end)
    {
#pragma unroll 1
        for (int t = t_begin;; t += kRing) {
            row<0>(t);
            if (t + 1 > t_end) break;
            row<1>(t + 1);
            if (t + 2 > t_end) break;
            row<2>(t + 2);
            if (t + 3 > t_end) break;
            row<3>(t + 3);
            if (t + 4 > t_end) break;
            row<4>(t + 4);
            if (t + 5 > t_end) break;
        }
    }
};

template <int PREC, bool RES, bool IMPL>
__global__ __launch_bounds__(kWaveLanes, Tuning<PREC>::kWaves) void k_fused(StepArgs a, const StripItem* items, int w0, int nw)
{
    const int w = w0 + (int)blockIdx.x;
    const StripItem it = items[w];
    if (it.unit < 0) return;   // padding of a per-XCD queue
    const CavityDesc c = a.desc[it.cav];
    __shared__ WaveLds<typename Storage<PREC>::T, Storage<PREC>::kExactFinal ? 9 : 0> sh;
    double acc[kPartials];
#pragma unroll
    for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
    March<PREC, RES, IMPL>(a, it, c, sh, acc);
    if (RES) {
        // wavefront sum in a fixed order
#pragma unroll
        for (int q5 = 0; q5 < kPartials; ++q5) {
            double v = acc[q5];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWaveLanes);
            if (threadIdx.x == 0) a.partial[(int64_t)it.unit * kPartials + q5] = v;
        }
    }
}

template <int PREC, bool IMPL>
hipError_t fused(const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    if (nw <= 0) return hipSuccess;
    if (residual)
        hipLaunchKernelGGL((k_fused<PREC, true, IMPL>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0, nw);
    else
        hipLaunchKernelGGL((k_fused<PREC, false, IMPL>), dim3(nw), dim3(kWaveLanes), 0, s, a, items, w0, nw);
    return hipGetLastError();
}

template <bool IMPL>
hipError_t fused_prec(int prec, const StepArgs& a, const StripItem* items, int w0, int nw, bool residual, hipStream_t s)
{
    switch (prec) {
    case P_FP64: return fused<P_FP64, IMPL>(a, items, w0, nw, residual, s);
    case P_FP32: return fused<P_FP32, IMPL>(a, items, w0, nw, residual, s);
    case P_FP16DEV: return fused<P_FP16DEV, IMPL>(a, items, w0, nw, residual, s);
    case P_FP32X: return fused<P_FP32X, IMPL>(a, items, w0, nw, residual, s);
    case P_FP32SR: return fused<P_FP32SR, IMPL>(a, items, w0, nw, residual, s);
    case P_FP32SRF: return fused<P_FP32SRF, IMPL>(a, items, w0, nw, residual, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// implicit_lambda is a handle option: every cavity of a launch has the same flag
hipError_t launch_fused_step(int prec, bool implicit_lambda, const StepArgs& a, const StripItem* items, int w0, int nw,
                             bool residual, hipStream_t s)
{
    return implicit_lambda ? fused_prec<true>(prec, a, items, w0, nw, residual, s)
                           : fused_prec<false>(prec, a, items, w0, nw, residual, s);
}

}  // namespace ifd
