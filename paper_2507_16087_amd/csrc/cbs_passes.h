// Device-side building blocks of the FFT passes (header of the per-size
// pass translation units): complex helpers, compile-time twiddles, in-register
// DFTs, Stockham stages through LDS, the three pass kernels and their launch
// helper.  See cbs_kernels.hip for the iteration these passes make up.
#pragma once
#include "cbs_internal.h"

#include <algorithm>
#include <utility>

namespace cbs {

// ---------------------------------------------------------------- complex --
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {   // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> rmul(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.im, a.re}; }   // i a
// 1 / a with the hardware reciprocal (1 ulp) in FP32, exact division in FP64.
template <typename T>
__device__ __forceinline__ cx<T> cinv_fast(cx<T> a) {
    const T n = a.re * a.re + a.im * a.im;
    T d;
    if constexpr (sizeof(T) == 4) d = __builtin_amdgcn_rcpf(n);
    else d = T(1) / n;
    return {a.re * d, -a.im * d};
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------- global memory --
// The solver's device pointers reach the kernels through the slot descriptor,
// so the compiler cannot tell them from LDS or scratch and would use flat
// memory instructions; flat accesses count against the LDS wait counter too,
// so every LDS exchange of an FFT would also wait for all loads and stores in
// flight.  The hot passes view their arrays through global-address-space
// pointers instead.
// (The host pass of the compiler parses these kernels too but emits no code
// for them; there the qualifier is left out.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#else
#define GLOBAL
#endif
template <typename T>
__device__ __forceinline__ GLOBAL T* gmem(T* p) {
    return (GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const GLOBAL T* gmem(const T* p) {
    return (const GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ T ldg(const GLOBAL T* p) {
    return *p;
}
// Non-temporal loads and stores for the streams the last-axis passes touch
// once per iteration (x, y and the medium read, x written): marked so, they
// leave more of the caches to the FFT work array w, which the next passes
// read again.
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const GLOBAL cx<T>* p) {
    using V = T __attribute__((ext_vector_type(2)));
    const V v = __builtin_nontemporal_load((const GLOBAL V*)p);
    return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_nt(GLOBAL cx<T>* p, cx<T> a) {
    using V = T __attribute__((ext_vector_type(2)));
    V v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, (GLOBAL V*)p);
}
__device__ __forceinline__ float ld_nt(const GLOBAL float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ld_nt(const GLOBAL double* p) { return __builtin_nontemporal_load(p); }

// ------------------------------------------------ compile-time twiddles --
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int i = 1; i < 24; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 24; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
constexpr double red_angle(int m, int R) {
    double a = 2.0 * kPi * (double)m / (double)R;
    return a > kPi ? a - 2.0 * kPi : a;
}

template <int... I, typename F>
__device__ __forceinline__ void sfor_(std::integer_sequence<int, I...>, F&& f) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_(std::make_integer_sequence<int, N>{}, static_cast<F&&>(f));
}

// v * exp(DIR 2 pi i M / R), exact for multiples of a quarter turn
template <int M, int R, int DIR, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> v) {
    constexpr int m = ((M % R) + R) % R;
    if constexpr (m == 0) {
        return v;
    } else if constexpr ((4 * m) % R == 0) {
        constexpr int q = (4 * m) / R;
        if constexpr (q == 2) return {-v.re, -v.im};
        else if constexpr ((q == 1) == (DIR > 0)) return {-v.im, v.re};
        else return {v.im, -v.re};
    } else {
        constexpr T c = (T)taylor_cos(red_angle(m, R));
        constexpr T s = (T)(DIR * taylor_sin(red_angle(m, R)));
        return {v.re * c - v.im * s, v.re * s + v.im * c};
    }
}

// ---------------------------------------------------- in-register DFTs --
// X_k = sum_n x_n exp(DIR 2 pi i n k / R), in place, natural order.
template <int R, int DIR>
struct Dft {
    static constexpr int R1 = (R % 4 == 0) ? 4 : ((R % 3 == 0) ? 3 : 2);
    static constexpr int R2 = R / R1;
    template <typename T>
    __device__ __forceinline__ static void run(cx<T>* v) {
        // R = R1 * R2: R2 DFTs of length R1 over n1 (stride R2), twiddle,
        // R1 DFTs of length R2 over n2; output index k1 + R1 k2.
        cx<T> t[R];
        sfor<R2>([&](auto N2) {
            constexpr int n2 = decltype(N2)::value;
            cx<T> a[R1];
            sfor<R1>([&](auto N1) { a[decltype(N1)::value] = v[n2 + R2 * decltype(N1)::value]; });
            Dft<R1, DIR>::run(a);
            sfor<R1>([&](auto K1) {
                constexpr int k1 = decltype(K1)::value;
                t[n2 * R1 + k1] = twc<n2 * k1, R, DIR>(a[k1]);
            });
        });
        sfor<R1>([&](auto K1) {
            constexpr int k1 = decltype(K1)::value;
            cx<T> b[R2];
            sfor<R2>([&](auto N2) { b[decltype(N2)::value] = t[decltype(N2)::value * R1 + k1]; });
            Dft<R2, DIR>::run(b);
            sfor<R2>([&](auto K2) { v[k1 + R1 * decltype(K2)::value] = b[decltype(K2)::value]; });
        });
    }
};
template <int DIR>
struct Dft<1, DIR> {
    template <typename T>
    __device__ __forceinline__ static void run(cx<T>*) {}
};
template <int DIR>
struct Dft<2, DIR> {
    template <typename T>
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a = v[0];
        v[0] = a + v[1];
        v[1] = a - v[1];
    }
};
template <int DIR>
struct Dft<3, DIR> {
    template <typename T>
    __device__ __forceinline__ static void run(cx<T>* v) {
        constexpr T h = (T)0.5;
        constexpr T s = (T)(DIR * 0.86602540378443864676372317075293618);
        cx<T> t = v[1] + v[2];
        cx<T> m = {v[0].re - h * t.re, v[0].im - h * t.im};
        cx<T> d = v[1] - v[2];
        cx<T> e = {-s * d.im, s * d.re};   // i s (v1 - v2)
        v[0] = v[0] + t;
        v[1] = m + e;
        v[2] = m - e;
    }
};
template <int DIR>
struct Dft<4, DIR> {
    template <typename T>
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
        cx<T> e = (DIR > 0) ? cx<T>{-d.im, d.re} : cx<T>{d.im, -d.re};   // DIR i d
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + e;
        v[3] = b - e;
    }
};

// ------------------------------------------------------------- FFT plans --
// N = R0 R1 R2 points; TPC threads cooperate on one column, each owning
// E = N / TPC elements (N / (R TPC) butterflies of every stage).
template <int N_, int R0_, int R1_, int R2_, int TPC_>
struct Plan {
    static constexpr int N = N_, R0 = R0_, R1 = R1_, R2 = R2_, TPC = TPC_;
    static constexpr int S = (R2 > 1) ? 3 : ((R1 > 1) ? 2 : 1);
    static constexpr int E = N / TPC;
    static_assert(R0 * R1 * R2 == N, "radices must multiply to N");
    static constexpr int radix(int s) { return s == 0 ? R0 : (s == 1 ? R1 : R2); }
};

// Stage s in execution order: forward runs R0, R1, R2; inverse runs them
// reversed so it can start from the forward transform's last-stage registers.
template <class P, int DIR>
struct Seq {
    static constexpr int r(int s) { return DIR < 0 ? P::radix(s) : P::radix(P::S - 1 - s); }
    static constexpr int ns(int s) {
        int a = 1;
        for (int i = 0; i < s; ++i) a *= r(i);
        return a;
    }
};

// LDS tile layouts.  COLS (column-fastest threads): element n of column c at
// lds[n * ldp + c], so a wave's columns hit consecutive words.  ROWS
// (lane-fastest threads): lds[c * ldp + n + n / 16], the pad word every 16
// elements keeping the stride-R Stockham scatters off a single bank.
enum Lay { COLS = 0, ROWS = 1 };
template <int LAY>
__device__ __forceinline__ int lidx(int n, int col, int ldp) {
    if constexpr (LAY == COLS) return n * ldp + col;
    else return col * ldp + n + (n >> 4);
}
template <int LAY>
constexpr int lds_pitch(int n, int pcols) {
    return LAY == COLS ? pcols + 1 : n + n / 16;
}

template <int N, int R, int TPC, int LAY, typename T>
__device__ __forceinline__ void lds_gather(cx<T>* v, const cx<T>* lds, int ldp, int col, int lane) {
    constexpr int NB = N / (R * TPC);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = lds[lidx<LAY>(lane + b * TPC + r * (N / R), col, ldp)];
}

template <int N, int R, int Ns, int TPC, int LAY, typename T>
__device__ __forceinline__ void lds_scatter(const cx<T>* v, cx<T>* lds, int ldp, int col, int lane) {
    constexpr int NB = N / (R * TPC);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = lane + b * TPC;
        const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx<LAY>(base + r * Ns, col, ldp)] = v[b * R + r];
    }
}

// Twiddle (stages after the first) and radix-R DFT on this thread's butterflies.
template <int N, int R, int Ns, int TPC, int DIR, typename T>
__device__ __forceinline__ void stage_compute(cx<T>* v, int lane, const cx<T>* __restrict__ tw) {
    constexpr int NB = N / (R * TPC);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (Ns > 1) {
            const int jm = (lane + b * TPC) % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[jm * r * (N / (Ns * R))];
                v[b * R + r] = (DIR < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
            }
        }
        Dft<R, DIR>::run(&v[b * R]);
    }
}

// Full transform of one column.  On entry v holds the first stage's inputs
// (elements lane + b TPC + r N/R); on exit v holds the outputs of the last
// stage, element lane + b TPC + r N/R_last in natural order.  The LDS tile
// must be free on entry; it is still being read on exit.
template <class P, int DIR, int LAY = COLS, typename T>
__device__ __forceinline__ void fft_regs(cx<T>* v, cx<T>* lds, int ldp, int col, int lane,
                                         const cx<T>* __restrict__ tw) {
    using Q = Seq<P, DIR>;
    constexpr int N = P::N, TPC = P::TPC;
    stage_compute<N, Q::r(0), 1, TPC, DIR>(v, lane, tw);
    if constexpr (P::S >= 2) {
        lds_scatter<N, Q::r(0), 1, TPC, LAY>(v, lds, ldp, col, lane);
        __syncthreads();
        lds_gather<N, Q::r(1), TPC, LAY>(v, lds, ldp, col, lane);
        stage_compute<N, Q::r(1), Q::ns(1), TPC, DIR>(v, lane, tw);
    }
    if constexpr (P::S >= 3) {
        __syncthreads();
        lds_scatter<N, Q::r(1), Q::ns(1), TPC, LAY>(v, lds, ldp, col, lane);
        __syncthreads();
        lds_gather<N, Q::r(2), TPC, LAY>(v, lds, ldp, col, lane);
        stage_compute<N, Q::r(2), Q::ns(2), TPC, DIR>(v, lane, tw);
    }
}

// The same transform on the first F of NF register arrays at once, each with
// its own LDS region (field_elems elements apart): one barrier per stage
// exchange covers every field.
template <class P, int DIR, int NF, typename T>
__device__ __forceinline__ void fft_regs_multi(cx<T> (*v)[P::E], int F, cx<T>* lds, int field_elems, int ldp,
                                               int col, int lane, const cx<T>* __restrict__ tw) {
    using Q = Seq<P, DIR>;
    constexpr int N = P::N, TPC = P::TPC;
#pragma unroll
    for (int f = 0; f < NF; ++f)
        if (f < F) stage_compute<N, Q::r(0), 1, TPC, DIR>(v[f], lane, tw);
    if constexpr (P::S >= 2) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < F) lds_scatter<N, Q::r(0), 1, TPC, COLS>(v[f], lds + f * field_elems, ldp, col, lane);
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < F) {
                lds_gather<N, Q::r(1), TPC, COLS>(v[f], lds + f * field_elems, ldp, col, lane);
                stage_compute<N, Q::r(1), Q::ns(1), TPC, DIR>(v[f], lane, tw);
            }
    }
    if constexpr (P::S >= 3) {
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < F) lds_scatter<N, Q::r(1), Q::ns(1), TPC, COLS>(v[f], lds + f * field_elems, ldp, col, lane);
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < F) {
                lds_gather<N, Q::r(2), TPC, COLS>(v[f], lds + f * field_elems, ldp, col, lane);
                stage_compute<N, Q::r(2), Q::ns(2), TPC, DIR>(v[f], lane, tw);
            }
    }
}

// Index of element (lane, b, r) of the last stage in natural order.
template <class P, int DIR>
__device__ __forceinline__ int out_index(int lane, int b, int r) {
    constexpr int Rl = Seq<P, DIR>::r(P::S - 1);
    return lane + b * P::TPC + r * (P::N / Rl);
}
template <class P, int DIR>
__device__ __forceinline__ int in_index(int lane, int b, int r) {
    constexpr int R0 = Seq<P, DIR>::r(0);
    return lane + b * P::TPC + r * (P::N / R0);
}

// Per-work-group copies of the small per-axis tables (FFT twiddles, layer
// profile, wavenumbers) live in LDS after the tile, so the FFT stages and the
// fused prologue / epilogue read them without touching the vector memory path.
template <typename T>
__host__ __device__ __forceinline__ size_t tile_bytes(size_t elems) {
    return (elems * sizeof(cx<T>) + 15) & ~size_t(15);
}
// ---------------------------------------------------------- pass modes --
enum Mode { CBS = 0, APPLY = 1 };

// Block reduction of two doubles; thread 0 gets the totals.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        red[2 * wid] = a;
        red[2 * wid + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) {
            a += red[2 * i];
            b += red[2 * i + 1];
        }
    }
}

// Final step of a norm reduction: the slot's control block from the two
// totals.  CBS: advance the iteration counter, relative update
// |dx| / |x_k| (not tested while x_k = 0, the first iteration), done on
// tolerance, cap, non-finite values or three consecutive updates above twice
// the iterate.  APPLY: |r|^2, |y|^2 and |r| for the refinement kernels.
// --------------------------------- passes A / E: last (contiguous) axis --
// One work-group owns P whole pencils of one field; TPC lane-fastest threads
// per pencil, so each stage-0 load and last-stage store of a pencil is one
// contiguous run.  grid = (pencils / P, F, slots).
//   KIND FIRST : prologue (CBS: w = B x + y; APPLY: w = x) -> forward FFT -> w
//   KIND LAST  : w -> inverse FFT -> epilogue (CBS: x += nu B (z - x) with
//                |dx|^2, |x|^2 partials; APPLY: w = y - D x / lam - z with
//                |r|^2, |y|^2 partials)
//   KIND FUSED : LAST's CBS epilogue, then the next iteration's prologue on
//                the same registers, forward FFT -> w.  The inverse transform
//                (radices reversed) leaves each thread holding exactly the
//                elements the forward transform's first stage needs.
enum Kind { FIRST = 0, LAST = 1, FUSED = 2 };

//   PF (LAST / FUSED): 0 loads x, y and the medium after the inverse
//   transform; 1 issues all three right after the w loads, so they travel
//   while the transform runs; 2 prefetches x and the medium only.
//   YS: sparse right-hand side -- velocity rows of y are zero and the
//   pressure row is read only on the pencils s.ypen flags.
template <class P, int MODE, int KIND, int PF, bool YS, typename T>
__global__ void __launch_bounds__(256) k_lastaxis(const Slot<T>* __restrict__ slots, Geom g, int pcols) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Slot<T>& s = slots[blockIdx.z];
    if (MODE == CBS && s.ctl->done) return;
    constexpr int N = P::N, E = P::E, TPC = P::TPC;
    constexpr int ldp = lds_pitch<ROWS>(N, 0);
    const int f = blockIdx.y;
    const int D = g.ndim, last = D - 1;
    const int tid = threadIdx.x;
    const int lane = tid % TPC, col = tid / TPC;
    const int pencil = blockIdx.x * pcols + col;
    // uniform tile bases; per-thread 32-bit offsets (pl + n) inside the tile
    const int64_t tile0 = (int64_t)blockIdx.x * pcols * N;
    const int64_t fbase = (int64_t)f * g.ncell + tile0;
    const uint32_t pl = (uint32_t)(col * N);
    // LDS: tile | twiddles (N) | layer profile of the last axis (N)
    // (the tile also hosts the 64-double block reduction, hence the floor)
    const size_t tab_off = max(tile_bytes<T>((size_t)pcols * ldp), (size_t)(64 * sizeof(double)));
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(smem_raw + tab_off);
    T* prof_l = reinterpret_cast<T*>(tw_l + N);
    {
        const GLOBAL T* __restrict__ src = gmem((f == last) ? s.gs[last] : s.gc[last]);
        const GLOBAL cx<T>* __restrict__ twg = gmem(s.tw[last]);
        for (int i = tid; i < N; i += blockDim.x) {
            tw_l[i] = twg[i];
            prof_l[i] = src[i];
        }
    }
    __syncthreads();
    const cx<T>* tw = tw_l;
    GLOBAL cx<T>* __restrict__ w = gmem(s.w) + fbase;
    GLOBAL cx<T>* __restrict__ x = gmem(s.x) + fbase;
    const GLOBAL cx<T>* __restrict__ y = gmem(s.y) + fbase;
    // this pencil's right-hand side is all zero (sparse y: a velocity row, or
    // a pressure pencil without a source cell)
    bool yzero = false;
    if constexpr (YS) yzero = f < g.ndim || !s.ypen[blockIdx.x * pcols + tid / P::TPC];
    auto yload = [&](int n) -> cx<T> {
        if constexpr (YS) {
            if (yzero) return cx<T>{T(0), T(0)};
        }
        return ld_nt(y + pl + n);
    };

    // per-pencil part of the layer rate for this field's row
    int ix[3];
    if (D == 3) {
        ix[1] = pencil % g.n[1];
        ix[0] = pencil / g.n[1];
    } else {
        ix[0] = pencil;
    }
    T colsum = 0;
    for (int d = 0; d < last; ++d) colsum += gmem((d == f) ? s.gs[d] : s.gc[d])[ix[d]];
    const T* lastprof = prof_l;
    const bool urow = f < D;
    const GLOBAL T* __restrict__ rb = gmem(s.rhobar) + (urow ? fbase : 0) + pl;
    const GLOBAL cx<T>* __restrict__ qv = gmem(s.q) + tile0 + pl;
    const T are = urow ? s.a1re : s.a2re;
    const T aim = s.adjoint ? -(urow ? s.a1im : s.a2im) : (urow ? s.a1im : s.a2im);
    const T il = urow ? s.inv_lam1 : s.inv_lam2;
    const T wim = s.adjoint ? -s.omega : s.omega;
    // medium value at element n: rhobar (real part) on velocity rows, q on
    // the pressure row
    auto medium = [&](int n) -> cx<T> {
        if (urow) return {ld_nt(rb + n), T(0)};
        return ld_nt(qv + n);
    };
    // diagonal D (conjugated for the adjoint) at element n from its medium value
    auto diag_m = [&](int n, cx<T> m) -> cx<T> {
        const T gam = s.gmax * (colsum + lastprof[n]);
        if (urow) return {m.re * gam, m.re * wim};
        const cx<T> dd = {gam * m.re - s.omega * m.im, gam * m.im + s.omega * m.re};
        return {dd.re, s.adjoint ? -dd.im : dd.im};
    };
    auto diag = [&](int n) -> cx<T> { return diag_m(n, medium(n)); };

    cx<T> v[E];
    using QF = Seq<P, -1>;
    using QI = Seq<P, 1>;
    if constexpr (KIND == FIRST) {
        constexpr int R0 = QF::r(0);
#pragma unroll
        for (int b = 0; b < N / (R0 * TPC); ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int n = in_index<P, -1>(lane, b, r);
                const cx<T> xv = ld_nt(x + pl + n);
                if constexpr (MODE == CBS) {
                    const cx<T> dd = diag(n);
                    const cx<T> bb = {T(1) - (dd.re - are) * il, -(dd.im - aim) * il};
                    v[b * R0 + r] = cmul(bb, xv) + yload(n);
                } else {
                    v[b * R0 + r] = xv;
                }
            }
    } else {
        constexpr int R0 = QI::r(0);
#pragma unroll
        for (int b = 0; b < N / (R0 * TPC); ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) v[b * R0 + r] = w[pl + in_index<P, 1>(lane, b, r)];
        constexpr int RL = QI::r(P::S - 1);   // == forward R0
        constexpr int EP = PF ? E : 1, EY = PF == 1 ? E : 1;
        cx<T> xp[EP], mp[EP], yp[EY];
        if constexpr (PF != 0) {
#pragma unroll
            for (int b = 0; b < N / (RL * TPC); ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int n = out_index<P, 1>(lane, b, r);
                    xp[b * RL + r] = ld_nt(x + pl + n);
                    mp[b * RL + r] = medium(n);
                    if constexpr (PF == 1) yp[b * RL + r] = yload(n);
                }
        }
        fft_regs<P, 1, ROWS>(v, lds, ldp, col, lane, tw);
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int b = 0; b < N / (RL * TPC); ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int n = out_index<P, 1>(lane, b, r);
                const int e = b * RL + r;
                const cx<T> z = v[e];
                const cx<T> xv = PF ? xp[PF ? e : 0] : ld_nt(x + pl + n);
                const cx<T> dd = PF ? diag_m(n, mp[PF ? e : 0]) : diag(n);
                if constexpr (MODE == CBS) {
                    const cx<T> bb = {T(1) - (dd.re - are) * il, -(dd.im - aim) * il};
                    const cx<T> dxv = rmul(s.nu, cmul(bb, z - xv));
                    const cx<T> xn = xv + dxv;
                    st_nt(x + pl + n, xn);
                    acc0 += (double)norm2(dxv);
                    acc1 += (double)norm2(xv);
                    if constexpr (KIND == FUSED) v[e] = cmul(bb, xn) + (PF == 1 ? yp[PF == 1 ? e : 0] : yload(n));
                } else {
                    const cx<T> yv = PF == 1 ? yp[PF == 1 ? e : 0] : yload(n);
                    const cx<T> rr = yv - rmul(il, cmul(dd, xv)) - z;
                    w[pl + n] = rr;
                    acc0 += (double)norm2(rr);
                    acc1 += (double)norm2(yv);
                }
            }
        // work-group partial sums (the tile is free again after this)
        double* red = reinterpret_cast<double*>(smem_raw);
        block_sum2(acc0, acc1, red);
        if (tid == 0) {
            const int64_t part = (int64_t)f * gridDim.x + blockIdx.x;
            gmem(s.partials)[2 * part] = acc0;
            gmem(s.partials)[2 * part + 1] = acc1;
        }
        if constexpr (KIND == LAST) return;
        __syncthreads();
    }
    // forward transform of the prepared registers, natural-order store
    fft_regs<P, -1, ROWS>(v, lds, ldp, col, lane, tw);
    constexpr int RLF = QF::r(P::S - 1);
#pragma unroll
    for (int b = 0; b < N / (RLF * TPC); ++b)
#pragma unroll
        for (int r = 0; r < RLF; ++r) w[pl + out_index<P, -1>(lane, b, r)] = v[b * RLF + r];
}

// XCD-aware tile order.  Work-groups are dispatched round-robin over the 8
// XCDs, each with its own L2.  When a tile's row segments are narrower than a
// 128-byte line, G neighbouring tiles share every line; this map sends those
// G tiles to the same XCD one after another, so each line is fetched from HBM
// once.  Identity when G = 1 or the grid does not split evenly.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb, int G) {
    constexpr unsigned X = 8;
    if (G <= 1 || nb % (X * (unsigned)G)) return b;
    const unsigned x = b % X, s = b / X;
    return ((s / (unsigned)G) * X + x) * (unsigned)G + (s % (unsigned)G);
}

// ------------------------------------------- pass B / D: strided axis --
// FFT along axis `axis` (< ndim - 1) of the w buffer, in place.  Tile = P
// adjacent columns along the last axis; the first stage loads straight from
// HBM and the last stage stores straight to HBM.  The inverse pass (DIR > 0)
// reads and writes non-temporally: its output is next read by the fused
// last-axis pass, which streams the whole grid anyway, so keeping it out of
// the caches leaves the memory-side cache to what the fused pass writes for
// the forward axis-1 pass that follows (8 % faster there, 2 % in the fused
// pass).  The other column passes keep their lines: each writes what the
// next one reads from the memory-side cache, and a non-temporal access to
// lines that are then rewritten in place costs the next reader its hits.
template <class P, int DIR, typename T>
__global__ void __launch_bounds__(256) k_strided(const Slot<T>* __restrict__ slots, Geom g, int axis,
                                                 int pcols, int ldp, int64_t es, int64_t ostride,
                                                 int nlast_tiles, int skip_done, int xg, int l0) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Slot<T>& s = slots[blockIdx.z];
    if (skip_done && s.ctl->done) return;
    const int tid = threadIdx.x;
    const int col = tid % pcols, lane = tid / pcols;
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x, xg);
    GLOBAL cx<T>* __restrict__ w = gmem(s.w) + (int64_t)blockIdx.y * g.ncell + (int64_t)(tile / nlast_tiles) * ostride + l0 +
                            (int64_t)(tile % nlast_tiles) * pcols;
    const uint32_t es32 = (uint32_t)es;
    cx<T> v[P::E];
    constexpr int NB0 = P::N / (Seq<P, DIR>::r(0) * P::TPC);
#pragma unroll
    for (int b = 0; b < NB0; ++b)
#pragma unroll
        for (int r = 0; r < Seq<P, DIR>::r(0); ++r) {
            const GLOBAL cx<T>* q = w + ((uint32_t)col + (uint32_t)in_index<P, DIR>(lane, b, r) * es32);
            if constexpr (DIR > 0) v[b * Seq<P, DIR>::r(0) + r] = ld_nt(q);
            else v[b * Seq<P, DIR>::r(0) + r] = *q;
        }
    // twiddles in LDS after the tile (first used after the first stage's barrier)
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(smem_raw + tile_bytes<T>((size_t)P::N * ldp));
    for (int i = tid; i < P::N; i += blockDim.x) tw_l[i] = gmem(s.tw[axis])[i];
    if constexpr (P::S == 1) __syncthreads();
    fft_regs<P, DIR>(v, lds, ldp, col, lane, tw_l);
    constexpr int Rl = Seq<P, DIR>::r(P::S - 1);
    constexpr int NBl = P::N / (Rl * P::TPC);
#pragma unroll
    for (int b = 0; b < NBl; ++b)
#pragma unroll
        for (int r = 0; r < Rl; ++r) {
            GLOBAL cx<T>* q = w + ((uint32_t)col + (uint32_t)out_index<P, DIR>(lane, b, r) * es32);
            if constexpr (DIR > 0) st_nt(q, v[b * Rl + r]);
            else *q = v[b * Rl + r];
        }
}

// ------------------------------------------------------ buffer access --
// Raw buffer loads and stores: a resource descriptor in scalar registers
// holds a base address and an extent in bytes, and each access adds a
// per-thread 32-bit byte offset (vector register) and a wave-uniform one
// (scalar register), dword 3 being the gfx9 raw-access format word.  Planes
// of different fields share the offsets, and element rows that differ by a
// uniform step share the vector offset, so the strided column passes keep
// one offset register per thread instead of a 64-bit address per element
// and field.  An offset beyond the extent reads zero and drops the write.
using bufres = __amdgpu_buffer_rsrc_t;
template <typename T>
__device__ __forceinline__ bufres make_res(const cx<T>* base, uint64_t bytes) {
    const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(base), (short)0, (int)n, 0x00020000);
}
template <typename T>
__device__ __forceinline__ cx<T> buf_load(bufres r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(bufres r, uint32_t voff, uint32_t soff, cx<T> v) {
    using V2 = unsigned int __attribute__((ext_vector_type(2)));
    using V4 = unsigned int __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 0);
    else __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, voff, soff, 0);
}

// ------------------------------------- pass C: axis 0 with the propagator --
// Forward FFT of all F fields along axis 0, per-wavevector operator, inverse
// FFT.  MODE CBS applies (L+I)^{-1} of App. B.1 (rank-one form, conjugate
// transpose for the adjoint); MODE APPLY applies the scaled staggered
// derivative block of L (negated for the adjoint).  1/prod(n) is folded in.
//   VAR 0: one LDS tile, fields in turn; 1: one region per field, every
//   exchange shared by all fields; 2: two regions, fields in pairs.
// NDIM (2 or 3) fixes the field count at compile time; the F planes of the
// tile are read and written through buffer resources that share offsets.
template <class P, int MODE, int VAR, int NDIM, typename T>
__global__ void __launch_bounds__(256) k_prop(const Slot<T>* __restrict__ slots, Geom g, int pcols, int ldp,
                                              int64_t es, int64_t ostride, int nlast_tiles, int xg, int l0) {
    constexpr int NR = VAR == 1 ? 4 : (VAR == 2 ? 2 : 1);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Slot<T>& s = slots[blockIdx.z];
    if (MODE == CBS && s.ctl->done) return;
    constexpr int N = P::N, E = P::E;
    constexpr int D = NDIM, F = NDIM + 1;
    const int tid = threadIdx.x;
    const int col = tid % pcols, lane = tid / pcols;
    const uint32_t es32 = (uint32_t)es;
    // LDS: NR field tiles | twiddles (N) | k0 S0 (N) | k0 (N)
    const int field_elems = (int)(tile_bytes<T>((size_t)N * ldp) / sizeof(cx<T>));
    cx<T>* tw_l = reinterpret_cast<cx<T>*>(smem_raw + (size_t)NR * field_elems * sizeof(cx<T>));
    cx<T>* g0_l = tw_l + N;
    T* k0_l = reinterpret_cast<T*>(g0_l + N);
    for (int i = tid; i < N; i += blockDim.x) {
        tw_l[i] = gmem(s.tw[0])[i];
        k0_l[i] = gmem(s.kv[0])[i];
        g0_l[i] = rmul(gmem(s.kv[0])[i], gmem(s.sh[0])[i]);
    }
    const cx<T>* tw = tw_l;
    using QF = Seq<P, -1>;
    using QI = Seq<P, 1>;
    constexpr int R0 = QF::r(0);
    constexpr int Rl = QF::r(P::S - 1);
    constexpr int RL = QI::r(P::S - 1);

    // first-stage inputs of every field of one tile, straight from HBM
    // element (lane + u) of a column sits at vo + u es bytes: one vector
    // offset per thread, the row step u es in a scalar register
    const uint32_t vo = ((uint32_t)col + (uint32_t)lane * es32) * (uint32_t)sizeof(cx<T>);
    auto soff = [&](int u) { return (uint32_t)u * es32 * (uint32_t)sizeof(cx<T>); };
    auto load = [&](cx<T> (&v)[4][E], const bufres (&res)[F]) {
#pragma unroll
        for (int b = 0; b < N / (R0 * P::TPC); ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const uint32_t so = soff(in_index<P, -1>(0, b, r));
#pragma unroll
                for (int f = 0; f < F; ++f) v[f][b * R0 + r] = buf_load<T>(res[f], vo, so);
            }
    };

    // transforms, operator and stores of one tile whose registers are loaded;
    // the LDS regions must be free on entry
    auto run = [&](cx<T> (&v)[4][E], int io, int il, const bufres (&res)[F]) {
        // wavevector components of this column (axes 1.., FFT order)
        T kc[2];
        cx<T> gc[2];   // k S for the column axes
        if (D == 3) {
            kc[0] = gmem(s.kv[1])[io];
            gc[0] = rmul(kc[0], gmem(s.sh[1])[io]);
            kc[1] = gmem(s.kv[2])[il];
            gc[1] = rmul(kc[1], gmem(s.sh[2])[il]);
        } else {
            kc[0] = gmem(s.kv[1])[il];
            gc[0] = rmul(kc[0], gmem(s.sh[1])[il]);
            kc[1] = 0;
            gc[1] = {0, 0};
        }
        if constexpr (NR == 4) {
            fft_regs_multi<P, -1, 4>(v, F, lds, field_elems, ldp, col, lane, tw);
        } else if constexpr (NR == 2) {
            fft_regs_multi<P, -1, 2>(v, 2, lds, field_elems, ldp, col, lane, tw);
            __syncthreads();
            fft_regs_multi<P, -1, 2>(v + 2, F - 2, lds, field_elems, ldp, col, lane, tw);
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (f < F) {
                    if (f > 0) __syncthreads();
                    fft_regs<P, -1>(v[f], lds, ldp, col, lane, tw);
                }
            }
        }

        // slot constants of the operator, conjugated for the adjoint (sign
        // flips of uniform values only, so they stay in scalar registers);
        // can carries the 1/prod(n) of the inverse transform
        const cx<T> ca = s.adjoint ? conjg(s.ca) : s.ca;
        const cx<T> cp = s.adjoint ? conjg(s.cp) : s.cp;
        const cx<T> can = s.adjoint ? conjg(s.can) : s.can;
        const T al12im = s.adjoint ? -s.al12.im : s.al12.im;
        const T ss = s.adjoint ? -s.s : s.s;   // sig s
        // per-wavevector operator on the registers
#pragma unroll
        for (int b = 0; b < N / (Rl * P::TPC); ++b) {
#pragma unroll
            for (int r = 0; r < Rl; ++r) {
                const int k0i = out_index<P, -1>(lane, b, r);
                const int e = b * Rl + r;
                const T k0 = k0_l[k0i];
                const cx<T> g0 = g0_l[k0i];
                cx<T> gg[3] = {g0, gc[0], gc[1]};
                const cx<T> wp = (D == 3) ? v[3][e] : v[2][e];
                // t = sum_eta conj(k_eta S_eta) w_eta
                cx<T> t = cmulc(v[0][e], gg[0]);
                t = t + cmulc(v[1][e], gg[1]);
                if (D == 3) t = t + cmulc(v[2][e], gg[2]);
                if constexpr (MODE == CBS) {
                    const T kk = k0 * k0 + kc[0] * kc[0] + kc[1] * kc[1];
                    const cx<T> mu = {kk + s.al12.re, al12im};
                    const cx<T> imu = rmul(s.inv_ntot, cinv_fast(mu));
                    // u_eta = ca (w_eta - g_eta t / mu) - i sig s g_eta wp / mu,
                    // p = -i sig s t / mu + cp wp / mu  (1/prod(n) inside imu)
                    const cx<T> tm = cmul(t, imu);
                    const cx<T> wpm = cmul(wp, imu);
                    if constexpr (sizeof(T) == 4) {
                        // fewer instructions: u_eta = (ca / prod n) w_eta - g_eta h
                        const cx<T> h = cmul(ca, tm) + rmul(ss, mul_i(wpm));
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            if (d < D) v[d][e] = cmul(can, v[d][e]) - cmul(gg[d], h);
                    } else {
                        // fewer live registers in FP64 (two waves per SIMD)
                        const cx<T> pm = rmul(ss, mul_i(wpm));
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            if (d < D) {
                                const cx<T> a = rmul(s.inv_ntot, v[d][e]) - cmul(gg[d], tm);
                                v[d][e] = cmul(ca, a) - cmul(gg[d], pm);
                            }
                        }
                    }
                    const cx<T> pz = cmul(cp, wpm) - rmul(ss, mul_i(tm));
                    if (D == 3) v[3][e] = pz;
                    else v[2][e] = pz;
                } else {
                    // (L - diag) x in scaled form: u_eta = i sig g_eta p / s ; p = i sig t / s
                    const T c = (s.adjoint ? -s.inv_ntot : s.inv_ntot) / s.s;
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        if (d < D) v[d][e] = rmul(c, mul_i(cmul(gg[d], wp)));
                    if (D == 3) v[3][e] = rmul(c, mul_i(t));
                    else v[2][e] = rmul(c, mul_i(t));
                }
            }
        }

        // inverse FFT from the registers; each field is stored as soon as
        // its transform is done, so its stores travel while the next
        // fields are transformed
        auto store = [&](int f) {
#pragma unroll
            for (int b = 0; b < N / (RL * P::TPC); ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r)
                    buf_store<T>(res[f], vo, soff(out_index<P, 1>(0, b, r)), v[f][b * RL + r]);
        };
        if constexpr (NR == 4) {
            __syncthreads();
            fft_regs_multi<P, 1, 4>(v, F, lds, field_elems, ldp, col, lane, tw);
#pragma unroll
            for (int f = 0; f < 4; ++f)
                if (f < F) store(f);
        } else if constexpr (NR == 2) {
            __syncthreads();
            fft_regs_multi<P, 1, 2>(v, 2, lds, field_elems, ldp, col, lane, tw);
            store(0);
            store(1);
            __syncthreads();
            fft_regs_multi<P, 1, 2>(v + 2, F - 2, lds, field_elems, ldp, col, lane, tw);
            store(2);
            if (F == 4) store(3);
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (f < F) {
                    __syncthreads();
                    fft_regs<P, 1>(v[f], lds, ldp, col, lane, tw);
                    store(f);
                }
            }
        }
    };

    // tile: index io along the middle axis (3-D), columns along the last
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x, xg);
    const int64_t toff = (int64_t)(tile / nlast_tiles) * ostride + l0 + (int64_t)(tile % nlast_tiles) * pcols;
    bufres res[F];
#pragma unroll
    for (int f = 0; f < F; ++f)
        res[f] = make_res<T>(s.w + (int64_t)f * g.ncell + toff, (uint64_t)(g.ncell - toff) * sizeof(cx<T>));
    cx<T> v[4][E];
    __syncthreads();   // tables staged
    load(v, res);
    run(v, (int)(tile / nlast_tiles), l0 + (int)(tile % nlast_tiles) * pcols + col, res);
}

// LDS one work-group may hold on gfx950 (160 KiB per compute unit); larger
// configurations are refused before launch.
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Launch one pass.  kind: 0 last-axis forward with prologue, 1 last-axis
// inverse with epilogue, 5 both fused across iterations, 2 strided forward,
// 3 strided inverse, 4 axis-0 propagator.
// FULL: every variant is compiled for this plan; otherwise only variant 0 of
// each pass (and the unpadded column tile, a launch-time choice).
template <typename T, class P, bool FULL>
static hipError_t launch_plan(int kind, int mode, const Slot<T>* slots, int nslots, const Geom& g, int axis,
                              int pcols, int variant, int l0, int lw, hipStream_t st) {
    if (!FULL && (variant & ~(4 | 16))) return hipErrorInvalidValue;
    const int N = P::N;
    // column tiles (strided and propagator passes) are padded by one element
    // per row unless variant bit 2 asks for the unpadded pitch
    const bool colpass = kind == 2 || kind == 3 || kind == 4;
    const int ldp = pcols + ((colpass && (variant & 4)) ? 0 : 1);
    if (colpass) variant &= 3;
    // tile + twiddles + (propagator) k0 S0 and k0 tables
    size_t lds = tile_bytes<T>((size_t)N * ldp) + (size_t)N * (2 * sizeof(cx<T>) + sizeof(T));
    if (lds < 64 * sizeof(double)) lds = 64 * sizeof(double);
    const dim3 block(pcols * P::TPC);
    const int F = g.ndim + 1;
    const int last = g.ndim - 1;
    if (kind == 0 || kind == 1 || kind == 5) {
        const int64_t tiles = g.ncell / ((int64_t)N * pcols);
        const dim3 grid((unsigned)tiles, F, nslots);
        const dim3 blk(pcols * P::TPC);
        const size_t lr = std::max(tile_bytes<T>((size_t)pcols * lds_pitch<ROWS>(N, 0)), (size_t)(64 * sizeof(double))) +
                          (size_t)N * (sizeof(cx<T>) + sizeof(T));
        if (lr > kMaxLdsBytes) return hipErrorInvalidConfiguration;
        // last-axis passes: variant bits 0-1 = prefetch of the inverse pass,
        // bit 4 = sparse right-hand side (kernels for it exist in FP64 for the
        // full-variant plans; elsewhere the dense y, always complete, is read)
        const bool ys = (variant & 16) && sizeof(T) == 8 && FULL;
        const int pf = variant & 3;
#define LA_LAUNCH(M, K, PF_, YS_) \
    hipLaunchKernelGGL((k_lastaxis<P, M, K, PF_, YS_, T>), grid, blk, lr, st, slots, g, pcols)
#define LA_YS(M, K, PF_)                                      \
    do {                                                      \
        if constexpr (sizeof(T) == 8 && FULL) {               \
            if (ys) LA_LAUNCH(M, K, PF_, true);               \
            else LA_LAUNCH(M, K, PF_, false);                 \
        } else {                                              \
            LA_LAUNCH(M, K, PF_, false);                      \
        }                                                     \
    } while (0)
        // residual (APPLY) passes run in FP64 only
        if (mode != CBS && sizeof(T) != 8) return hipErrorInvalidValue;
        if (kind == 0) {
            if (mode == CBS) LA_YS(CBS, FIRST, 0);
            else if constexpr (sizeof(T) == 8) LA_LAUNCH(APPLY, FIRST, 0, false);
        } else if (kind == 1) {
            if (mode == CBS) {
                if constexpr (FULL) {
                    if (pf == 1) LA_LAUNCH(CBS, LAST, 1, false);
                    else if (pf == 2) LA_LAUNCH(CBS, LAST, 2, false);
                    else LA_LAUNCH(CBS, LAST, 0, false);
                } else {
                    LA_LAUNCH(CBS, LAST, 0, false);
                }
            } else if constexpr (sizeof(T) == 8) {
                if constexpr (FULL) {
                    if (pf == 1) LA_YS(APPLY, LAST, 1);
                    else if (pf == 2) LA_YS(APPLY, LAST, 2);
                    else LA_YS(APPLY, LAST, 0);
                } else {
                    LA_LAUNCH(APPLY, LAST, 0, false);
                }
            }
        } else {
            if constexpr (FULL) {
                if (pf == 1) LA_YS(CBS, FUSED, 1);
                else if (pf == 2) LA_YS(CBS, FUSED, 2);
                else LA_YS(CBS, FUSED, 0);
            } else {
                LA_LAUNCH(CBS, FUSED, 0, false);
            }
        }
#undef LA_YS
#undef LA_LAUNCH
    } else {
        // strided along `axis`; columns run along the last axis in groups of pcols
        int64_t es = 1;
        for (int d = axis + 1; d < g.ndim; ++d) es *= g.n[d];
        // columns [l0, l0 + lw) of the last axis (lw = 0: all of it)
        if (lw == 0) lw = g.n[last];
        if (l0 < 0 || lw <= 0 || l0 + lw > g.n[last] || lw % pcols || l0 % pcols) return hipErrorInvalidValue;
        const int nlast_tiles = lw / pcols;
        // the remaining ("other") axis: the one that is neither `axis` nor last
        int other = -1;
        for (int d = 0; d < g.ndim - 1; ++d)
            if (d != axis) other = d;
        int64_t ostride = 0;
        int nother = 1;
        if (other >= 0) {
            ostride = 1;
            for (int d = other + 1; d < g.ndim; ++d) ostride *= g.n[d];
            nother = g.n[other];
        }
        const unsigned tiles = (unsigned)(nlast_tiles * nother);
        // tiles sharing each 128-byte line (adjacent along the last axis)
        int xg = (int)(128 / ((size_t)pcols * sizeof(cx<T>)));
        if (xg < 1 || nlast_tiles % xg) xg = 1;
        if (kind == 4) {
            const dim3 grid(tiles, 1, nslots);
            const int nr = variant == 1 ? 4 : (variant == 2 ? 2 : 1);
            const size_t lp = lds + (size_t)(nr - 1) * tile_bytes<T>((size_t)N * ldp);
            if (lp > kMaxLdsBytes) return hipErrorInvalidConfiguration;
#define PROP_LAUNCH(M, V)                                                                                     \
    do {                                                                                                      \
        if (g.ndim == 3)                                                                                      \
            hipLaunchKernelGGL((k_prop<P, M, V, 3, T>), grid, block, lp, st, slots, g, pcols, ldp, es, ostride, \
                               nlast_tiles, xg, l0);                                                          \
        else                                                                                                  \
            hipLaunchKernelGGL((k_prop<P, M, V, 2, T>), grid, block, lp, st, slots, g, pcols, ldp, es, ostride, \
                               nlast_tiles, xg, l0);                                                          \
    } while (0)
            if (mode != CBS && sizeof(T) != 8) return hipErrorInvalidValue;
            if (mode == CBS) {
                if constexpr (FULL) {
                    if (variant == 1) PROP_LAUNCH(CBS, 1);
                    else if (variant == 2) PROP_LAUNCH(CBS, 2);
                    else PROP_LAUNCH(CBS, 0);
                } else {
                    PROP_LAUNCH(CBS, 0);
                }
            } else if constexpr (sizeof(T) == 8) {
                if constexpr (FULL) {
                    if (variant == 1) PROP_LAUNCH(APPLY, 1);
                    else if (variant == 2) PROP_LAUNCH(APPLY, 2);
                    else PROP_LAUNCH(APPLY, 0);
                } else {
                    PROP_LAUNCH(APPLY, 0);
                }
            }
#undef PROP_LAUNCH
        } else {
            if (lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
            const dim3 grid(tiles, F, nslots);
            const int skip = mode == CBS ? 1 : 0;
            if (kind == 2)
                hipLaunchKernelGGL((k_strided<P, -1, T>), grid, block, lds, st, slots, g, axis, pcols, ldp, es,
                                   ostride, nlast_tiles, skip, xg, l0);
            else
                hipLaunchKernelGGL((k_strided<P, 1, T>), grid, block, lds, st, slots, g, axis, pcols, ldp, es,
                                   ostride, nlast_tiles, skip, xg, l0);
        }
    }
    return hipGetLastError();
}

}  // namespace cbs
