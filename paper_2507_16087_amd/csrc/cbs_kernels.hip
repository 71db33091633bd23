// gfx950 kernels of the iterative Born solver (arXiv 2507.16087, Algorithm 1
// on the staggered first-order system of App. B.1).
//
// One CBS iteration (eq. BornAlt: x <- x + nu B [(L+I)^{-1}(B x + y) - x]) on
// an n0 x n1 x n2 grid with F = ndim + 1 complex fields is a set of passes
// over HBM, each a batch of 1-D FFTs along one axis:
//   pass A  axis 2 (contiguous): w = B x + y formed on load, forward FFT
//   pass B  axis 1 (strided)   : forward FFT                        (3-D only)
//   pass C  axis 0 (strided)   : forward FFT, (L+I)^{-1} per wavevector with
//                                all F fields in registers, inverse FFT
//   pass D  axis 1 (strided)   : inverse FFT                        (3-D only)
//   pass E  axis 2 (contiguous): inverse FFT, x += nu B (z - x) with the
//                                |dx|^2, |x|^2 partial sums
// In steady state E and the next iteration's A are one kernel (the fused
// kind): the inverse transform runs its radices in reverse order, so the
// registers it ends with are exactly the forward transform's first-stage
// inputs.  A two-level reduction kernel then folds the partial sums in index
// order, advances the iteration counter and raises the slot's stop flag.
// The same passes with a different middle operator (i k S / sqrt(lam1 lam2))
// and epilogue (r = y - D x / lam - z) evaluate the scaled true residual
// y - (L+V) x used by iterative refinement.
//
// FFTs are Stockham radix-R stages (R in 2..16, including 3, 6, 12): every
// thread owns whole butterflies, the first stage loads straight from HBM and
// the last stage stores straight to HBM in natural order, and stages exchange
// through an LDS tile.  Strided passes map threads column-fastest (a tile of P
// adjacent columns reads P-element row segments); contiguous passes map them
// lane-fastest along each pencil, so loads and stores run along cache lines.
#include "cbs_passes.h"
#include "cbs_plans.h"

namespace cbs {

__device__ __forceinline__ void cell_coords(const Geom& g, int64_t cell, int* ix) {
    int64_t r = cell;
    for (int d = g.ndim - 1; d >= 0; --d) {
        ix[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
}


template <bool CBSMODE>
__device__ void finalize_ctl(Ctl* c, double a, double b) {
    if (!CBSMODE) {
        c->res2 = a;
        c->rhs2 = b;
        c->scale = sqrt(a);
        c->res_done += 1;
        return;
    }
    const int it = c->iter + 1;
    c->iter = it;
    const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
    c->rel_update = rel;
    c->xnorm2 = b;
    int done = RUNNING;
    if (!isfinite(a) || !isfinite(b)) {
        done = DIVERGED;
    } else {
        c->grow = (it >= 3 && rel > 2.0) ? c->grow + 1 : 0;
        if (c->grow >= 3) done = DIVERGED;
        else if (b > 0.0 && rel <= c->tol) done = CONVERGED;
        else if (it >= c->max_iter) done = CAPPED;
    }
    c->done = done;
}


// ---------------------------------------------------------- reductions --
// Two levels, one launch: grid = (blocks, slots); block b folds partial pairs
// [b * kReduceChunk, (b + 1) * kReduceChunk) into chunks[b]; the block that
// arrives last folds the chunk sums with all its threads (thread t takes
// chunks t, t + 256, ... in order, then the block's fixed tree), so the
// totals do not depend on scheduling, and finalises the slot's control block
// (finalize_ctl).
template <typename T, bool CBSMODE>
__global__ void __launch_bounds__(256) k_reduce(const Slot<T>* slots, int nparts) {
    __shared__ double red[16];
    __shared__ int last;
    const Slot<T>& s = slots[blockIdx.y];
    Ctl* c = s.ctl;
    if (CBSMODE && c->done) return;
    const double* p = s.partials;
    const int b0 = blockIdx.x * kReduceChunk;
    const int b1 = min(nparts, b0 + kReduceChunk);
    double a = 0.0, b = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        a += p[2 * i];
        b += p[2 * i + 1];
    }
    block_sum2(a, b, red);
    if (threadIdx.x == 0) {
        s.chunks[2 * blockIdx.x] = a;
        s.chunks[2 * blockIdx.x + 1] = b;
        __threadfence();
        last = atomicAdd(&c->arrive, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    a = 0.0;
    b = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
        a += ((volatile double*)s.chunks)[2 * i];
        b += ((volatile double*)s.chunks)[2 * i + 1];
    }
    block_sum2(a, b, red);
    if (threadIdx.x != 0) return;
    c->arrive = 0;
    finalize_ctl<CBSMODE>(c, a, b);
}

__global__ void k_ctl_reset(Ctl* c, int max_iter, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->done = RUNNING;
        c->iter = 0;
        c->max_iter = max_iter;
        c->grow = 0;
        c->tol = tol;
        c->rel_update = 0.0;
        c->xnorm2 = 0.0;
    }
}

// every field of a control block to zero (a kernel, so that no memset node
// lands in a caller's captured graph)
__global__ void k_ctl_clear(Ctl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = Ctl{};
}

// ------------------------------------------------------ slab exchange --
// Layouts of F planes of an n0 x n1 x n2 grid split into G parts:
//   0 whole grid      [f][i0][i1][i2]
//   1 axis-0 slabs    part g = i0 / s (s = n0 / G): [g][f][i0 % s][i1][i2]
//   2 axis-1 pencils  part h = i1 / t (t = n1 / G): [h][f][i0][i1 % t][i2]
// k_relayout copies every element from one layout to another, walking the
// destination in memory order; from layout 1 to 2 and back it is the
// all-to-all exchange of a solve split over G devices.
struct SplitDims {
    int F, n0, n1, n2, G;
};

__device__ __forceinline__ int64_t split_offset(int lay, const SplitDims& d, int f, int i0, int i1, int i2) {
    if (lay == 0) return (((int64_t)f * d.n0 + i0) * d.n1 + i1) * d.n2 + i2;
    if (lay == 1) {
        const int s = d.n0 / d.G;
        return (int64_t)(i0 / s) * d.F * s * d.n1 * d.n2 + (((int64_t)f * s + i0 % s) * d.n1 + i1) * d.n2 + i2;
    }
    const int t = d.n1 / d.G;
    return (int64_t)(i1 / t) * d.F * d.n0 * t * d.n2 + (((int64_t)f * d.n0 + i0) * t + i1 % t) * d.n2 + i2;
}

__device__ __forceinline__ void split_coords(int lay, const SplitDims& d, int64_t e, int* f, int* i0, int* i1,
                                             int* i2) {
    if (lay == 0) {
        *i2 = (int)(e % d.n2);
        e /= d.n2;
        *i1 = (int)(e % d.n1);
        e /= d.n1;
        *i0 = (int)(e % d.n0);
        *f = (int)(e / d.n0);
    } else if (lay == 1) {
        const int s = d.n0 / d.G;
        const int64_t part = (int64_t)d.F * s * d.n1 * d.n2;
        const int g = (int)(e / part);
        e %= part;
        *i2 = (int)(e % d.n2);
        e /= d.n2;
        *i1 = (int)(e % d.n1);
        e /= d.n1;
        *i0 = g * s + (int)(e % s);
        *f = (int)(e / s);
    } else {
        const int t = d.n1 / d.G;
        const int64_t part = (int64_t)d.F * d.n0 * t * d.n2;
        const int h = (int)(e / part);
        e %= part;
        *i2 = (int)(e % d.n2);
        e /= d.n2;
        *i1 = h * t + (int)(e % t);
        e /= t;
        *i0 = (int)(e % d.n0);
        *f = (int)(e / d.n0);
    }
}

template <typename E>
__global__ void __launch_bounds__(256) k_relayout(const E* __restrict__ src, int src_lay, E* __restrict__ dst,
                                                  int dst_lay, SplitDims d) {
    const int64_t total = (int64_t)d.F * d.n0 * d.n1 * d.n2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int f, i0, i1, i2;
        split_coords(dst_lay, d, e, &f, &i0, &i1, &i2);
        dst[e] = src[split_offset(src_lay, d, f, i0, i1, i2)];
    }
}

// Per-pencil flags of a sparse right-hand side: flag[k] = 1 if any of the n
// values of pencil k (of one field plane) is non-zero.  One wave per pencil.
__global__ void __launch_bounds__(256) k_pencil_flags(const cx<double>* __restrict__ plane, int64_t pencils, int n,
                                                      unsigned char* __restrict__ flag) {
    const int64_t pc = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pc >= pencils) return;
    const int lane = threadIdx.x & 63;
    int nz = 0;
    for (int j = lane; j < n; j += 64) {
        const cx<double> v = plane[pc * n + j];
        nz |= (v.re != 0.0 || v.im != 0.0);
    }
    nz = __any(nz);
    if (lane == 0) flag[pc] = (unsigned char)(nz ? 1 : 0);
}

// ------------------------------------------------------- elementwise --
template <typename T>
__global__ void k_zero(cx<T>* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = {T(0), T(0)};
}

// y = C^{-1/2} s_hat for every field, written at both precisions (either
// destination nullable).  kind PHYSICAL forms s_hat from the physical
// sources (rhobar s_u, q s_p); EQUATION takes them as given.  su may be null.
__global__ void k_rhs(Geom g, const cx<double>* sp, const cx<double>* su, const double* rhobar,
                      const cx<double>* q, int physical, double il1s, double il2s, cx<double>* y64,
                      cx<float>* y32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int F = g.ndim + 1;
    if (i >= g.ncell * F) return;
    const int f = (int)(i / g.ncell);
    const int64_t cell = i % g.ncell;
    cx<double> v;
    if (f < g.ndim) {
        v = su ? su[i] : cx<double>{0.0, 0.0};
        if (physical) v = rmul(rhobar[i], v);
        v = rmul(il1s, v);
    } else {
        v = sp[cell];
        if (physical) v = cmul(q[cell], v);
        v = rmul(il2s, v);
    }
    if (y64) y64[i] = v;
    if (y32) y32[i] = {(float)v.re, (float)v.im};
}

// x = C^{1/2} (u, p) from physical fields (u nullable).
__global__ void k_scale_in(Geom g, const cx<double>* p, const cx<double>* u, double sl1, double sl2,
                           cx<double>* x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int F = g.ndim + 1;
    if (i >= g.ncell * F) return;
    const int f = (int)(i / g.ncell);
    if (f < g.ndim) x[i] = u ? rmul(sl1, u[i]) : cx<double>{0.0, 0.0};
    else x[i] = rmul(sl2, p[i % g.ncell]);
}

// (u, p) = C^{-1/2} x into complex128 outputs (u nullable); T = state precision.
template <typename T>
__global__ void k_unscale(Geom g, const cx<T>* x, double il1s, double il2s, cx<double>* p, cx<double>* u) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int F = g.ndim + 1;
    if (i >= g.ncell * F) return;
    const int f = (int)(i / g.ncell);
    const cx<double> v = {(double)x[i].re, (double)x[i].im};
    if (f < g.ndim) {
        if (u) u[i] = rmul(il1s, v);
    } else {
        p[i % g.ncell] = rmul(il2s, v);
    }
}

// physical residual C^{1/2} r from the scaled residual r
__global__ void k_residual_out(Geom g, const cx<double>* r, double sl1, double sl2, cx<double>* rp,
                               cx<double>* ru) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int F = g.ndim + 1;
    if (i >= g.ncell * F) return;
    const int f = (int)(i / g.ncell);
    if (f < g.ndim) {
        if (ru) ru[i] = rmul(sl1, r[i]);
    } else if (rp) {
        rp[i % g.ncell] = rmul(sl2, r[i]);
    }
}

// refinement: inner right-hand side r / |r| in FP32 (|r| read on device)
__global__ void k_convert(const cx<double>* r, cx<float>* y32, int64_t n, const Ctl* c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = c->scale > 0.0 ? 1.0 / c->scale : 0.0;
    y32[i] = {(float)(r[i].re * inv), (float)(r[i].im * inv)};
}

// refinement: x64 += |r| d32
__global__ void k_accumulate(cx<double>* x, const cx<float>* d, int64_t n, const Ctl* c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sc = c->scale;
    x[i] = {x[i].re + sc * (double)d[i].re, x[i].im + sc * (double)d[i].im};
}

// Misfit gradient (adjoint-state) per cell; see cbs_gradient in cbs.h.
__global__ void k_gradient(Geom g, const double* c, const double* rho, const double* alpha,
                           const cx<double>* q, const double* gcen0, const double* gcen1,
                           const double* gcen2, const double* gst0, const double* gst1,
                           const double* gst2, double gmax, double omega, const cx<double>* sp,
                           const cx<double>* su, const cx<double>* p, const cx<double>* u,
                           const cx<double>* lp, const cx<double>* lu, double* gc, double* grho,
                           double* galpha, int collocated) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.ncell) return;
    int ix[3];
    cell_coords(g, i, ix);
    const double* gcen[3] = {gcen0, gcen1, gcen2};
    const double* gst[3] = {gst0, gst1, gst2};
    double gsum = 0.0;
    for (int d = 0; d < g.ndim; ++d) gsum += gcen[d][ix[d]];
    const double gam = gmax * gsum;
    const double cv = c[i], rv = rho[i], av = alpha[i];
    const cx<double> iwg = {gam, omega};
    // conj(lambda_p) (s_p - (gamma + i w) p): common factor of the pressure row
    const cx<double> core = cmulc(sp[i] - cmul(iwg, p[i]), lp[i]);
    const cx<double> dq_dc = {-2.0 / (cv * cv * cv * rv), 2.0 * av / (omega * cv * cv * rv)};
    const cx<double> dq_dal = {0.0, -2.0 / (omega * rv * cv)};
    const cx<double> qv = q[i];
    const cx<double> dq_drho = {-qv.re / rv, -qv.im / rv};
    if (gc) gc[i] = cmul(core, dq_dc).re;
    if (galpha) galpha[i] = cmul(core, dq_dal).re;
    if (grho) {
        double gr = cmul(core, dq_drho).re;
        if (u && lu && collocated) {
            // collocated: the velocity rows at this cell carry rho(x) itself
            for (int e = 0; e < g.ndim; ++e) {
                const int64_t k = (int64_t)e * g.ncell + i;
                const cx<double> sv = su ? su[k] : cx<double>{0.0, 0.0};
                gr += cmulc(sv - cmul(iwg, u[k]), lu[k]).re;
            }
        } else if (u && lu) {
            for (int e = 0; e < g.ndim; ++e) {
                // rhobar_e at this cell and at the cell one step back along e
                int jx[3] = {ix[0], ix[1], ix[2]};
                jx[e] = (jx[e] - 1 + g.n[e]) % g.n[e];
                int64_t j = 0;
                for (int d = 0; d < g.ndim; ++d) j = j * g.n[d] + (d < g.ndim ? jx[d] : 0);
                for (int which = 0; which < 2; ++which) {
                    const int64_t cell = which ? j : i;
                    const int* cc = which ? jx : ix;
                    double gs = 0.0;
                    for (int d = 0; d < g.ndim; ++d) gs += (d == e) ? gst[d][cc[d]] : gcen[d][cc[d]];
                    const cx<double> iwe = {gmax * gs, omega};
                    const int64_t k = (int64_t)e * g.ncell + cell;
                    const cx<double> sv = su ? su[k] : cx<double>{0.0, 0.0};
                    gr += 0.5 * cmulc(sv - cmul(iwe, u[k]), lu[k]).re;
                }
            }
        }
        grho[i] = gr;
    }
}

// ------------------------------------------------------------ dispatch --
int plan_tpc(int n, bool wide) {
#define TPC_CASE(G_, N_, A, B, C, T_) \
    if (n == N_) return T_;
    if (wide) { CBS_PLANS_WIDE(TPC_CASE) }
    CBS_PLANS(TPC_CASE)
#undef TPC_CASE
    return 0;
}

bool plan_has_wide(int n) {
#define WIDE_CASE(G_, N_, A, B, C, T_) \
    if (n == N_) return true;
    CBS_PLANS_WIDE(WIDE_CASE)
#undef WIDE_CASE
    return false;
}

static int plan_group(int n) {
#define GROUP_CASE(G_, N_, A, B, C, T_) \
    if (n == N_) return G_;
    CBS_PLANS(GROUP_CASE)
#undef GROUP_CASE
    return -1;
}

// per-group launchers (cbs_pass_group.hip, one object per group)
template <int G, typename T>
hipError_t launch_group(int kind, int mode, const Slot<T>* slots, int nslots, const Geom& g, int axis, int n,
                        int pcols, bool wide, int variant, hipStream_t st, int l0, int lw);

// 1-D grids: the one axis is the contiguous one, so the per-wavevector
// operator of pass C runs on its own between the forward (A) and inverse (E)
// last-axis passes, one thread per wavenumber on the spectrum in w.  MODE CBS
// applies (L+I)^{-1} of App. B.1 in its rank-one form with one velocity
// field (conjugate transpose for the adjoint); MODE APPLY applies the scaled
// staggered derivative block of L (negated for the adjoint).  1/n is folded
// in as in pass C.
template <int MODE, typename T>
__global__ void __launch_bounds__(256) k_op1(const Slot<T>* __restrict__ slots, int n) {
    const Slot<T>& s = slots[blockIdx.y];
    if (MODE == CBS && s.ctl->done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<T>* w = s.w;
    const cx<T> wu = w[i], wp = w[n + i];
    const T k = s.kv[0][i];
    const cx<T> gk = rmul(k, s.sh[0][i]);   // k S
    const cx<T> t = cmulc(wu, gk);           // conj(k S) w_u
    if constexpr (MODE == CBS) {
        const bool adj = s.adjoint != 0;
        const cx<T> ca = adj ? conjg(s.ca) : s.ca;
        const cx<T> cp = adj ? conjg(s.cp) : s.cp;
        const T ss = adj ? -s.s : s.s;
        const cx<T> mu = {k * k + s.al12.re, adj ? -s.al12.im : s.al12.im};
        const cx<T> imu = rmul(s.inv_ntot, cinv_fast(mu));
        const cx<T> tm = cmul(t, imu), wpm = cmul(wp, imu);
        // u = ca (w_u - k S t / mu) - i sig s k S w_p / mu ; p = -i sig s t / mu + cp w_p / mu
        w[i] = cmul(ca, rmul(s.inv_ntot, wu) - cmul(gk, tm)) - cmul(gk, rmul(ss, mul_i(wpm)));
        w[n + i] = cmul(cp, wpm) - rmul(ss, mul_i(tm));
    } else {
        const T c = (s.adjoint ? -s.inv_ntot : s.inv_ntot) / s.s;
        w[i] = rmul(c, mul_i(cmul(gk, wp)));
        w[n + i] = rmul(c, mul_i(t));
    }
}

template <typename T>
hipError_t launch_pass(int kind, int mode, const Slot<T>* slots, int nslots, const Geom& g, int axis, int n,
                       int pcols, bool wide, int variant, hipStream_t st, int l0, int lw) {
    if (kind == 6) {
        // 1-D operator pass (kind 6): the whole grid is one spectrum of n points
        if (g.ndim != 1 || n != g.n[0] || (mode != CBS && sizeof(T) != 8)) return hipErrorInvalidValue;
        const dim3 grid((unsigned)((n + 255) / 256), (unsigned)nslots);
        if (mode == CBS) hipLaunchKernelGGL((k_op1<CBS, T>), grid, dim3(256), 0, st, slots, n);
        else hipLaunchKernelGGL((k_op1<APPLY, T>), grid, dim3(256), 0, st, slots, n);
        return hipGetLastError();
    }
    switch (plan_group(n)) {
#define GROUP_LAUNCH(G_) \
    case G_: return launch_group<G_, T>(kind, mode, slots, nslots, g, axis, n, pcols, wide, variant, st, l0, lw);
        GROUP_LAUNCH(0)
        GROUP_LAUNCH(1)
        GROUP_LAUNCH(2)
        GROUP_LAUNCH(3)
        GROUP_LAUNCH(4)
        GROUP_LAUNCH(5)
        GROUP_LAUNCH(6)
        GROUP_LAUNCH(7)
        GROUP_LAUNCH(8)
        GROUP_LAUNCH(9)
        GROUP_LAUNCH(10)
#undef GROUP_LAUNCH
        default: return hipErrorInvalidValue;
    }
}
static_assert(CBS_PLAN_GROUPS == 11, "one GROUP_LAUNCH per plan group");

bool plan_has_variants(int n) {
    const int gr = plan_group(n);
    return gr >= 0 && gr < CBS_FULL_VARIANT_GROUPS;
}

template hipError_t launch_pass<float>(int, int, const Slot<float>*, int, const Geom&, int, int, int, bool, int,
                                       hipStream_t, int, int);
template hipError_t launch_pass<double>(int, int, const Slot<double>*, int, const Geom&, int, int, int, bool, int,
                                        hipStream_t, int, int);

template <typename T>
hipError_t launch_reduce(bool cbs_mode, const Slot<T>* slots, int nparts, int nslots, hipStream_t st) {
    const dim3 grid((unsigned)((nparts + kReduceChunk - 1) / kReduceChunk), nslots);
    if (cbs_mode)
        hipLaunchKernelGGL((k_reduce<T, true>), grid, dim3(256), 0, st, slots, nparts);
    else
        hipLaunchKernelGGL((k_reduce<T, false>), grid, dim3(256), 0, st, slots, nparts);
    return hipGetLastError();
}
template hipError_t launch_reduce<float>(bool, const Slot<float>*, int, int, hipStream_t);
template hipError_t launch_reduce<double>(bool, const Slot<double>*, int, int, hipStream_t);

hipError_t launch_ctl_reset(Ctl* c, int max_iter, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, c, max_iter, tol);
    return hipGetLastError();
}

// Streaming copy for bandwidth measurement: work-group b copies the b-th
// contiguous chunk of kProbeChunk 16-byte vectors, four nontemporal loads in
// flight per thread before their stores.
constexpr size_t kProbeChunk = 1024;   // 16 KiB
using v4u = unsigned int __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_stream_copy(const v4u* __restrict__ src, v4u* __restrict__ dst, size_t n) {
    const size_t base = (size_t)blockIdx.x * kProbeChunk;
    const size_t end = base + kProbeChunk < n ? base + kProbeChunk : n;
    size_t i = base + threadIdx.x;
    for (; i + 768 < end; i += 1024) {
        const v4u a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + 256);
        const v4u c = __builtin_nontemporal_load(src + i + 512), d = __builtin_nontemporal_load(src + i + 768);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + 256);
        __builtin_nontemporal_store(c, dst + i + 512);
        __builtin_nontemporal_store(d, dst + i + 768);
    }
    for (; i < end; i += 256) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
    const size_t n = bytes / sizeof(v4u);
    const size_t grid = (n + kProbeChunk - 1) / kProbeChunk;
    if (n == 0 || grid > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)grid), dim3(256), 0, st, static_cast<const v4u*>(src),
                       static_cast<v4u*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_ctl_clear(Ctl* c, hipStream_t st) {
    hipLaunchKernelGGL(k_ctl_clear, dim3(1), dim3(64), 0, st, c);
    return hipGetLastError();
}

template <typename E>
hipError_t launch_relayout(const E* src, int src_lay, E* dst, int dst_lay, int F, const int* n, int G,
                           hipStream_t st) {
    const SplitDims d{F, n[0], n[1], n[2], G};
    const int64_t total = (int64_t)F * n[0] * n[1] * n[2];
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL((k_relayout<E>), dim3(blocks), dim3(256), 0, st, src, src_lay, dst, dst_lay, d);
    return hipGetLastError();
}
template hipError_t launch_relayout<cx<double>>(const cx<double>*, int, cx<double>*, int, int, const int*, int,
                                                hipStream_t);
template hipError_t launch_relayout<cx<float>>(const cx<float>*, int, cx<float>*, int, int, const int*, int,
                                               hipStream_t);
template hipError_t launch_relayout<double>(const double*, int, double*, int, int, const int*, int, hipStream_t);
template hipError_t launch_relayout<float>(const float*, int, float*, int, int, const int*, int, hipStream_t);

hipError_t launch_pencil_flags(const cx<double>* plane, int64_t pencils, int n, unsigned char* flag,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_pencil_flags, dim3((unsigned)((pencils + 3) / 4)), dim3(256), 0, st, plane, pencils, n, flag);
    return hipGetLastError();
}

static inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <typename T>
hipError_t launch_zero(cx<T>* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_zero<T>), grid1(n), dim3(256), 0, st, p, n);
    return hipGetLastError();
}
template hipError_t launch_zero<float>(cx<float>*, int64_t, hipStream_t);
template hipError_t launch_zero<double>(cx<double>*, int64_t, hipStream_t);

hipError_t launch_rhs(const Geom& g, const cx<double>* sp, const cx<double>* su, const double* rhobar,
                      const cx<double>* q, int physical, double il1s, double il2s, cx<double>* y64,
                      cx<float>* y32, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs, grid1(g.ncell * (g.ndim + 1)), dim3(256), 0, st, g, sp, su, rhobar, q, physical,
                       il1s, il2s, y64, y32);
    return hipGetLastError();
}

hipError_t launch_scale_in(const Geom& g, const cx<double>* p, const cx<double>* u, double sl1, double sl2,
                           cx<double>* x, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_in, grid1(g.ncell * (g.ndim + 1)), dim3(256), 0, st, g, p, u, sl1, sl2, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_unscale(const Geom& g, const cx<T>* x, double il1s, double il2s, cx<double>* p,
                          cx<double>* u, hipStream_t st) {
    hipLaunchKernelGGL((k_unscale<T>), grid1(g.ncell * (g.ndim + 1)), dim3(256), 0, st, g, x, il1s, il2s, p, u);
    return hipGetLastError();
}
template hipError_t launch_unscale<float>(const Geom&, const cx<float>*, double, double, cx<double>*,
                                          cx<double>*, hipStream_t);
template hipError_t launch_unscale<double>(const Geom&, const cx<double>*, double, double, cx<double>*,
                                           cx<double>*, hipStream_t);

hipError_t launch_residual_out(const Geom& g, const cx<double>* r, double sl1, double sl2, cx<double>* rp,
                               cx<double>* ru, hipStream_t st) {
    hipLaunchKernelGGL(k_residual_out, grid1(g.ncell * (g.ndim + 1)), dim3(256), 0, st, g, r, sl1, sl2, rp, ru);
    return hipGetLastError();
}

hipError_t launch_convert(const cx<double>* r, cx<float>* y32, int64_t n, const Ctl* c, hipStream_t st) {
    hipLaunchKernelGGL(k_convert, grid1(n), dim3(256), 0, st, r, y32, n, c);
    return hipGetLastError();
}

hipError_t launch_accumulate(cx<double>* x, const cx<float>* d, int64_t n, const Ctl* c, hipStream_t st) {
    hipLaunchKernelGGL(k_accumulate, grid1(n), dim3(256), 0, st, x, d, n, c);
    return hipGetLastError();
}

hipError_t launch_gradient(const Geom& g, const double* c, const double* rho, const double* alpha,
                           const cx<double>* q, const double* const* gcen, const double* const* gst, double gmax,
                           double omega, const cx<double>* sp, const cx<double>* su, const cx<double>* p,
                           const cx<double>* u, const cx<double>* lp, const cx<double>* lu, double* gc,
                           double* grho, double* galpha, int collocated, hipStream_t st) {
    hipLaunchKernelGGL(k_gradient, grid1(g.ncell), dim3(256), 0, st, g, c, rho, alpha, q, gcen[0], gcen[1],
                       gcen[2], gst[0], gst[1], gst[2], gmax, omega, sp, su, p, u, lp, lu, gc, grho, galpha,
                       collocated);
    return hipGetLastError();
}

}  // namespace cbs