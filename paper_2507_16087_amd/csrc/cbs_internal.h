// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbs {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

// Partial-sum pairs one reduction block folds.
constexpr int kReduceChunk = 1024;

// Per-solve control block in device memory.  Written by the reduction
// kernels, read by every pass kernel (a finished slot's passes exit at once)
// and polled by the host every few iterations.
struct Ctl {
    int done;            // 0 running, 1 converged, 2 iteration cap, 3 diverged
    int iter;            // iterations of the current CBS run
    int max_iter;        // cap of the current CBS run
    int grow;            // consecutive iterations with relative update > 2
    double tol;          // relative-update tolerance of the current run
    double rel_update;   // last relative update
    double xnorm2;       // |x_{k+1}|^2 of the last iteration
    double res2;         // |r|^2 of the last residual evaluation
    double rhs2;         // |y|^2 of the last residual evaluation
    double scale;        // |r| used by the refinement convert/accumulate kernels
    int res_done;        // residual evaluations since reset
    int arrive;          // blocks of the current reduction that have finished
};

enum Done { RUNNING = 0, CONVERGED = 1, CAPPED = 2, DIVERGED = 3 };

// Everything one solve's kernels need, at working precision T.  Lives in
// device memory (one per slot); the kernels read it with scalar loads.
template <typename T>
struct Slot {
    cx<T>* x;             // state, F planes
    cx<T>* w;             // FFT work buffer, F planes (residual lands here)
    const cx<T>* y;       // right-hand side, F planes
    const T* rhobar;      // staggered density, ndim planes
    const cx<T>* q;       // 1 / (rho c_cx^2)
    const T* gc[3];       // layer profile r^2 at cell centres, per axis
    const T* gs[3];       // layer profile r^2 at staggered points, per axis
    const T* kv[3];       // wavenumbers per axis, FFT order
    const cx<T>* sh[3];   // exp(i k dx / 2) per axis
    const cx<T>* tw[3];   // exp(-2 pi i m / n) per axis
    T omega, gmax, nu;
    T a1re, a1im, a2re, a2im;
    T inv_lam1, inv_lam2; // 1 / lam
    T s;                  // sqrt(lam1 lam2)
    T inv_ntot;           // 1 / prod(n)
    cx<T> al1, al2;       // a + lam
    cx<T> ca;             // lam1 / al1
    cx<T> can;            // lam1 / al1 / prod(n)
    cx<T> cp;             // lam2 * al1
    cx<T> al12;           // al1 * al2
    int adjoint;
    int pad;
    // sparse right-hand side (kernels built with a sparse-y flag only): the
    // velocity rows of y are zero and its pressure row is read only on
    // pencils whose flag is set (one byte per pencil of a field plane)
    const unsigned char* ypen;
    Ctl* ctl;
    double* partials;     // 2 doubles per work-group of the last pass
    double* chunks;       // 2 doubles per block of the reduction
};


struct Geom {
    int ndim;
    int n[3];             // unused axes = 1
    int64_t ncell;
};

}  // namespace cbs
