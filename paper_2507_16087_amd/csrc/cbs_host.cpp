// Host runtime of the iterative Born solver: medium planner (Algorithm 1
// preprocessing), workspace layout, iteration drivers (plain FP64 and FP32
// with FP64 iterative refinement), and the C ABI of include/cbs.h.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <cstdio>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "cbs.h"
#include "cbs_internal.h"

using cd = std::complex<double>;

namespace cbs {
// kernels (cbs_kernels.hip)
template <typename T>
hipError_t launch_pass(int kind, int mode, const Slot<T>* slots, int nslots, const Geom& g, int axis, int n,
                       int pcols, bool wide, int variant, hipStream_t st, int l0 = 0, int lw = 0);
template <typename T>
hipError_t launch_reduce(bool cbs_mode, const Slot<T>* slots, int nparts, int nslots, hipStream_t st);
hipError_t launch_ctl_reset(Ctl* c, int max_iter, double tol, hipStream_t st);
hipError_t launch_ctl_clear(Ctl* c, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
hipError_t launch_pencil_flags(const cx<double>* plane, int64_t pencils, int n, unsigned char* flag,
                               hipStream_t st);
template <typename T>
hipError_t launch_zero(cx<T>* p, int64_t n, hipStream_t st);
hipError_t launch_rhs(const Geom& g, const cx<double>* sp, const cx<double>* su, const double* rhobar,
                      const cx<double>* q, int physical, double il1s, double il2s, cx<double>* y64,
                      cx<float>* y32, hipStream_t st);
hipError_t launch_scale_in(const Geom& g, const cx<double>* p, const cx<double>* u, double sl1, double sl2,
                           cx<double>* x, hipStream_t st);
template <typename T>
hipError_t launch_unscale(const Geom& g, const cx<T>* x, double il1s, double il2s, cx<double>* p,
                          cx<double>* u, hipStream_t st);
hipError_t launch_residual_out(const Geom& g, const cx<double>* r, double sl1, double sl2, cx<double>* rp,
                               cx<double>* ru, hipStream_t st);
hipError_t launch_convert(const cx<double>* r, cx<float>* y32, int64_t n, const Ctl* c, hipStream_t st);
hipError_t launch_accumulate(cx<double>* x, const cx<float>* d, int64_t n, const Ctl* c, hipStream_t st);
hipError_t launch_gradient(const Geom& g, const double* c, const double* rho, const double* alpha,
                           const cx<double>* q, const double* const* gcen, const double* const* gst, double gmax,
                           double omega, const cx<double>* sp, const cx<double>* su, const cx<double>* p,
                           const cx<double>* u, const cx<double>* lp, const cx<double>* lu, double* gc,
                           double* grho, double* galpha, int collocated, hipStream_t st);
int plan_tpc(int n, bool wide);
bool plan_has_wide(int n);
bool plan_has_variants(int n);
enum { MODE_CBS = 0, MODE_APPLY = 1 };
}  // namespace cbs

using namespace cbs;

#define HIPOK(expr)                                   \
    do {                                              \
        if ((expr) != hipSuccess) return CBS_E_DEVICE; \
    } while (0)

namespace {

// Axis lengths with a compiled FFT plan: every 2^a 3^b in [4, 512].
bool size_supported(int64_t n) { return n >= 4 && n <= 512 && plan_tpc((int)n, false) > 0; }

// ----------------------------------------------------------- pass config --
// The passes of one iteration, and the column-tile width of each.
struct Pass {
    int kind;    // 0 contiguous forward (+prologue), 1 contiguous inverse (+epilogue),
                 // 2 strided forward, 3 strided inverse, 4 axis-0 propagator,
                 // 6 operator alone on the spectrum (1-D grids)
    int axis;
    int n;
    int pcols;
    bool wide;
    int variant;   // propagator: LDS regions (bits 0-1: 0 one, 1 per field, 2 two);
                   // last-axis inverse: prefetch (0 none, 1 x y medium, 2 x medium);
                   // strided and propagator: bit 2 = unpadded column tile
};

struct PassSet {
    Pass p[5];
    int count;
    int nparts;    // partial-sum slots written by the last pass
    // 3-D: the middle passes (forward axis 1, propagator, inverse axis 1) run
    // block by block over this many equal ranges of last-axis columns, so a
    // block's data is still in the memory-side cache for its next pass
    int cblocks = 1;
};

int pow2_floor_div(int64_t total, int cap) {
    int p = 1;
    while (p * 2 <= cap && total % (p * 2) == 0) p *= 2;
    return p;
}

// The default pass along the contiguous last axis (kind 0 forward with the
// prologue, 1 inverse with the epilogue).
Pass contig_pass(const Geom& g, int kind, bool fp64) {
    Pass p{};
    p.kind = kind;
    p.axis = g.ndim - 1;
    p.n = g.n[p.axis];
    p.wide = false;
    const int tpc = std::max(1, plan_tpc(p.n, false));
    const int64_t pencils = g.ncell / g.n[p.axis];
    // whole pencils per work-group: at most 256 threads and ~40 KiB of LDS
    const size_t pencil_lds = (size_t)(p.n + p.n / 16) * (fp64 ? 16 : 8);
    const int lds_cap = (int)std::max<size_t>(1, (40 * 1024) / pencil_lds);
    p.pcols = pow2_floor_div(pencils, std::min(256 / tpc, lds_cap));
    return p;
}

PassSet make_passes(const Geom& g, bool fp64) {
    PassSet ps{};
    const int last = g.ndim - 1;
    const int pstr = fp64 ? 8 : 16;   // columns per strided tile: 128-byte row segments
    auto strided = [&](int kind, int axis, bool wide) {
        Pass p{};
        p.kind = kind;
        p.axis = axis;
        p.n = g.n[axis];
        p.wide = wide && plan_has_wide(p.n);
        const int tpc = std::max(1, plan_tpc(p.n, p.wide));   // every length here has a plan
        p.pcols = pow2_floor_div(g.n[last], std::min(pstr, 256 / tpc));
        return p;
    };
    auto contig = [&](int kind) { return contig_pass(g, kind, fp64); };
    int k = 0;
    ps.p[k++] = contig(0);
    if (g.ndim == 3) ps.p[k++] = strided(2, 1, false);
    if (g.ndim == 1) {
        // one axis, the contiguous one: the operator alone on the spectrum
        Pass p{};
        p.kind = 6;
        p.axis = 0;
        p.n = g.n[0];
        p.pcols = 1;
        ps.p[k++] = p;
    } else {
        ps.p[k++] = strided(4, 0, fp64);
    }
    if (g.ndim == 3) ps.p[k++] = strided(3, 1, false);
    ps.p[k++] = contig(1);
    ps.count = k;
    const Pass& lp = ps.p[k - 1];
    ps.nparts = (int)((g.ndim + 1) * (g.ncell / ((int64_t)lp.n * lp.pcols)));
    return ps;
}

// ------------------------------------------------------------- planner --
// Periodic distance of position t from the interior [L, n-1-L], over L+1/2.
double layer_frac(double t, int n, int L) {
    if (L <= 0) return 0.0;
    const double lo = L, hi = n - 1 - L;
    if (t >= lo && t <= hi) return 0.0;
    const double d = (t > hi) ? std::min(t - hi, lo + n - t) : std::min(lo - t, t + n - hi);
    return d / (L + 0.5);
}

struct Circle {
    double x, y, r;
};

bool in_circle(const Circle& c, double px, double py) {
    return std::hypot(px - c.x, py - c.y) <= c.r * (1.0 + 1e-12) + 1e-300;
}

Circle from2(double ax, double ay, double bx, double by) {
    return {(ax + bx) * 0.5, (ay + by) * 0.5, 0.5 * std::hypot(ax - bx, ay - by)};
}

Circle from3(double ax, double ay, double bx, double by, double cx_, double cy_) {
    const double ux = bx - ax, uy = by - ay, vx = cx_ - ax, vy = cy_ - ay;
    const double d = 2.0 * (ux * vy - uy * vx);
    if (std::fabs(d) < 1e-300) {
        Circle c1 = from2(ax, ay, bx, by), c2 = from2(ax, ay, cx_, cy_), c3 = from2(bx, by, cx_, cy_);
        Circle best = c1;
        if (c2.r > best.r) best = c2;
        if (c3.r > best.r) best = c3;
        return best;
    }
    const double u2 = ux * ux + uy * uy, v2 = vx * vx + vy * vy;
    const double ox = (vy * u2 - uy * v2) / d, oy = (ux * v2 - vx * u2) / d;
    return {ax + ox, ay + oy, std::hypot(ox, oy)};
}

// Run body(lo, hi) over [0, n) in contiguous chunks, one per host thread (at
// most 16), the first on the calling thread.  Chunks are returned in order by
// the caller's own bookkeeping, so results do not depend on the thread count.
// An exception thrown in any chunk (an allocation failing) is rethrown on
// the calling thread after every chunk has finished.
template <class F>
void parallel_chunks(int64_t n, int nchunks, F&& body) {
    std::vector<std::exception_ptr> err(nchunks);
    auto run = [&](int c) {
        try {
            body(c, n * c / nchunks, n * (c + 1) / nchunks);
        } catch (...) {
            err[c] = std::current_exception();
        }
    };
    std::vector<std::thread> pool;
    for (int c = 1; c < nchunks; ++c) pool.emplace_back(run, c);
    run(0);
    for (std::thread& t : pool) t.join();
    for (const std::exception_ptr& e : err)
        if (e) std::rethrow_exception(e);
}

int plan_threads(int64_t n) {
    if (n < (1 << 16)) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::min<unsigned>(16, std::max(1u, hw));
}

// Smallest circle enclosing the points (Welzl's incremental algorithm).  A
// pre-filter first drops the points that cannot lie on the circle: those
// strictly inside the octagon spanned by the extreme points in eight
// directions (interior to the convex hull), copies of an octagon vertex (the
// vertex itself is kept once), and points exactly on an octagon edge strictly
// between its ends (on a chord of the enclosing disk, hence inside it).  The
// last two matter for media with many equal values (a water background puts
// millions of cells on one point) or values on a line (every cell outside
// the absorbing layer has a purely imaginary velocity diagonal).  The scans
// run on host threads; ties and the order of the kept points are those of a
// serial scan.
Circle min_circle(const std::vector<cd>& pts) {
    const size_t n = pts.size();
    if (n == 0) return {0, 0, 0};
    const double dirs[8][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
    const int nt = plan_threads((int64_t)n);
    std::vector<std::array<size_t, 8>> cext(nt);
    std::vector<std::array<double, 8>> cbest(nt);
    parallel_chunks((int64_t)n, nt, [&](int c, int64_t lo, int64_t hi) {
        std::array<size_t, 8>& ext = cext[c];
        std::array<double, 8>& best = cbest[c];
        ext.fill(0);
        best.fill(-INFINITY);
        for (int64_t i = lo; i < hi; ++i)
            for (int d = 0; d < 8; ++d) {
                const double v = pts[i].real() * dirs[d][0] + pts[i].imag() * dirs[d][1];
                if (v > best[d]) {
                    best[d] = v;
                    ext[d] = (size_t)i;
                }
            }
    });
    size_t ext[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double best[8];
    for (int d = 0; d < 8; ++d) best[d] = -INFINITY;
    for (int c = 0; c < nt; ++c)   // chunk order: the first maximum wins, as in one scan
        for (int d = 0; d < 8; ++d)
            if (cbest[c][d] > best[d]) {
                best[d] = cbest[c][d];
                ext[d] = cext[c][d];
            }
    std::vector<cd> poly;
    for (int d = 0; d < 8; ++d) {
        const cd p = pts[ext[d]];
        if (poly.empty() || std::abs(poly.back() - p) > 0) poly.push_back(p);
    }
    while (poly.size() > 1 && std::abs(poly.front() - poly.back()) == 0) poly.pop_back();
    const size_t m = poly.size();
    std::vector<std::vector<cd>> ckeep(nt);
    parallel_chunks((int64_t)n, nt, [&](int c, int64_t lo, int64_t hi) {
        std::vector<cd>& keep = ckeep[c];
        for (int64_t i = lo; i < hi; ++i) {
            const cd p = pts[i];
            bool inside = m >= 3, drop = false;
            for (size_t e = 0; e < m && !drop; ++e) {
                const cd a = poly[e], b = poly[(e + 1) % m];
                if (p == a) {
                    drop = true;   // a vertex value: the vertex is kept below
                    break;
                }
                const double ex = b.real() - a.real(), ey = b.imag() - a.imag();
                const double px = p.real() - a.real(), py = p.imag() - a.imag();
                const double cr = ex * py - ey * px;
                if (cr == 0.0) {
                    const double t = ex * px + ey * py, len2 = ex * ex + ey * ey;
                    if (t > 0.0 && t < len2) drop = true;   // on the edge, between its ends
                }
                // counter-clockwise octagon: interior points are strictly left of
                // every edge, by a relative margin of 1e-9
                if (!(cr > 0.0 && cr * cr > 1e-18 * (ex * ex + ey * ey) * (px * px + py * py))) inside = false;
            }
            if (!drop && !inside) keep.push_back(p);
        }
    });
    std::vector<cd> keep(poly.begin(), poly.end());
    for (const std::vector<cd>& k : ckeep) keep.insert(keep.end(), k.begin(), k.end());
    // deterministic shuffle
    uint64_t s = 0x2545F4914F6CDD1Dull;
    for (size_t i = keep.size(); i > 1; --i) {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        std::swap(keep[i - 1], keep[s % i]);
    }
    Circle c{keep[0].real(), keep[0].imag(), 0.0};
    for (size_t i = 1; i < keep.size(); ++i) {
        if (in_circle(c, keep[i].real(), keep[i].imag())) continue;
        c = {keep[i].real(), keep[i].imag(), 0.0};
        for (size_t j = 0; j < i; ++j) {
            if (in_circle(c, keep[j].real(), keep[j].imag())) continue;
            c = from2(keep[i].real(), keep[i].imag(), keep[j].real(), keep[j].imag());
            for (size_t k = 0; k < j; ++k)
                if (!in_circle(c, keep[k].real(), keep[k].imag()))
                    c = from3(keep[i].real(), keep[i].imag(), keep[j].real(), keep[j].imag(), keep[k].real(),
                              keep[k].imag());
        }
    }
    return c;
}

double median(std::vector<double>& v) {
    const size_t n = v.size(), h = n / 2;
    std::nth_element(v.begin(), v.begin() + h, v.end());
    const double hi = v[h];
    if (n % 2) return hi;
    const double lo = *std::max_element(v.begin(), v.begin() + h);
    return 0.5 * (lo + hi);
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace

// ---------------------------------------------------------------- medium --
// Per-pass GPU time accounting: HIP event pairs around every pass launch,
// harvested whenever the driver synchronises.  Groups: 0 FP32 CBS, 1 FP64
// CBS, 2 FP64 residual; slots 0..4 = passes in launch order, 5 = reduction.
struct PassTiming {
    bool on = false;
    int mask = 0x3f;   // pass slots bracketed with events (bit k = slot k)
    std::vector<hipEvent_t> ev;
    std::vector<int> tag;
    size_t used = 0;
    double ms[3][6] = {};
    int64_t cnt[3][6] = {};
};

struct cbs_medium_s {
    PassTiming timing;
    Geom g;
    cbs_grid grid;
    double gmax, beta, nu;
    cd a1, a2;
    double lam1, lam2;
    PassSet ps64, ps32;
    bool tuned64 = false, tuned32 = false;
    std::mutex tune_mu;   // first solves on several threads tune the pass sets once
    void* dev = nullptr;
    // device pointers into dev
    double *rhobar64, *c64, *rho64, *alpha64;
    cx<double>* q64;
    float* rhobar32;
    cx<float>* q32;
    double *gc64[3], *gs64[3], *kv64[3];
    cx<double> *sh64[3], *tw64[3];
    float *gc32[3], *gs32[3], *kv32[3];
    cx<float> *sh32[3], *tw32[3];
};

namespace {

template <typename T>
struct Tables;
template <>
struct Tables<double> {
    static void fill(const cbs_medium_s* m, Slot<double>& s) {
        s.rhobar = m->rhobar64;
        s.q = m->q64;
        for (int d = 0; d < 3; ++d) {
            s.gc[d] = m->gc64[d];
            s.gs[d] = m->gs64[d];
            s.kv[d] = m->kv64[d];
            s.sh[d] = m->sh64[d];
            s.tw[d] = m->tw64[d];
        }
    }
};
template <>
struct Tables<float> {
    static void fill(const cbs_medium_s* m, Slot<float>& s) {
        s.rhobar = m->rhobar32;
        s.q = m->q32;
        for (int d = 0; d < 3; ++d) {
            s.gc[d] = m->gc32[d];
            s.gs[d] = m->gs32[d];
            s.kv[d] = m->kv32[d];
            s.sh[d] = m->sh32[d];
            s.tw[d] = m->tw32[d];
        }
    }
};

template <typename T>
cx<T> tocx(cd v) {
    return {(T)v.real(), (T)v.imag()};
}

template <typename T>
Slot<T> make_slot(const cbs_medium_s* m, cx<T>* x, cx<T>* w, const cx<T>* y, Ctl* ctl, double* partials,
                  int adjoint, double* chunks) {
    Slot<T> s{};
    s.x = x;
    s.w = w;
    s.y = y;
    Tables<T>::fill(m, s);
    s.omega = (T)m->grid.omega;
    s.gmax = (T)m->gmax;
    s.nu = (T)m->nu;
    s.a1re = (T)m->a1.real();
    s.a1im = (T)m->a1.imag();
    s.a2re = (T)m->a2.real();
    s.a2im = (T)m->a2.imag();
    s.inv_lam1 = (T)(1.0 / m->lam1);
    s.inv_lam2 = (T)(1.0 / m->lam2);
    s.s = (T)std::sqrt(m->lam1 * m->lam2);
    s.inv_ntot = (T)(1.0 / (double)m->g.ncell);
    const cd al1 = m->a1 + m->lam1, al2 = m->a2 + m->lam2;
    s.al1 = tocx<T>(al1);
    s.al2 = tocx<T>(al2);
    s.ca = tocx<T>(m->lam1 / al1);
    s.can = tocx<T>(m->lam1 / al1 / (double)m->g.ncell);
    s.cp = tocx<T>(m->lam2 * al1);
    s.al12 = tocx<T>(al1 * al2);
    s.adjoint = adjoint;
    s.ctl = ctl;
    s.partials = partials;
    s.chunks = chunks;
    return s;
}

hipError_t timing_begin(PassTiming& t, int tag, hipStream_t st) {
    if (t.used + 2 > t.ev.size()) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            t.ev.push_back(e);
            t.tag.push_back(0);
        }
    }
    t.tag[t.used] = tag;
    return hipEventRecord(t.ev[t.used], st);
}

hipError_t timing_end(PassTiming& t, hipStream_t st) {
    hipError_t r = hipEventRecord(t.ev[t.used + 1], st);
    t.used += 2;
    return r;
}

// Fold recorded event pairs into the per-pass totals (stream already synced).
// Launches that found their slot finished return at once; they are left out
// (shorter than a quarter of the longest launch of the same pass in the batch).
void timing_harvest(PassTiming& t) {
    std::vector<float> dur(t.used / 2, -1.f);
    float mx[24] = {};
    for (size_t i = 0; i + 1 < t.used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]) == hipSuccess) {
            dur[i / 2] = ms;
            mx[t.tag[i]] = std::max(mx[t.tag[i]], ms);
        }
    }
    for (size_t i = 0; i + 1 < t.used; i += 2) {
        const float ms = dur[i / 2];
        if (ms < 0.f || ms < 0.25f * mx[t.tag[i]]) continue;
        const int g = t.tag[i] / 8, k = t.tag[i] % 8;
        t.ms[g][k] += ms;
        t.cnt[g][k] += 1;
    }
    t.used = 0;
}

// One CBS iteration (MODE_CBS) or one residual evaluation (MODE_APPLY) for
// nslots same-shape slots.  A CBS iteration ends with the fused pass that
// updates x and already transforms the next iteration's B x + y along the
// last axis, so only the first iteration of a run (start) launches the
// stand-alone prologue pass.
// Passes of one iteration for a set of same-shape slots.  In CBS mode the
// stand-alone prologue pass runs only over `starts` (slots whose CBS run
// begins with this iteration); the other passes run over `all`.
// yflags: OR-ed into the variant of the last-axis launches (16: the slots'
// right-hand side is sparse, see Slot::ypen).
template <typename T>
hipError_t run_passes_set(const Geom& g, PassTiming* tp, const PassSet& ps, int mode, const Slot<T>* all,
                          int nall, const Slot<T>* starts, int nstart, hipStream_t st, int yflags = 0) {
    const bool timed = tp && tp->on;
    const int group = mode == MODE_APPLY ? 2 : (sizeof(T) == 8 ? 1 : 0);
    auto launch = [&](int i, int l0, int lw) -> hipError_t {
        const Pass& p = ps.p[i];
        const bool pro = mode == MODE_CBS && i == 0;
        const int kind = (mode == MODE_CBS && i == ps.count - 1) ? 5 : p.kind;
        const int slot = i == ps.count - 1 ? 4 : i;
        const bool ev = timed && ((tp->mask >> slot) & 1);
        if (ev && timing_begin(*tp, group * 8 + slot, st) != hipSuccess) return hipErrorUnknown;
        const int variant = (p.kind == 0 || p.kind == 1) ? (p.variant | yflags) : p.variant;
        hipError_t e = launch_pass<T>(kind, mode, pro ? starts : all, pro ? nstart : nall, g, p.axis, p.n, p.pcols,
                                      p.wide, variant, st, l0, lw);
        if (e != hipSuccess) return e;
        if (ev && timing_end(*tp, st) != hipSuccess) return hipErrorUnknown;
        return hipSuccess;
    };
    hipError_t e;
    if (!(mode == MODE_CBS && nstart == 0) && (e = launch(0, 0, 0)) != hipSuccess) return e;
    if (ps.count == 5 && ps.cblocks > 1) {
        // middle passes block by block over the last-axis columns
        const int lw = g.n[g.ndim - 1] / ps.cblocks;
        for (int b = 0; b < ps.cblocks; ++b)
            for (int i = 1; i <= 3; ++i)
                if ((e = launch(i, b * lw, lw)) != hipSuccess) return e;
    } else {
        for (int i = 1; i < ps.count - 1; ++i)
            if ((e = launch(i, 0, 0)) != hipSuccess) return e;
    }
    if ((e = launch(ps.count - 1, 0, 0)) != hipSuccess) return e;
    const bool ev = timed && ((tp->mask >> 5) & 1);
    if (ev && timing_begin(*tp, group * 8 + 5, st) != hipSuccess) return hipErrorUnknown;
    e = launch_reduce<T>(mode == MODE_CBS, all, ps.nparts, nall, st);
    if (e != hipSuccess) return e;
    if (ev && timing_end(*tp, st) != hipSuccess) return hipErrorUnknown;
    return hipSuccess;
}

template <typename T>
hipError_t run_passes(cbs_medium_s* m, const PassSet& ps, int mode, const Slot<T>* dslots, int nslots,
                      hipStream_t st, bool start = true, int yflags = 0) {
    return run_passes_set<T>(m->g, &m->timing, ps, mode, dslots, nslots, dslots, start ? nslots : 0, st, yflags);
}

// ------------------------------------------------------------ autotuner --
// For every pass of an iteration, time the candidate FFT plans (the default
// radix split, and the wider one with fewer elements per thread where it
// exists) at every admissible tile width on the caller's workspace, and keep
// the fastest.  Winners are cached per (shape, precision) for the process, so
// every medium of one shape runs the same kernels (results of a solve do not
// depend on which other solves ran first).  CBS_AUTOTUNE=0 keeps the defaults.
struct TuneKey {
    int ndim, n0, n1, n2, fp64, prop_variant, last_variant, strided_variant, cblocks;
    bool operator<(const TuneKey& o) const {
        return std::tie(ndim, n0, n1, n2, fp64, prop_variant, last_variant, strided_variant, cblocks) <
               std::tie(o.ndim, o.n0, o.n1, o.n2, o.fp64, o.prop_variant, o.last_variant, o.strided_variant,
                        o.cblocks);
    }
};

// Variants a pass kind may take: the propagator's LDS layouts (0 one tile
// reused field by field, 1 one region per field, 2 two regions with fields in
// pairs); the last-axis inverse pass's prefetch (0 none, 1 x, y and medium,
// 2 x and medium).  Bit 2 of a strided or propagator variant drops the
// one-element row padding of the column tile.
std::vector<int> variants_of(int kind, int n) {
    const bool all = plan_has_variants(n);   // else only variant 0 is compiled
    if (kind == 4) return all ? std::vector<int>{0, 1, 2, 4, 5, 6} : std::vector<int>{0, 4};
    if (kind == 1) return all ? std::vector<int>{0, 1, 2} : std::vector<int>{0};
    if (kind == 2 || kind == 3) return {0, 4};
    return {0};
}

// CBS_PROP_VARIANT pins the propagator pass, CBS_LAST_VARIANT the last-axis
// inverse pass and CBS_STRIDED_VARIANT the strided passes to one of their
// variants; unset, all compete.
// The raw pin of a pass kind from the environment (-1 unset), before any
// check against a length's plans: part of the tuning cache key.
int env_pin(int kind) {
    const char* name = kind == 4 ? "CBS_PROP_VARIANT" : (kind == 1 ? "CBS_LAST_VARIANT" : "CBS_STRIDED_VARIANT");
    const char* e = std::getenv(name);
    if (!e || e[0] < '0' || e[0] > '9') return -1;
    char* end = nullptr;
    const long v = std::strtol(e, &end, 10);
    return (end && *end == 0 && v < 64) ? (int)v : -1;
}

int forced_variant(int kind, int n) {
    const char* name = kind == 4 ? "CBS_PROP_VARIANT" : (kind == 1 ? "CBS_LAST_VARIANT" : "CBS_STRIDED_VARIANT");
    const char* e = std::getenv(name);
    if (!e || e[0] < '0' || e[0] > '9') return -1;
    char* end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (!end || *end != 0) return -1;
    for (int ok : variants_of(kind, n))
        if (ok == v) return (int)v;
    return -1;
}
std::mutex g_tune_mu;
std::map<TuneKey, PassSet> g_tune_cache;

// CBS_COLUMN_BLOCKS pins the block count of the middle passes (1, 2, 4, 8).
int forced_cblocks() {
    const char* e = std::getenv("CBS_COLUMN_BLOCKS");
    if (!e) return -1;
    const int v = std::atoi(e);
    return (v == 1 || v == 2 || v == 4 || v == 8) ? v : -1;
}

// Blocks must split the last axis into whole column tiles of every middle pass.
bool cblocks_valid(const Geom& g, const PassSet& ps, int blocks) {
    if (ps.count != 5) return blocks == 1;
    const int nl = g.n[g.ndim - 1];
    if (nl % blocks) return false;
    for (int i = 1; i <= 3; ++i)
        if ((nl / blocks) % ps.p[i].pcols) return false;
    return true;
}

std::vector<Pass> pass_candidates(const Geom& g, const Pass& base, bool fp64) {
    std::vector<Pass> out;
    const int last = g.ndim - 1;
    const bool lastaxis = base.kind == 0 || base.kind == 1;
    for (int wide = 0; wide < 2; ++wide) {
        if (wide && !plan_has_wide(base.n)) continue;
        const int tpc = plan_tpc(base.n, wide != 0);
        int cap = 256 / tpc;
        int64_t total;
        if (lastaxis) {
            total = g.ncell / g.n[last];
            const size_t pencil_lds = (size_t)(base.n + base.n / 16) * (fp64 ? 16 : 8);
            cap = std::min<int>(cap, (int)std::max<size_t>(1, (64 * 1024) / pencil_lds));
        } else {
            total = g.n[last];
            cap = std::min(cap, fp64 ? 16 : 32);
        }
        // a pinned column-block count needs tiles that split each block evenly
        const int pin = forced_cblocks();
        const bool middle = g.ndim == 3 && (base.kind == 2 || base.kind == 3 || base.kind == 4);
        const int lw = (middle && pin > 1 && g.n[last] % pin == 0) ? g.n[last] / pin : 0;
        for (int pc = 1; pc <= cap; pc *= 2) {
            if (total % pc) break;
            if (lw && lw % pc) break;
            if (pc * tpc < 64 && pc * 2 <= cap && total % (pc * 2) == 0 && !(lw && lw % (pc * 2)))
                continue;   // at least a wave
            Pass p = base;
            p.wide = wide != 0;
            p.pcols = pc;
            const int pinned = forced_variant(base.kind, base.n);
            for (int v : variants_of(base.kind, base.n)) {
                if (pinned >= 0 && v != pinned) continue;
                p.variant = v;
                out.push_back(p);
            }
        }
    }
    return out;
}

template <typename T>
float time_pass(cbs_medium_s* m, int kind, const Slot<T>* dslot, const Pass& p, hipStream_t st) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.f;
    }
    float ms = -1.f;
    auto once = [&]() {
        return launch_pass<T>(kind, MODE_CBS, dslot, 1, m->g, p.axis, p.n, p.pcols, p.wide, p.variant, st) ==
               hipSuccess;
    };
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) ok = once();
    const int reps = 6;
    ok = ok && hipEventRecord(a, st) == hipSuccess;
    for (int i = 0; i < reps && ok; ++i) ok = once();
    ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, a, b) == hipSuccess) ms /= reps;
    else ms = -1.f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// Time of one iteration's passes with the middle chain run block by block.
template <typename T>
float time_middle(cbs_medium_s* m, const PassSet& ps, int blocks, const Slot<T>* dslot, hipStream_t st) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.f;
    }
    const int lw = m->g.n[m->g.ndim - 1] / blocks;
    // one steady-state iteration: the middle chain block by block, then the
    // fused last-axis pass, so each block count is timed with the cache
    // contents the solve gives it (the forward axis-1 pass reads what the
    // fused pass wrote)
    auto once = [&]() {
        for (int bl = 0; bl < blocks; ++bl)
            for (int i = 1; i <= 3; ++i) {
                const Pass& p = ps.p[i];
                if (launch_pass<T>(p.kind, MODE_CBS, dslot, 1, m->g, p.axis, p.n, p.pcols, p.wide, p.variant, st,
                                   bl * lw, lw) != hipSuccess)
                    return false;
            }
        const Pass& lp = ps.p[ps.count - 1];
        return launch_pass<T>(5, MODE_CBS, dslot, 1, m->g, lp.axis, lp.n, lp.pcols, lp.wide, lp.variant, st) ==
               hipSuccess;
    };
    // the fastest of three rounds of four iterations
    float ms = -1.f;
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) ok = once();
    const int reps = 4;
    for (int round = 0; round < 3 && ok; ++round) {
        ok = hipEventRecord(a, st) == hipSuccess;
        for (int i = 0; i < reps && ok; ++i) ok = once();
        ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
        float t = 0.f;
        if (ok && hipEventElapsedTime(&t, a, b) == hipSuccess) {
            t /= reps;
            if (ms < 0.f || t < ms) ms = t;
        } else {
            ok = false;
        }
    }
    if (!ok) ms = -1.f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

template <typename T>
cbs_status tune_set(cbs_medium_s* m, PassSet& ps, Slot<T>* dslot, cx<T>* x, cx<T>* w, cx<T>* y, Ctl* ctl,
                    double* part, double* chunks, hipStream_t st) {
    const int64_t nf = (int64_t)(m->g.ndim + 1) * m->g.ncell;
    HIPOK(launch_zero<T>(x, nf, st));
    HIPOK(launch_zero<T>(w, nf, st));
    HIPOK(launch_zero<T>(y, nf, st));
    HIPOK(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
    HIPOK(launch_ctl_reset(ctl, INT32_MAX, -1.0, st));   // candidates never see a finished slot
    Slot<T> h = make_slot<T>(m, x, w, y, ctl, part, 0, chunks);
    HIPOK(hipMemcpyAsync(dslot, &h, sizeof(h), hipMemcpyHostToDevice, st));
    HIPOK(hipStreamSynchronize(st));
    const bool fp64 = sizeof(T) == 8;
    for (int i = 0; i < ps.count; ++i) {
        const int kind = (i == ps.count - 1) ? 5 : ps.p[i].kind;
        float best = -1.f;
        Pass pick = ps.p[i];
        if (ps.p[i].kind == 6) continue;   // one configuration
        for (const Pass& c : pass_candidates(m->g, ps.p[i], fp64)) {
            const float t = time_pass<T>(m, kind, dslot, c, st);
            if (t > 0.f && (best < 0.f || t < best)) {
                best = t;
                pick = c;
            }
        }
        ps.p[i] = pick;
    }
    // block count of the middle passes, timed as a chain with the plans above
    ps.cblocks = 1;
    if (ps.count == 5) {
        const int pin = forced_cblocks();
        float best = -1.f;
        for (int blocks : {1, 2, 4, 8}) {
            if ((pin > 0 && blocks != pin) || !cblocks_valid(m->g, ps, blocks)) continue;
            const float t = time_middle<T>(m, ps, blocks, dslot, st);
            if (t > 0.f && (best < 0.f || t < best)) {
                best = t;
                ps.cblocks = blocks;
            }
        }
    }
    const Pass& lp = ps.p[ps.count - 1];
    ps.nparts = (int)((m->g.ndim + 1) * (m->g.ncell / ((int64_t)lp.n * lp.pcols)));
    return CBS_OK;
}

struct Layout {
    size_t off_slot64, off_ctl64, off_part64, off_chunk64, off_x64, off_w64, off_y64, off_ypen64;
    size_t off_slot32, off_ctl32, off_part32, off_chunk32, off_d32, off_w32, off_y32;
    size_t total;
};

Layout layout_for(const Geom& g, int prec) {
    Layout L{};
    const size_t nf = (size_t)(g.ndim + 1) * g.ncell;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.off_slot64 = take(sizeof(Slot<double>));
    L.off_ctl64 = take(sizeof(Ctl));
    // partial sums: one pair per work-group of the last pass, at any tile width
    const size_t maxparts = (size_t)(g.ndim + 1) * (g.ncell / g.n[g.ndim - 1]);
    const size_t maxchunks = (maxparts + kReduceChunk - 1) / kReduceChunk;
    L.off_part64 = take(sizeof(double) * 2 * maxparts);
    L.off_chunk64 = take(sizeof(double) * 2 * maxchunks);
    L.off_x64 = take(nf * sizeof(cx<double>));
    L.off_w64 = take(nf * sizeof(cx<double>));
    L.off_y64 = take(nf * sizeof(cx<double>));
    L.off_ypen64 = take((size_t)(g.ncell / g.n[g.ndim - 1]));   // pencil flags of a sparse y
    if (prec == CBS_FP32_REFINED) {
        L.off_slot32 = take(sizeof(Slot<float>));
        L.off_ctl32 = take(sizeof(Ctl));
        L.off_part32 = take(sizeof(double) * 2 * maxparts);
        L.off_chunk32 = take(sizeof(double) * 2 * maxchunks);
        L.off_d32 = take(nf * sizeof(cx<float>));
        L.off_w32 = take(nf * sizeof(cx<float>));
        L.off_y32 = take(nf * sizeof(cx<float>));
    }
    L.total = o;
    return L;
}

Layout layout_for(const cbs_medium_s* m, int prec) { return layout_for(m->g, prec); }

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}


bool autotune_enabled() {
    const char* e = std::getenv("CBS_AUTOTUNE");
    return !(e && e[0] == '0');
}

// ------------------------------------------------------- tune file --
// CBS_TUNE_FILE names a text file that keeps tuned pass sets across
// processes, one line per (device architecture, shape, precision, pins):
//   cbs-tune-v1 <arch> <ndim> <n0> <n1> <n2> <fp64> <4 pins> <count> <cblocks>
//               then <kind> <axis> <n> <pcols> <wide> <variant> per pass.
// A line is used only if it describes a valid set for the shape; a process
// that tunes a key the file lacks appends its line.  Unset: nothing is read
// or written.
const char* tune_file() {
    const char* e = std::getenv("CBS_TUNE_FILE");
    return (e && e[0]) ? e : nullptr;
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');   // feature suffixes do not change the plans
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string tune_prefix(const std::string& arch, const TuneKey& k) {
    std::ostringstream o;
    o << "cbs-tune-v1 " << arch << ' ' << k.ndim << ' ' << k.n0 << ' ' << k.n1 << ' ' << k.n2 << ' ' << k.fp64
      << ' ' << k.prop_variant << ' ' << k.last_variant << ' ' << k.strided_variant << ' ' << k.cblocks;
    return o.str();
}

// A pass set read from the file must match the shape's pass sequence and
// stay inside what the tuner itself could have chosen.
bool plausible(const Geom& g, const PassSet& def, const PassSet& ps) {
    if (ps.count != def.count) return false;
    const int last = g.ndim - 1;
    for (int i = 0; i < ps.count; ++i) {
        const Pass &p = ps.p[i], &d = def.p[i];
        if (p.kind != d.kind || p.axis != d.axis || p.n != d.n) return false;
        if (p.kind == 6 && (p.pcols != 1 || p.wide || p.variant)) return false;
        if (p.wide && !plan_has_wide(p.n)) return false;
        const int tpc = plan_tpc(p.n, p.wide);
        if (p.pcols < 1 || (p.pcols & (p.pcols - 1)) || tpc <= 0 || p.pcols * tpc > 256) return false;
        const int64_t total = (p.kind == 0 || p.kind == 1) ? g.ncell / g.n[last] : g.n[last];
        if (total % p.pcols) return false;
        const std::vector<int> vs = variants_of(p.kind, p.n);
        if (std::find(vs.begin(), vs.end(), p.variant) == vs.end()) return false;
    }
    return ps.cblocks == 1 || ((ps.cblocks == 2 || ps.cblocks == 4 || ps.cblocks == 8) && cblocks_valid(g, ps, ps.cblocks));
}

bool tune_file_lookup(const Geom& g, const TuneKey& key, const PassSet& def, PassSet* out) {
    const char* path = tune_file();
    if (!path) return false;
    const std::string arch = device_arch();
    if (arch.empty()) return false;
    const std::string prefix = tune_prefix(arch, key) + ' ';
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char buf[1024];
    while (!found && std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (line.compare(0, prefix.size(), prefix) != 0) continue;
        std::istringstream in(line.substr(prefix.size()));
        PassSet ps{};
        if (!(in >> ps.count >> ps.cblocks) || ps.count < 1 || ps.count > 5) continue;
        bool ok = true;
        for (int i = 0; i < ps.count && ok; ++i) {
            Pass& p = ps.p[i];
            int wide = 0;
            ok = static_cast<bool>(in >> p.kind >> p.axis >> p.n >> p.pcols >> wide >> p.variant);
            p.wide = wide != 0;
        }
        if (!ok || !plausible(g, def, ps)) continue;
        const Pass& lp = ps.p[ps.count - 1];
        ps.nparts = (int)((g.ndim + 1) * (g.ncell / ((int64_t)lp.n * lp.pcols)));
        *out = ps;
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_file_append(const TuneKey& key, const PassSet& ps) {
    const char* path = tune_file();
    if (!path) return;
    const std::string arch = device_arch();
    if (arch.empty()) return;
    std::ostringstream o;
    o << tune_prefix(arch, key) << ' ' << ps.count << ' ' << ps.cblocks;
    for (int i = 0; i < ps.count; ++i) {
        const Pass& p = ps.p[i];
        o << ' ' << p.kind << ' ' << p.axis << ' ' << p.n << ' ' << p.pcols << ' ' << (p.wide ? 1 : 0) << ' '
          << p.variant;
    }
    o << '\n';
    FILE* f = std::fopen(path, "a");
    if (!f) return;   // the file is an optimisation: a failed write changes nothing else
    const std::string line = o.str();
    (void)std::fwrite(line.data(), 1, line.size(), f);
    std::fclose(f);
}

// Tune the pass sets this precision uses, on the caller's workspace (its
// contents are scratch here), or take them from the process cache.
cbs_status ensure_tuned(cbs_medium_s* m, int prec, void* ws, hipStream_t st) {
    // Pass sets change only here, under the medium's lock, and only until
    // they are marked tuned; solves read them after this call returns.
    std::lock_guard<std::mutex> mlk(m->tune_mu);
    if (!autotune_enabled()) {
        if (m->tuned64 && m->tuned32) return CBS_OK;
        for (PassSet* ps : {&m->ps64, &m->ps32}) {
            for (int i = 0; i < ps->count; ++i)
                if (ps->p[i].kind >= 1 && ps->p[i].kind <= 4)
                    ps->p[i].variant = std::max(0, forced_variant(ps->p[i].kind, ps->p[i].n));
            const int blocks = forced_cblocks();
            ps->cblocks = (blocks > 0 && cblocks_valid(m->g, *ps, blocks)) ? blocks : 1;
        }
        m->tuned64 = m->tuned32 = true;
        return CBS_OK;
    }
    const Layout L = layout_for(m, prec);
    const Geom& g = m->g;
    for (int fp64 = 1; fp64 >= 0; --fp64) {
        if (!fp64 && prec != CBS_FP32_REFINED) continue;
        bool& done = fp64 ? m->tuned64 : m->tuned32;
        if (done) continue;
        PassSet& ps = fp64 ? m->ps64 : m->ps32;
        const TuneKey key{g.ndim, g.n[0], g.n[1], g.n[2], fp64, env_pin(4), env_pin(1), env_pin(2),
                          forced_cblocks()};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it == g_tune_cache.end()) {
                PassSet from_file;
                if (tune_file_lookup(g, key, make_passes(g, fp64 != 0), &from_file))
                    it = g_tune_cache.emplace(key, from_file).first;
            }
            if (it != g_tune_cache.end()) {
                ps = it->second;
                done = true;
                continue;
            }
        }
        cbs_status cs;
        if (fp64)
            cs = tune_set<double>(m, ps, at<Slot<double>>(ws, L.off_slot64), at<cx<double>>(ws, L.off_x64),
                                  at<cx<double>>(ws, L.off_w64), at<cx<double>>(ws, L.off_y64),
                                  at<Ctl>(ws, L.off_ctl64), at<double>(ws, L.off_part64),
                                  at<double>(ws, L.off_chunk64), st);
        else
            cs = tune_set<float>(m, ps, at<Slot<float>>(ws, L.off_slot32), at<cx<float>>(ws, L.off_d32),
                                 at<cx<float>>(ws, L.off_w32), at<cx<float>>(ws, L.off_y32),
                                 at<Ctl>(ws, L.off_ctl32), at<double>(ws, L.off_part32),
                                 at<double>(ws, L.off_chunk32), st);
        if (cs != CBS_OK) return cs;
        done = true;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = ps;
        tune_file_append(key, ps);
    }
    return CBS_OK;
}

cbs_status validate_grid(const cbs_grid* g) {
    if (!g) return CBS_E_INVALID;
    if (g->ndim < 1 || g->ndim > 3) return CBS_E_UNSUPPORTED;
    if (!(g->dx > 0) || !(g->omega > 0) || !std::isfinite(g->dx) || !std::isfinite(g->omega))
        return CBS_E_INVALID;
    for (int d = 0; d < g->ndim; ++d) {
        if (!size_supported(g->n[d])) return CBS_E_UNSUPPORTED;
        if (g->pml_cells < 0 || 2 * (int64_t)g->pml_cells >= g->n[d]) return CBS_E_INVALID;
    }
    const double beta = g->beta == 0 ? 0.95 : g->beta;
    const double nu = g->nu == 0 ? 0.9 : g->nu;
    if (!(beta > 0) || !std::isfinite(beta)) return CBS_E_INVALID;
    if (!(nu > 0) || !std::isfinite(nu)) return CBS_E_INVALID;
    if (g->shift_rule != 0 && g->shift_rule != 1) return CBS_E_INVALID;
    if (g->collocated != 0 && g->collocated != 1) return CBS_E_INVALID;
    return CBS_OK;
}

// Host part of the medium planner (Algorithm 1 preprocessing): layer
// profiles, q and the staggered densities, the diagonal values, the shifts
// a1, a2 (minimum enclosing circle or median) and the scales lam1, lam2
// (eq. C).  Inputs are validated host arrays of g.ncell values.
struct HostPlan {
    std::vector<double> prof_c[3], prof_s[3];   // layer r^2 at centres / staggered points
    std::vector<cd> q;                          // (1 - 2i alpha c / omega) / (rho c^2)
    std::vector<double> rb;                     // staggered densities, ndim planes
    cd a1, a2;
    double lam1 = 0, lam2 = 0, gmax = 0, beta = 0, nu = 0;
};

void plan_medium(const cbs_grid& grid, const Geom& g, const double* hc, const double* hr, const double* ha,
                 HostPlan* hp) {
    hp->gmax = grid.pml_gamma_max > 0 ? grid.pml_gamma_max : grid.omega;
    hp->beta = grid.beta == 0 ? 0.95 : grid.beta;
    hp->nu = grid.nu == 0 ? 0.9 : grid.nu;
    const double w = grid.omega;
    const int L = grid.pml_cells;
    const int D = g.ndim;
    const int64_t N = g.ncell;

    // per-axis layer profiles r^2 at centres and staggered points
    std::vector<double>* prof_c = hp->prof_c;
    std::vector<double>* prof_s = hp->prof_s;
    for (int d = 0; d < 3; ++d) {
        prof_c[d].assign(g.n[d], 0.0);
        prof_s[d].assign(g.n[d], 0.0);
        if (d >= D) continue;
        const double half = grid.collocated ? 0.0 : 0.5;   // velocity rows' position
        for (int i = 0; i < g.n[d]; ++i) {
            const double rc = layer_frac(i, g.n[d], L), rs = layer_frac(i + half, g.n[d], L);
            prof_c[d][i] = rc * rc;
            prof_s[d][i] = rs * rs;
        }
    }
    // q, staggered density, diagonal values for the shifts
    std::vector<cd>& q = hp->q;
    std::vector<double>& rb = hp->rb;
    q.assign(N, cd());
    rb.assign((size_t)D * N, 0.0);
    std::vector<cd> Du((size_t)D * N), Dp(N);
    int64_t stride[3] = {1, 1, 1};
    for (int d = D - 2; d >= 0; --d) stride[d] = stride[d + 1] * g.n[d + 1];
    const int nt = plan_threads(N);
    parallel_chunks(N, nt, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            int ix[3] = {0, 0, 0};
            int64_t r = i;
            for (int d = D - 1; d >= 0; --d) {
                ix[d] = (int)(r % g.n[d]);
                r /= g.n[d];
            }
            const double cc = hc[i];
            q[i] = cd(1.0, -2.0 * ha[i] * cc / w) / (hr[i] * cc * cc);
            double gsum = 0.0;
            for (int d = 0; d < D; ++d) gsum += prof_c[d][ix[d]];
            const double gam = hp->gmax * gsum;
            Dp[i] = cd(gam, w) * q[i];
            for (int e = 0; e < D; ++e) {
                const int64_t nb = (ix[e] + 1 < g.n[e]) ? i + stride[e] : i - (int64_t)(g.n[e] - 1) * stride[e];
                const double rbar = grid.collocated ? hr[i] : 0.5 * (hr[i] + hr[nb]);
                rb[(size_t)e * N + i] = rbar;
                double gs = 0.0;
                for (int d = 0; d < D; ++d) gs += (d == e) ? prof_s[d][ix[d]] : prof_c[d][ix[d]];
                Du[(size_t)e * N + i] = cd(rbar * (hp->gmax * gs), rbar * w);
            }
        }
    });
    // shifts (Algorithm 1 preprocessing) and scales (eq. C)
    if (grid.shift_rule == 1) {
        std::vector<double> v(Du.size());
        for (size_t i = 0; i < Du.size(); ++i) v[i] = Du[i].real();
        const double r1 = median(v);
        for (size_t i = 0; i < Du.size(); ++i) v[i] = Du[i].imag();
        hp->a1 = cd(r1, median(v));
        v.resize(Dp.size());
        for (size_t i = 0; i < Dp.size(); ++i) v[i] = Dp[i].real();
        const double r2 = median(v);
        for (size_t i = 0; i < Dp.size(); ++i) v[i] = Dp[i].imag();
        hp->a2 = cd(r2, median(v));
    } else {
        Circle c1 = min_circle(Du), c2 = min_circle(Dp);
        hp->a1 = cd(c1.x, c1.y);
        hp->a2 = cd(c2.x, c2.y);
    }
    // max |D - a| (a maximum: exact whatever the chunking)
    auto max_dist = [&](const std::vector<cd>& v, cd a) {
        const int nc = plan_threads((int64_t)v.size());
        std::vector<double> cm(nc, 0.0);
        parallel_chunks((int64_t)v.size(), nc, [&](int c, int64_t lo, int64_t hi) {
            double r = 0.0;
            for (int64_t i = lo; i < hi; ++i) r = std::max(r, std::abs(v[i] - a));
            cm[c] = r;
        });
        return *std::max_element(cm.begin(), cm.end());
    };
    const double r1 = max_dist(Du, hp->a1), r2 = max_dist(Dp, hp->a2);
    hp->lam1 = std::max(r1, 1e-3 * std::abs(hp->a1)) / hp->beta;
    hp->lam2 = std::max(r2, 1e-3 * std::abs(hp->a2)) / hp->beta;
}

// Host copies of c, rho, alpha (from host or device memory), checked:
// c > 0, rho > 0, alpha >= 0, all finite.
cbs_status host_medium(const Geom& g, const double* c, const double* rho, const double* alpha, int32_t ptr_kind,
                       hipStream_t st, std::vector<double>* hc, std::vector<double>* hr, std::vector<double>* ha) {
    const int64_t N = g.ncell;
    hc->resize(N);
    hr->resize(N);
    ha->resize(N);
    if (ptr_kind == CBS_PTR_DEVICE) {
        HIPOK(hipMemcpyAsync(hc->data(), c, N * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPOK(hipMemcpyAsync(hr->data(), rho, N * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPOK(hipMemcpyAsync(ha->data(), alpha, N * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPOK(hipStreamSynchronize(st));
    } else {
        std::memcpy(hc->data(), c, N * sizeof(double));
        std::memcpy(hr->data(), rho, N * sizeof(double));
        std::memcpy(ha->data(), alpha, N * sizeof(double));
    }
    for (int64_t i = 0; i < N; ++i) {
        const double cv = (*hc)[i], rv = (*hr)[i], av = (*ha)[i];
        if (!(cv > 0) || !(rv > 0) || !(av >= 0) || !std::isfinite(cv) || !std::isfinite(rv) || !std::isfinite(av))
            return CBS_E_INVALID;
    }
    return CBS_OK;
}

Geom geom_of(const cbs_grid& grid) {
    Geom g{};
    g.ndim = grid.ndim;
    g.ncell = 1;
    for (int d = 0; d < 3; ++d) g.n[d] = d < grid.ndim ? (int)grid.n[d] : 1;
    for (int d = 0; d < grid.ndim; ++d) g.ncell *= g.n[d];
    return g;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Frees a partly built medium (device block included) unless released.
struct MediumOwner {
    cbs_medium_s* m;
    ~MediumOwner() {
        if (!m) return;
        if (m->dev) (void)hipFree(m->dev);
        delete m;
    }
};

cbs_status create_medium(const cbs_grid* grid, const double* c, const double* rho, const double* alpha,
                                int32_t ptr_kind, void* hip_stream, cbs_medium* out) {
    cbs_status vs = validate_grid(grid);
    if (vs != CBS_OK) return vs;
    if (!c || !rho || !alpha) return CBS_E_INVALID;
    if (ptr_kind != CBS_PTR_HOST && ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom g = geom_of(*grid);
    const int D = g.ndim;
    const int64_t N = g.ncell;
    std::vector<double> hc, hr, ha;
    cbs_status hs = host_medium(g, c, rho, alpha, ptr_kind, st, &hc, &hr, &ha);
    if (hs != CBS_OK) return hs;

    cbs_medium_s* m = new (std::nothrow) cbs_medium_s();
    if (!m) return CBS_E_NOMEM;
    MediumOwner own{m};
    m->g = g;
    m->grid = *grid;
    const double dx = grid->dx;
    HostPlan hp;
    plan_medium(*grid, g, hc.data(), hr.data(), ha.data(), &hp);
    m->gmax = hp.gmax;
    m->a1 = hp.a1;
    m->a2 = hp.a2;
    m->lam1 = hp.lam1;
    m->lam2 = hp.lam2;
    m->beta = hp.beta;
    m->nu = hp.nu;
    const std::vector<double>* prof_c = hp.prof_c;
    const std::vector<double>* prof_s = hp.prof_s;
    const std::vector<cd>& q = hp.q;
    const std::vector<double>& rb = hp.rb;

    // device block: FP64 medium, FP32 medium, physical fields, axis tables
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t o_rb64 = take(sizeof(double) * D * N), o_q64 = take(sizeof(cx<double>) * N);
    const size_t o_rb32 = take(sizeof(float) * D * N), o_q32 = take(sizeof(cx<float>) * N);
    const size_t o_c = take(sizeof(double) * N), o_r = take(sizeof(double) * N), o_a = take(sizeof(double) * N);
    size_t o_tab64[3][5], o_tab32[3][5];
    for (int d = 0; d < 3; ++d) {
        for (int t = 0; t < 3; ++t) o_tab64[d][t] = take(sizeof(double) * g.n[d]);
        for (int t = 3; t < 5; ++t) o_tab64[d][t] = take(sizeof(cx<double>) * g.n[d]);
        for (int t = 0; t < 3; ++t) o_tab32[d][t] = take(sizeof(float) * g.n[d]);
        for (int t = 3; t < 5; ++t) o_tab32[d][t] = take(sizeof(cx<float>) * g.n[d]);
    }
    if (hipMalloc(&m->dev, off) != hipSuccess) {
        m->dev = nullptr;
        return CBS_E_NOMEM;
    }
    char* base = static_cast<char*>(m->dev);
    m->rhobar64 = reinterpret_cast<double*>(base + o_rb64);
    m->q64 = reinterpret_cast<cx<double>*>(base + o_q64);
    m->rhobar32 = reinterpret_cast<float*>(base + o_rb32);
    m->q32 = reinterpret_cast<cx<float>*>(base + o_q32);
    m->c64 = reinterpret_cast<double*>(base + o_c);
    m->rho64 = reinterpret_cast<double*>(base + o_r);
    m->alpha64 = reinterpret_cast<double*>(base + o_a);

    // Upload: the FP64 planes straight from the planner's arrays
    // (std::complex<double> has the two-double layout of cx<double>), the FP32
    // planes converted on host threads, the small per-axis tables staged in one
    // buffer; one synchronisation at the end.
    std::vector<float> rb32((size_t)D * N);
    std::vector<cx<float>> q32(N);
    parallel_chunks(N, plan_threads(N), [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            q32[i] = {(float)q[i].real(), (float)q[i].imag()};
            for (int e = 0; e < D; ++e) rb32[(size_t)e * N + i] = (float)rb[(size_t)e * N + i];
        }
    });
    const size_t tab0 = o_tab64[0][0];   // the tables follow the planes
    std::vector<char> tabs(off - tab0, 0);
    auto tput = [&](size_t o, const void* src, size_t bytes) { std::memcpy(tabs.data() + (o - tab0), src, bytes); };
    for (int d = 0; d < 3; ++d) {
        const int n = g.n[d];
        std::vector<double> kv(n);
        std::vector<cx<double>> sh(n), tw(n);
        std::vector<float> kv32(n), gc32(n), gs32(n);
        std::vector<cx<float>> sh32(n), tw32(n);
        for (int j = 0; j < n; ++j) {
            const int fidx = (j < (n + 1) / 2) ? j : j - n;   // FFT order
            kv[j] = d < D ? 2.0 * M_PI * fidx / (n * dx) : 0.0;
            sh[j] = {std::cos(kv[j] * dx / 2), std::sin(kv[j] * dx / 2)};
            if (grid->collocated) {
                // collocated derivative symbol i k, Nyquist bin zeroed, no shift
                if (n % 2 == 0 && j == n / 2) kv[j] = 0.0;
                sh[j] = {1.0, 0.0};
            }
            const double ang = -2.0 * M_PI * (double)j / (double)n;
            tw[j] = {std::cos(ang), std::sin(ang)};
            kv32[j] = (float)kv[j];
            sh32[j] = {(float)sh[j].re, (float)sh[j].im};
            tw32[j] = {(float)tw[j].re, (float)tw[j].im};
            gc32[j] = (float)prof_c[d][j];
            gs32[j] = (float)prof_s[d][j];
        }
        tput(o_tab64[d][0], prof_c[d].data(), sizeof(double) * n);
        tput(o_tab64[d][1], prof_s[d].data(), sizeof(double) * n);
        tput(o_tab64[d][2], kv.data(), sizeof(double) * n);
        tput(o_tab64[d][3], sh.data(), sizeof(cx<double>) * n);
        tput(o_tab64[d][4], tw.data(), sizeof(cx<double>) * n);
        tput(o_tab32[d][0], gc32.data(), sizeof(float) * n);
        tput(o_tab32[d][1], gs32.data(), sizeof(float) * n);
        tput(o_tab32[d][2], kv32.data(), sizeof(float) * n);
        tput(o_tab32[d][3], sh32.data(), sizeof(cx<float>) * n);
        tput(o_tab32[d][4], tw32.data(), sizeof(cx<float>) * n);
        m->gc64[d] = reinterpret_cast<double*>(base + o_tab64[d][0]);
        m->gs64[d] = reinterpret_cast<double*>(base + o_tab64[d][1]);
        m->kv64[d] = reinterpret_cast<double*>(base + o_tab64[d][2]);
        m->sh64[d] = reinterpret_cast<cx<double>*>(base + o_tab64[d][3]);
        m->tw64[d] = reinterpret_cast<cx<double>*>(base + o_tab64[d][4]);
        m->gc32[d] = reinterpret_cast<float*>(base + o_tab32[d][0]);
        m->gs32[d] = reinterpret_cast<float*>(base + o_tab32[d][1]);
        m->kv32[d] = reinterpret_cast<float*>(base + o_tab32[d][2]);
        m->sh32[d] = reinterpret_cast<cx<float>*>(base + o_tab32[d][3]);
        m->tw32[d] = reinterpret_cast<cx<float>*>(base + o_tab32[d][4]);
    }
    static_assert(sizeof(cd) == sizeof(cx<double>), "complex layouts differ");
    hipError_t ce = hipSuccess;
    auto h2d = [&](size_t o, const void* src, size_t bytes) {
        if (ce == hipSuccess) ce = hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, st);
    };
    h2d(o_rb64, rb.data(), sizeof(double) * D * N);
    h2d(o_q64, q.data(), sizeof(cx<double>) * N);
    h2d(o_rb32, rb32.data(), sizeof(float) * D * N);
    h2d(o_q32, q32.data(), sizeof(cx<float>) * N);
    h2d(o_c, hc.data(), sizeof(double) * N);
    h2d(o_r, hr.data(), sizeof(double) * N);
    h2d(o_a, ha.data(), sizeof(double) * N);
    h2d(tab0, tabs.data(), tabs.size());
    if (ce != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return CBS_E_DEVICE;
    m->ps64 = make_passes(g, true);
    m->ps32 = make_passes(g, false);
    own.m = nullptr;
    *out = m;
    return CBS_OK;
}

// No C++ exception crosses the C ABI: a failed host allocation is
// CBS_E_NOMEM, anything else CBS_E_INVALID.
template <class F>
cbs_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return CBS_E_NOMEM;
    } catch (...) {
        return CBS_E_INVALID;
    }
}

}  // namespace

extern "C" {

cbs_status cbs_create_medium(const cbs_grid* grid, const double* c, const double* rho, const double* alpha,
                             int32_t ptr_kind, void* hip_stream, cbs_medium* out) {
    if (!out) return CBS_E_INVALID;
    *out = nullptr;
    return guarded([&] { return create_medium(grid, c, rho, alpha, ptr_kind, hip_stream, out); });
}

cbs_status cbs_destroy_medium(cbs_medium m) {
    if (!m) return CBS_E_INVALID;
    for (hipEvent_t e : m->timing.ev) (void)hipEventDestroy(e);
    if (m->dev) (void)hipFree(m->dev);
    delete m;
    return CBS_OK;
}

cbs_status cbs_medium_scalars(cbs_medium m, double out[8]) {
    if (!m || !out) return CBS_E_INVALID;
    out[0] = m->a1.real();
    out[1] = m->a1.imag();
    out[2] = m->a2.real();
    out[3] = m->a2.imag();
    out[4] = m->lam1;
    out[5] = m->lam2;
    out[6] = m->beta;
    out[7] = m->nu;
    return CBS_OK;
}

cbs_status cbs_plan_scalars(const cbs_grid* grid, const double* c, const double* rho, const double* alpha,
                            double out[8]) {
    if (!out) return CBS_E_INVALID;
    cbs_status vs = validate_grid(grid);
    if (vs != CBS_OK) return vs;
    if (!c || !rho || !alpha) return CBS_E_INVALID;
    return guarded([&] {
        const Geom g = geom_of(*grid);
        std::vector<double> hc, hr, ha;
        cbs_status hs = host_medium(g, c, rho, alpha, CBS_PTR_HOST, nullptr, &hc, &hr, &ha);
        if (hs != CBS_OK) return hs;
        HostPlan hp;
        plan_medium(*grid, g, hc.data(), hr.data(), ha.data(), &hp);
        const double v[8] = {hp.a1.real(), hp.a1.imag(), hp.a2.real(), hp.a2.imag(),
                             hp.lam1,      hp.lam2,      hp.beta,      hp.nu};
        std::memcpy(out, v, sizeof v);
        return CBS_OK;
    });
}

cbs_status cbs_set_scalars(cbs_medium m, const double in[6]) {
    if (!m || !in) return CBS_E_INVALID;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(in[i])) return CBS_E_INVALID;
    if (!(in[4] > 0) || !(in[5] > 0)) return CBS_E_INVALID;
    m->a1 = cd(in[0], in[1]);
    m->a2 = cd(in[2], in[3]);
    m->lam1 = in[4];
    m->lam2 = in[5];
    return CBS_OK;
}

cbs_status cbs_workspace_bytes(cbs_medium m, int32_t prec, int32_t batch, size_t* bytes) {
    if (!m || !bytes || batch < 1) return CBS_E_INVALID;
    if (prec != CBS_FP64 && prec != CBS_FP32_REFINED) return CBS_E_INVALID;
    *bytes = layout_for(m, prec).total * (size_t)batch;
    return CBS_OK;
}

}  // extern "C"

namespace {

// Stage host or device sources into device complex128 arrays.  Host data is
// copied into `stage` (at least (ndim + 1) * ncell complex128).
cbs_status stage_sources(const cbs_medium_s* m, const void* s_p, const void* s_u, int ptr_kind, cx<double>* stage,
                         const cx<double>** dsp, const cx<double>** dsu, hipStream_t st) {
    const int64_t N = m->g.ncell;
    const int D = m->g.ndim;
    if (ptr_kind == CBS_PTR_DEVICE) {
        *dsp = static_cast<const cx<double>*>(s_p);
        *dsu = static_cast<const cx<double>*>(s_u);
        return CBS_OK;
    }
    // stage layout: [u planes D*N][p N]
    if (s_u) HIPOK(hipMemcpyAsync(stage, s_u, sizeof(cx<double>) * D * N, hipMemcpyHostToDevice, st));
    HIPOK(hipMemcpyAsync(stage + (size_t)D * N, s_p, sizeof(cx<double>) * N, hipMemcpyHostToDevice, st));
    HIPOK(hipStreamSynchronize(st));
    *dsp = stage + (size_t)D * N;
    *dsu = s_u ? stage : nullptr;
    return CBS_OK;
}

// Write (u, p) = C^{-1/2} x to the caller's outputs.
template <typename T>
cbs_status write_outputs(const cbs_medium_s* m, const cx<T>* x, void* p_out, void* u_out, int ptr_kind,
                         cx<double>* stage, hipStream_t st) {
    const int64_t N = m->g.ncell;
    const int D = m->g.ndim;
    const double il1s = 1.0 / std::sqrt(m->lam1), il2s = 1.0 / std::sqrt(m->lam2);
    if (ptr_kind == CBS_PTR_DEVICE) {
        HIPOK(launch_unscale<T>(m->g, x, il1s, il2s, static_cast<cx<double>*>(p_out),
                                static_cast<cx<double>*>(u_out), st));
        HIPOK(hipStreamSynchronize(st));
        return CBS_OK;
    }
    HIPOK(launch_unscale<T>(m->g, x, il1s, il2s, stage + (size_t)D * N, stage, st));
    if (p_out) HIPOK(hipMemcpyAsync(p_out, stage + (size_t)D * N, sizeof(cx<double>) * N, hipMemcpyDeviceToHost, st));
    if (u_out) HIPOK(hipMemcpyAsync(u_out, stage, sizeof(cx<double>) * D * N, hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    return CBS_OK;
}

cbs_status read_ctl(cbs_medium_s* m, const Ctl* d, Ctl* h, hipStream_t st) {
    HIPOK(hipMemcpyAsync(h, d, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    if (m->timing.on) timing_harvest(m->timing);
    return CBS_OK;
}

cbs_status solve_impl(cbs_medium m, const void* s_p, const void* s_u, const cbs_solve_opts* o, void* p_out,
                      void* u_out, void* ws, size_t wsb, cbs_solve_info* info, void* hip_stream, int adjoint) {
    const double t0 = now_s();
    if (!m || !s_p || !o || !p_out || !ws) return CBS_E_INVALID;
    if (o->prec != CBS_FP64 && o->prec != CBS_FP32_REFINED) return CBS_E_INVALID;
    if (o->ptr_kind != CBS_PTR_HOST && o->ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    if (o->rhs_kind != CBS_RHS_PHYSICAL && o->rhs_kind != CBS_RHS_EQUATION) return CBS_E_INVALID;
    if (!(o->tol >= 0) || o->max_iter < 1 || o->max_iter > 0x7fffffff) return CBS_E_INVALID;
    const Layout L = layout_for(m, o->prec);
    if (wsb < L.total) return CBS_E_NOMEM;
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom& g = m->g;
    const int64_t nf = (int64_t)(g.ndim + 1) * g.ncell;
    const int check = o->check_every > 0 ? o->check_every : 32;
    cbs_status ts = ensure_tuned(m, o->prec, ws, st);
    if (ts != CBS_OK) return ts;

    Slot<double>* dslot64 = at<Slot<double>>(ws, L.off_slot64);
    Ctl* ctl64 = at<Ctl>(ws, L.off_ctl64);
    cx<double>* x64 = at<cx<double>>(ws, L.off_x64);
    cx<double>* w64 = at<cx<double>>(ws, L.off_w64);
    cx<double>* y64 = at<cx<double>>(ws, L.off_y64);
    double* part64 = at<double>(ws, L.off_part64);

    // right-hand side y = C^{-1/2} s_hat (FP64)
    const cx<double>*dsp = nullptr, *dsu = nullptr;
    cbs_status cs = stage_sources(m, s_p, s_u, o->ptr_kind, w64, &dsp, &dsu, st);
    if (cs != CBS_OK) return cs;
    HIPOK(launch_rhs(g, dsp, dsu, m->rhobar64, m->q64, o->rhs_kind == CBS_RHS_PHYSICAL, 1.0 / std::sqrt(m->lam1),
                     1.0 / std::sqrt(m->lam2), y64, nullptr, st));
    HIPOK(launch_zero<double>(x64, nf, st));
    HIPOK(hipMemsetAsync(ctl64, 0, sizeof(Ctl), st));
    Slot<double> h64 = make_slot<double>(m, x64, w64, y64, ctl64, part64, adjoint, at<double>(ws, L.off_chunk64));
    // without a velocity source the FP64 right-hand side is sparse: zero
    // velocity rows and pressure sources on few pencils (point sources, a
    // bowl); the FP64 last-axis passes then read y only where it is non-zero
    int yflags = 0;
    if (!dsu) {
        unsigned char* ypen = at<unsigned char>(ws, L.off_ypen64);
        const int nl = g.n[g.ndim - 1];
        HIPOK(launch_pencil_flags(y64 + (size_t)g.ndim * g.ncell, g.ncell / nl, nl, ypen, st));
        h64.ypen = ypen;
        yflags = 16;
    }
    HIPOK(hipMemcpyAsync(dslot64, &h64, sizeof(h64), hipMemcpyHostToDevice, st));

    cbs_solve_info inf{};
    inf.rel_residual = -1.0;
    Ctl hc{};
    int status = CBS_NOT_CONVERGED;

    if (o->prec == CBS_FP64) {
        const bool by_res = o->stop_rule == CBS_STOP_RESIDUAL;
        HIPOK(launch_ctl_reset(ctl64, (int)o->max_iter, by_res ? -1.0 : o->tol, st));
        int64_t launched = 0;
        // the fused pass leaves the next iteration's transformed B x + y in w;
        // a residual evaluation reuses w, so the iteration after it restarts
        // from the stand-alone prologue pass
        bool start = true;
        while (true) {
            const int64_t chunk = std::min<int64_t>(check, o->max_iter - launched);
            for (int64_t k = 0; k < chunk; ++k) {
                HIPOK(run_passes<double>(m, m->ps64, MODE_CBS, dslot64, 1, st, start, yflags));
                start = false;
            }
            launched += chunk;
            if (by_res) {
                HIPOK(run_passes<double>(m, m->ps64, MODE_APPLY, dslot64, 1, st, true, yflags));
                inf.residual_evals++;
                start = true;
            }
            if ((cs = read_ctl(m, ctl64, &hc, st)) != CBS_OK) return cs;
            inf.iterations = hc.iter;
            inf.rel_update = hc.rel_update;
            if (by_res) {
                inf.rel_residual = hc.rhs2 > 0 ? std::sqrt(hc.res2 / hc.rhs2) : 0.0;
                if (!std::isfinite(inf.rel_residual)) {
                    status = CBS_E_DIVERGED;
                    break;
                }
                if (inf.rel_residual <= o->tol) {
                    status = CBS_OK;
                    break;
                }
            }
            if (hc.done == CONVERGED) {
                status = CBS_OK;
                break;
            }
            if (hc.done == DIVERGED) {
                status = CBS_E_DIVERGED;
                break;
            }
            if (hc.done == CAPPED || launched >= o->max_iter) {
                status = CBS_NOT_CONVERGED;
                break;
            }
        }
        if (status != CBS_E_DIVERGED) {
            cs = write_outputs<double>(m, x64, p_out, u_out, o->ptr_kind, w64, st);
            if (cs != CBS_OK) return cs;
        }
    } else {
        // FP32 inner CBS with FP64 residual and accumulation
        Slot<float>* dslot32 = at<Slot<float>>(ws, L.off_slot32);
        Ctl* ctl32 = at<Ctl>(ws, L.off_ctl32);
        cx<float>* d32 = at<cx<float>>(ws, L.off_d32);
        cx<float>* w32 = at<cx<float>>(ws, L.off_w32);
        cx<float>* y32 = at<cx<float>>(ws, L.off_y32);
        double* part32 = at<double>(ws, L.off_part32);
        HIPOK(hipMemsetAsync(ctl32, 0, sizeof(Ctl), st));
        Slot<float> h32 = make_slot<float>(m, d32, w32, y32, ctl32, part32, adjoint, at<double>(ws, L.off_chunk32));
        HIPOK(hipMemcpyAsync(dslot32, &h32, sizeof(h32), hipMemcpyHostToDevice, st));
        const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-3;
        const int max_outer = o->max_outer > 0 ? o->max_outer : 10000;
        const int64_t max_inner = o->max_inner > 0 ? o->max_inner : 256;
        // x64 = 0 so the first residual is y: evaluate it with the APPLY passes
        int64_t total = 0;
        for (int outer = 0;; ++outer) {
            HIPOK(run_passes<double>(m, m->ps64, MODE_APPLY, dslot64, 1, st, true, yflags));
            inf.residual_evals++;
            if ((cs = read_ctl(m, ctl64, &hc, st)) != CBS_OK) return cs;
            inf.rel_residual = hc.rhs2 > 0 ? std::sqrt(hc.res2 / hc.rhs2) : 0.0;
            inf.outer = outer;
            if (!std::isfinite(inf.rel_residual)) {
                status = CBS_E_DIVERGED;
                break;
            }
            if (inf.rel_residual <= o->tol) {
                status = CBS_OK;
                break;
            }
            if (outer >= max_outer || total >= o->max_iter) {
                status = CBS_NOT_CONVERGED;
                break;
            }
            HIPOK(launch_convert(w64, y32, nf, ctl64, st));
            HIPOK(launch_zero<float>(d32, nf, st));
            const int64_t cap = std::min<int64_t>(o->max_iter - total, max_inner);
            HIPOK(launch_ctl_reset(ctl32, (int)cap, inner_tol, st));
            Ctl ic{};
            int64_t launched = 0;
            while (true) {
                const int64_t chunk = std::min<int64_t>(check, cap - launched);
                for (int64_t k = 0; k < chunk; ++k)
                    HIPOK(run_passes<float>(m, m->ps32, MODE_CBS, dslot32, 1, st, launched + k == 0));
                launched += chunk;
                if ((cs = read_ctl(m, ctl32, &ic, st)) != CBS_OK) return cs;
                if (ic.done != RUNNING || launched >= cap) break;
            }
            total += ic.iter;
            inf.rel_update = ic.rel_update;
            if (ic.done == DIVERGED) {
                status = CBS_E_DIVERGED;
                break;
            }
            HIPOK(launch_accumulate(x64, d32, nf, ctl64, st));
        }
        inf.iterations = total;
        if (status != CBS_E_DIVERGED) {
            cs = write_outputs<double>(m, x64, p_out, u_out, o->ptr_kind, w64, st);
            if (cs != CBS_OK) return cs;
        }
    }
    inf.status = status;
    inf.seconds = now_s() - t0;
    if (info) *info = inf;
    return (cbs_status)status;
}

}  // namespace

namespace cbs {
// Body of cbs_residual.  no_alloc: the allocation-free entry point's path --
// no tuning (the pass set the medium holds is used as it stands: tuned by an
// earlier call, or the default plans) and the control block cleared by a
// kernel rather than a memset; nothing here allocates.
cbs_status residual_impl(cbs_medium m, const void* s_p, const void* s_u, const void* p, const void* u,
                         int32_t adjoint, int32_t rhs_kind, int32_t ptr_kind, double* rel_residual, void* r_p,
                         void* r_u, void* workspace, size_t ws_bytes, hipStream_t st, bool no_alloc) {
    if (!m || !s_p || !p || !workspace) return CBS_E_INVALID;
    if (ptr_kind != CBS_PTR_HOST && ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    if (rhs_kind != CBS_RHS_PHYSICAL && rhs_kind != CBS_RHS_EQUATION) return CBS_E_INVALID;
    const Layout L = layout_for(m, CBS_FP64);
    if (ws_bytes < L.total) return CBS_E_NOMEM;
    const Geom& g = m->g;
    const int64_t N = g.ncell;
    const int D = g.ndim;
    PassSet ps;
    if (no_alloc) {
        std::lock_guard<std::mutex> lk(m->tune_mu);
        ps = m->ps64;
    } else {
        cbs_status ts = guarded([&] { return ensure_tuned(m, CBS_FP64, workspace, st); });
        if (ts != CBS_OK) return ts;
        ps = m->ps64;
    }
    Slot<double>* dslot = at<Slot<double>>(workspace, L.off_slot64);
    Ctl* ctl = at<Ctl>(workspace, L.off_ctl64);
    cx<double>* x = at<cx<double>>(workspace, L.off_x64);
    cx<double>* w = at<cx<double>>(workspace, L.off_w64);
    cx<double>* y = at<cx<double>>(workspace, L.off_y64);
    double* part = at<double>(workspace, L.off_part64);
    // sources -> y (staged through w), fields -> x (staged through w)
    const cx<double>*dsp = nullptr, *dsu = nullptr;
    cbs_status cs = stage_sources(m, s_p, s_u, ptr_kind, w, &dsp, &dsu, st);
    if (cs != CBS_OK) return cs;
    HIPOK(launch_rhs(g, dsp, dsu, m->rhobar64, m->q64, rhs_kind == CBS_RHS_PHYSICAL, 1.0 / std::sqrt(m->lam1),
                     1.0 / std::sqrt(m->lam2), y, nullptr, st));
    const cx<double>*dp = nullptr, *du = nullptr;
    cs = stage_sources(m, p, u, ptr_kind, w, &dp, &du, st);
    if (cs != CBS_OK) return cs;
    HIPOK(launch_scale_in(g, dp, du, std::sqrt(m->lam1), std::sqrt(m->lam2), x, st));
    if (no_alloc) HIPOK(launch_ctl_clear(ctl, st));
    else HIPOK(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
    Slot<double> h = make_slot<double>(m, x, w, y, ctl, part, adjoint ? 1 : 0, at<double>(workspace, L.off_chunk64));
    HIPOK(hipMemcpyAsync(dslot, &h, sizeof(h), hipMemcpyHostToDevice, st));
    // the allocation-free path never records pass timing (its events would be
    // created on first use)
    HIPOK(run_passes_set<double>(g, no_alloc ? nullptr : &m->timing, ps, MODE_APPLY, dslot, 1, dslot, 1, st));
    Ctl hc{};
    if (no_alloc) {
        HIPOK(hipMemcpyAsync(&hc, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIPOK(hipStreamSynchronize(st));
    } else if ((cs = read_ctl(m, ctl, &hc, st)) != CBS_OK) {
        return cs;
    }
    if (rel_residual) *rel_residual = hc.rhs2 > 0 ? std::sqrt(hc.res2 / hc.rhs2) : 0.0;
    if (r_p || r_u) {
        const double sl1 = std::sqrt(m->lam1), sl2 = std::sqrt(m->lam2);
        if (ptr_kind == CBS_PTR_DEVICE) {
            HIPOK(launch_residual_out(g, w, sl1, sl2, static_cast<cx<double>*>(r_p), static_cast<cx<double>*>(r_u),
                                      st));
        } else {
            // x is free now: use it as the staging area
            HIPOK(launch_residual_out(g, w, sl1, sl2, x + (size_t)D * N, x, st));
            if (r_p) HIPOK(hipMemcpyAsync(r_p, x + (size_t)D * N, sizeof(cx<double>) * N, hipMemcpyDeviceToHost, st));
            if (r_u) HIPOK(hipMemcpyAsync(r_u, x, sizeof(cx<double>) * D * N, hipMemcpyDeviceToHost, st));
        }
        HIPOK(hipStreamSynchronize(st));
    }
    return CBS_OK;
}

// Bytes of device memory cbs_residual's kernels use beyond inputs and outputs.
size_t residual_workspace_bytes(cbs_medium m) { return layout_for(m, CBS_FP64).total; }
}  // namespace cbs

extern "C" {

cbs_status cbs_solve(cbs_medium m, const void* s_p, const void* s_u, const cbs_solve_opts* opts, void* p_out,
                     void* u_out, void* workspace, size_t ws_bytes, cbs_solve_info* info, void* hip_stream) {
    return guarded([&] { return solve_impl(m, s_p, s_u, opts, p_out, u_out, workspace, ws_bytes, info, hip_stream, 0); });
}

cbs_status cbs_solve_adjoint(cbs_medium m, const void* s_p, const void* s_u, const cbs_solve_opts* opts,
                             void* p_out, void* u_out, void* workspace, size_t ws_bytes, cbs_solve_info* info,
                             void* hip_stream) {
    return guarded([&] { return solve_impl(m, s_p, s_u, opts, p_out, u_out, workspace, ws_bytes, info, hip_stream, 1); });
}

cbs_status cbs_residual(cbs_medium m, const void* s_p, const void* s_u, const void* p, const void* u,
                        int32_t adjoint, int32_t rhs_kind, int32_t ptr_kind, double* rel_residual, void* r_p,
                        void* r_u, void* workspace, size_t ws_bytes, void* hip_stream) {
    return residual_impl(m, s_p, s_u, p, u, adjoint, rhs_kind, ptr_kind, rel_residual, r_p, r_u, workspace,
                         ws_bytes, (hipStream_t)hip_stream, false);
}

cbs_status cbs_gradient(cbs_medium m, const void* s_p, const void* s_u, const void* p, const void* u,
                        const void* lp, const void* lu, int32_t ptr_kind, double* g_c, double* g_rho,
                        double* g_alpha, void* hip_stream) {
    if (!m || !s_p || !p || !lp) return CBS_E_INVALID;
    if (ptr_kind != CBS_PTR_HOST && ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom& g = m->g;
    const int64_t N = g.ncell;
    const int D = g.ndim;
    const double* gcen[3] = {m->gc64[0], m->gc64[1], m->gc64[2]};
    const double* gst[3] = {m->gs64[0], m->gs64[1], m->gs64[2]};
    if (ptr_kind == CBS_PTR_DEVICE) {
        HIPOK(launch_gradient(g, m->c64, m->rho64, m->alpha64, m->q64, gcen, gst, m->gmax, m->grid.omega,
                              static_cast<const cx<double>*>(s_p), static_cast<const cx<double>*>(s_u),
                              static_cast<const cx<double>*>(p), static_cast<const cx<double>*>(u),
                              static_cast<const cx<double>*>(lp), static_cast<const cx<double>*>(lu), g_c, g_rho,
                              g_alpha, m->grid.collocated, st));
        HIPOK(hipStreamSynchronize(st));
        return CBS_OK;
    }
    // host pointers: stage everything through one temporary device block
    const size_t cN = sizeof(cx<double>) * N, rN = sizeof(double) * N;
    const size_t bytes = 3 * cN + 3 * (size_t)D * cN + 3 * rN;
    char* tmp = nullptr;
    if (hipMalloc(&tmp, bytes) != hipSuccess) return CBS_E_NOMEM;
    cx<double>* dsp = reinterpret_cast<cx<double>*>(tmp);
    cx<double>* dp = dsp + N;
    cx<double>* dlp = dp + N;
    cx<double>* dsu = dlp + N;
    cx<double>* du = dsu + (size_t)D * N;
    cx<double>* dlu = du + (size_t)D * N;
    double* dgc = reinterpret_cast<double*>(dlu + (size_t)D * N);
    double* dgr = dgc + N;
    double* dga = dgr + N;
    cbs_status rc = CBS_OK;
    auto h2d = [&](void* dst, const void* src, size_t b) {
        if (src && hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st) != hipSuccess) rc = CBS_E_DEVICE;
    };
    h2d(dsp, s_p, cN);
    h2d(dp, p, cN);
    h2d(dlp, lp, cN);
    h2d(dsu, s_u, D * cN);
    h2d(du, u, D * cN);
    h2d(dlu, lu, D * cN);
    if (rc == CBS_OK &&
        launch_gradient(g, m->c64, m->rho64, m->alpha64, m->q64, gcen, gst, m->gmax, m->grid.omega, dsp,
                        s_u ? dsu : nullptr, dp, u ? du : nullptr, dlp, lu ? dlu : nullptr, dgc, dgr, dga,
                        m->grid.collocated, st) != hipSuccess)
        rc = CBS_E_DEVICE;
    if (rc == CBS_OK) {
        if (g_c && hipMemcpyAsync(g_c, dgc, rN, hipMemcpyDeviceToHost, st) != hipSuccess) rc = CBS_E_DEVICE;
        if (g_rho && hipMemcpyAsync(g_rho, dgr, rN, hipMemcpyDeviceToHost, st) != hipSuccess) rc = CBS_E_DEVICE;
        if (g_alpha && hipMemcpyAsync(g_alpha, dga, rN, hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = CBS_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) rc = CBS_E_DEVICE;
    (void)hipFree(tmp);
    return rc;
}

cbs_status cbs_pass_config(cbs_medium m, int32_t prec, int32_t out[20]) {
    if (!m || !out) return CBS_E_INVALID;
    if (prec != CBS_FP64 && prec != CBS_FP32_REFINED) return CBS_E_INVALID;
    const PassSet& ps = prec == CBS_FP64 ? m->ps64 : m->ps32;
    for (int i = 0; i < 5; ++i) {
        const bool have = i < ps.count;
        out[4 * i + 0] = have ? ps.p[i].kind : -1;
        out[4 * i + 1] = have ? ps.p[i].n : 0;
        out[4 * i + 2] = have ? ps.p[i].pcols : 0;
        const int blocks = (have && ps.count == 5 && i >= 1 && i <= 3) ? ps.cblocks : 1;
        out[4 * i + 3] = have ? ((ps.p[i].wide ? 1 : 0) | (ps.p[i].variant << 1) | (blocks << 5)) : 0;
    }
    return CBS_OK;
}

cbs_status cbs_pass_timing(cbs_medium m, int32_t enable) {
    if (!m) return CBS_E_INVALID;
    PassTiming& t = m->timing;
    if (enable) {
        std::memset(t.ms, 0, sizeof(t.ms));
        std::memset(t.cnt, 0, sizeof(t.cnt));
        t.used = 0;
    }
    t.on = enable != 0;
    return CBS_OK;
}

cbs_status cbs_pass_timing_slots(cbs_medium m, int32_t slot_mask) {
    if (!m || slot_mask < 0 || slot_mask > 0x3f) return CBS_E_INVALID;
    m->timing.mask = slot_mask;
    return CBS_OK;
}

cbs_status cbs_pass_timing_read(cbs_medium m, double ms[18], int64_t launches[18]) {
    if (!m || !ms || !launches) return CBS_E_INVALID;
    for (int g = 0; g < 3; ++g)
        for (int k = 0; k < 6; ++k) {
            ms[g * 6 + k] = m->timing.ms[g][k];
            launches[g * 6 + k] = m->timing.cnt[g][k];
        }
    return CBS_OK;
}

cbs_status cbs_stream_probe(const void* src, void* dst, size_t bytes, int32_t reps, double* gbs,
                            void* hip_stream) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
    if (!src || !dst || !gbs || (a | b) % 16 || bytes == 0 || bytes % 16 || reps < 1) return CBS_E_INVALID;
    if ((a < b && b - a < bytes) || (b <= a && a - b < bytes)) return CBS_E_INVALID;   // overlapping
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CBS_E_DEVICE;
    }
    bool ok = launch_stream_copy(src, dst, bytes, st) == hipSuccess;   // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int i = 0; i < reps && ok; ++i) ok = launch_stream_copy(src, dst, bytes, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return CBS_E_DEVICE;
    *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return CBS_OK;
}

}  // extern "C"

// =================================================== batched slots ======
// Continuous batching of same-shape solves.  Each slot owns a region laid out
// exactly like a single solve's workspace; its kernels, plans and
// refinement steps are the ones cbs_solve runs, and a slot's arithmetic never
// reads another slot's data, so its result is the same alone or in a mix.
namespace {

enum Phase { PH_FREE = 0, PH_RES = 1, PH_CBS = 2, PH_DONE = 3 };

struct BatchSlot {
    int phase = PH_FREE;
    cbs_medium_s* m = nullptr;
    cbs_solve_opts o{};
    bool start = true;
    int status = CBS_NOT_CONVERGED;
    int64_t iters = 0, res_evals = 0;
    int outer = 0;
    double rel_res = -1.0, rel_upd = 0.0, t0 = 0.0;
    Slot<double> h64{};
    Slot<float> h32{};
};

}  // namespace

struct cbs_batch_s {
    Geom g{};
    int prec = 0, maxs = 0;
    char* ws = nullptr;
    size_t header = 0, slot_bytes = 0;
    Layout L{};
    hipStream_t st = nullptr;
    PassSet ps64{}, ps32{};
    bool have_plans = false;
    std::vector<BatchSlot> s;
    Slot<double>* dc64 = nullptr;   // device: [0, maxs) all, [maxs, 2 maxs) starts
    Slot<float>* dc32 = nullptr;
    Slot<double>* hc64 = nullptr;   // pinned staging of the same
    Slot<float>* hc32 = nullptr;
    Ctl* hctl = nullptr;            // pinned: one control block per slot
    // instantiated graphs of `iterations` CBS iterations, keyed by
    // (slots, starting slots, iterations); the descriptors they read are
    // refreshed in place before each launch
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
    bool use_graphs = true;
    char* region(int i) const { return ws + header + (size_t)i * slot_bytes; }
};

namespace {

cbs_status batch_geom(const cbs_grid* grid, Geom* g) {
    cbs_status vs = validate_grid(grid);
    if (vs != CBS_OK) return vs;
    *g = geom_of(*grid);
    return CBS_OK;
}

size_t batch_header(int maxs) {
    return align_up(2 * (size_t)maxs * sizeof(Slot<double>)) + align_up(2 * (size_t)maxs * sizeof(Slot<float>));
}

cbs_status batch_residual_phase(cbs_batch_s* b) {
    std::vector<int> idx;
    for (int i = 0; i < b->maxs; ++i)
        if (b->s[i].phase == PH_RES) idx.push_back(i);
    if (idx.empty()) return CBS_OK;
    const int n = (int)idx.size();
    for (int k = 0; k < n; ++k) b->hc64[k] = b->s[idx[k]].h64;
    HIPOK(hipMemcpyAsync(b->dc64, b->hc64, sizeof(Slot<double>) * n, hipMemcpyHostToDevice, b->st));
    HIPOK(run_passes_set<double>(b->g, nullptr, b->ps64, MODE_APPLY, b->dc64, n, b->dc64, 0, b->st));
    for (int k = 0; k < n; ++k)
        HIPOK(hipMemcpyAsync(&b->hctl[idx[k]], b->s[idx[k]].h64.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, b->st));
    HIPOK(hipStreamSynchronize(b->st));
    const int64_t nf = (int64_t)(b->g.ndim + 1) * b->g.ncell;
    for (int i : idx) {
        BatchSlot& sl = b->s[i];
        const Ctl& c = b->hctl[i];
        sl.res_evals++;
        sl.rel_res = c.rhs2 > 0 ? std::sqrt(c.res2 / c.rhs2) : 0.0;
        const int max_outer = sl.o.max_outer > 0 ? sl.o.max_outer : 10000;
        if (!std::isfinite(sl.rel_res)) {
            sl.status = CBS_E_DIVERGED;
            sl.phase = PH_DONE;
        } else if (sl.rel_res <= sl.o.tol) {
            sl.status = CBS_OK;
            sl.phase = PH_DONE;
        } else if (sl.outer >= max_outer || sl.iters >= sl.o.max_iter) {
            sl.status = CBS_NOT_CONVERGED;
            sl.phase = PH_DONE;
        } else {
            const double inner_tol = sl.o.inner_tol > 0 ? sl.o.inner_tol : 1e-3;
            HIPOK(launch_convert(sl.h64.w, const_cast<cx<float>*>(sl.h32.y), nf, sl.h64.ctl, b->st));
            HIPOK(launch_zero<float>(sl.h32.x, nf, b->st));
            const int64_t max_inner = sl.o.max_inner > 0 ? sl.o.max_inner : 256;
            HIPOK(launch_ctl_reset(sl.h32.ctl, (int)std::min<int64_t>(sl.o.max_iter - sl.iters, max_inner),
                                   inner_tol, b->st));
            sl.phase = PH_CBS;
            sl.start = true;
        }
    }
    return CBS_OK;
}

template <typename T>
cbs_status batch_cbs_phase(cbs_batch_s* b, int iterations, Slot<T>* dc, Slot<T>* hc, const PassSet& ps) {
    std::vector<int> idx, starts;
    for (int i = 0; i < b->maxs; ++i)
        if (b->s[i].phase == PH_CBS) {
            idx.push_back(i);
            if (b->s[i].start) starts.push_back(i);
        }
    if (idx.empty()) return CBS_OK;
    const int n = (int)idx.size(), ns = (int)starts.size();
    auto desc = [&](int i) -> const Slot<T>& {
        if constexpr (sizeof(T) == 8) return b->s[i].h64;
        else return b->s[i].h32;
    };
    for (int k = 0; k < n; ++k) hc[k] = desc(idx[k]);
    for (int k = 0; k < ns; ++k) hc[b->maxs + k] = desc(starts[k]);
    HIPOK(hipMemcpyAsync(dc, hc, sizeof(Slot<T>) * n, hipMemcpyHostToDevice, b->st));
    if (ns) HIPOK(hipMemcpyAsync(dc + b->maxs, hc + b->maxs, sizeof(Slot<T>) * ns, hipMemcpyHostToDevice, b->st));
    if (b->use_graphs) {
        const auto key = std::make_tuple(n, ns, iterations);
        auto itg = b->graphs.find(key);
        if (itg == b->graphs.end()) {
            hipGraph_t graph = nullptr;
            HIPOK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
            hipError_t ce = hipSuccess;
            for (int it = 0; it < iterations && ce == hipSuccess; ++it)
                ce = run_passes_set<T>(b->g, nullptr, ps, MODE_CBS, dc, n, dc + b->maxs, it == 0 ? ns : 0, b->st);
            const hipError_t ee = hipStreamEndCapture(b->st, &graph);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return CBS_E_DEVICE;
            }
            hipGraphExec_t exec = nullptr;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return CBS_E_DEVICE;
            itg = b->graphs.emplace(key, exec).first;
        }
        HIPOK(hipGraphLaunch(itg->second, b->st));
    } else {
        for (int it = 0; it < iterations; ++it)
            HIPOK(run_passes_set<T>(b->g, nullptr, ps, MODE_CBS, dc, n, dc + b->maxs, it == 0 ? ns : 0, b->st));
    }
    for (int i : idx) {
        b->s[i].start = false;
        HIPOK(hipMemcpyAsync(&b->hctl[i], desc(i).ctl, sizeof(Ctl), hipMemcpyDeviceToHost, b->st));
    }
    HIPOK(hipStreamSynchronize(b->st));
    const int64_t nf = (int64_t)(b->g.ndim + 1) * b->g.ncell;
    for (int i : idx) {
        BatchSlot& sl = b->s[i];
        const Ctl& c = b->hctl[i];
        if (c.done == RUNNING) continue;
        sl.rel_upd = c.rel_update;
        if (b->prec == CBS_FP64) {
            sl.iters = c.iter;
            sl.status = c.done == CONVERGED ? CBS_OK : (c.done == DIVERGED ? CBS_E_DIVERGED : CBS_NOT_CONVERGED);
            sl.phase = PH_DONE;
        } else {
            sl.iters += c.iter;
            if (c.done == DIVERGED) {
                sl.status = CBS_E_DIVERGED;
                sl.phase = PH_DONE;
            } else {
                HIPOK(launch_accumulate(sl.h64.x, sl.h32.x, nf, sl.h64.ctl, b->st));
                sl.outer++;
                sl.phase = PH_RES;
            }
        }
    }
    return CBS_OK;
}

// One step of every active slot: residual phase (refined precision), then
// `iterations` CBS iterations; done_mask marks finished slots.
cbs_status batch_step(cbs_batch_s* b, int32_t iterations, uint8_t* done_mask) {
    cbs_status cs = CBS_OK;
    if (b->prec == CBS_FP32_REFINED) {
        if ((cs = batch_residual_phase(b)) != CBS_OK) return cs;
        cs = batch_cbs_phase<float>(b, iterations, b->dc32, b->hc32, b->ps32);
    } else {
        cs = batch_cbs_phase<double>(b, iterations, b->dc64, b->hc64, b->ps64);
    }
    if (cs != CBS_OK) return cs;
    if (done_mask)
        for (int i = 0; i < b->maxs; ++i) done_mask[i] = b->s[i].phase == PH_DONE ? 1 : 0;
    return CBS_OK;
}

}  // namespace

extern "C" {

cbs_status cbs_batch_workspace_bytes(const cbs_grid* grid, int32_t prec, int32_t max_slots, size_t* bytes) {
    if (!bytes || max_slots < 1 || max_slots > 4096) return CBS_E_INVALID;
    if (prec != CBS_FP64 && prec != CBS_FP32_REFINED) return CBS_E_INVALID;
    Geom g{};
    cbs_status cs = batch_geom(grid, &g);
    if (cs != CBS_OK) return cs;
    *bytes = batch_header(max_slots) + (size_t)max_slots * layout_for(g, prec).total;
    return CBS_OK;
}

cbs_status cbs_batch_create(const cbs_grid* grid, int32_t prec, int32_t max_slots, void* workspace,
                            size_t ws_bytes, void* hip_stream, cbs_batch* out) {
    if (!out || !workspace) return CBS_E_INVALID;
    *out = nullptr;
    size_t need = 0;
    cbs_status cs = cbs_batch_workspace_bytes(grid, prec, max_slots, &need);
    if (cs != CBS_OK) return cs;
    if (ws_bytes < need) return CBS_E_NOMEM;
    cbs_batch_s* b = new (std::nothrow) cbs_batch_s();
    if (!b) return CBS_E_NOMEM;
    batch_geom(grid, &b->g);
    b->prec = prec;
    b->maxs = max_slots;
    b->ws = static_cast<char*>(workspace);
    b->st = (hipStream_t)hip_stream;
    b->L = layout_for(b->g, prec);
    b->slot_bytes = b->L.total;
    b->header = batch_header(max_slots);
    b->s.resize(max_slots);
    {
        const char* e = std::getenv("CBS_BATCH_GRAPHS");
        b->use_graphs = !(e && e[0] == '0');
    }
    b->dc64 = reinterpret_cast<Slot<double>*>(b->ws);
    b->dc32 = reinterpret_cast<Slot<float>*>(b->ws + align_up(2 * (size_t)max_slots * sizeof(Slot<double>)));
    if (hipHostMalloc((void**)&b->hc64, 2 * sizeof(Slot<double>) * max_slots) != hipSuccess ||
        hipHostMalloc((void**)&b->hc32, 2 * sizeof(Slot<float>) * max_slots) != hipSuccess ||
        hipHostMalloc((void**)&b->hctl, sizeof(Ctl) * max_slots) != hipSuccess) {
        cbs_batch_destroy(b);
        return CBS_E_NOMEM;
    }
    *out = b;
    return CBS_OK;
}

cbs_status cbs_batch_destroy(cbs_batch b) {
    if (!b) return CBS_E_INVALID;
    (void)hipStreamSynchronize(b->st);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->hc64) (void)hipHostFree(b->hc64);
    if (b->hc32) (void)hipHostFree(b->hc32);
    if (b->hctl) (void)hipHostFree(b->hctl);
    delete b;
    return CBS_OK;
}

cbs_status cbs_batch_submit(cbs_batch b, cbs_medium m, const void* s_p, const void* s_u, const cbs_solve_opts* o,
                            int32_t* slot) {
    if (!b || !m || !s_p || !o || !slot) return CBS_E_INVALID;
    if (o->prec != b->prec) return CBS_E_INVALID;
    if (o->ptr_kind != CBS_PTR_HOST && o->ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    if (o->rhs_kind != CBS_RHS_PHYSICAL && o->rhs_kind != CBS_RHS_EQUATION) return CBS_E_INVALID;
    if (!(o->tol >= 0) || o->max_iter < 1 || o->max_iter > 0x7fffffff) return CBS_E_INVALID;
    if (b->prec == CBS_FP64 && o->stop_rule != CBS_STOP_UPDATE) return CBS_E_UNSUPPORTED;
    for (int d = 0; d < 3; ++d)
        if (m->g.n[d] != b->g.n[d] || m->g.ndim != b->g.ndim) return CBS_E_INVALID;
    int i = 0;
    while (i < b->maxs && b->s[i].phase != PH_FREE) ++i;
    if (i == b->maxs) return CBS_E_NOMEM;
    char* ws = b->region(i);
    if (!b->have_plans) {
        cbs_status ts = guarded([&] { return ensure_tuned(m, b->prec, ws, b->st); });
        if (ts != CBS_OK) return ts;
        b->ps64 = m->ps64;
        b->ps32 = m->ps32;
        b->have_plans = true;
    }
    const Layout& L = b->L;
    const Geom& g = b->g;
    const int64_t nf = (int64_t)(g.ndim + 1) * g.ncell;
    BatchSlot& sl = b->s[i];
    sl = BatchSlot();
    sl.t0 = now_s();
    sl.m = m;
    sl.o = *o;
    cx<double>* x64 = at<cx<double>>(ws, L.off_x64);
    cx<double>* w64 = at<cx<double>>(ws, L.off_w64);
    cx<double>* y64 = at<cx<double>>(ws, L.off_y64);
    const cx<double>*dsp = nullptr, *dsu = nullptr;
    cbs_status cs = stage_sources(m, s_p, s_u, o->ptr_kind, w64, &dsp, &dsu, b->st);
    if (cs != CBS_OK) return cs;
    HIPOK(launch_rhs(g, dsp, dsu, m->rhobar64, m->q64, o->rhs_kind == CBS_RHS_PHYSICAL, 1.0 / std::sqrt(m->lam1),
                     1.0 / std::sqrt(m->lam2), y64, nullptr, b->st));
    HIPOK(launch_zero<double>(x64, nf, b->st));
    Ctl* ctl64 = at<Ctl>(ws, L.off_ctl64);
    HIPOK(hipMemsetAsync(ctl64, 0, sizeof(Ctl), b->st));
    sl.h64 = make_slot<double>(m, x64, w64, y64, ctl64, at<double>(ws, L.off_part64), 0,
                               at<double>(ws, L.off_chunk64));
    if (b->prec == CBS_FP32_REFINED) {
        Ctl* ctl32 = at<Ctl>(ws, L.off_ctl32);
        HIPOK(hipMemsetAsync(ctl32, 0, sizeof(Ctl), b->st));
        sl.h32 = make_slot<float>(m, at<cx<float>>(ws, L.off_d32), at<cx<float>>(ws, L.off_w32),
                                  at<cx<float>>(ws, L.off_y32), ctl32, at<double>(ws, L.off_part32), 0,
                                  at<double>(ws, L.off_chunk32));
        sl.phase = PH_RES;
    } else {
        HIPOK(launch_ctl_reset(ctl64, (int)o->max_iter, o->tol, b->st));
        sl.phase = PH_CBS;
        sl.start = true;
    }
    *slot = i;
    return CBS_OK;
}

cbs_status cbs_batch_step(cbs_batch b, int32_t iterations, uint8_t* done_mask) {
    if (!b || iterations < 1) return CBS_E_INVALID;
    return guarded([&] { return batch_step(b, iterations, done_mask); });
}

cbs_status cbs_batch_retire(cbs_batch b, int32_t slot, void* p_out, void* u_out, int32_t ptr_kind,
                            cbs_solve_info* info) {
    if (!b || slot < 0 || slot >= b->maxs) return CBS_E_INVALID;
    BatchSlot& sl = b->s[slot];
    if (sl.phase != PH_DONE) return CBS_E_INVALID;
    if (ptr_kind != CBS_PTR_HOST && ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    if (sl.status != CBS_E_DIVERGED && p_out) {
        cbs_status cs = write_outputs<double>(sl.m, sl.h64.x, p_out, u_out, ptr_kind, sl.h64.w, b->st);
        if (cs != CBS_OK) return cs;
    }
    if (info) {
        cbs_solve_info inf{};
        inf.iterations = sl.iters;
        inf.outer = sl.outer;
        inf.status = sl.status;
        inf.rel_update = sl.rel_upd;
        inf.rel_residual = sl.rel_res;
        inf.seconds = now_s() - sl.t0;
        inf.residual_evals = sl.res_evals;
        *info = inf;
    }
    const int st = sl.status;
    sl = BatchSlot();
    return (cbs_status)st;
}

}  // extern "C"

// ------------------------------------------------------------ slab split --
// One solve split along axis 0 into G parts, run the way G devices would run
// it, on the current device: part g owns planes [g s, (g+1) s) of x, y, the
// work array and the medium (s = n0 / G) and runs the last-axis and axis-1
// passes on them; an all-to-all exchange turns the parts into axis-1 pencil
// groups (part h owns rows [h t, (h+1) t), t = n1 / G, for every axis-0
// index) for the axis-0 pass with the propagator, whose wavenumber tables are
// offset to part h's rows, and a second exchange turns them back; the norm
// partial sums of all parts are folded by one reduction (the all-reduce).
// Every pass is launched per part, at the part's own shape.
namespace cbs {
template <typename E>
hipError_t launch_relayout(const E* src, int src_lay, E* dst, int dst_lay, int F, const int* n, int G,
                           hipStream_t st);
}

namespace {

enum { LAY_WHOLE = 0, LAY_SLAB = 1, LAY_PENCIL = 2 };

struct SplitLayout {
    size_t off_ctl64, off_slots64, off_part64, off_chunk64, off_x64, off_w64, off_y64, off_p64, off_rb64;
    size_t off_ctl32, off_slots32, off_part32, off_chunk32, off_d32, off_w32, off_y32, off_p32, off_rb32;
    size_t total;
};

SplitLayout split_layout_for(const Geom& g, int prec, int G) {
    SplitLayout L{};
    const size_t F = (size_t)g.ndim + 1, N = (size_t)g.ncell, D = (size_t)g.ndim;
    const size_t maxparts = F * (N / (size_t)g.n[g.ndim - 1]);   // one pair per pencil at most, all parts
    const size_t maxchunks = (maxparts + kReduceChunk - 1) / kReduceChunk;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.off_ctl64 = take(sizeof(Ctl));
    L.off_slots64 = take(sizeof(Slot<double>) * (2 * (size_t)G + 1));
    L.off_part64 = take(sizeof(double) * 2 * maxparts);
    L.off_chunk64 = take(sizeof(double) * 2 * maxchunks);
    L.off_x64 = take(F * N * sizeof(cx<double>));
    L.off_w64 = take(F * N * sizeof(cx<double>));
    L.off_y64 = take(F * N * sizeof(cx<double>));
    L.off_p64 = take(F * N * sizeof(cx<double>));
    L.off_rb64 = take(D * N * sizeof(double));
    if (prec == CBS_FP32_REFINED) {
        L.off_ctl32 = take(sizeof(Ctl));
        L.off_slots32 = take(sizeof(Slot<float>) * (2 * (size_t)G + 1));
        L.off_part32 = take(sizeof(double) * 2 * maxparts);
        L.off_chunk32 = take(sizeof(double) * 2 * maxchunks);
        L.off_d32 = take(F * N * sizeof(cx<float>));
        L.off_w32 = take(F * N * sizeof(cx<float>));
        L.off_y32 = take(F * N * sizeof(cx<float>));
        L.off_p32 = take(F * N * sizeof(cx<float>));
        L.off_rb32 = take(D * N * sizeof(float));
    }
    // the tuner runs on the same workspace with the unsplit layout
    L.total = std::max(o, layout_for(g, prec).total);
    return L;
}

cbs_status split_check(const cbs_medium_s* m, int G) {
    if (!m || G < 1 || G > 64) return CBS_E_INVALID;
    if (m->g.ndim != 3) return CBS_E_UNSUPPORTED;
    if (m->g.n[0] % G || m->g.n[1] % G) return CBS_E_UNSUPPORTED;
    return CBS_OK;
}

// The passes of one part: the tuned plans of the whole grid where their
// tile widths fit the part's shapes, the default plans otherwise.
PassSet split_passes(const cbs_medium_s* m, const PassSet& tuned, const Geom& gs, bool fp64) {
    PassSet ps = tuned;
    ps.cblocks = 1;
    // only the last-axis passes see the slab's own pencil count (its axis 0,
    // n0 / parts planes, is never transformed, and may have no plan)
    const int64_t pencils = gs.ncell / gs.n[2];
    for (int i : {0, ps.count - 1})
        if (ps.p[i].pcols < 1 || pencils % ps.p[i].pcols) ps.p[i] = contig_pass(gs, ps.p[i].kind, fp64);
    const Pass& lp = ps.p[ps.count - 1];
    ps.nparts = (int)((gs.ndim + 1) * (gs.ncell / ((int64_t)lp.n * lp.pcols)));
    (void)m;
    return ps;
}

template <typename T>
struct SplitRun {
    Geom gs, gp;               // one part's slab and pencil-group shapes
    int G;
    int n[3];
    PassSet ps;
    const Slot<T>* slots;      // device: G slab slots, G pencil slots, the reduction slot
    cx<T>* w_slab;
    cx<T>* w_pen;
};

// Slot descriptors of every part (host side), uploaded by the caller.
template <typename T>
void split_slots(const cbs_medium_s* m, const SplitRun<T>& r, cx<T>* x, cx<T>* y, const T* rb, const cx<T>* q,
                 T* const* gc, T* const* gsp, T* const* kv, cx<T>* const* sh, Ctl* ctl, double* part,
                 double* chunks, Slot<T>* out) {
    const int G = r.G;
    const int64_t sc = r.gs.ncell, pc = r.gp.ncell;
    const int F = 4, D = 3;
    const int s = r.n[0] / G, t = r.n[1] / G;
    for (int g = 0; g < G; ++g) {
        Slot<T> sl = make_slot<T>(m, x + (int64_t)g * F * sc, r.w_slab + (int64_t)g * F * sc,
                                  y + (int64_t)g * F * sc, ctl, part + (int64_t)g * r.ps.nparts * 2, 0, chunks);
        sl.rhobar = rb + (int64_t)g * D * sc;
        sl.q = q + (int64_t)g * sc;
        sl.gc[0] = gc[0] + (int64_t)g * s;
        sl.gs[0] = gsp[0] + (int64_t)g * s;
        out[g] = sl;
        Slot<T> pn = make_slot<T>(m, nullptr, r.w_pen + (int64_t)g * F * pc, nullptr, ctl, nullptr, 0, chunks);
        pn.kv[1] = kv[1] + (int64_t)g * t;
        pn.sh[1] = sh[1] + (int64_t)g * t;
        out[G + g] = pn;
    }
    out[2 * G] = make_slot<T>(m, nullptr, nullptr, nullptr, ctl, part, 0, chunks);
}

// One CBS iteration (or one residual evaluation) of the split solve.
template <typename T>
hipError_t split_iteration(const SplitRun<T>& r, int mode, bool start, hipStream_t st) {
    const Pass* P = r.ps.p;
    const Slot<T>* slab = r.slots;
    const Slot<T>* pen = r.slots + r.G;
    hipError_t e;
    auto pass = [&](int kind, const Slot<T>* sl, const Geom& g, const Pass& p) {
        return launch_pass<T>(kind, mode, sl, 1, g, p.axis, p.n, p.pcols, p.wide, p.variant, st, 0, 0);
    };
    for (int g = 0; g < r.G; ++g) {
        if ((mode == MODE_APPLY || start) && (e = pass(0, slab + g, r.gs, P[0])) != hipSuccess) return e;
        if ((e = pass(2, slab + g, r.gs, P[1])) != hipSuccess) return e;
    }
    if ((e = launch_relayout<cx<T>>(r.w_slab, LAY_SLAB, r.w_pen, LAY_PENCIL, 4, r.n, r.G, st)) != hipSuccess)
        return e;
    for (int h = 0; h < r.G; ++h)
        if ((e = pass(4, pen + h, r.gp, P[2])) != hipSuccess) return e;
    if ((e = launch_relayout<cx<T>>(r.w_pen, LAY_PENCIL, r.w_slab, LAY_SLAB, 4, r.n, r.G, st)) != hipSuccess)
        return e;
    for (int g = 0; g < r.G; ++g) {
        if ((e = pass(3, slab + g, r.gs, P[3])) != hipSuccess) return e;
        if ((e = pass(mode == MODE_CBS ? 5 : 1, slab + g, r.gs, P[4])) != hipSuccess) return e;
    }
    return launch_reduce<T>(mode == MODE_CBS, r.slots + 2 * r.G, r.G * r.ps.nparts, 1, st);
}

template <typename T>
SplitRun<T> split_run(const cbs_medium_s* m, const PassSet& tuned, int G, cx<T>* w_slab, cx<T>* w_pen,
                      const Slot<T>* dslots) {
    SplitRun<T> r{};
    r.G = G;
    for (int d = 0; d < 3; ++d) r.n[d] = m->g.n[d];
    r.gs = Geom{3, {r.n[0] / G, r.n[1], r.n[2]}, (int64_t)(r.n[0] / G) * r.n[1] * r.n[2]};
    r.gp = Geom{3, {r.n[0], r.n[1] / G, r.n[2]}, (int64_t)r.n[0] * (r.n[1] / G) * r.n[2]};
    r.ps = split_passes(m, tuned, r.gs, sizeof(T) == 8);
    r.slots = dslots;
    r.w_slab = w_slab;
    r.w_pen = w_pen;
    return r;
}

cbs_status solve_split_impl(cbs_medium m, int G, const void* s_p, const void* s_u, const cbs_solve_opts* o,
                            void* p_out, void* u_out, void* ws, size_t wsb, cbs_solve_info* info,
                            void* hip_stream) {
    const double t0 = now_s();
    cbs_status cs = split_check(m, G);
    if (cs != CBS_OK) return cs;
    if (!s_p || !o || !p_out || !ws) return CBS_E_INVALID;
    if (o->prec != CBS_FP64 && o->prec != CBS_FP32_REFINED) return CBS_E_INVALID;
    if (o->ptr_kind != CBS_PTR_HOST && o->ptr_kind != CBS_PTR_DEVICE) return CBS_E_INVALID;
    if (o->rhs_kind != CBS_RHS_PHYSICAL && o->rhs_kind != CBS_RHS_EQUATION) return CBS_E_INVALID;
    if (o->stop_rule != CBS_STOP_UPDATE && o->stop_rule != CBS_STOP_RESIDUAL) return CBS_E_INVALID;
    if (!(o->tol >= 0) || o->max_iter < 1 || o->max_iter > 0x7fffffff) return CBS_E_INVALID;
    const SplitLayout L = split_layout_for(m->g, o->prec, G);
    if (wsb < L.total) return CBS_E_NOMEM;
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom& g = m->g;
    const int64_t N = g.ncell, nf = 4 * N;
    const int check = o->check_every > 0 ? o->check_every : 32;
    if ((cs = ensure_tuned(m, o->prec, ws, st)) != CBS_OK) return cs;
    const int n[3] = {g.n[0], g.n[1], g.n[2]};

    Ctl* ctl64 = at<Ctl>(ws, L.off_ctl64);
    Slot<double>* dslots64 = at<Slot<double>>(ws, L.off_slots64);
    cx<double>* x64 = at<cx<double>>(ws, L.off_x64);
    cx<double>* w64 = at<cx<double>>(ws, L.off_w64);
    cx<double>* y64 = at<cx<double>>(ws, L.off_y64);
    cx<double>* p64 = at<cx<double>>(ws, L.off_p64);
    double* rb64 = at<double>(ws, L.off_rb64);
    const SplitRun<double> r64 = split_run<double>(m, m->ps64, G, w64, p64, dslots64);

    // right-hand side in the whole-grid layout (staged through the pencil
    // array), then split into parts; the medium's staggered densities too
    const cx<double>*dsp = nullptr, *dsu = nullptr;
    if ((cs = stage_sources(m, s_p, s_u, o->ptr_kind, w64, &dsp, &dsu, st)) != CBS_OK) return cs;
    HIPOK(launch_rhs(g, dsp, dsu, m->rhobar64, m->q64, o->rhs_kind == CBS_RHS_PHYSICAL, 1.0 / std::sqrt(m->lam1),
                     1.0 / std::sqrt(m->lam2), p64, nullptr, st));
    HIPOK(launch_relayout<cx<double>>(p64, LAY_WHOLE, y64, LAY_SLAB, 4, n, G, st));
    HIPOK(launch_relayout<double>(m->rhobar64, LAY_WHOLE, rb64, LAY_SLAB, 3, n, G, st));
    HIPOK(launch_zero<double>(x64, nf, st));
    HIPOK(launch_ctl_clear(ctl64, st));
    {
        std::vector<Slot<double>> hs(2 * G + 1);
        split_slots<double>(m, r64, x64, y64, rb64, m->q64, m->gc64, m->gs64, m->kv64, m->sh64, ctl64,
                            at<double>(ws, L.off_part64), at<double>(ws, L.off_chunk64), hs.data());
        HIPOK(hipMemcpyAsync(dslots64, hs.data(), sizeof(Slot<double>) * hs.size(), hipMemcpyHostToDevice, st));
        HIPOK(hipStreamSynchronize(st));
    }

    cbs_solve_info inf{};
    inf.rel_residual = -1.0;
    Ctl hc{};
    int status = CBS_NOT_CONVERGED;
    if (o->prec == CBS_FP64) {
        const bool by_res = o->stop_rule == CBS_STOP_RESIDUAL;
        HIPOK(launch_ctl_reset(ctl64, (int)o->max_iter, by_res ? -1.0 : o->tol, st));
        int64_t launched = 0;
        bool start = true;
        while (true) {
            const int64_t chunk = std::min<int64_t>(check, o->max_iter - launched);
            for (int64_t k = 0; k < chunk; ++k) {
                HIPOK(split_iteration<double>(r64, MODE_CBS, start, st));
                start = false;
            }
            launched += chunk;
            if (by_res) {
                HIPOK(split_iteration<double>(r64, MODE_APPLY, true, st));
                inf.residual_evals++;
                start = true;
            }
            if ((cs = read_ctl(m, ctl64, &hc, st)) != CBS_OK) return cs;
            inf.iterations = hc.iter;
            inf.rel_update = hc.rel_update;
            if (by_res) {
                inf.rel_residual = hc.rhs2 > 0 ? std::sqrt(hc.res2 / hc.rhs2) : 0.0;
                if (!std::isfinite(inf.rel_residual)) {
                    status = CBS_E_DIVERGED;
                    break;
                }
                if (inf.rel_residual <= o->tol) {
                    status = CBS_OK;
                    break;
                }
            }
            if (hc.done == CONVERGED) {
                status = CBS_OK;
                break;
            }
            if (hc.done == DIVERGED) {
                status = CBS_E_DIVERGED;
                break;
            }
            if (hc.done == CAPPED || launched >= o->max_iter) break;
        }
    } else {
        Ctl* ctl32 = at<Ctl>(ws, L.off_ctl32);
        Slot<float>* dslots32 = at<Slot<float>>(ws, L.off_slots32);
        cx<float>* d32 = at<cx<float>>(ws, L.off_d32);
        cx<float>* w32 = at<cx<float>>(ws, L.off_w32);
        cx<float>* y32 = at<cx<float>>(ws, L.off_y32);
        cx<float>* p32 = at<cx<float>>(ws, L.off_p32);
        float* rb32 = at<float>(ws, L.off_rb32);
        const SplitRun<float> r32 = split_run<float>(m, m->ps32, G, w32, p32, dslots32);
        HIPOK(launch_relayout<float>(m->rhobar32, LAY_WHOLE, rb32, LAY_SLAB, 3, n, G, st));
        HIPOK(launch_ctl_clear(ctl32, st));
        {
            std::vector<Slot<float>> hs(2 * G + 1);
            split_slots<float>(m, r32, d32, y32, rb32, m->q32, m->gc32, m->gs32, m->kv32, m->sh32, ctl32,
                               at<double>(ws, L.off_part32), at<double>(ws, L.off_chunk32), hs.data());
            HIPOK(hipMemcpyAsync(dslots32, hs.data(), sizeof(Slot<float>) * hs.size(), hipMemcpyHostToDevice, st));
            HIPOK(hipStreamSynchronize(st));
        }
        const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-3;
        const int max_outer = o->max_outer > 0 ? o->max_outer : 10000;
        const int64_t max_inner = o->max_inner > 0 ? o->max_inner : 256;
        int64_t total = 0;
        for (int outer = 0;; ++outer) {
            HIPOK(split_iteration<double>(r64, MODE_APPLY, true, st));
            inf.residual_evals++;
            if ((cs = read_ctl(m, ctl64, &hc, st)) != CBS_OK) return cs;
            inf.rel_residual = hc.rhs2 > 0 ? std::sqrt(hc.res2 / hc.rhs2) : 0.0;
            inf.outer = outer;
            if (!std::isfinite(inf.rel_residual)) {
                status = CBS_E_DIVERGED;
                break;
            }
            if (inf.rel_residual <= o->tol) {
                status = CBS_OK;
                break;
            }
            if (outer >= max_outer || total >= o->max_iter) break;
            HIPOK(launch_convert(w64, y32, nf, ctl64, st));
            HIPOK(launch_zero<float>(d32, nf, st));
            const int64_t cap = std::min<int64_t>(o->max_iter - total, max_inner);
            HIPOK(launch_ctl_reset(ctl32, (int)cap, inner_tol, st));
            Ctl ic{};
            int64_t launched = 0;
            while (true) {
                const int64_t chunk = std::min<int64_t>(check, cap - launched);
                for (int64_t k = 0; k < chunk; ++k)
                    HIPOK(split_iteration<float>(r32, MODE_CBS, launched + k == 0, st));
                launched += chunk;
                if ((cs = read_ctl(m, ctl32, &ic, st)) != CBS_OK) return cs;
                if (ic.done != RUNNING || launched >= cap) break;
            }
            total += ic.iter;
            inf.rel_update = ic.rel_update;
            if (ic.done == DIVERGED) {
                status = CBS_E_DIVERGED;
                break;
            }
            HIPOK(launch_accumulate(x64, d32, nf, ctl64, st));
        }
        inf.iterations = total;
    }
    if (status != CBS_E_DIVERGED) {
        // the parts' state back in the whole-grid layout, then unscaled out
        HIPOK(launch_relayout<cx<double>>(x64, LAY_SLAB, p64, LAY_WHOLE, 4, n, G, st));
        if ((cs = write_outputs<double>(m, p64, p_out, u_out, o->ptr_kind, w64, st)) != CBS_OK) return cs;
    }
    inf.status = status;
    inf.seconds = now_s() - t0;
    if (info) *info = inf;
    return (cbs_status)status;
}

}  // namespace

extern "C" {

cbs_status cbs_split_workspace_bytes(cbs_medium m, int32_t prec, int32_t parts, size_t* bytes) {
    const cbs_status cs = split_check(m, parts);
    if (cs != CBS_OK) return cs;
    if (!bytes || (prec != CBS_FP64 && prec != CBS_FP32_REFINED)) return CBS_E_INVALID;
    *bytes = split_layout_for(m->g, prec, parts).total;
    return CBS_OK;
}

cbs_status cbs_solve_split(cbs_medium m, int32_t parts, const void* s_p, const void* s_u,
                           const cbs_solve_opts* opts, void* p_out, void* u_out, void* workspace, size_t ws_bytes,
                           cbs_solve_info* info, void* hip_stream) {
    return guarded(
        [&] { return solve_split_impl(m, parts, s_p, s_u, opts, p_out, u_out, workspace, ws_bytes, info, hip_stream); });
}

}  // extern "C"
