// Host-side planning (no HIP): pencil tiles, tile DAG, stream placement,
// twiddle tables.
#include "plan.hpp"

#include <math.h>

#include <algorithm>

#include "fft_lengths.hpp"
#include "stage_args.hpp"

namespace fft3d {

bool boxes_overlap(const Box& a, const Box& b)
{
    for (int d = 0; d < 3; ++d)
        if (a.hi[d] <= b.lo[d] || b.hi[d] <= a.lo[d]) return false;
    return true;
}

void split_range(int64_t n, int p, int i, int64_t* lo, int64_t* hi)
{
    const int64_t q = n / p, r = n % p;
    *lo = i * q + std::min<int64_t>(i, r);
    *hi = *lo + q + (i < r ? 1 : 0);
}

// x ranges are the lanes of the y and z stages' row tiles: their edges are
// rounded to whole cache lines (granule values) when every tile keeps at
// least two lines, so no tile starts its rows in the middle of a line
// (otherwise balanced as split_range)
void split_x(int64_t n, int p, int i, int64_t granule, int64_t* lo, int64_t* hi)
{
    if (p > 1 && n / p >= 2 * granule) {
        auto edge = [&](int k) -> int64_t {
            if (k >= p) return n;
            return std::min<int64_t>(n, ((int64_t)k * n / p + granule / 2) / granule * granule);
        };
        *lo = edge(i);
        *hi = edge(i + 1);
        return;
    }
    split_range(n, p, i, lo, hi);
}

std::vector<Box> stage_boxes(const PlanDesc& d, int axis)
{
    const int64_t ext[3] = {d.nxc(), d.ny, d.nz};
    // the two axes a pencil of this orientation is split along, over p1 x p2
    int s1, s2;
    if (axis == 0) { s1 = 1; s2 = 2; }
    else if (axis == 1) { s1 = 0; s2 = 2; }
    else { s1 = 0; s2 = 1; }
    std::vector<Box> out;
    for (int j2 = 0; j2 < d.p2; ++j2) {
        for (int j1 = 0; j1 < d.p1; ++j1) {
            Box b;
            b.lo[axis] = 0;
            b.hi[axis] = ext[axis];
            if (s1 == 0) split_x(ext[0], d.p1, j1, d.dtype == 1 ? 8 : 16, &b.lo[0], &b.hi[0]);
            else split_range(ext[s1], d.p1, j1, &b.lo[s1], &b.hi[s1]);
            split_range(ext[s2], d.p2, j2, &b.lo[s2], &b.hi[s2]);
            out.push_back(b);
        }
    }
    return out;
}

static Stage mk(int kind, int axis, int n, int conj, int weight, double scale, int src, int dst)
{
    Stage s;
    s.kind = kind; s.axis = axis; s.n = n; s.conj = conj; s.weight = weight;
    s.scale = scale; s.src = src; s.dst = dst;
    return s;
}

std::vector<Stage> op_stages(const PlanDesc& d, int op)
{
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const double inv_n = 1.0 / ((double)d.nx * (double)d.ny * (double)d.nz);
    std::vector<Stage> s;
    if (!d.r2c && d.staging == STAGING_FUSED_XY) {
        switch (op) {
        case OP_FORWARD:  // the planes (x and y), then z in place
            s.push_back(mk(K_C2C_XY, 0, nx, 0, 0, 1.0, BUF_IN, BUF_OUT));
            s.push_back(mk(K_C2C, 2, nz, 0, 0, 1.0, BUF_OUT, BUF_OUT));
            break;
        case OP_INVERSE:  // mirrored: z, then the planes
        case OP_BACKWARD:
            s.push_back(mk(K_C2C, 2, nz, 1, 0, 1.0, BUF_IN, BUF_OUT));
            s.push_back(mk(K_C2C_XY, 0, nx, 1, 0, op == OP_INVERSE ? inv_n : 1.0, BUF_OUT, BUF_OUT));
            break;
        default:
            break;
        }
        return s;
    }
    if (!d.r2c && d.staging == STAGING_SWAP_YZ) {
        // x, y, z in both directions; the y stage writes the workspace in
        // SWAP_YZ order, the z stage reads it back into the output
        const bool fwd = op == OP_FORWARD;
        if (op != OP_FORWARD && op != OP_INVERSE && op != OP_BACKWARD) return s;
        const int cj = fwd ? 0 : 1;
        s.push_back(mk(K_C2C, 0, nx, cj, 0, 1.0, BUF_IN, BUF_OUT));
        s.push_back(mk(K_C2C, 1, ny, cj, 0, 1.0, BUF_OUT, BUF_WS));
        s.back().lay_dst = LAY_SWAP_YZ;
        s.push_back(mk(K_C2C, 2, nz, cj, 0, op == OP_INVERSE ? inv_n : 1.0, BUF_WS, BUF_OUT));
        s.back().lay_src = LAY_SWAP_YZ;
        return s;
    }
    if (!d.r2c) {
        switch (op) {
        case OP_FORWARD:  // x, y, z (Alg. 1)
            s.push_back(mk(K_C2C, 0, nx, 0, 0, 1.0, BUF_IN, BUF_OUT));
            s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_OUT, BUF_OUT));
            s.push_back(mk(K_C2C, 2, nz, 0, 0, 1.0, BUF_OUT, BUF_OUT));
            break;
        case OP_INVERSE:   // mirrored: z, y, x
        case OP_BACKWARD:
            s.push_back(mk(K_C2C, 2, nz, 1, 0, 1.0, BUF_IN, BUF_OUT));
            s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_OUT, BUF_OUT));
            s.push_back(mk(K_C2C, 0, nx, 1, 0, op == OP_INVERSE ? inv_n : 1.0, BUF_OUT, BUF_OUT));
            break;
        default:
            break;
        }
        return s;
    }
    if (d.zbc != Z_PERIODIC) {
        // (Periodic, Periodic, Bounded): DFT along x (half spectrum) and y,
        // DCT-II (Neumann) or DST-II (Dirichlet) along z; the inverse divides
        // by 2 Nz along z (DCT-III / DST-III) and by Nx Ny as the periodic one
        const bool dst = d.zbc == Z_DIRICHLET;
        const int fwd_z = dst ? R2R_DST2 : R2R_DCT2, inv_z = dst ? R2R_DST3 : R2R_DCT3;
        const int pz = dst ? R2R_POISSON_D : R2R_POISSON_N;
        auto r2r = [&](int mode, int weight, double scale, int src, int dst_buf) {
            Stage st = mk(K_R2R_Z, 2, nz, 0, weight, scale, src, dst_buf);
            st.r2r = mode;
            return st;
        };
        switch (op) {
        case OP_FORWARD:
            s.push_back(mk(K_R2C_X, 0, nx, 0, 0, 1.0, BUF_IN, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(r2r(fwd_z, 0, 1.0, BUF_WS, BUF_OUT));
            break;
        case OP_INVERSE:
            s.push_back(r2r(inv_z, 0, 0.5, BUF_IN, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2R_X, 0, nx, 0, 0, inv_n, BUF_WS, BUF_OUT));
            break;
        case OP_BACKWARD:  // transposes in reverse order: DCT-II^T, DFT_y^H, r2c^T
            s.push_back(r2r(inv_z, 1, 1.0, BUF_IN, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2R_X, 0, nx, 0, 1, 1.0, BUF_WS, BUF_OUT));
            break;
        case OP_POISSON:  // the z stage folds forward, multiplier and inverse (1/(2N) in all)
            s.push_back(mk(K_R2C_X, 0, nx, 0, 0, 1.0, BUF_IN, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(r2r(pz, 0, 0.5 * inv_n, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2R_X, 0, nx, 0, 0, 1.0, BUF_WS, BUF_OUT));
            break;
        case OP_POISSON_ADJ:  // as the periodic adjoint; the fused z stage is symmetric
            s.push_back(mk(K_R2C_X, 0, nx, 0, 1, 1.0, BUF_IN, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(r2r(pz, 0, 0.5 * inv_n, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
            s.push_back(mk(K_C2R_X, 0, nx, 0, 1, 1.0, BUF_WS, BUF_OUT));
            break;
        default:
            break;
        }
        return s;
    }
    if (d.staging == STAGING_SWAP_YZ && op == OP_FORWARD) {
        // x writes the output, y moves it into the workspace with y and z
        // swapped, z reads the workspace rows back into the output: no stage
        // reads lines at the plane stride
        s.push_back(mk(K_R2C_X, 0, nx, 0, 0, 1.0, BUF_IN, BUF_OUT));
        s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_OUT, BUF_WS));
        s.back().lay_dst = LAY_SWAP_YZ;
        s.push_back(mk(K_C2C, 2, nz, 0, 0, 1.0, BUF_WS, BUF_OUT));
        s.back().lay_src = LAY_SWAP_YZ;
        return s;
    }
    switch (op) {
    case OP_FORWARD:
        // x and y in the workspace (rows on cache-line bounds), z writes the output
        s.push_back(mk(K_R2C_X, 0, nx, 0, 0, 1.0, BUF_IN, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
        s.push_back(mk(K_C2C, 2, nz, 0, 0, 1.0, BUF_WS, BUF_OUT));
        break;
    case OP_INVERSE:
    case OP_BACKWARD:
        // the input half spectrum is left intact: z reads it into the workspace
        s.push_back(mk(K_C2C, 2, nz, 1, 0, 1.0, BUF_IN, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
        if (op == OP_INVERSE) s.push_back(mk(K_C2R_X, 0, nx, 0, 0, inv_n, BUF_WS, BUF_OUT));
        else s.push_back(mk(K_C2R_X, 0, nx, 0, 1, 1.0, BUF_WS, BUF_OUT));  // adjoint of r2c
        break;
    case OP_POISSON:
        s.push_back(mk(K_R2C_X, 0, nx, 0, 0, 1.0, BUF_IN, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
        s.push_back(mk(K_POISSON_Z, 2, nz, 0, 0, inv_n, BUF_WS, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
        s.push_back(mk(K_C2R_X, 0, nx, 0, 0, 1.0, BUF_WS, BUF_OUT));
        break;
    case OP_POISSON_ADJ:
        // adjoint of each forward step, in reverse order:
        //   c2r^T = (x2 interior bins) r2c, (y inverse)^T = y forward,
        //   z stage (real multiplier) is self-adjoint, (y forward)^T = y inverse,
        //   r2c^T = c2r of (interior bins x1/2)
        s.push_back(mk(K_R2C_X, 0, nx, 0, 1, 1.0, BUF_IN, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 0, 0, 1.0, BUF_WS, BUF_WS));
        s.push_back(mk(K_POISSON_Z, 2, nz, 0, 0, inv_n, BUF_WS, BUF_WS));
        s.push_back(mk(K_C2C, 1, ny, 1, 0, 1.0, BUF_WS, BUF_WS));
        s.push_back(mk(K_C2R_X, 0, nx, 0, 1, 1.0, BUF_WS, BUF_OUT));
        break;
    default:
        break;
    }
    return s;
}

void place_tasks(Pipeline& p, int nstreams)
{
    if (nstreams < 1) nstreams = 1;
    p.nstreams = nstreams;
    std::vector<double> load(nstreams, 0.0);
    for (auto& t : p.tasks) {
        std::vector<int> aff(nstreams, 0);
        for (int d : t.deps) aff[p.tasks[d].stream]++;
        int best = 0;
        for (int s = 1; s < nstreams; ++s) {
            if (load[s] < load[best] || (load[s] == load[best] && aff[s] > aff[best])) best = s;
        }
        t.stream = best;
        load[best] += t.cost;
    }
    // Event waits: a task waits, per other stream, on the last of its producers
    // there, unless an earlier task of its own stream already waited on that
    // producer or a later task of that stream.
    std::vector<std::vector<int>> seen(nstreams, std::vector<int>(nstreams, -1));
    for (size_t i = 0; i < p.tasks.size(); ++i) {
        Task& t = p.tasks[i];
        t.waits.clear();
        std::vector<int> last(nstreams, -1);
        for (int d : t.deps) {
            const int s = p.tasks[d].stream;
            if (s != t.stream) last[s] = std::max(last[s], d);
        }
        for (int s = 0; s < nstreams; ++s) {
            if (last[s] > seen[t.stream][s]) {
                t.waits.push_back(last[s]);
                seen[t.stream][s] = last[s];
            }
        }
    }
}

Pipeline build_pipeline(const PlanDesc& d, int op, int nstreams)
{
    Pipeline p;
    p.stages = op_stages(d, op);
    int prev_begin = -1, prev_end = -1;
    for (int si = 0; si < (int)p.stages.size(); ++si) {
        const int begin = (int)p.tasks.size();
        for (const Box& b : stage_boxes(d, p.stages[si].axis)) {
            Task t;
            t.stage = si;
            t.box = b;
            t.cost = (double)b.count();
            for (int q = prev_begin; q >= 0 && q < prev_end; ++q)
                if (boxes_overlap(p.tasks[q].box, b)) t.deps.push_back(q);
            p.tasks.push_back(t);
        }
        prev_begin = begin;
        prev_end = (int)p.tasks.size();
    }
    issue_order(p);
    place_tasks(p, nstreams);
    return p;
}

void issue_order(Pipeline& p)
{
    // Immediate dispatch (the paper's data-dependency queue, Sec. IV-D): a
    // tile is issued as soon as its producers are, deeper stages first.  A
    // consumer then runs right after the tiles that wrote its input, while
    // that data is still in the GPU's caches.
    const int n = (int)p.tasks.size();
    std::vector<int> missing(n, 0);
    std::vector<std::vector<int>> users(n);
    for (int i = 0; i < n; ++i) {
        missing[i] = (int)p.tasks[i].deps.size();
        for (int d : p.tasks[i].deps) users[d].push_back(i);
    }
    std::vector<char> ready(n, 0), done(n, 0);
    for (int i = 0; i < n; ++i) ready[i] = missing[i] == 0;
    std::vector<int> order;
    order.reserve(n);
    for (int step = 0; step < n; ++step) {
        int best = -1;
        for (int i = 0; i < n; ++i) {
            if (!ready[i] || done[i]) continue;
            if (best < 0 || p.tasks[i].stage > p.tasks[best].stage) best = i;
        }
        done[best] = 1;
        order.push_back(best);
        for (int u : users[best])
            if (--missing[u] == 0) ready[u] = 1;
    }
    std::vector<int> pos(n);
    for (int k = 0; k < n; ++k) pos[order[k]] = k;
    std::vector<Task> re(n);
    for (int k = 0; k < n; ++k) {
        re[k] = p.tasks[order[k]];
        for (int& d : re[k].deps) d = pos[d];
        std::sort(re[k].deps.begin(), re[k].deps.end());
    }
    p.tasks.swap(re);
}

// cos and sin of (pi/2) * num / n for 0 <= num <= n, evaluated on an angle
// of at most pi/4 so the small-angle end keeps full relative accuracy.
static void quarter_turn(int64_t num, int64_t n, long double* c, long double* s)
{
    const long double half_pi = 1.57079632679489661923132169163975144L;
    if (2 * num <= n) {
        const long double a = half_pi * (long double)num / (long double)n;
        *c = cosl(a);
        *s = sinl(a);
    } else {
        const long double a = half_pi * (long double)(n - num) / (long double)n;
        *c = sinl(a);
        *s = cosl(a);
    }
}

void twiddles_f64(int64_t n, double* out)
{
    for (int64_t m = 0; m < n; ++m) {
        // angle 2 pi m / n = (pi/2) * 4m / n; fold into [0, pi/2] by symmetry
        int64_t k = 4 * m;           // in units of (pi/2)/n, within [0, 4n)
        const bool lower = k > 2 * n;  // angle in (pi, 2 pi): sin negative
        if (lower) k = 4 * n - k;
        const bool second = k > n;  // angle in (pi/2, pi]: cos negative
        if (second) k = 2 * n - k;
        long double c, s;
        quarter_turn(k, n, &c, &s);
        if (second) c = -c;
        if (lower) s = -s;
        out[2 * m] = (double)c;
        out[2 * m + 1] = (double)(-s);  // forward root: exp(-i angle)
    }
}

void twiddles_f32(int64_t n, float* out)
{
    std::vector<double> d((size_t)(2 * n));
    twiddles_f64(n, d.data());
    for (int64_t i = 0; i < 2 * n; ++i) out[i] = (float)d[(size_t)i];
}

}  // namespace fft3d

namespace fft3d {

int64_t pass_twiddles_f64(int64_t n, double* out, int ord)
{
    if (!length_supported(n)) return -1;
    const RadixPlan rp = radix_plan((int)n, ord);
    const int64_t total = pass_table_size(rp);
    if (!out || total == 0) return total;
    std::vector<double> w((size_t)(2 * n));
    twiddles_f64(n, w.data());
    for (int p = 1; p < rp.np; ++p) {
        const int R = rp.r[p], ns = radix_ns(rp, p), step = (int)n / (ns * R);
        const int off = pass_table_offset(rp, p);
        for (int k = 0; k < ns; ++k) {
            for (int r = 0; r < R; ++r) {
                const int64_t m = ((int64_t)r * k * step) % n;
                out[2 * (off + k * R + r)] = w[(size_t)(2 * m)];
                out[2 * (off + k * R + r) + 1] = w[(size_t)(2 * m + 1)];
            }
        }
    }
    return total;
}

int64_t pass_twiddles_f32(int64_t n, float* out, int ord)
{
    const int64_t total = pass_twiddles_f64(n, nullptr, ord);
    if (!out || total <= 0) return total;
    std::vector<double> d((size_t)(2 * total));
    pass_twiddles_f64(n, d.data(), ord);
    for (int64_t i = 0; i < 2 * total; ++i) out[i] = (float)d[(size_t)i];
    return total;
}

}  // namespace fft3d

namespace fft3d {

std::vector<std::vector<int>> place_batch(const std::vector<double>& cost, int nstreams)
{
    if (nstreams < 1) nstreams = 1;
    std::vector<int> order(cost.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::vector<int>> per(nstreams);
    std::vector<double> load(nstreams, 0.0);
    for (int f : order) {
        int best = 0;
        for (int s = 1; s < nstreams; ++s)
            if (load[s] < load[best]) best = s;
        per[best].push_back(f);
        load[best] += cost[f];
    }
    return per;
}

}  // namespace fft3d
