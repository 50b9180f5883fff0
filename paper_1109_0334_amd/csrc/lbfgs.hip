// lbfgs.hip -- projected L-BFGS polish of parameter points on the discrete-adjoint gradient
// (afm_polish), and the top-k selection that hands swarm optima to it (used by afm_invert).
//
// The paper stops at the swarm (Sec. 3.4); once the swarm sits in the basin of the global
// minimum a few quasi-Newton steps on the exact gradient reach the bottom far faster.  The
// iteration, in normalised coordinates z in [0,1]^D:
//   d = -H g (two-loop recursion over the last 5 pairs, H0 = s'y / y'y), trial points
//   z_k = clamp(z + 2^-k d, 0, 1) for k = 0..20, accept the first with
//   J(z_k) <= J(z) + 1e-4 g'(z_k - z) and g'(z_k - z) < 0 (backtracking Armijo), store the pair
//   (s, y) unless s'y <= 1e-12 |s||y|.
// All 21 trial points of every polished point are evaluated in one batched misfit launch (the
// batches are small, so the extra trajectories cost no wall time), and every step of the loop is
// a fixed sequence of kernel launches: no host round-trip, capturable in a graph.
#include <climits>

#include "afm_internal.hpp"

namespace afm {

namespace {

constexpr int kHist = 5;

__device__ inline double to_theta(double z, double lo, double hi, int32_t lg) {
    if (lg) return ::exp(::log(lo) + z * (::log(hi) - ::log(lo)));
    return lo + z * (hi - lo);
}

__device__ inline double dtheta_dz(double z, double lo, double hi, int32_t lg) {
    if (lg) return to_theta(z, lo, hi, 1) * (::log(hi) - ::log(lo));
    return hi - lo;
}

struct Box {
    double lo[kMaxParams], hi[kMaxParams];
    int32_t lg[kMaxParams];
};

// theta = map(z) for n points ([D][n] each)
__global__ void k_lb_theta(int64_t n, int32_t D, const double *z, double *theta, Box b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < D; ++j) theta[j * n + i] = to_theta(z[j * n + i], b.lo[j], b.hi[j], b.lg[j]);
}

// z-gradient from the SI gradient: g_z = g_theta * dtheta/dz (in place), and reset state.
__global__ void k_lb_start(int64_t n, int32_t D, const double *z, double *g, int32_t *cnt,
                           int32_t *head, int32_t *done, const int32_t *status, Box b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < D; ++j) g[j * n + i] *= dtheta_dz(z[j * n + i], b.lo[j], b.hi[j], b.lg[j]);
    cnt[i] = 0;
    head[i] = 0;
    done[i] = status[i] != 0;
}

// Direction by the two-loop recursion and the 21 trial points (layout: trial t = i * L + k).
__global__ void k_lb_dir(int64_t n, int32_t D, int32_t L, const double *z, const double *g,
                         const double *S, const double *Y, const double *rho, const int32_t *cnt,
                         const int32_t *head, const int32_t *done, double *ttheta, double *dec,
                         Box b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nt = n * L;
    double q[kMaxParams], d[kMaxParams], al[kHist];
    for (int j = 0; j < D; ++j) q[j] = g[j * n + i];
    const int hn = cnt[i], hd = head[i];
    for (int k = 0; k < hn; ++k) {
        const int h = (hd - 1 - k + kHist) % kHist;
        double sq = 0.0;
        for (int j = 0; j < D; ++j) sq += S[((int64_t)h * D + j) * n + i] * q[j];
        al[h] = rho[(int64_t)h * n + i] * sq;
        for (int j = 0; j < D; ++j) q[j] -= al[h] * Y[((int64_t)h * D + j) * n + i];
    }
    double gamma = 1.0;
    if (hn > 0) {
        const int h = (hd - 1 + kHist) % kHist;
        double sy = 0.0, yy = 0.0;
        for (int j = 0; j < D; ++j) {
            const double sj = S[((int64_t)h * D + j) * n + i], yj = Y[((int64_t)h * D + j) * n + i];
            sy += sj * yj;
            yy += yj * yj;
        }
        gamma = sy / yy;
    }
    for (int j = 0; j < D; ++j) d[j] = gamma * q[j];
    for (int k = hn - 1; k >= 0; --k) {
        const int h = (hd - 1 - k + kHist) % kHist;
        double yd = 0.0;
        for (int j = 0; j < D; ++j) yd += Y[((int64_t)h * D + j) * n + i] * d[j];
        const double be = rho[(int64_t)h * n + i] * yd;
        for (int j = 0; j < D; ++j) d[j] += S[((int64_t)h * D + j) * n + i] * (al[h] - be);
    }
    double alpha = 1.0;
    for (int k = 0; k < L; ++k, alpha *= 0.5) {
        const int64_t t = i * L + k;
        double dc = 0.0;
        for (int j = 0; j < D; ++j) {
            const double zj = z[j * n + i];
            double zk = zj - alpha * d[j];
            zk = zk < 0.0 ? 0.0 : (zk > 1.0 ? 1.0 : zk);
            dc += g[j * n + i] * (zk - zj);
            ttheta[j * nt + t] = to_theta(zk, b.lo[j], b.hi[j], b.lg[j]);
        }
        dec[t] = done[i] ? INFINITY : dc;
    }
}

// Accept the first trial satisfying Armijo; otherwise the point is finished.
__global__ void k_lb_select(int64_t n, int32_t D, int32_t L, const double *z, const double *g,
                            const double *J, const double *Jt, const double *dec,
                            const int32_t *cnt, const int32_t *head, const double *S,
                            const double *Y, const double *rho, double *znew, double *Jnew,
                            int32_t *done) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int acc = -1;
    if (!done[i]) {
        for (int k = 0; k < L; ++k) {
            const int64_t t = i * L + k;
            if (Jt[t] <= J[i] + 1e-4 * dec[t] && dec[t] < 0.0) {
                acc = k;
                break;
            }
        }
    }
    if (acc < 0) {
        done[i] = 1;
        for (int j = 0; j < D; ++j) znew[j * n + i] = z[j * n + i];
        Jnew[i] = J[i];
        return;
    }
    // recompute the accepted point exactly as k_lb_dir did
    double q[kMaxParams], d[kMaxParams], al[kHist];
    for (int j = 0; j < D; ++j) q[j] = g[j * n + i];
    const int hn = cnt[i], hd = head[i];
    for (int k = 0; k < hn; ++k) {
        const int h = (hd - 1 - k + kHist) % kHist;
        double sq = 0.0;
        for (int j = 0; j < D; ++j) sq += S[((int64_t)h * D + j) * n + i] * q[j];
        al[h] = rho[(int64_t)h * n + i] * sq;
        for (int j = 0; j < D; ++j) q[j] -= al[h] * Y[((int64_t)h * D + j) * n + i];
    }
    double gamma = 1.0;
    if (hn > 0) {
        const int h = (hd - 1 + kHist) % kHist;
        double sy = 0.0, yy = 0.0;
        for (int j = 0; j < D; ++j) {
            const double sj = S[((int64_t)h * D + j) * n + i], yj = Y[((int64_t)h * D + j) * n + i];
            sy += sj * yj;
            yy += yj * yj;
        }
        gamma = sy / yy;
    }
    for (int j = 0; j < D; ++j) d[j] = gamma * q[j];
    for (int k = hn - 1; k >= 0; --k) {
        const int h = (hd - 1 - k + kHist) % kHist;
        double yd = 0.0;
        for (int j = 0; j < D; ++j) yd += Y[((int64_t)h * D + j) * n + i] * d[j];
        const double be = rho[(int64_t)h * n + i] * yd;
        for (int j = 0; j < D; ++j) d[j] += S[((int64_t)h * D + j) * n + i] * (al[h] - be);
    }
    const double alpha = ::ldexp(1.0, -acc);
    for (int j = 0; j < D; ++j) {
        double zk = z[j * n + i] - alpha * d[j];
        znew[j * n + i] = zk < 0.0 ? 0.0 : (zk > 1.0 ? 1.0 : zk);
    }
    Jnew[i] = Jt[i * L + acc];
}

// History update with the new gradient (SI in gnew, converted here), then move to znew.
__global__ void k_lb_update(int64_t n, int32_t D, double *z, double *g, double *J,
                            const double *znew, double *gnew, const double *Jnew,
                            const int32_t *stnew, double *S, double *Y, double *rho, int32_t *cnt,
                            int32_t *head, int32_t *done, Box b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (done[i]) return;
    if (stnew[i] != 0) {
        done[i] = 1;
        return;
    }
    double s[kMaxParams], y[kMaxParams], sy = 0.0, ss = 0.0, yy = 0.0;
    for (int j = 0; j < D; ++j) {
        const double zn = znew[j * n + i];
        const double gz = gnew[j * n + i] * dtheta_dz(zn, b.lo[j], b.hi[j], b.lg[j]);
        gnew[j * n + i] = gz;
        s[j] = zn - z[j * n + i];
        y[j] = gz - g[j * n + i];
        sy += s[j] * y[j];
        ss += s[j] * s[j];
        yy += y[j] * y[j];
    }
    if (sy > 1e-12 * ::sqrt(ss) * ::sqrt(yy)) {
        const int h = head[i];
        for (int j = 0; j < D; ++j) {
            S[((int64_t)h * D + j) * n + i] = s[j];
            Y[((int64_t)h * D + j) * n + i] = y[j];
        }
        rho[(int64_t)h * n + i] = 1.0 / sy;
        head[i] = (h + 1) % kHist;
        if (cnt[i] < kHist) cnt[i] += 1;
    }
    for (int j = 0; j < D; ++j) {
        z[j * n + i] = znew[j * n + i];
        g[j * n + i] = gnew[j * n + i];
    }
    J[i] = Jnew[i];
}

__global__ void k_copy(int64_t n, const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Per swarm (one workgroup each): the k particles with the lowest pbest_J (ties to the lowest
// index), copied as polish points s*k + r with their target row and period count.
__global__ void __launch_bounds__(256) k_topk(int32_t D, int32_t P, int32_t S, int32_t k,
                                              const double *pbest_J, const double *pbest_z,
                                              int32_t *taken, double *zsel, int32_t *tsel,
                                              const int32_t *ncyc, int32_t *nsel,
                                              const double *sbase, double *bsel) {
    const int32_t s = blockIdx.x;
    const int64_t n = (int64_t)S * P, base = (int64_t)s * P, m = (int64_t)S * k;
    for (int32_t p = threadIdx.x; p < P; p += blockDim.x) taken[base + p] = 0;
    __syncthreads();
    __shared__ double sv[4];
    __shared__ int si[4];
    __shared__ int pick;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int32_t r = 0; r < k; ++r) {
        double bv = INFINITY;
        int bi = INT_MAX;
        for (int32_t p = threadIdx.x; p < P; p += blockDim.x) {
            if (taken[base + p]) continue;
            const double v = pbest_J[base + p];
            if (v < bv || (v == bv && p < bi) || bi == INT_MAX) {
                if (bi == INT_MAX || v < bv || (v == bv && p < bi)) {
                    bv = v;
                    bi = p;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (oi != INT_MAX && (bi == INT_MAX || ov < bv || (ov == bv && oi < bi))) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            sv[wave] = bv;
            si[wave] = bi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
                if (si[w] != INT_MAX && (bi == INT_MAX || sv[w] < bv || (sv[w] == bv && si[w] < bi))) {
                    bv = sv[w];
                    bi = si[w];
                }
            pick = bi;
            if (bi != INT_MAX) taken[base + bi] = 1;
        }
        __syncthreads();
        if (threadIdx.x < D && pick != INT_MAX)
            zsel[(int64_t)threadIdx.x * m + (int64_t)s * k + r] = pbest_z[(int64_t)threadIdx.x * n + base + pick];
        if (threadIdx.x == 0) {
            tsel[(int64_t)s * k + r] = s;
            if (ncyc) nsel[(int64_t)s * k + r] = ncyc[s];
        }
        if (sbase && threadIdx.x < kMaxParams)
            bsel[(int64_t)threadIdx.x * m + (int64_t)s * k + r] = sbase[(int64_t)threadIdx.x * S + s];
        __syncthreads();
    }
}

// Per swarm: the best polished point replaces the swarm best when it is lower.
__global__ void k_merge(int32_t D, int32_t S, int32_t k, const double *zsel, const double *Jsel,
                        double *gbest_z, double *gbest_J) {
    const int32_t s = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= S) return;
    const int64_t m = (int64_t)S * k;
    int best = -1;
    double bv = gbest_J[s];
    for (int r = 0; r < k; ++r) {
        const double v = Jsel[(int64_t)s * k + r];
        if (v < bv) {
            bv = v;
            best = r;
        }
    }
    if (best >= 0) {
        gbest_J[s] = bv;
        for (int j = 0; j < D; ++j) gbest_z[(int64_t)j * S + s] = zsel[(int64_t)j * m + (int64_t)s * k + best];
    }
}

Box make_box(const afm_plan *plan) {
    Box b{};
    for (int j = 0; j < kMaxParams; ++j) {
        b.lo[j] = plan->prob.lo[j];
        b.hi[j] = plan->prob.hi[j];
        b.lg[j] = plan->prob.log_scale[j];
    }
    return b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Workspace of a polish of n points (doubles unless noted), carved from one allocation.
struct PolishWs {
    double *theta, *g, *gnew, *znew, *J, *Jnew, *S, *Y, *rho, *ttheta, *Jt, *dec;
    int32_t *cnt, *head, *done, *st, *stt;
};

size_t polish_ws_bytes(int64_t n, int32_t D, int32_t L) {
    const size_t nd = sizeof(double) * (size_t)n, ni = sizeof(int32_t) * (size_t)n;
    return align256(nd * D) * 4 + align256(nd) * 2 + align256(nd * D * kHist) * 2 +
           align256(nd * kHist) + align256(nd * D * L) + align256(nd * L) * 2 + align256(ni) * 4 +
           align256(ni * L);
}

static PolishWs carve(void *base, int64_t n, int32_t D, int32_t L) {
    char *p = (char *)base;
    const size_t nd = sizeof(double) * (size_t)n, ni = sizeof(int32_t) * (size_t)n;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return r;
    };
    PolishWs w;
    w.theta = (double *)take(nd * D);
    w.g = (double *)take(nd * D);
    w.gnew = (double *)take(nd * D);
    w.znew = (double *)take(nd * D);
    w.J = (double *)take(nd);
    w.Jnew = (double *)take(nd);
    w.S = (double *)take(nd * D * kHist);
    w.Y = (double *)take(nd * D * kHist);
    w.rho = (double *)take(nd * kHist);
    w.ttheta = (double *)take(nd * D * L);
    w.Jt = (double *)take(nd * L);
    w.dec = (double *)take(nd * L);
    w.cnt = (int32_t *)take(ni);
    w.head = (int32_t *)take(ni);
    w.done = (int32_t *)take(ni);
    w.st = (int32_t *)take(ni);
    w.stt = (int32_t *)take(ni * L);
    return w;
}

// Enqueue `steps` L-BFGS iterations on n points z [D][n] (in/out) with the given targets.
hipError_t enqueue_polish(afm_plan *plan, void *ws, int64_t n, double *z,
                          const int32_t *target_id, const double *targets, int32_t n_targets,
                          const int32_t *n_cycles, const double *base, int32_t steps, int32_t kc,
                          double *J_out, hipStream_t s) {
    const int32_t D = plan->prob.n_free, L = 21;
    const int32_t prec = polish_prec(plan);
    PolishWs w = carve(ws, n, D, L);
    const Box b = make_box(plan);
    const unsigned blocks = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_lb_theta, dim3(blocks), dim3(64), 0, s, n, D, z, w.theta, b);
    GradArgs ga{};
    ga.n = n;
    ga.ld = n;
    ga.theta = w.theta;
    ga.n_cycles = n_cycles;
    ga.target_id = target_id;
    ga.targets = targets;
    ga.n_targets = n_targets;
    ga.J = w.J;
    ga.dJ = w.g;
    ga.status = w.st;
    ga.kc = kc;
    ga.base = base;
    ga.base_ld = n;
    // one lane per mode while the groups fit one wave per SIMD (same bits, shorter streams)
    ga.mp = plan->kc.nm > 1 && n * 4 <= 65536;
    ga.form = grad_default_form(plan);
    ga.seg = (float *)((char *)ws + align256(polish_ws_bytes(n, D, L)));
    ga.ckpt = (float *)((char *)ga.seg + align256(grad_seg_bytes(plan, prec, n, kc, ga.form)));
    hipError_t e = launch_grad_p(plan, prec, ga, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lb_start, dim3(blocks), dim3(64), 0, s, n, D, (const double *)z, w.g,
                       w.cnt, w.head, w.done, (const int32_t *)w.st, b);
    FwdArgs fa{};
    fa.n = n * L;
    fa.ld = n * L;
    fa.theta = w.ttheta;
    fa.n_cycles = n_cycles;
    fa.target_id = target_id;
    fa.targets = targets;
    fa.n_targets = n_targets;
    fa.group = L;
    fa.base = base;
    fa.base_ld = n;
    fa.J = w.Jt;
    fa.status = w.stt;
    for (int32_t it = 0; it < steps; ++it) {
        hipLaunchKernelGGL(k_lb_dir, dim3(blocks), dim3(64), 0, s, n, D, L, (const double *)z,
                           (const double *)w.g, (const double *)w.S, (const double *)w.Y,
                           (const double *)w.rho, (const int32_t *)w.cnt,
                           (const int32_t *)w.head, (const int32_t *)w.done, w.ttheta, w.dec, b);
        e = launch_forward_p(plan, prec, fa, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lb_select, dim3(blocks), dim3(64), 0, s, n, D, L, (const double *)z,
                           (const double *)w.g, (const double *)w.J, (const double *)w.Jt,
                           (const double *)w.dec, (const int32_t *)w.cnt,
                           (const int32_t *)w.head, (const double *)w.S, (const double *)w.Y,
                           (const double *)w.rho, w.znew, w.Jnew, w.done);
        hipLaunchKernelGGL(k_lb_theta, dim3(blocks), dim3(64), 0, s, n, D, (const double *)w.znew,
                           w.theta, b);
        ga.J = w.Jt;  // gradient pass re-evaluates J at znew; keep the line-search value
        ga.dJ = w.gnew;
        ga.status = w.st;
        e = launch_grad_p(plan, prec, ga, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lb_update, dim3(blocks), dim3(64), 0, s, n, D, z, w.g, w.J,
                           (const double *)w.znew, w.gnew, (const double *)w.Jnew,
                           (const int32_t *)w.st, w.S, w.Y, w.rho, w.cnt, w.head, w.done, b);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (J_out) {
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(64), 0, s, n, (const double *)w.J, J_out);
        e = hipGetLastError();
    }
    return e;
}

hipError_t enqueue_topk(const afm_plan *plan, const afm_swarm &sw, int32_t k, int32_t *taken,
                        double *zsel, int32_t *tsel, const int32_t *ncyc, int32_t *nsel,
                        const double *swarm_base, double *bsel, hipStream_t s) {
    hipLaunchKernelGGL(k_topk, dim3((unsigned)sw.swarms), dim3(256), 0, s, sw.n_dim, sw.particles,
                       sw.swarms, k, (const double *)sw.pbest_J, (const double *)sw.pbest_z, taken,
                       zsel, tsel, ncyc, nsel, swarm_base, bsel);
    return hipGetLastError();
}

hipError_t enqueue_merge(const afm_swarm &sw, int32_t k, const double *zsel, const double *Jsel,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_merge, dim3((unsigned)((sw.swarms + 63) / 64)), dim3(64), 0, s, sw.n_dim,
                       sw.swarms, k, zsel, Jsel, sw.gbest_z, sw.gbest_J);
    return hipGetLastError();
}

size_t polish_total_bytes(const afm_plan *plan, int64_t n, int32_t kc) {
    const int32_t D = plan->prob.n_free, L = 21, prec = polish_prec(plan);
    return align256(polish_ws_bytes(n, D, L)) +
           align256(grad_seg_bytes(plan, prec, n, kc, grad_default_form(plan))) +
           grad_ckpt_bytes(plan, prec, n, kc) + 256;
}

}  // namespace afm
