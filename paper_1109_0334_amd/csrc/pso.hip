// pso.hip -- particle swarm optimisation kernels (paper Sec. 3.4, Eq. 8).
//
// Swarm state is structure-of-arrays in HBM ([D][S*P] rows), so the per-particle loops read and
// write coalesced rows.  One workgroup owns one swarm: personal bests, the swarm-best argmin
// (wavefront shuffles, then LDS across the workgroup's waves) and the velocity/position move
// happen in a single launch per generation.  The move is FP64 with contraction disabled and a
// fixed evaluation order, so any IEEE implementation that evaluates it the same way -- the CPU
// oracle included -- reproduces it bit for bit given the same misfits.
#include <climits>

#include "afm_internal.hpp"

namespace afm {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32 bijection; in
// each round words 0 and 2 are multiplied (full 64-bit product) by the two round multipliers,
// the high halves are xored with the other two words and the round key, and the key advances
// by the two Weyl increments.
__device__ inline void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Uniform double in [0, 1) from the top 27 bits of a and the top 26 bits of b (exact).
__device__ inline double unit53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Random words for (swarm, iteration, particle, dimension, purpose):
// key (seed_lo, swarm), counter (iter, particle, dim << 8 | purpose, seed_hi).
__device__ inline void stream_words(uint64_t seed, int32_t swarm, int32_t iter, int32_t particle,
                                    int32_t dim, uint32_t purpose, uint32_t out[4]) {
    philox10((uint32_t)iter, (uint32_t)particle, ((uint32_t)dim << 8) | purpose,
             (uint32_t)(seed >> 32), (uint32_t)seed, (uint32_t)swarm, out);
}

struct PsoArgs {
    int32_t D, P, S;
    double *z, *v, *pbest_z, *pbest_J, *gbest_z, *gbest_J, *theta;
    int32_t *gen;
    const double *J;
    uint64_t seed;
    int32_t iter, is_last;
    double cutoff, w, c1, c2, vmax;
    double lo[kMaxParams], hi[kMaxParams];
    int32_t lg[kMaxParams];
};

// normalised coordinate -> SI parameter
__device__ inline double to_theta(double z, double lo, double hi, int32_t lg) {
    if (lg) return ::exp(::log(lo) + z * (::log(hi) - ::log(lo)));
    return lo + z * (hi - lo);
}

__global__ void __launch_bounds__(256) k_swarm_init(PsoArgs a) {
    const int64_t n = (int64_t)a.S * a.P;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int32_t s = (int32_t)(t / a.P), p = (int32_t)(t % a.P);
        for (int j = 0; j < a.D; ++j) {
            uint32_t rz[4], rv[4];
            stream_words(a.seed, s, 0, p, j, 1u, rz);
            stream_words(a.seed, s, 0, p, j, 2u, rv);
            const double z0 = unit53(rz[0], rz[1]);
            const int64_t ij = (int64_t)j * n + t;
            a.z[ij] = z0;
            a.v[ij] = unit53(rv[0], rv[1]) - z0;
            a.pbest_z[ij] = z0;
            a.theta[ij] = to_theta(z0, a.lo[j], a.hi[j], a.lg[j]);
        }
        a.pbest_J[t] = INFINITY;
    }
    if (t < a.S) {
        a.gbest_J[t] = INFINITY;
        a.gen[t] = -1;
        for (int j = 0; j < a.D; ++j) a.gbest_z[(int64_t)j * a.S + t] = 0.0;
    }
}

// (value, index) lexicographic minimum: lowest value, ties to the lowest index.
__device__ inline void better(double &bv, int &bi, double v, int i) {
    if (v < bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
    }
}

__global__ void __launch_bounds__(256) k_pso_step(PsoArgs a) {
#pragma clang fp contract(off)
    const int32_t s = blockIdx.x;
    const int32_t P = a.P, D = a.D;
    const int64_t n = (int64_t)a.S * P, base = (int64_t)s * P;
    // 1. personal bests (strict improvement; non-finite misfits count as +inf)
    for (int32_t p = threadIdx.x; p < P; p += blockDim.x) {
        double Jg = a.J[base + p];
        if (!isfinite(Jg)) Jg = INFINITY;
        if (Jg < a.pbest_J[base + p]) {
            a.pbest_J[base + p] = Jg;
            for (int j = 0; j < D; ++j) a.pbest_z[(int64_t)j * n + base + p] = a.z[(int64_t)j * n + base + p];
        }
    }
    // 2. swarm best: lane-local scan, 64-lane shuffle tree, then across waves through LDS
    double bv = INFINITY;
    int bi = INT_MAX;
    for (int32_t p = threadIdx.x; p < P; p += blockDim.x) better(bv, bi, a.pbest_J[base + p], p);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        better(bv, bi, ov, oi);
    }
    __shared__ double s_v[4];
    __shared__ int s_i[4];
    __shared__ double s_gz[kMaxParams];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_v[wave] = bv;
        s_i[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) better(bv, bi, s_v[w], s_i[w]);
        a.gbest_J[s] = bv;
        for (int j = 0; j < D; ++j) {
            const double g = a.pbest_z[(int64_t)j * n + base + bi];
            a.gbest_z[(int64_t)j * a.S + s] = g;
            s_gz[j] = g;
        }
        if (a.gen[s] < 0 && ::sqrt(bv) <= a.cutoff) a.gen[s] = a.iter;
    }
    __syncthreads();
    if (a.is_last) return;
    // 3. Eq. 8 move, clamped velocity, positions kept in the box
    for (int32_t p = threadIdx.x; p < P; p += blockDim.x) {
        for (int j = 0; j < D; ++j) {
            uint32_t r[4];
            stream_words(a.seed, s, a.iter, p, j, 0u, r);
            const double r1 = unit53(r[0], r[1]), r2 = unit53(r[2], r[3]);
            const int64_t ij = (int64_t)j * n + base + p;
            const double zj = a.z[ij];
            const double t1 = a.w * a.v[ij];
            const double t2 = (a.c1 * r1) * (a.pbest_z[ij] - zj);
            const double t3 = (a.c2 * r2) * (s_gz[j] - zj);
            double vn = (t1 + t2) + t3;
            if (vn > a.vmax) vn = a.vmax;
            if (vn < -a.vmax) vn = -a.vmax;
            double zn = zj + vn;
            if (zn < 0.0) {
                zn = 0.0;
                vn = 0.0;
            }
            if (zn > 1.0) {
                zn = 1.0;
                vn = 0.0;
            }
            a.z[ij] = zn;
            a.v[ij] = vn;
            a.theta[ij] = to_theta(zn, a.lo[j], a.hi[j], a.lg[j]);
        }
    }
}

__global__ void k_gather_best(PsoArgs a, double *best_theta, double *best_J, int32_t *gen) {
    const int32_t s = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= a.S) return;
    for (int j = 0; j < a.D; ++j)
        best_theta[(int64_t)j * a.S + s] = to_theta(a.gbest_z[(int64_t)j * a.S + s], a.lo[j], a.hi[j], a.lg[j]);
    best_J[s] = a.gbest_J[s];
    gen[s] = a.gen[s];
}

PsoArgs make_args(const afm_plan *plan, const afm_swarm &sw) {
    PsoArgs a{};
    a.D = sw.n_dim;
    a.P = sw.particles;
    a.S = sw.swarms;
    a.z = sw.z;
    a.v = sw.v;
    a.pbest_z = sw.pbest_z;
    a.pbest_J = sw.pbest_J;
    a.gbest_z = sw.gbest_z;
    a.gbest_J = sw.gbest_J;
    a.theta = sw.theta;
    a.gen = sw.gen_to_cutoff;
    a.w = plan->pso_w;
    a.c1 = plan->pso_c1;
    a.c2 = plan->pso_c2;
    a.vmax = plan->pso_vmax;
    for (int j = 0; j < kMaxParams; ++j) {
        a.lo[j] = plan->prob.lo[j];
        a.hi[j] = plan->prob.hi[j];
        a.lg[j] = plan->prob.log_scale[j];
    }
    return a;
}

}  // namespace

hipError_t launch_swarm_init(const afm_plan *plan, const afm_swarm &sw, uint64_t seed,
                             hipStream_t s) {
    PsoArgs a = make_args(plan, sw);
    a.seed = seed;
    const int64_t n = (int64_t)sw.swarms * sw.particles;
    const int64_t cover = n > sw.swarms ? n : sw.swarms;
    hipLaunchKernelGGL(k_swarm_init, dim3((unsigned)((cover + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pso_step(const afm_plan *plan, const afm_swarm &sw, const double *J,
                           uint64_t seed, int32_t iter, int32_t is_last, double cutoff,
                           hipStream_t s) {
    PsoArgs a = make_args(plan, sw);
    a.J = J;
    a.seed = seed;
    a.iter = iter;
    a.is_last = is_last;
    a.cutoff = cutoff;
    // one workgroup per swarm; small swarms use a single wave
    const int block = sw.particles <= 64 ? 64 : (sw.particles <= 128 ? 128 : 256);
    hipLaunchKernelGGL(k_pso_step, dim3((unsigned)sw.swarms), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather_best(const afm_plan *plan, const afm_swarm &sw, double *best_theta,
                              double *best_J, int32_t *gen, hipStream_t s) {
    PsoArgs a = make_args(plan, sw);
    hipLaunchKernelGGL(k_gather_best, dim3((unsigned)((sw.swarms + 255) / 256)), dim3(256), 0, s,
                       a, best_theta, best_J, gen);
    return hipGetLastError();
}

}  // namespace afm
