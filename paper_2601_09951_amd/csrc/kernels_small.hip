// kernels_small.hip -- the whole per-bond-length loop of Algorithm 1
// (arXiv 2601.09951, Section 4.2) in one persistent launch for small states.
//
// One workgroup owns one instance (one bond length or parameter point, Eq. 7)
// and keeps everything on chip for all iterations: psi and lambda in LDS,
// gate matrices, parameters and Adam moments in LDS.  Each iteration runs
//   prepare e_ref -> gates (Eqs. 4-5) -> lambda = H psi, E = <psi|lambda>
//   -> reverse sweep g_l = Im<lambda|G_l|psi> with U_l^dag on both
//   -> dE/dtheta -> Adam (Section 3.4) or gradient descent,
// and after the last step the energy at the final parameters.  There is no
// host round trip and no HBM traffic inside the loop apart from the tiny
// term tables (cache resident) and the per-step energy store.
#include "internal.h"

namespace vqe {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b)
{
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ uint32_t insert_zeros(uint32_t j, int nfix, const uint8_t *pos)
{
    for (int i = 0; i < nfix; ++i) {
        const uint32_t p = pos[i];
        j = ((j >> p) << (p + 1)) | (j & ((1u << p) - 1u));
    }
    return j;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// workgroup sum in fixed order; valid in every thread after the call
__device__ __forceinline__ double block_sum_all(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ void gate_matrix(int kind, double a, double2 *m)
{
    double s, c;
    sincos(0.5 * a, &s, &c);
    double2 u00 = {0, 0}, u01 = {0, 0}, u10 = {0, 0}, u11 = {0, 0};
    switch (kind) {
    case VQE_GATE_RX: u00 = {c, 0}; u01 = {0, -s}; u10 = {0, -s}; u11 = {c, 0}; break;
    case VQE_GATE_RY:
    case VQE_GATE_SINGLE_EXC:
    case VQE_GATE_DOUBLE_EXC: u00 = {c, 0}; u01 = {-s, 0}; u10 = {s, 0}; u11 = {c, 0}; break;
    case VQE_GATE_RZ: u00 = {c, -s}; u11 = {c, s}; break;
    case VQE_GATE_H: {
        const double r = 0.70710678118654752440;
        u00 = {r, 0}; u01 = {r, 0}; u10 = {r, 0}; u11 = {-r, 0};
        break;
    }
    case VQE_GATE_X:
    case VQE_GATE_CNOT: u01 = {1, 0}; u10 = {1, 0}; break;
    case VQE_GATE_CZ: u00 = {1, 0}; u11 = {-1, 0}; break;
    }
    m[0] = u00;
    m[1] = u01;
    m[2] = u10;
    m[3] = u11;
}

__device__ __forceinline__ void term_sums(const TermDev *__restrict__ terms, int tb, int tm, int te,
                                          uint32_t b, double &A, double &B)
{
    A = 0.0;
    B = 0.0;
    for (int t = tb; t < tm; ++t) {
        const TermDev d = terms[t];
        A += (__popc(d.zloc & b) & 1) ? -d.w : d.w;
    }
    for (int t = tm; t < te; ++t) {
        const TermDev d = terms[t];
        B += (__popc(d.zloc & b) & 1) ? -d.w : d.w;
    }
}

struct SmallLayout {
    int D, G, P, NPG, nw;
    size_t psi, lam, mats, th, mom, vel, grd, red, bred, total;
};

__host__ __device__ inline SmallLayout small_layout(int n, int G, int P, int NPG, int nthreads)
{
    SmallLayout L;
    L.D = 1 << n;
    L.G = G;
    L.P = P;
    L.NPG = NPG;
    L.nw = nthreads / 64;
    size_t o = 0;
    L.psi = o; o += (size_t)16 * L.D;
    L.lam = o; o += (size_t)16 * L.D;
    L.mats = o; o += (size_t)64 * G;
    L.th = o; o += (size_t)8 * P;
    L.mom = o; o += (size_t)8 * P;
    L.vel = o; o += (size_t)8 * P;
    L.grd = o; o += (size_t)8 * P;
    L.red = o; o += (size_t)8 * NPG * L.nw;
    L.bred = o; o += (size_t)8 * L.nw;
    L.total = o;
    return L;
}

struct SmallKernelArgs {
    SmallRunArgs a;
    const OpDesc *rops;      // reverse single-pass ops
    const int32_t *pmap_off; // [P+1]
    const int32_t *pmap_idx;
    int n_pgates;
    int nthreads;
};

__global__ __launch_bounds__(256) void k_small_run(SmallKernelArgs ka)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallRunArgs &a = ka.a;
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, ka.n_pgates, blockDim.x);
    double2 *psi = reinterpret_cast<double2 *>(smem + L.psi);
    double2 *lam = reinterpret_cast<double2 *>(smem + L.lam);
    double2 *mats = reinterpret_cast<double2 *>(smem + L.mats);
    double *th = reinterpret_cast<double *>(smem + L.th);
    double *mom = reinterpret_cast<double *>(smem + L.mom);
    double *vel = reinterpret_cast<double *>(smem + L.vel);
    double *grd = reinterpret_cast<double *>(smem + L.grd);
    double *red = reinterpret_cast<double *>(smem + L.red);
    double *bred = reinterpret_cast<double *>(smem + L.bred);

    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int inst = blockIdx.x;
    const int D = L.D, G = L.G, P = L.P;
    const int32_t *to = a.toff + (size_t)(a.shared_ham ? 0 : inst) * a.n_groups * 3;
    double *energies = a.energies + (size_t)inst * (a.iters + 1);

    for (int p = tid; p < P; p += bs) {
        th[p] = a.theta[(size_t)inst * P + p];
        mom[p] = 0.0;
        vel[p] = 0.0;
    }
    __syncthreads();

    for (int it = 0; it <= a.iters; ++it) {
        // gate matrices at the current parameters; reference state
        for (int g = tid; g < G; g += bs) {
            const GateDev gd = a.gates[g];
            gate_matrix(gd.kind, gd.pidx >= 0 ? th[gd.pidx] : gd.fixed, mats + 4 * g);
        }
        for (int j = tid; j < D; j += bs) {
            psi[j] = make_double2(j == (int)a.ref ? 1.0 : 0.0, 0.0);
            lam[j] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        // U(theta) e_ref
        for (int q = 0; q < G; ++q) {
            const OpDesc o = a.ops[q];
            const double2 u00 = mats[4 * o.gate], u01 = mats[4 * o.gate + 1];
            const double2 u10 = mats[4 * o.gate + 2], u11 = mats[4 * o.gate + 3];
            const int np = D >> o.nfix;
            for (int j = tid; j < np; j += bs) {
                const uint32_t p0 = insert_zeros((uint32_t)j, o.nfix, o.fixpos) | o.fixed_bits;
                const uint32_t p1 = p0 ^ o.m;
                const double2 x = psi[p0], y = psi[p1];
                if (o.cls == CLS_SWAP) {
                    psi[p0] = y;
                    psi[p1] = x;
                } else if (o.cls == CLS_DIAG) {
                    psi[p0] = cmul(u00, x);
                    psi[p1] = cmul(u11, y);
                } else {
                    psi[p0] = cadd(cmul(u00, x), cmul(u01, y));
                    psi[p1] = cadd(cmul(u10, x), cmul(u11, y));
                }
            }
            __syncthreads();
        }
        // lambda = H psi (paired over (b, b ^ f)); E = Re <psi|lambda>
        for (int q = 0; q < a.n_groups; ++q) {
            const GroupDev gd = a.groups[q];
            const int tb = to[gd.ugroup * 3], tm = to[gd.ugroup * 3 + 1], te = to[gd.ugroup * 3 + 2];
            if (te == tb) continue;
            if (gd.floc == 0) {
                for (int j = tid; j < D; j += bs) {
                    double A, B;
                    term_sums(a.terms, tb, tm, te, (uint32_t)j, A, B);
                    const double2 x = psi[j];
                    lam[j] = cadd(lam[j], make_double2(A * x.x, A * x.y));
                }
            } else {
                const uint32_t pv = gd.pivot;
                for (int j = tid; j < (D >> 1); j += bs) {
                    const uint32_t b = (((uint32_t)j >> pv) << (pv + 1)) | ((uint32_t)j & ((1u << pv) - 1u));
                    const uint32_t bf = b ^ gd.floc;
                    double A, B;
                    term_sums(a.terms, tb, tm, te, b, A, B);
                    const double2 x0 = psi[b], x1 = psi[bf];
                    lam[bf] = cadd(lam[bf], make_double2(A * x0.x - B * x0.y, A * x0.y + B * x0.x));
                    lam[b] = cadd(lam[b], make_double2(A * x1.x + B * x1.y, A * x1.y - B * x1.x));
                }
            }
            __syncthreads();
        }
        double e = 0.0;
        for (int j = tid; j < D; j += bs) e += psi[j].x * lam[j].x + psi[j].y * lam[j].y;
        e = block_sum_all(e, bred);
        if (tid == 0) energies[it] = e;
        if (it == a.iters) break;

        // reverse sweep
        for (int i = tid; i < L.NPG * L.nw; i += bs) red[i] = 0.0;
        __syncthreads();
        for (int q = 0; q < G; ++q) {
            const OpDesc o = ka.rops[q];
            const double2 v00 = cconj(mats[4 * o.gate]), v01 = cconj(mats[4 * o.gate + 2]);
            const double2 v10 = cconj(mats[4 * o.gate + 1]), v11 = cconj(mats[4 * o.gate + 3]);
            const int np = D >> o.nfix;
            const bool param = o.pgate >= 0;
            double acc = 0.0;
            for (int j = tid; j < np; j += bs) {
                const uint32_t p0 = insert_zeros((uint32_t)j, o.nfix, o.fixpos) | o.fixed_bits;
                const uint32_t p1 = p0 ^ o.m;
                const double2 x = psi[p0], y = psi[p1];
                const double2 lx = lam[p0], ly = lam[p1];
                if (param) {
                    if (o.gen == GEN_Y)
                        acc += -(lx.x * y.x + lx.y * y.y) + (ly.x * x.x + ly.y * x.y);
                    else if (o.gen == GEN_X)
                        acc += (lx.x * y.y - lx.y * y.x) + (ly.x * x.y - ly.y * x.x);
                    else
                        acc += (lx.x * x.y - lx.y * x.x) - (ly.x * y.y - ly.y * y.x);
                }
                if (o.cls == CLS_SWAP) {
                    psi[p0] = y;
                    psi[p1] = x;
                    lam[p0] = ly;
                    lam[p1] = lx;
                } else if (o.cls == CLS_DIAG) {
                    psi[p0] = cmul(v00, x);
                    psi[p1] = cmul(v11, y);
                    lam[p0] = cmul(v00, lx);
                    lam[p1] = cmul(v11, ly);
                } else {
                    psi[p0] = cadd(cmul(v00, x), cmul(v01, y));
                    psi[p1] = cadd(cmul(v10, x), cmul(v11, y));
                    lam[p0] = cadd(cmul(v00, lx), cmul(v01, ly));
                    lam[p1] = cadd(cmul(v10, lx), cmul(v11, ly));
                }
            }
            if (param) {
                acc = wave_sum(acc);
                if (lane == 0) red[o.pgate * L.nw + wave] = acc;
            }
            __syncthreads();
        }
        // dE/dtheta_p and the optimiser step
        for (int p = tid; p < P; p += bs) {
            double gp = 0.0;
            for (int e2 = ka.pmap_off[p]; e2 < ka.pmap_off[p + 1]; ++e2) {
                const int pg = ka.pmap_idx[e2];
                double s = 0.0;
                for (int w = 0; w < L.nw; ++w) s += red[pg * L.nw + w];
                gp += s;
            }
            grd[p] = gp;
            if (a.opt == VQE_OPT_ADAM) {
                const double mi = a.b1 * mom[p] + (1.0 - a.b1) * gp;
                const double vi = a.b2 * vel[p] + (1.0 - a.b2) * gp * gp;
                mom[p] = mi;
                vel[p] = vi;
                const double c1 = 1.0 - pow(a.b1, (double)(it + 1));
                const double c2 = 1.0 - pow(a.b2, (double)(it + 1));
                th[p] -= a.lr * (mi / c1) / (sqrt(vi / c2) + a.eps);
            } else {
                th[p] -= a.lr * gp;
            }
        }
        __syncthreads();
    }
    for (int p = tid; p < P; p += bs) a.theta[(size_t)inst * P + p] = th[p];
}

}  // namespace

int small_run_supported(int n, int n_gates, int n_params, int n_pgates, int max_terms)
{
    (void)max_terms;
    if (n > 10 || n_gates > 1024 || n_params > 1024) return 0;
    const int nthreads = n <= 7 ? 64 : (n == 8 ? 128 : 256);
    const SmallLayout L = small_layout(n, n_gates, n_params, n_pgates, nthreads);
    return L.total <= 150 * 1024;
}

hipError_t launch_small_run(const SmallRunArgs &a, const OpDesc *rops, const int32_t *pmap_off,
                            const int32_t *pmap_idx, int n_pgates, int64_t batch, hipStream_t s)
{
    const int nthreads = a.n <= 7 ? 64 : (a.n == 8 ? 128 : 256);
    SmallKernelArgs ka;
    ka.a = a;
    ka.rops = rops;
    ka.pmap_off = pmap_off;
    ka.pmap_idx = pmap_idx;
    ka.n_pgates = n_pgates;
    ka.nthreads = nthreads;
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, n_pgates, nthreads);
    if (L.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_small_run),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_small_run, dim3((unsigned)batch), dim3(nthreads), L.total, s, ka);
    return hipGetLastError();
}

}  // namespace vqe
