// kernels_small.hip -- the whole per-bond-length loop of Algorithm 1
// (arXiv 2601.09951, Section 4.2) in one persistent launch for small states.
//
// One workgroup owns one instance (one bond length or parameter point, Eq. 7)
// and keeps everything on chip for all iterations: psi and lambda in LDS,
// gate matrices, parameters and Adam moments in LDS, and the instance's
// Hamiltonian.  Each iteration runs
//   prepare e_ref -> gates (Eqs. 4-5) -> lambda = H psi, E = <psi|lambda>
//   -> reverse sweep g_l = Im<lambda|G_l|psi> with U_l^dag on both
//   -> dE/dtheta -> Adam (Section 3.4) or gradient descent,
// and after the last step the energy at the final parameters.
//
// The Hamiltonian is held in one of two forms:
//  * table form: for every flip group f the diagonal D_f[b] = s_f(b ^ f)
//    with s_f(b) = sum_{t in f} kappa_t (-1)^{z_t . b}, so that
//    lambda[b] = sum_f D_f[b] psi[b ^ f] is a barrier-free gather (H in
//    XOR-offset diagonal storage, built once per launch);
//  * term form (when the table does not fit LDS): terms staged in LDS and
//    summed per pair of each flip group.
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

__device__ __forceinline__ uint32_t insert_zeros(uint32_t j, uint64_t pack, int nfix)
{
    for (int i = 0; i < nfix; ++i) {
        const uint32_t p = (uint32_t)(pack >> (6 * i)) & 63u;
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

// compact per-op record kept in LDS
struct SmallOp {
    uint32_t m, fixed_bits;
    uint64_t fixpack;   // 6-bit fields: ascending fixed positions
    int32_t gate, pgate;
    int16_t cls, gen;
    int32_t nfix;
};

struct SmallLayout {
    int D, G, P, NPG, NG, nw, nterms, mode;
    size_t psi, lam, mats, th, mom, vel, grd, red, bred, ops, rops, gf, tab, toff, tz, tw, total;
};

// mode 1: real table, 2: complex table, 0: term form
__host__ __device__ inline SmallLayout small_layout(int n, int G, int P, int NPG, int NG, int nterms,
                                                    int nthreads, int mode)
{
    SmallLayout L;
    L.D = 1 << n;
    L.G = G;
    L.P = P;
    L.NPG = NPG;
    L.NG = NG;
    L.nterms = nterms;
    L.mode = mode;
    L.nw = nthreads / 64;
    size_t o = 0;
    auto take = [&](size_t bytes, size_t align) {
        o = (o + align - 1) / align * align;
        size_t r = o;
        o += bytes;
        return r;
    };
    L.psi = take((size_t)16 * L.D, 16);
    L.lam = take((size_t)16 * L.D, 16);
    L.mats = take((size_t)64 * G, 16);
    L.th = take((size_t)8 * P, 8);
    L.mom = take((size_t)8 * P, 8);
    L.vel = take((size_t)8 * P, 8);
    L.grd = take((size_t)8 * P, 8);
    L.red = take((size_t)8 * NPG * L.nw, 8);
    L.bred = take((size_t)8 * L.nw, 8);
    L.ops = take(sizeof(SmallOp) * G, 16);
    L.rops = take(sizeof(SmallOp) * G, 16);
    L.gf = take((size_t)8 * NG, 8);  // uint32 flip, uint32 pivot
    if (mode == 1) {
        L.tab = take((size_t)8 * NG * L.D, 16);
        L.toff = L.tz = L.tw = o;
    } else if (mode == 2) {
        L.tab = take((size_t)16 * NG * L.D, 16);
        L.toff = L.tz = L.tw = o;
    } else {
        L.tab = o;
        L.toff = take((size_t)12 * NG, 4);
        L.tz = take((size_t)4 * nterms, 4);
        L.tw = take((size_t)8 * nterms, 8);
    }
    L.total = o;
    return L;
}

__device__ __forceinline__ SmallOp pack_op(const OpDesc &o)
{
    SmallOp s;
    s.m = o.m;
    s.fixed_bits = o.fixed_bits;
    uint64_t pk = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) pk |= (uint64_t)o.fixpos[i] << (6 * i);
    s.fixpack = pk;
    s.gate = o.gate;
    s.pgate = o.pgate;
    s.cls = o.cls;
    s.gen = o.gen;
    s.nfix = o.nfix;
    return s;
}

struct SmallKernelArgs {
    SmallRunArgs a;
    const OpDesc *rops;      // reverse single-pass ops
    const int32_t *pmap_off; // [P+1]
    const int32_t *pmap_idx;
    int n_pgates;
    int mode;
    int max_inst_terms;
};

__global__ __launch_bounds__(256) void k_small_run(SmallKernelArgs ka)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallRunArgs &a = ka.a;
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, ka.n_pgates, a.n_groups, ka.max_inst_terms,
                                       blockDim.x, ka.mode);
    double2 *psi = reinterpret_cast<double2 *>(smem + L.psi);
    double2 *lam = reinterpret_cast<double2 *>(smem + L.lam);
    double2 *mats = reinterpret_cast<double2 *>(smem + L.mats);
    double *th = reinterpret_cast<double *>(smem + L.th);
    double *mom = reinterpret_cast<double *>(smem + L.mom);
    double *vel = reinterpret_cast<double *>(smem + L.vel);
    double *red = reinterpret_cast<double *>(smem + L.red);
    double *bred = reinterpret_cast<double *>(smem + L.bred);
    SmallOp *fops = reinterpret_cast<SmallOp *>(smem + L.ops);
    SmallOp *rops = reinterpret_cast<SmallOp *>(smem + L.rops);
    uint32_t *gf = reinterpret_cast<uint32_t *>(smem + L.gf);
    double *tabr = reinterpret_cast<double *>(smem + L.tab);
    double2 *tabc = reinterpret_cast<double2 *>(smem + L.tab);
    int32_t *stoff = reinterpret_cast<int32_t *>(smem + L.toff);
    uint32_t *tz = reinterpret_cast<uint32_t *>(smem + L.tz);
    double *tw = reinterpret_cast<double *>(smem + L.tw);

    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int inst = blockIdx.x;
    const int D = L.D, G = L.G, P = L.P, NG = L.NG;
    const int32_t *to = a.toff + (size_t)(a.shared_ham ? 0 : inst) * NG * 3;
    double *energies = a.energies + (size_t)inst * (a.iters + 1);

    // ---- one-time staging: parameters, ops, groups, the Hamiltonian
    for (int p = tid; p < P; p += bs) {
        th[p] = a.theta[(size_t)inst * P + p];
        mom[p] = 0.0;
        vel[p] = 0.0;
    }
    for (int q = tid; q < G; q += bs) {
        fops[q] = pack_op(a.ops[q]);
        rops[q] = pack_op(ka.rops[q]);
    }
    for (int g = tid; g < NG; g += bs) {
        gf[2 * g] = a.groups[g].floc;
        gf[2 * g + 1] = a.groups[g].pivot;
    }
    __syncthreads();
    if (ka.mode != 0) {
        // D_g[b] = sum_t kappa_t (-1)^{z_t . (b ^ f_g)}
        for (int i = tid; i < NG * D; i += bs) {
            const int g = i / D;
            const uint32_t b = (uint32_t)(i - g * D);
            const int ug = a.groups[g].ugroup;
            const int tb = to[ug * 3], tm = to[ug * 3 + 1], te = to[ug * 3 + 2];
            const uint32_t bb = b ^ gf[2 * g];
            double re = 0.0, im = 0.0;
            for (int t = tb; t < tm; ++t) {
                const TermDev d = a.terms[t];
                re += (__popc(d.zloc & bb) & 1) ? -d.w : d.w;
            }
            for (int t = tm; t < te; ++t) {
                const TermDev d = a.terms[t];
                im += (__popc(d.zloc & bb) & 1) ? -d.w : d.w;
            }
            if (ka.mode == 1)
                tabr[i] = re;
            else
                tabc[i] = make_double2(re, im);
        }
    } else {
        // stage this instance's terms (contiguous in the term table)
        const int t0 = to[0];
        for (int g = tid; g < NG; g += bs) {
            const int ug = a.groups[g].ugroup;
            stoff[3 * g] = to[ug * 3] - t0;
            stoff[3 * g + 1] = to[ug * 3 + 1] - t0;
            stoff[3 * g + 2] = to[ug * 3 + 2] - t0;
        }
        const int t1 = to[(NG - 1) * 3 + 2];
        for (int t = tid; t < t1 - t0; t += bs) {
            tz[t] = a.terms[t0 + t].zloc;
            tw[t] = a.terms[t0 + t].w;
        }
    }
    __syncthreads();

    double b1t = 1.0, b2t = 1.0;  // beta1^t, beta2^t for Adam's bias corrections
    for (int it = 0; it <= a.iters; ++it) {
        // gate matrices at the current parameters; reference state
        for (int g = tid; g < G; g += bs) {
            const GateDev gd = a.gates[g];
            gate_matrix(gd.kind, gd.pidx >= 0 ? th[gd.pidx] : gd.fixed, mats + 4 * g);
        }
        for (int j = tid; j < D; j += bs) psi[j] = make_double2(j == (int)a.ref ? 1.0 : 0.0, 0.0);
        __syncthreads();
        // U(theta) e_ref
        for (int q = 0; q < G; ++q) {
            const SmallOp o = fops[q];
            const double2 u00 = mats[4 * o.gate], u01 = mats[4 * o.gate + 1];
            const double2 u10 = mats[4 * o.gate + 2], u11 = mats[4 * o.gate + 3];
            const int np = D >> o.nfix;
            for (int j = tid; j < np; j += bs) {
                const uint32_t p0 = insert_zeros((uint32_t)j, o.fixpack, o.nfix) | o.fixed_bits;
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
        // lambda = H psi; E = Re <psi|lambda>
        double e = 0.0;
        if (ka.mode != 0) {
            for (int b = tid; b < D; b += bs) {
                double2 acc = make_double2(0.0, 0.0);
                if (ka.mode == 1) {
                    for (int g = 0; g < NG; ++g) {
                        const double d = tabr[g * D + b];
                        const double2 x = psi[b ^ gf[2 * g]];
                        acc.x += d * x.x;
                        acc.y += d * x.y;
                    }
                } else {
                    for (int g = 0; g < NG; ++g) acc = cadd(acc, cmul(tabc[g * D + b], psi[b ^ gf[2 * g]]));
                }
                lam[b] = acc;
                const double2 x = psi[b];
                e += x.x * acc.x + x.y * acc.y;
            }
        } else {
            for (int j = tid; j < D; j += bs) lam[j] = make_double2(0.0, 0.0);
            __syncthreads();
            for (int g = 0; g < NG; ++g) {
                const uint32_t f = gf[2 * g], pv = gf[2 * g + 1];
                const int tb = stoff[3 * g], tm = stoff[3 * g + 1], te = stoff[3 * g + 2];
                if (te == tb) continue;
                if (f == 0) {
                    for (int j = tid; j < D; j += bs) {
                        double A = 0.0;
                        for (int t = tb; t < tm; ++t) A += (__popc(tz[t] & (uint32_t)j) & 1) ? -tw[t] : tw[t];
                        const double2 x = psi[j];
                        lam[j] = cadd(lam[j], make_double2(A * x.x, A * x.y));
                    }
                } else {
                    for (int j = tid; j < (D >> 1); j += bs) {
                        const uint32_t b = (((uint32_t)j >> pv) << (pv + 1)) | ((uint32_t)j & ((1u << pv) - 1u));
                        const uint32_t bf = b ^ f;
                        double A = 0.0, B = 0.0;
                        for (int t = tb; t < tm; ++t) A += (__popc(tz[t] & b) & 1) ? -tw[t] : tw[t];
                        for (int t = tm; t < te; ++t) B += (__popc(tz[t] & b) & 1) ? -tw[t] : tw[t];
                        const double2 x0 = psi[b], x1 = psi[bf];
                        lam[bf] = cadd(lam[bf], make_double2(A * x0.x - B * x0.y, A * x0.y + B * x0.x));
                        lam[b] = cadd(lam[b], make_double2(A * x1.x + B * x1.y, A * x1.y - B * x1.x));
                    }
                }
                __syncthreads();
            }
            for (int j = tid; j < D; j += bs) e += psi[j].x * lam[j].x + psi[j].y * lam[j].y;
        }
        e = block_sum_all(e, bred);  // also orders the lambda writes before the reverse sweep
        if (tid == 0) energies[it] = e;
        if (it == a.iters) break;

        // reverse sweep
        for (int q = 0; q < G; ++q) {
            const SmallOp o = rops[q];
            const double2 v00 = cconj(mats[4 * o.gate]), v01 = cconj(mats[4 * o.gate + 2]);
            const double2 v10 = cconj(mats[4 * o.gate + 1]), v11 = cconj(mats[4 * o.gate + 3]);
            const int np = D >> o.nfix;
            const bool param = o.pgate >= 0;
            double acc = 0.0;
            for (int j = tid; j < np; j += bs) {
                const uint32_t p0 = insert_zeros((uint32_t)j, o.fixpack, o.nfix) | o.fixed_bits;
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
        b1t *= a.b1;
        b2t *= a.b2;
        for (int p = tid; p < P; p += bs) {
            double gp = 0.0;
            for (int e2 = ka.pmap_off[p]; e2 < ka.pmap_off[p + 1]; ++e2) {
                const int pg = ka.pmap_idx[e2];
                double s = 0.0;
                for (int w = 0; w < L.nw; ++w) s += red[pg * L.nw + w];
                gp += s;
            }
            if (a.opt == VQE_OPT_ADAM) {
                const double mi = a.b1 * mom[p] + (1.0 - a.b1) * gp;
                const double vi = a.b2 * vel[p] + (1.0 - a.b2) * gp * gp;
                mom[p] = mi;
                vel[p] = vi;
                const double c1 = 1.0 - b1t;
                const double c2 = 1.0 - b2t;
                th[p] -= a.lr * (mi / c1) / (sqrt(vi / c2) + a.eps);
            } else {
                th[p] -= a.lr * gp;
            }
        }
        __syncthreads();
    }
    for (int p = tid; p < P; p += bs) a.theta[(size_t)inst * P + p] = th[p];
}

constexpr size_t kSmallLdsMax = 160 * 1024 - 1024;

int choose_block(int n)
{
    if (n <= 6) return 64;
    if (n <= 8) return 128;
    return 256;
}

}  // namespace

// 1 if the persistent loop can run this problem; *mode_out gets the Hamiltonian form
int small_run_plan(int n, int n_gates, int n_params, int n_pgates, int n_groups, int max_inst_terms,
                   int has_imag, int *mode_out, size_t *lds_out)
{
    if (n > 10 || n_gates > 2048 || n_params > 2048) return 0;
    const int nt = choose_block(n);
    int mode = has_imag ? 2 : 1;
    SmallLayout L = small_layout(n, n_gates, n_params, n_pgates, n_groups, max_inst_terms, nt, mode);
    if (L.total > kSmallLdsMax) {
        mode = 0;
        L = small_layout(n, n_gates, n_params, n_pgates, n_groups, max_inst_terms, nt, mode);
        if (L.total > kSmallLdsMax) return 0;
    }
    *mode_out = mode;
    *lds_out = L.total;
    return 1;
}

hipError_t launch_small_run(const SmallRunArgs &a, const OpDesc *rops, const int32_t *pmap_off,
                            const int32_t *pmap_idx, int n_pgates, int mode, int max_inst_terms,
                            int64_t batch, hipStream_t s)
{
    const int nthreads = choose_block(a.n);
    SmallKernelArgs ka;
    ka.a = a;
    ka.rops = rops;
    ka.pmap_off = pmap_off;
    ka.pmap_idx = pmap_idx;
    ka.n_pgates = n_pgates;
    ka.mode = mode;
    ka.max_inst_terms = max_inst_terms;
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, n_pgates, a.n_groups, max_inst_terms,
                                       nthreads, mode);
    if (L.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_small_run),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_small_run, dim3((unsigned)batch), dim3(nthreads), L.total, s, ka);
    return hipGetLastError();
}

}  // namespace vqe
