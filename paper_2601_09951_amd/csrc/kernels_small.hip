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
#include <type_traits>

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

// Sums over the 64 lanes, the same in every lane, in a fixed order: by
// butterfly shuffles, or (wave_sum_dpp, shorter latency on a single wave) by
// DPP lane permutations forming quad, half-row and row sums (no LDS traffic)
// and the four row sums added through readlane in row order.  Every lane of
// the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);  // every lane has a source
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
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

// the 2x2 of a gate kind from c = cos(a/2), s = sin(a/2)
__device__ __forceinline__ void gate_matrix_cs(int kind, double c, double s, double2 *m)
{
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

__device__ __forceinline__ void gate_matrix(int kind, double a, double2 *m)
{
    double s, c;
    sincos(0.5 * a, &s, &c);
    gate_matrix_cs(kind, c, s, m);
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
    int D, G, P, NPG, NG, nw, nterms, mode, defer;
    size_t psi, lam, mats, th, mom, vel, grd, red, bred, ops, rops, gf, gdev, poff, pidx, tab, toff, tz, tw, total;
};

// mode 1: real table, 2: complex table, 0: term form.  defer: per-thread
// gradient partials [NPG][nthreads] kept in LDS and summed once after the
// reverse sweep (else one workgroup reduction per parametric gate)
__host__ __device__ inline SmallLayout small_layout(int n, int G, int P, int NPG, int NG, int nterms,
                                                    int nthreads, int mode, int defer)
{
    SmallLayout L;
    L.D = 1 << n;
    L.G = G;
    L.P = P;
    L.NPG = NPG;
    L.NG = NG;
    L.nterms = nterms;
    L.mode = mode;
    L.defer = defer;
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
    L.red = take((size_t)8 * NPG * (defer ? nthreads : L.nw), 8);
    L.bred = take((size_t)8 * L.nw, 8);
    L.ops = take(sizeof(SmallOp) * G, 16);
    L.rops = take(sizeof(SmallOp) * G, 16);
    L.gf = take((size_t)8 * NG, 8);  // uint32 flip, uint32 pivot
    L.gdev = take(sizeof(GateDev) * G, 16);
    L.poff = take((size_t)4 * (P + 1), 4);
    L.pidx = take((size_t)4 * (NPG > 0 ? NPG : 1), 4);
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
    int defer;
};

__global__ __launch_bounds__(256) void k_small_run(SmallKernelArgs ka)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallRunArgs &a = ka.a;
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, ka.n_pgates, a.n_groups, ka.max_inst_terms,
                                       blockDim.x, ka.mode, ka.defer);
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
    GateDev *gdev = reinterpret_cast<GateDev *>(smem + L.gdev);
    int32_t *poff = reinterpret_cast<int32_t *>(smem + L.poff);
    int32_t *pidx = reinterpret_cast<int32_t *>(smem + L.pidx);
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
        gdev[q] = a.gates[q];
    }
    for (int p = tid; p <= P; p += bs) poff[p] = ka.pmap_off[p];
    for (int i = tid; i < ka.n_pgates; i += bs) pidx[i] = ka.pmap_idx[i];
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
            const GateDev gd = gdev[g];
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
#pragma unroll 4
                    for (int g = 0; g < NG; ++g) {
                        const double d = tabr[g * D + b];
                        const double2 x = psi[b ^ gf[2 * g]];
                        acc.x += d * x.x;
                        acc.y += d * x.y;
                    }
                } else {
#pragma unroll 4
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
                if (L.defer) {
                    red[o.pgate * bs + tid] = acc;
                } else {
                    acc = wave_sum(acc);
                    if (lane == 0) red[o.pgate * L.nw + wave] = acc;
                }
            }
            __syncthreads();
        }
        // dE/dtheta_p and the optimiser step
        b1t *= a.b1;
        b2t *= a.b2;
        for (int p = tid; p < P; p += bs) {
            double gp = 0.0;
            for (int e2 = poff[p]; e2 < poff[p + 1]; ++e2) {
                const int pg = pidx[e2];
                double s = 0.0;
                if (L.defer) {
                    // fixed order: four interleaved partial sums over the threads' partials
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    for (int t = 0; t < bs; t += 4) {
                        s0 += red[pg * bs + t];
                        s1 += red[pg * bs + t + 1];
                        s2 += red[pg * bs + t + 2];
                        s3 += red[pg * bs + t + 3];
                    }
                    s = (s0 + s1) + (s2 + s3);
                } else {
                    for (int w = 0; w < L.nw; ++w) s += red[pg * L.nw + w];
                }
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

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The same loop for states of at most 8 qubits with the Hamiltonian as
// XOR-offset diagonals, built for latency.  An iteration is a chain of
// dependent steps (gate after gate, then H psi, then the reverse sweep, then
// the optimiser step); on this hardware a dependent FP64 operation costs tens
// of cycles, an LDS round trip about 70 and a workgroup barrier with the wave
// skew it waits for well over 100, so every link of the chain is cut to its
// data dependence:
//  * the gate chains (forward and reverse) and the optimiser step run on one
//    wave, which needs no workgroup barrier between dependent steps: a
//    wave's LDS operations execute in issue order, so a wave-level fence
//    (a compiler code-motion barrier) is all that orders one gate's writes
//    before the next gate's reads; only H psi, whose work is spread over all
//    amplitudes, uses every wave, with one barrier on each side;
//  * when every gate matrix is real for every angle and the Hamiltonian is
//    a real matrix, the state stays real and the loop runs on f64
//    amplitudes (a template variant): half the LDS bytes, a fifth of the
//    FP64 work per gate;
//  * a lane holds one pair of a gate, two when a gate has more pairs than
//    lanes (one-qubit gates at 8 qubits; a template parameter); the byte
//    offsets of every op's pairs are tabulated once per launch (the reverse
//    chain reads the forward rows backwards), lanes without a pair use
//    zeroed trash slots, and the gate matrices are laid out in op order (the
//    reverse ones already conjugate-transposed);
//  * the forward sweep records each lane's pair values after every gate in
//    a history buffer in global memory; the reverse sweep reads psi back
//    from it (kHistAhead ops ahead) instead of undoing the gates on psi, so
//    only lambda is carried back;
//  * the optimiser step writes the next iteration's matrices of each
//    parameter's gates directly (U = A cos(a/2) + B sin(a/2) with A, B
//    tabulated per parametric gate; cos and sin by rotating the stored pair
//    through the half step); constant gates keep theirs; with one gate per
//    parameter the lanes that sum a gate's partials step its parameter;
//  * lambda = H psi uses eight interleaved accumulators, one amplitude per
//    thread; at 8 qubits with a real state, at most 64 flip groups and gates
//    of at most 64 pairs four extra waves do it, each thread holding its
//    amplitude's row of the table and its partners in registers for the
//    whole launch, so only psi is read from LDS;
//  * a gate's gradient partials go to an LDS row per parametric gate, one
//    per lane, summed in fixed order after the sweep; with several waves
//    the last one sums the energy during the reverse sweep.
struct FastLayout {
    size_t psi, lam, matf, matr, cs, fcs, th, mom, vel, gpart, gsum, epart, finf, rinf, ptf, ptr, pq, mab, gdev, poff,
        pidx, gf, tab, total;
};

// padding ops after the last op of the gate chains: no pairs, zero
// matrices, gate index G (a spare history row)
constexpr int kFastPad = 4;

__host__ __device__ inline int fast_threads(int n) { return n <= 6 ? 64 : (1 << n); }

// entries per op in the pair tables: the pair count 2^n / 2, at least 64
__host__ __device__ inline int fast_row(int n) { return n >= 8 ? (1 << (n - 1)) : 64; }

__host__ __device__ inline FastLayout fast_layout(int n, int G, int P, int NPG, int NG, int complex_tab,
                                                  bool regtab = false)
{
    FastLayout L;
    const size_t D = (size_t)1 << n, H = D / 2 > 0 ? D / 2 : 1, nt = (size_t)fast_threads(n) + (regtab ? 64 : 0);
    const size_t npg = NPG > 0 ? NPG : 1;
    size_t o = 0;
    auto take = [&](size_t bytes, size_t align) {
        o = (o + align - 1) / align * align;
        size_t r = o;
        o += bytes;
        return r;
    };
    L.psi = take(16 * (D + 128), 16);  // + two trash slots per lane for lanes without a pair
    L.lam = take(16 * (D + 128), 16);
    L.matf = take((size_t)64 * (G + kFastPad), 16);  // + padding ops (branch-free prefetch)
    L.matr = take((size_t)64 * (G + kFastPad), 16);
    L.cs = take((size_t)16 * (P > 0 ? P : 1), 16);
    L.fcs = take((size_t)16 * G, 16);
    L.th = take((size_t)8 * P, 8);
    L.mom = take((size_t)8 * P, 8);
    L.vel = take((size_t)8 * P, 8);
    L.gpart = take((size_t)8 * 64 * (npg + 1), 16);  // per parametric gate (+ a spare row), one partial per lane
    L.gsum = take((size_t)8 * (npg > 8 ? npg : 8), 8);  // one sum per parametric gate (8: block sum scratch)
    L.epart = take(8 * nt, 8);
    L.finf = take((size_t)8 * (G + kFastPad), 8);  // {gen | (pgate + 1) << 8, gate} per op
    L.rinf = take((size_t)8 * (G + kFastPad), 8);
    L.ptf = take(4 * (size_t)(G + kFastPad) * fast_row(n), 4);  // pair t of op q at [q][t]
    L.ptr = L.ptf;  // the reverse chain reads the forward rows backwards
    L.pq = take((size_t)8 * npg, 8);            // per parametric gate: forward and reverse op
    L.mab = take((size_t)256 * npg, 16);        // per parametric gate: U = A cos + B sin, forward and reverse
    L.gdev = take(sizeof(GateDev) * G, 16);
    L.poff = take((size_t)4 * (P + 1), 4);
    L.pidx = take((size_t)4 * npg, 4);
    const size_t ng8 = (size_t)(NG + 7) / 8 * 8;  // groups padded with zero diagonals
    L.gf = take(4 * ng8, 16);
    L.tab = take(regtab ? 0 : (complex_tab ? 16 : 8) * ng8 * D, 16);  // in registers with regtab
    L.total = o;
    return L;
}

// Register-held Hamiltonian rows: at 8 qubits with a real state, at most
// kRegGroups flip groups and at most 64 pairs per gate, one wave runs the
// gate chains and four more waves run H psi, each thread keeping its
// amplitude's diagonal entries for all groups in registers for the whole
// launch, so H psi reads only psi from LDS.  (A complex state at 8 qubits
// has a one-qubit RX or RZ, 128 pairs, so it never meets the pair limit.)
constexpr int kRegGroups = 64;

__host__ __device__ inline bool fast_regtab(int n, int NG, bool real_state, int max_pairs)
{
    return n == 8 && real_state && NG <= kRegGroups && max_pairs <= 64;
}

__device__ __forceinline__ uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// u x + v y with balanced dependency chains
__device__ __forceinline__ double2 mac2(double2 u, double2 x, double2 v, double2 y)
{
    const double r0 = fma(u.x, x.x, -u.y * x.y), r1 = fma(v.x, y.x, -v.y * y.y);
    const double i0 = fma(u.x, x.y, u.y * x.x), i1 = fma(v.x, y.y, v.y * y.x);
    return make_double2(r0 + r1, i0 + i1);
}

// the same with real amplitudes and real matrix entries (a state that stays
// real: every gate matrix real for every angle, a real Hamiltonian)
__device__ __forceinline__ double mac2(double u, double x, double v, double y) { return fma(u, x, v * y); }

// amplitude helpers for the complex (double2) and the real (double) state
__device__ __forceinline__ void amp_fma(double2 &acc, double d, double2 x)
{
    acc.x = fma(d, x.x, acc.x);
    acc.y = fma(d, x.y, acc.y);
}
__device__ __forceinline__ void amp_fma(double &acc, double d, double x) { acc = fma(d, x, acc); }
__device__ __forceinline__ double amp_add(double a, double b) { return a + b; }
__device__ __forceinline__ double2 amp_add(double2 a, double2 b) { return cadd(a, b); }
__device__ __forceinline__ double amp_dot(double2 x, double2 y) { return x.x * y.x + x.y * y.y; }  // Re x* y
__device__ __forceinline__ double amp_dot(double x, double y) { return x * y; }
__device__ __forceinline__ void amp_set(double2 &a, double v) { a = make_double2(v, 0.0); }
__device__ __forceinline__ void amp_set(double &a, double v) { a = v; }
// a gate matrix entry as the chain applies it (the real state takes the real part)
__device__ __forceinline__ void mat_get(double2 &d, const double2 &m) { d = m; }
__device__ __forceinline__ void mat_get(double &d, const double2 &m) { d = m.x; }

// Orders the calling wave's LDS writes before its later LDS reads by other
// lanes: LDS operations of one wave execute in issue order, so no wait is
// needed, only that the compiler moves no memory operation across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// op q's pair entries of this lane (pairs lane + 64 s; the rows are padded
// to at least 64 entries, so no lane needs a bound) and its matrix; ops G..
// are padding (no pairs, zero matrices), so the prefetch of later ops needs
// no branch.  An entry holds the byte offsets of the pair's two amplitudes
// in the state (first | second << 16); a lane without a pair gets its own
// two trash slots past the state, which hold zeros, so no lane branches or
// masks its partial
template <int SP, typename T>
__device__ __forceinline__ void fast_tables(const uint32_t *pt, const double2 *mat, int q, int row, int HP, int lane,
                                            uint32_t (&pe)[SP], T (&u)[4])
{
#pragma unroll
    for (int s = 0; s < SP; ++s) pe[s] = pt[row * HP + lane + 64 * s];
#pragma unroll
    for (int k = 0; k < 4; ++k) mat_get(u[k], mat[4 * q + k]);
}

// the amplitude at a byte offset of a state
template <typename T>
__device__ __forceinline__ T &amp_at(T *st, uint32_t off)
{
    return *reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(st) + off);
}
template <typename T>
__device__ __forceinline__ const T &amp_at(const T *st, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const unsigned char *>(st) + off);
}

// bit 4 of an op's info word: the op has more pairs than lanes, so the
// second pair slot is in use (a wave-uniform test)
constexpr int kTwoSlots = 16;

// pair slots per lane: a gate on 2^n amplitudes has at most 2^n / 2 pairs
__host__ __device__ constexpr int fast_slots(int n) { return n >= 8 ? 2 : 1; }

// One gate op as the gate wave sees it: the lane's pair table entries, the
// op's matrix and info word and the state values read on the lane's pairs
// (psi after the gate, which the reverse sweep needs, comes separately from
// the forward history).  The chains below alternate two of these buffers over the ops
// (op q in buffer q & 1): while op q computes, the pairs of op q + 1 are
// already read and the tables of op q + 2 are on their way, so each op costs
// one LDS read latency plus its arithmetic, and no value is moved between
// registers (a move would have to wait for its load).  T is the amplitude
// type: double2, or double for a state that stays real.
template <int SP, typename T>
struct FastOp {
    uint32_t pe[SP];
    T u[4];
    int info;  // gen | two-slot flag | (pgate + 1) << 8
    T x[SP], y[SP];  // the state on the pairs before the op
};

// psi on the lane's pairs after a gate (forward history, reverse sweep)
template <int SP, typename T>
struct FastHist {
    T hx[SP], hy[SP];
};

// op q of a chain; its pair table row is q forward, and for the reverse
// chain (the gates in reverse order on the same pairs) the row of forward op
// G - 1 - q (rows G.. are the padding ops either way)
template <int SP, typename T>
__device__ __forceinline__ void fast_op_load(FastOp<SP, T> &o, const uint32_t *pt, const double2 *mat,
                                             const int2 *inf, int q, int row, int HP, int lane)
{
    fast_tables<SP>(pt, mat, q, row, HP, lane, o.pe, o.u);
    o.info = inf[q].x;  // the word the chains use (a 32-bit load: no second register in flight)
}
__device__ __forceinline__ int rev_row(int q, int G) { return q < G ? G - 1 - q : q; }

// read the op's pairs of a state (psi forward, lambda reverse)
template <int SP, typename T>
__device__ __forceinline__ void fast_op_read(FastOp<SP, T> &o, const T *st, int D, int lane)
{
    const bool two = SP > 1 && (ufirst((uint32_t)o.info) & kTwoSlots);
#pragma unroll
    for (int s = 0; s < SP; ++s)
        if (s == 0 || two) {
            o.x[s] = amp_at(st, o.pe[s] & 0xFFFFu);
            o.y[s] = amp_at(st, o.pe[s] >> 16);
        }
}

// forward op q (gate q): update the lane's pairs of psi and record them
// after the gate in hist[q][slot][lane] (global memory, off the chain)
template <int SP, typename T>
__device__ __forceinline__ void fast_fwd_step(const FastOp<SP, T> &o, T *psi, T *__restrict__ hist, int q, int lane)
{
    const bool two = SP > 1 && (ufirst((uint32_t)o.info) & kTwoSlots);
    T *hq = hist + (size_t)q * (SP * 128) + 2 * lane;
#pragma unroll
    for (int s = 0; s < SP; ++s)
        if (s == 0 || two) {
            const T nx = mac2(o.u[0], o.x[s], o.u[1], o.y[s]), ny = mac2(o.u[2], o.x[s], o.u[3], o.y[s]);
            amp_at(psi, o.pe[s] & 0xFFFFu) = nx;
            amp_at(psi, o.pe[s] >> 16) = ny;
            hq[128 * s] = nx;
            hq[128 * s + 1] = ny;
        }
    wave_lds_sync();
}

// Im <lam|G|psi> on one pair (a, b of lambda, x, y of psi) for the op's generator
__device__ __forceinline__ double pair_grad(int gen, double2 a, double2 b, double2 x, double2 y)
{
    const double gy = (b.x * x.x + b.y * x.y) - (a.x * y.x + a.y * y.y);
    const double gx = (a.x * y.y - a.y * y.x) + (b.x * x.y - b.y * x.x);
    const double gz = (a.x * x.y - a.y * x.x) - (b.x * y.y - b.y * y.x);
    return gen == GEN_Y ? gy : (gen == GEN_X ? gx : gz);
}
// real states: only Y-type generators (RY, the excitations) keep the state
// real, and Im <lam|G|psi> = b x - a y
__device__ __forceinline__ double pair_grad(int, double a, double b, double x, double y) { return b * x - a * y; }

// reverse op: U^dagger on the lane's pairs of lambda; returns the lane's
// gradient partial Im <lam|G|psi> (psi from the history); psi itself is not
// carried back
template <int SP, typename T>
__device__ __forceinline__ double fast_rev_step(const FastOp<SP, T> &o, const FastHist<SP, T> &h, T *lam, int D,
                                                int lane)
{
    const uint32_t cd = ufirst((uint32_t)o.info);
    const bool two = SP > 1 && (cd & kTwoSlots);
    const int gen = (int)(cd & 15u);
    double g = 0.0;
#pragma unroll
    for (int s = 0; s < SP; ++s)
        if (s == 0 || two) {
            const T a = o.x[s], b = o.y[s];
            amp_at(lam, o.pe[s] & 0xFFFFu) = mac2(o.u[0], a, o.u[1], b);
            amp_at(lam, o.pe[s] >> 16) = mac2(o.u[2], a, o.u[3], b);
            const double gs = pair_grad(gen, a, b, h.hx[s], h.hy[s]);  // zero on trash slots
            g = s == 0 ? gs : g + gs;
        }
    wave_lds_sync();
    return g;
}

// the forward chain U(theta) e_ref on one wave, two ops per trip; the first
// op acts on the reference basis state (ref_off: its byte offset), so its
// pair values follow from its table entry without an LDS read
template <int SP, typename T>
__device__ __forceinline__ void fast_forward(T *psi, const uint32_t *ptf, const double2 *matf, const int2 *finf,
                                             T *__restrict__ hist, int G, int HP, int D, uint32_t ref_off, int lane)
{
    FastOp<SP, T> A, B;
    fast_op_load(A, ptf, matf, finf, 0, 0, HP, lane);
    fast_op_load(B, ptf, matf, finf, 1, 1, HP, lane);
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        amp_set(A.x[s], (A.pe[s] & 0xFFFFu) == ref_off ? 1.0 : 0.0);
        amp_set(A.y[s], (A.pe[s] >> 16) == ref_off ? 1.0 : 0.0);
    }
    for (int q = 0; q < G; q += 2) {
        fast_fwd_step(A, psi, hist, q, lane);
        if (q + 1 >= G) break;
        fast_op_read(B, psi, D, lane);
        fast_op_load(A, ptf, matf, finf, q + 2, q + 2, HP, lane);
        fast_fwd_step(B, psi, hist, q + 1, lane);
        fast_op_read(A, psi, D, lane);
        fast_op_load(B, ptf, matf, finf, q + 3, q + 3, HP, lane);
    }
}

// the history of reverse op q: gate G - 1 - q (the host checks that the
// reverse plan lists the gates in exactly that order), padding ops read the
// spare row G; no table read, so the load's address is ready at once
template <int SP, typename T>
__device__ __forceinline__ void fast_hist_load(FastHist<SP, T> &h, const T *__restrict__ hist, int G, int q,
                                               int lane)
{
    const int gate = q < G ? G - 1 - q : G;
    const T *hq = hist + (size_t)gate * (SP * 128) + 2 * lane;
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        h.hx[s] = hq[128 * s];
        h.hy[s] = hq[128 * s + 1];
    }
}

template <int SP, typename T>
__device__ __forceinline__ void fast_rev_op(FastOp<SP, T> &cur, const FastHist<SP, T> &h, FastOp<SP, T> &nxt, T *lam,
                                            double *gpart, const uint32_t *ptr, const double2 *matr,
                                            const int2 *rinf, int npg, int qload, int G, int HP, int D, int lane)
{
    const double g = fast_rev_step(cur, h, lam, D, lane);
    fast_op_read(nxt, lam, D, lane);
    const int pg = (int)(ufirst((uint32_t)cur.info) >> 8) - 1;
    gpart[(pg >= 0 ? pg : npg) * 64 + lane] = g;  // row npg: ops without a parameter
    fast_op_load(cur, ptr, matr, rinf, qload, rev_row(qload, G), HP, lane);
}

// the reverse chain on one wave (leaving after op G - 1); the history of op
// q is loaded kHistAhead ops ahead (a global-memory round trip spans
// several ops), the tables two ops ahead
constexpr int kHistAhead = 8;

template <int SP, typename T>
__device__ __forceinline__ void fast_reverse(T *lam, const uint32_t *ptr, const double2 *matr, const int2 *rinf,
                                             const T *__restrict__ hist, double *gpart, int npg, int G, int HP, int D,
                                             int lane)
{
    FastOp<SP, T> ops[2];
    FastHist<SP, T> hs[kHistAhead];
    const int last = G + kFastPad - 1;
    fast_op_load(ops[0], ptr, matr, rinf, 0, rev_row(0, G), HP, lane);
    fast_op_load(ops[1], ptr, matr, rinf, 1, rev_row(1, G), HP, lane);
#pragma unroll
    for (int j = 0; j < kHistAhead; ++j) fast_hist_load(hs[j], hist, G, j, lane);
    fast_op_read(ops[0], lam, D, lane);
    // whole blocks of eight unguarded steps (each history buffer keeps its
    // registers, and every step finds the same history loads in flight),
    // then the last G mod 8 ops, whose history is already loaded
    int q = 0;
    for (; q + kHistAhead <= G; q += kHistAhead) {
#pragma unroll
        for (int j = 0; j < kHistAhead; ++j) {
            fast_rev_op(ops[j & 1], hs[j], ops[(j + 1) & 1], lam, gpart, ptr, matr, rinf, npg, min(q + j + 2, last),
                        G, HP, D, lane);
            fast_hist_load(hs[j], hist, G, q + j + kHistAhead, lane);
        }
    }
#pragma unroll
    for (int j = 0; j < kHistAhead; ++j)
        if (q + j < G)
            fast_rev_op(ops[j & 1], hs[j], ops[(j + 1) & 1], lam, gpart, ptr, matr, rinf, npg, min(q + j + 2, last), G,
                        HP, D, lane);
    // the last block prefetched spare rows nobody reads; wait for them here
    // (s_waitcnt vmcnt(0), gfx9 encoding), so no load is in flight when the
    // next forward chain starts and its stores need no wait of their own
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// the sum of parametric gate row's 64 lane partials in fixed order: each of
// the four lanes of a quad adds 16 partials (part = lane & 3), then a quad
// sum leaves the total in all four lanes (rows past NPG give zero)
__device__ __forceinline__ double row_sum(const double *gpart, int row, int NPG, int part)
{
    double s0 = 0.0, s1 = 0.0;
    if (row < NPG) {
        const double2 *v = reinterpret_cast<const double2 *>(gpart + row * 64 + part * 16);
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
            const double2 a = v[j], b = v[j + 1];
            s0 = j == 0 ? a.x + a.y : s0 + (a.x + a.y);
            s1 = j == 0 ? b.x + b.y : s1 + (b.x + b.y);
        }
    }
    double t = s0 + s1;
    t += dpp_move<0xB1>(t);  // quad_perm [1, 0, 3, 2]
    t += dpp_move<0x4E>(t);  // quad_perm [2, 3, 0, 1]
    return t;
}

// per parametric gate the sum of its 64 lane partials, 16 gates per pass
__device__ __forceinline__ void gate_sums(const double *gpart, double *gsum, int NPG, int lane)
{
    for (int r0 = 0; r0 < NPG; r0 += 16) {
        const int row = r0 + (lane >> 2), part = lane & 3;
        const double t = row_sum(gpart, row, NPG, part);
        if (part == 0 && row < NPG) gsum[row] = t;
    }
}

// the parameters are the parametric gates: one gate per parameter, gate j
// holding parameter j, at most 16 (then the lane that sums gate j's partials
// steps parameter j at once, without a round trip through LDS)
constexpr int kDirectParams = 16;

// the next iteration's matrix of a rotation, U = A cos(t/2) + B sin(t/2),
// into dst[0..3] (ab[0..3] = A, ab[4..7] = B); with real coefficients only
// the real parts are written (the imaginary parts stay zero)
__device__ __forceinline__ void rot_store(double2 *dst, const double2 *ab, double cn, double sn)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        dst[k] = make_double2(fma(ab[k].x, cn, ab[4 + k].x * sn), fma(ab[k].y, cn, ab[4 + k].y * sn));
}
__device__ __forceinline__ void rot_store(double2 *dst, const double *ab, double cn, double sn)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) reinterpret_cast<double *>(dst + k)[0] = fma(ab[k], cn, ab[4 + k] * sn);
}

// H psi of one amplitude from register-held rows: sum over the first NR
// groups of tv[g] psi[ad[g]] (ad: the amplitude's partner in group g, fixed
// for the launch), eight interleaved accumulators; no branch and no table
// read between the loads, so they issue back to back
template <int NR, typename T>
__device__ __forceinline__ T rows_gather(const T *psi, const double (&tv)[kRegGroups],
                                         const uint32_t (&ad)[kRegGroups])
{
    T sacc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) amp_set(sacc[k], 0.0);
#pragma unroll
    for (int g = 0; g < NR; ++g) amp_fma(sacc[g & 7], tv[g], psi[ad[g]]);
    return amp_add(amp_add(amp_add(sacc[0], sacc[1]), amp_add(sacc[2], sacc[3])),
                   amp_add(amp_add(sacc[4], sacc[5]), amp_add(sacc[6], sacc[7])));
}

// SP: pair slots per lane of the gate wave, 2 only when some op has more
// pairs than lanes (one-qubit gates at 8 qubits)
// RT: the register-held Hamiltonian rows (NT = 320: the gate wave, then
// four waves for H psi with one amplitude per thread)
// RS: the state stays real (every gate matrix is real for every angle, the
// reference is a basis state and the Hamiltonian is a real matrix), so psi,
// lambda and the history hold real amplitudes: half the LDS bytes per pair
// and a fifth of the FP64 work per gate on the chain
template <int NT, int SP, bool CT, bool RT, bool RS>
__global__ __launch_bounds__(NT) void k_small_fast(SmallKernelArgs ka)
{
    using T = typename std::conditional<RS, double, double2>::type;
    constexpr int NW = NT / 64;
    static_assert(SP == 1 || (SP == 2 && NT >= 256), "pair slots per lane");
    static_assert(!RT || (NT == 320 && RS), "register rows: 8 qubits, real state");
    static_assert(!RS || !CT, "a real state needs a real Hamiltonian");
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallRunArgs &a = ka.a;
    const FastLayout L = fast_layout(a.n, a.n_gates, a.n_params, ka.n_pgates, a.n_groups, CT, RT);
    T *psi = reinterpret_cast<T *>(smem + L.psi);
    T *lam = reinterpret_cast<T *>(smem + L.lam);
    double2 *matf = reinterpret_cast<double2 *>(smem + L.matf);
    double2 *matr = reinterpret_cast<double2 *>(smem + L.matr);
    double2 *cs = reinterpret_cast<double2 *>(smem + L.cs);
    double2 *fcs = reinterpret_cast<double2 *>(smem + L.fcs);
    double *th = reinterpret_cast<double *>(smem + L.th);
    double *mom = reinterpret_cast<double *>(smem + L.mom);
    double *vel = reinterpret_cast<double *>(smem + L.vel);
    double *gpart = reinterpret_cast<double *>(smem + L.gpart);
    double *gsum = reinterpret_cast<double *>(smem + L.gsum);
    double *epart = reinterpret_cast<double *>(smem + L.epart);
    int2 *finf = reinterpret_cast<int2 *>(smem + L.finf);
    int2 *rinf = reinterpret_cast<int2 *>(smem + L.rinf);
    uint32_t *ptf = reinterpret_cast<uint32_t *>(smem + L.ptf);
    uint32_t *ptr = reinterpret_cast<uint32_t *>(smem + L.ptr);
    GateDev *gdev = reinterpret_cast<GateDev *>(smem + L.gdev);
    int32_t *poff = reinterpret_cast<int32_t *>(smem + L.poff);
    int32_t *pidx = reinterpret_cast<int32_t *>(smem + L.pidx);
    uint32_t *gf = reinterpret_cast<uint32_t *>(smem + L.gf);
    double *tabr = reinterpret_cast<double *>(smem + L.tab);
    double2 *tabc = reinterpret_cast<double2 *>(smem + L.tab);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int inst = blockIdx.x;
    const int D = 1 << a.n, HP = fast_row(a.n);
    const int G = a.n_gates, P = a.n_params, NG = a.n_groups, NG8 = (NG + 7) / 8 * 8, NPG = ka.n_pgates;
    const int32_t *to = a.toff + (size_t)(a.shared_ham ? 0 : inst) * NG * 3;
    double *energies = a.energies + (size_t)inst * (a.iters + 1);
    T *hist = reinterpret_cast<T *>(a.hist) + (size_t)inst * (G + 1) * (SP * 128);

    // ---- one-time staging (ops G and G + 1 pad the tables and are never applied)
    for (int p = tid; p < P; p += NT) {
        const double t = a.theta[(size_t)inst * P + p];
        th[p] = t;
        mom[p] = 0.0;
        vel[p] = 0.0;
        double sn, cn;
        sincos(0.5 * t, &sn, &cn);
        cs[p] = make_double2(cn, sn);
    }
    for (int q = tid; q < G + kFastPad; q += NT) {
        if (q < G) {
            const OpDesc f = a.ops[q], r = ka.rops[q];
            const int f2 = (D >> pack_op(f).nfix) > 64 ? kTwoSlots : 0;
            const int r2 = (D >> pack_op(r).nfix) > 64 ? kTwoSlots : 0;
            finf[q] = make_int2(f.gen | f2 | ((f.pgate + 1) << 8), f.gate);
            rinf[q] = make_int2(r.gen | r2 | ((r.pgate + 1) << 8), r.gate);
            const GateDev gd = a.gates[q];
            gdev[q] = gd;
            double sn, cn;
            sincos(0.5 * gd.fixed, &sn, &cn);
            fcs[q] = make_double2(cn, sn);
        } else {
            finf[q] = rinf[q] = make_int2(0, G);
        }
    }
    // pair table of the forward ops (the reverse ops are the same pairs in
    // reverse order): op q, pair t -> byte offsets of p0 | p1 << 16; past the
    // op's pair count the trash slots D + 2 l, D + 2 l + 1 of lane l = t mod 64
    for (int w = tid; w < (G + kFastPad) * HP; w += NT) {
        const int q = w / HP, t = w % HP;
        uint32_t p0 = (uint32_t)(D + 2 * (t & 63)), p1 = p0 + 1u;
        if (q < G) {
            const SmallOp o = pack_op(a.ops[q]);
            if (t < (D >> o.nfix)) {
                p0 = insert_zeros((uint32_t)t, o.fixpack, o.nfix) | o.fixed_bits;
                p1 = p0 ^ o.m;
            }
        }
        ptf[w] = (p0 * (uint32_t)sizeof(T)) | (p1 * (uint32_t)sizeof(T)) << 16;
    }
    for (int i = tid; i < 128; i += NT) {  // the trash slots hold zeros (gates keep them zero)
        amp_set(psi[D + i], 0.0);
        amp_set(lam[D + i], 0.0);
    }
    for (int k = tid; k < 4 * kFastPad; k += NT) {
        matf[4 * G + k] = make_double2(0.0, 0.0);
        matr[4 * G + k] = make_double2(0.0, 0.0);
    }
    for (int p = tid; p <= P; p += NT) poff[p] = ka.pmap_off[p];
    for (int i = tid; i < NPG; i += NT) pidx[i] = ka.pmap_idx[i];
    for (int g = tid; g < NG8; g += NT) gf[g] = g < NG ? a.groups[g].floc : 0u;
    __syncthreads();
    // D_g[b] = sum_t kappa_t (-1)^{z_t . (b ^ f_g)}; zero rows pad the groups
    for (int i = tid; i < (RT ? 0 : NG8 * D); i += NT) {
        const int g = i >> a.n;
        const uint32_t b = (uint32_t)(i & (D - 1));
        double re = 0.0, im = 0.0;
        if (g < NG) {
            const int ug = a.groups[g].ugroup;
            const int tb = to[ug * 3], tm = to[ug * 3 + 1], te = to[ug * 3 + 2];
            const uint32_t bb = b ^ gf[g];
            for (int t = tb; t < tm; ++t) {
                const TermDev d = a.terms[t];
                re += (__popc(d.zloc & bb) & 1) ? -d.w : d.w;
            }
            for (int t = tm; t < te; ++t) {
                const TermDev d = a.terms[t];
                im += (__popc(d.zloc & bb) & 1) ? -d.w : d.w;
            }
        }
        if (CT)
            tabc[i] = make_double2(re, im);
        else
            tabr[i] = re;
    }
    __syncthreads();

    // the first iteration's matrices in op order (forward U, reverse
    // U^dagger); afterwards the optimiser step rewrites the parametric ones.
    // A rotation's 2x2 is A cos(a/2) + B sin(a/2) with constant A, B, kept
    // per parametric gate for both directions (mab: A fwd, B fwd, A rev, B rev).
    for (int w = tid; w < 2 * G; w += NT) {
        const int rev = w >= G, q = rev ? w - G : w;
        const int2 inf = (rev ? rinf : finf)[q];
        const GateDev gd = gdev[inf.y];
        const double2 c = gd.pidx >= 0 ? cs[gd.pidx] : fcs[inf.y];
        double2 m[4], ma[4], mb[4];
        gate_matrix_cs(gd.kind, c.x, c.y, m);
        gate_matrix_cs(gd.kind, 1.0, 0.0, ma);
        gate_matrix_cs(gd.kind, 0.0, 1.0, mb);
        double2 *dst = (rev ? matr : matf) + 4 * q;
        const int order[4] = {0, rev ? 2 : 1, rev ? 1 : 2, 3};  // U^dagger: transpose and conjugate
        const int pg = (inf.x >> 8) - 1;
        const bool rot = gd.kind == VQE_GATE_RX || gd.kind == VQE_GATE_RY || gd.kind == VQE_GATE_RZ ||
                         gd.kind == VQE_GATE_SINGLE_EXC || gd.kind == VQE_GATE_DOUBLE_EXC;
        double2 *ab = reinterpret_cast<double2 *>(smem + L.mab) + (pg >= 0 ? pg : 0) * 16 + (rev ? 8 : 0);
        int2 *pq = reinterpret_cast<int2 *>(smem + L.pq);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 v = m[order[k]], va = ma[order[k]], vb = mb[order[k]];
            dst[k] = rev ? cconj(v) : v;
            if (pg >= 0) {
                ab[k] = rev ? cconj(va) : va;
                ab[4 + k] = rev ? cconj(vb) : vb;
            }
        }
        if (pg >= 0) {  // a constant gate kind with a parameter keeps its matrix (q = -1: never rewritten)
            if (rev)
                pq[pg].y = rot ? q : -1;
            else
                pq[pg].x = rot ? q : -1;
        }
    }
    __syncthreads();

    if (RT && wave >= 1) {
        // H psi waves: amplitude b's diagonal entries of every group in
        // registers (groups past NG are zero), then per iteration the same
        // barriers as the gate wave's loop
        const uint32_t b = (uint32_t)(tid - 64);
        double tv[kRegGroups];
        uint32_t ad[kRegGroups];  // partners b ^ f_g (b itself for the zero rows)
#pragma unroll
        for (int g = 0; g < kRegGroups; ++g) {
            double re = 0.0;
            ad[g] = g < NG ? b ^ gf[g] : b;
            if (g < NG) {
                const int ug = a.groups[g].ugroup;
                const int tb = to[ug * 3], tm = to[ug * 3 + 1];
                const uint32_t bb = b ^ gf[g];
                for (int t = tb; t < tm; ++t) {
                    const TermDev d = a.terms[t];
                    re += (__popc(d.zloc & bb) & 1) ? -d.w : d.w;
                }
            }
            tv[g] = re;
        }
        for (int it = 0; it <= a.iters; ++it) {
            __syncthreads();  // psi is final
            T acc;  // the groups in whole blocks of eight (zero rows pad the last)
            switch ((NG + 7) >> 3) {
            case 1: acc = rows_gather<8>(psi, tv, ad); break;
            case 2: acc = rows_gather<16>(psi, tv, ad); break;
            case 3: acc = rows_gather<24>(psi, tv, ad); break;
            case 4: acc = rows_gather<32>(psi, tv, ad); break;
            case 5: acc = rows_gather<40>(psi, tv, ad); break;
            case 6: acc = rows_gather<48>(psi, tv, ad); break;
            case 7: acc = rows_gather<56>(psi, tv, ad); break;
            default: acc = rows_gather<64>(psi, tv, ad); break;
            }
            lam[b] = acc;
            const double e = amp_dot(psi[b], acc);
            epart[b] = e;
            __syncthreads();  // lambda is final
            if (it == a.iters) {
                const double sE = block_sum_all(e, gsum);
                (void)sE;
                break;
            }
            if (wave == NW - 1) {  // the energy's sum beside the reverse sweep
                double sE = 0.0;
                for (int t = lane; t < D; t += 64) sE += epart[t];
                sE = wave_sum(sE);
                if (lane == 0) energies[it] = sE;
            }
        }
        __syncthreads();
        return;
    }

    const bool mine = !RT && tid < D;  // this thread's amplitude b = tid in H psi
    double b1t = 1.0, b2t = 1.0;  // beta1^t, beta2^t for Adam's bias corrections
    const int2 *pq = reinterpret_cast<const int2 *>(smem + L.pq);
    const double2 *mab = reinterpret_cast<const double2 *>(smem + L.mab);
    bool direct = NPG == P && P <= kDirectParams;  // the same in every thread
    for (int p = 0; p < P && direct; ++p) direct = poff[p] == p && pidx[p] == p;

    // optimiser step of parameter p (gradient gp, gates pidx[e0..e1), the
    // first one's op slots q0 and coefficients ab), then the next
    // iteration's matrices of its gates
    // the parameter's state (angle, half-angle pair, Adam moments), read by
    // the caller before the gradient so that it lands during the sums
    struct ParamState {
        double t0, m0, v0;
        double2 c0;
    };
    auto param_load = [&](int p) {
        ParamState ps;
        ps.t0 = th[p];
        ps.c0 = cs[p];
        ps.m0 = mom[p];
        ps.v0 = vel[p];
        return ps;
    };
    auto param_step = [&](int p, double gp, int e0, int e1, int2 q0, const T (&ab)[16], const ParamState &ps,
                          double rc1, double rc2) {
        const double t0 = ps.t0;
        const double2 c0 = ps.c0;
        double t = t0;
        if (a.opt == VQE_OPT_ADAM) {
            const double mi = a.b1 * ps.m0 + (1.0 - a.b1) * gp;
            const double vi = a.b2 * ps.v0 + (1.0 - a.b2) * gp * gp;
            mom[p] = mi;
            vel[p] = vi;
            t -= a.lr * (mi * rc1) / (sqrt(vi * rc2) + a.eps);
        } else {
            t -= a.lr * gp;
        }
        th[p] = t;
        // cos and sin of the new half angle: the old pair rotated by the half
        // step d (|d| < 1/16: Taylor series to d^9, error below 1e-19), else
        // from scratch
        const double d = 0.5 * (t - t0);
        double sn, cn;
        if (fabs(d) < 0.0625) {
            const double d2 = d * d;
            const double cd = fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 40320, -1.0 / 720), 1.0 / 24), -0.5), 1.0);
            const double sd = d * fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 362880, -1.0 / 5040), 1.0 / 120), -1.0 / 6), 1.0);
            cn = fma(c0.x, cd, -c0.y * sd);
            sn = fma(c0.y, cd, c0.x * sd);
        } else {
            sincos(0.5 * t, &sn, &cn);
        }
        cs[p] = make_double2(cn, sn);
        if (e0 < e1) {
            if (q0.x >= 0) rot_store(matf + 4 * q0.x, ab, cn, sn);
            if (q0.y >= 0) rot_store(matr + 4 * q0.y, ab + 8, cn, sn);
        }
        for (int e2 = e0 + 1; e2 < e1; ++e2) {  // further gates sharing the parameter
            const int j = pidx[e2];
            const int2 qq = pq[j];
            T abj[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) mat_get(abj[k], mab[j * 16 + k]);
            if (qq.x >= 0) rot_store(matf + 4 * qq.x, abj, cn, sn);
            if (qq.y >= 0) rot_store(matr + 4 * qq.y, abj + 8, cn, sn);
        }
    };
    for (int it = 0; it <= a.iters; ++it) {
        if (wave == 0) {
            for (int b = lane; b < D; b += 64) amp_set(psi[b], b == (int)a.ref ? 1.0 : 0.0);
            wave_lds_sync();
            fast_forward<SP>(psi, ptf, matf, finf, hist, G, HP, D, a.ref * (uint32_t)sizeof(T), lane);  // U(theta) e_ref
        }
        __syncthreads();

        // lambda = H psi with the XOR-offset diagonals, eight interleaved
        // accumulators; this thread's part of E = Re <psi|lambda>
        double e = 0.0;
        if (mine) {
            const uint32_t b = (uint32_t)tid;
            T sacc[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) amp_set(sacc[k], 0.0);
            for (int g = 0; g < NG8; g += 8) {
                const uint4 fa = *reinterpret_cast<const uint4 *>(gf + g);
                const uint4 fb = *reinterpret_cast<const uint4 *>(gf + g + 4);
                const uint32_t fk[8] = {fa.x, fa.y, fa.z, fa.w, fb.x, fb.y, fb.z, fb.w};
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const T x = psi[b ^ fk[k]];
                    if constexpr (CT)
                        sacc[k] = cadd(sacc[k], cmul(tabc[(g + k) * D + b], x));
                    else
                        amp_fma(sacc[k], tabr[(g + k) * D + b], x);
                }
            }
            const T acc = amp_add(amp_add(amp_add(sacc[0], sacc[1]), amp_add(sacc[2], sacc[3])),
                                  amp_add(amp_add(sacc[4], sacc[5]), amp_add(sacc[6], sacc[7])));
            lam[b] = acc;
            e = amp_dot(psi[b], acc);
        }
        if (!RT) epart[tid] = e;
        __syncthreads();
        if (it == a.iters) {
            const double sE = block_sum_all(e, gsum);
            if (tid == 0) energies[it] = sE;
            break;
        }

        b1t *= a.b1;
        b2t *= a.b2;
        if (wave == 0) {
            // reverse sweep: g_l = Im <lambda|G_l|psi>, then U_l^dagger on both states
            fast_reverse<SP>(lam, ptr, matr, rinf, hist, gpart, NPG, G, HP, D, lane);
            wave_lds_sync();  // the last partials before their sums
            const double rc1 = 1.0 / (1.0 - b1t), rc2 = 1.0 / (1.0 - b2t);
            if (direct) {
                // gate p's quad sums its partials; its first lane steps parameter p
                const int p = min(lane >> 2, P - 1);
                const int2 q0 = pq[p];
                T ab[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) mat_get(ab[k], mab[p * 16 + k]);
                const ParamState ps = param_load(p);
                const double gp = row_sum(gpart, lane >> 2, NPG, lane & 3);
                if ((lane & 3) == 0 && (lane >> 2) < P) param_step(p, gp, p, p + 1, q0, ab, ps, rc1, rc2);
            } else {
                gate_sums(gpart, gsum, NPG, lane);
                wave_lds_sync();
                for (int p = lane; p < P; p += 64) {
                    const int e0 = poff[p], e1 = poff[p + 1];
                    // the parameter's first gate: its op slots and matrix
                    // coefficients, read before the update so they land during
                    // its arithmetic
                    const int j0 = e0 < e1 ? pidx[e0] : 0;  // row 0 exists (at least one is laid out)
                    const int2 q0 = pq[j0];
                    T ab[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) mat_get(ab[k], mab[j0 * 16 + k]);
                    const ParamState ps = param_load(p);
                    double gp = 0.0;
                    for (int e2 = e0; e2 < e1; ++e2) gp += gsum[pidx[e2]];
                    param_step(p, gp, e0, e1, q0, ab, ps, rc1, rc2);
                }
            }
            if (NW == 1) {
                const double sE = wave_sum_dpp(e);  // one wave: epart[tid] is this lane's e
                if (lane == 0) energies[it] = sE;
            }
            wave_lds_sync();
        } else if (wave == NW - 1) {
            // the energy's sum beside the reverse sweep
            double sE = 0.0;
            for (int t = lane; t < D; t += 64) sE += epart[t];
            sE = wave_sum(sE);
            if (lane == 0) energies[it] = sE;
        }
    }
    __syncthreads();
    for (int p = tid; p < P; p += NT) a.theta[(size_t)inst * P + p] = th[p];
}

constexpr size_t kSmallLdsMax = 160 * 1024 - 1024;
constexpr int kSmallFast = 1 << 5;  // mode flag: k_small_fast

constexpr int kSmallReal = 1 << 6;  // mode flag: the state stays real

inline void (*fast_kernel(int n, bool complex_tab, bool two_slots, bool regtab, bool real))(SmallKernelArgs)
{
    if (real) {  // real table only: the planner takes the real state only with a real Hamiltonian
        if (n <= 6) return k_small_fast<64, 1, false, false, true>;
        if (n == 7) return k_small_fast<128, 1, false, false, true>;
        if (regtab) return k_small_fast<320, 1, false, true, true>;  // one pair slot only (two would spill)
        return two_slots ? k_small_fast<256, 2, false, false, true> : k_small_fast<256, 1, false, false, true>;
    }
    if (n <= 6) return complex_tab ? k_small_fast<64, 1, true, false, false> : k_small_fast<64, 1, false, false, false>;
    if (n == 7)
        return complex_tab ? k_small_fast<128, 1, true, false, false> : k_small_fast<128, 1, false, false, false>;
    if (two_slots)
        return complex_tab ? k_small_fast<256, 2, true, false, false> : k_small_fast<256, 2, false, false, false>;
    return complex_tab ? k_small_fast<256, 1, true, false, false> : k_small_fast<256, 1, false, false, false>;
}

int choose_block(int n)
{
    if (n <= 6) return 64;
    if (n <= 8) return 128;
    return 256;
}

}  // namespace

size_t small_fast_hist_bytes(int n, int n_gates)
{
    return (size_t)(n_gates + 1) * fast_slots(n) * 128 * sizeof(double2);
}

// 1 if the persistent loop can run this problem; *mode_out gets the Hamiltonian form
int small_run_plan(int n, int n_gates, int n_params, int n_pgates, int n_groups, int max_inst_terms,
                   int has_imag, int real_gates, int max_pairs, int *mode_out, size_t *lds_out)
{
    if (n > 10 || n_gates > 2048 || n_params > 2048) return 0;
    // up to 8 qubits with the Hamiltonian as a table: the latency-built kernel,
    // sized with the layout of the variant that will run (register rows keep
    // no table in LDS)
    if (n <= 8 && n_gates <= 1024) {
        const bool rt = fast_regtab(n, n_groups, real_gates && !has_imag, max_pairs);
        const FastLayout W = fast_layout(n, n_gates, n_params, n_pgates, n_groups, has_imag, rt);
        if (W.total <= kSmallLdsMax) {
            *mode_out = (has_imag ? 2 : 1) | kSmallFast | (real_gates && !has_imag ? kSmallReal : 0);
            *lds_out = W.total;
            return 1;
        }
    }
    const int nt = choose_block(n);
    // preference: Hamiltonian table with deferred gradient sums, table, terms with deferred sums, terms
    const int tmode = has_imag ? 2 : 1;
    const int order[4][2] = {{tmode, 1}, {tmode, 0}, {0, 1}, {0, 0}};
    for (auto &o : order) {
        const SmallLayout L = small_layout(n, n_gates, n_params, n_pgates, n_groups, max_inst_terms, nt, o[0], o[1]);
        if (L.total <= kSmallLdsMax) {
            *mode_out = o[0] | (o[1] << 4);
            *lds_out = L.total;
            return 1;
        }
    }
    return 0;
}

const char *small_run_variant(const SmallRunArgs &a, int mode, int max_pairs)
{
    if (!(mode & kSmallFast)) return "k_small_run (persistent loop)";
    const bool real = mode & kSmallReal;
    if (fast_regtab(a.n, a.n_groups, real, max_pairs)) return "k_small_fast (real state, register rows)";
    return real ? "k_small_fast (real state, table)" : "k_small_fast (persistent loop, table)";
}

hipError_t launch_small_run(const SmallRunArgs &a, const OpDesc *rops, const int32_t *pmap_off,
                            const int32_t *pmap_idx, int n_pgates, int mode, int max_inst_terms, int max_pairs,
                            int64_t batch, hipStream_t s)
{
    SmallKernelArgs ka;
    ka.a = a;
    ka.rops = rops;
    ka.pmap_off = pmap_off;
    ka.pmap_idx = pmap_idx;
    ka.n_pgates = n_pgates;
    ka.mode = mode & 15;
    ka.defer = (mode >> 4) & 1;
    ka.max_inst_terms = max_inst_terms;
    if (mode & kSmallFast) {
        const bool rt = fast_regtab(a.n, a.n_groups, mode & kSmallReal, max_pairs);
        const int nt = fast_threads(a.n) + (rt ? 64 : 0);
        const FastLayout W = fast_layout(a.n, a.n_gates, a.n_params, n_pgates, a.n_groups, ka.mode == 2, rt);
        void (*kern)(SmallKernelArgs) = fast_kernel(a.n, ka.mode == 2, max_pairs > 64, rt, mode & kSmallReal);
        if (W.total > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)W.total);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)batch), dim3(nt), W.total, s, ka);
        return hipGetLastError();
    }
    const int nthreads = choose_block(a.n);
    const SmallLayout L = small_layout(a.n, a.n_gates, a.n_params, n_pgates, a.n_groups, max_inst_terms,
                                       nthreads, ka.mode, ka.defer);
    if (L.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_small_run),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_small_run, dim3((unsigned)batch), dim3(nthreads), L.total, s, ka);
    return hipGetLastError();
}

}  // namespace vqe
