// kernels.hip -- gfx950 kernels of the VQE hot path (arXiv 2601.09951):
// reference-state preparation (Eq. 4), tile passes that apply many gates per
// HBM round trip (Eqs. 4-5), flip-group Pauli sweeps for <psi|H|psi> and
// H psi (Eq. 2), the adjoint reverse sweep, fixed-order reductions and the
// Adam update (Section 3.4).
//
// All state arithmetic is complex128 (double2, re/im interleaved).  A tile
// pass stages 2^k amplitudes in LDS: the low c index bits are contiguous in
// HBM (runs of 2^c * 16 bytes per wavefront access), the remaining k - c
// tile bits are gathered through a per-pass offset table.  Each workgroup
// walks tiles t = blockIdx.x, blockIdx.x + gridDim.x, ... of one instance
// (blockIdx.y), so the per-instance reduction tree does not depend on the
// batch size.
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

// u x + v y with one multiply and three FMAs per component (16 FP64
// instructions per 2x2 pair update instead of 20 for two products and a sum)
__device__ __forceinline__ double2 cmac(double2 u, double2 x, double2 v, double2 y)
{
    return make_double2(fma(u.x, x.x, fma(-u.y, x.y, fma(v.x, y.x, -v.y * y.y))),
                        fma(u.x, x.y, fma(u.y, x.x, fma(v.x, y.y, v.y * y.x))));
}

// zero bits inserted at the ascending positions packed 6 bits apiece in `pack`
__device__ __forceinline__ uint32_t insert_zeros(uint32_t j, uint64_t pack, int nfix)
{
    for (int i = 0; i < nfix; ++i) {
        const uint32_t p = (uint32_t)(pack >> (6 * i)) & 63u;
        j = ((j >> p) << (p + 1)) | (j & ((1u << p) - 1u));
    }
    return j;
}

// the fixed positions of an op as one register word (compile-time indices only)
__device__ __forceinline__ uint64_t fix_pack(const OpDesc &o)
{
    uint64_t pk = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) pk |= (uint64_t)o.fixpos[i] << (6 * i);
    return pk;
}

// geometry is read through a device pointer (uniform scalar loads)
__device__ __forceinline__ uint64_t tile_base(const TileGeom *__restrict__ gp, int nout, int64_t t)
{
    uint64_t base = 0;
    for (int i = 0; i < nout; ++i)
        if ((t >> i) & 1) base |= 1ull << gp->opos[i];
    return base;
}

// tile bases from an LDS table of the tile-number bits' index masks (obit[i]
// = 1 << opos[i], filled by fill_obit): LDS reads do not wait on outstanding
// global loads, as the byte loads of the geometry would
__device__ __forceinline__ void fill_obit(const TileGeom *__restrict__ gp, int nout, uint64_t *obit)
{
    for (int i = threadIdx.x; i < nout; i += blockDim.x) obit[i] = 1ull << gp->opos[i];
}

__device__ __forceinline__ uint64_t tile_base_l(const uint64_t *obit, int nout, int64_t t)
{
    uint64_t base = 0;
    for (int i = 0; i < nout; ++i)
        if ((t >> i) & 1) base |= obit[i];
    return base;
}

// offsets of the gathered (non-contiguous) part of a tile
__device__ __forceinline__ void fill_hoff(const TileGeom *__restrict__ gp, int k, int c, uint64_t *hoff)
{
    const int nh = 1 << (k - c);
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        uint64_t o = 0;
        for (int i = 0; i < k - c; ++i)
            if ((h >> i) & 1) o |= 1ull << gp->tpos[c + i];
        hoff[h] = o;
    }
}

// XOR swizzle of an LDS tile index: bits 4..7 folded into bits 0..3, so that
// 16-amplitude sub-cubes strided in any four bits spread over all banks
__device__ __forceinline__ uint32_t swz(uint32_t i) { return i ^ ((i >> 4) & 15u); }

// Streaming a tile between HBM and LDS.  Tile element j lives at
// base + hoff[j >> c] + (j & lowm) in HBM (the low c bits are contiguous) and
// at j (or swz(j)) in LDS.  NB elements per thread are read from HBM before
// the first LDS write, so that every CU keeps tens of kilobytes of reads in
// flight; one outstanding 16-byte load per thread leaves the passes far below
// HBM bandwidth.  Lanes past the tile's end re-read their first element (in
// bounds) so that every load is unconditional and the batch stays in
// registers; only the writes are predicated.
template <int NB, bool SWZ>
__device__ __forceinline__ void tile_in(double2 *tile, const double2 *__restrict__ src, uint64_t base,
                                        const uint64_t *hoff, int T, int c)
{
    const uint32_t lowm = (1u << c) - 1u;
    for (int j0 = threadIdx.x; j0 < T; j0 += NB * kThreads) {
        double rx[NB], ry[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads < T ? j0 + u * kThreads : j0;
            const double2 v = src[base + hoff[j >> c] + (j & lowm)];
            rx[u] = v.x;
            ry[u] = v.y;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads;
            if (j < T) tile[SWZ ? swz(j) : j] = make_double2(rx[u], ry[u]);
        }
    }
}

// both states of the adjoint pass (same element offsets)
template <int NB, bool SWZ>
__device__ __forceinline__ void tile_in2(double2 *ta, double2 *tb, const double2 *__restrict__ a,
                                         const double2 *__restrict__ b, uint64_t base, const uint64_t *hoff, int T,
                                         int c)
{
    const uint32_t lowm = (1u << c) - 1u;
    for (int j0 = threadIdx.x; j0 < T; j0 += NB * kThreads) {
        double ax[NB], ay[NB], bx[NB], by[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads < T ? j0 + u * kThreads : j0;
            const uint64_t gi = base + hoff[j >> c] + (j & lowm);
            const double2 va = a[gi], vb = b[gi];
            ax[u] = va.x;
            ay[u] = va.y;
            bx[u] = vb.x;
            by[u] = vb.y;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads;
            if (j < T) {
                ta[SWZ ? swz(j) : j] = make_double2(ax[u], ay[u]);
                tb[SWZ ? swz(j) : j] = make_double2(bx[u], by[u]);
            }
        }
    }
}

template <int NB, bool SWZ>
__device__ __forceinline__ void tile_out(const double2 *tile, double2 *__restrict__ dst, uint64_t base,
                                         const uint64_t *hoff, int T, int c)
{
    const uint32_t lowm = (1u << c) - 1u;
    for (int j0 = threadIdx.x; j0 < T; j0 += NB * kThreads) {
        double rx[NB], ry[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads < T ? j0 + u * kThreads : j0;
            const double2 v = tile[SWZ ? swz(j) : j];
            rx[u] = v.x;
            ry[u] = v.y;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads;
            if (j < T) dst[base + hoff[j >> c] + (j & lowm)] = make_double2(rx[u], ry[u]);
        }
    }
}

template <int NB, bool SWZ>
__device__ __forceinline__ void tile_out2(const double2 *ta, const double2 *tb, double2 *__restrict__ a,
                                          double2 *__restrict__ b, uint64_t base, const uint64_t *hoff, int T, int c)
{
    const uint32_t lowm = (1u << c) - 1u;
    for (int j0 = threadIdx.x; j0 < T; j0 += NB * kThreads) {
        double ax[NB], ay[NB], bx[NB], by[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads < T ? j0 + u * kThreads : j0;
            const double2 va = ta[SWZ ? swz(j) : j], vb = tb[SWZ ? swz(j) : j];
            ax[u] = va.x;
            ay[u] = va.y;
            bx[u] = vb.x;
            by[u] = vb.y;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kThreads;
            if (j < T) {
                const uint64_t gi = base + hoff[j >> c] + (j & lowm);
                a[gi] = make_double2(ax[u], ay[u]);
                b[gi] = make_double2(bx[u], by[u]);
            }
        }
    }
}

// An amplitude read field by field: a register array filled this way stays
// in registers even where a stage stores it back unchanged (a whole-struct
// copy from LDS into the array and back can leave the array in scratch).
__device__ __forceinline__ double2 lds_get(const double2 *p)
{
    double2 r;
    r.x = p->x;
    r.y = p->y;
    return r;
}

// Workgroup barrier that orders LDS only: outstanding global loads (a tile
// prefetch) stay in flight across it, which __syncthreads would drain.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the 64 lanes, identical in every lane, in a fixed order: DPP
// lane permutations (no LDS traffic) form quad, half-row and row sums, and
// the four row sums are added through readlane in row order.  Every lane
// must be active.  The moves carry no "old" value: the quad permutations,
// mirrors and row rotations give every lane a source, and the row broadcasts
// below leave only rows whose values the final lane never reads (a zero
// "old" would cost one extra move per DPP instruction).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

// The same sum, complete in lane 63 only (fixed order): the row sums are
// carried across rows by row_bcast:15 (rows 1, 3) and row_bcast:31 (rows 2,
// 3), so no readlane round trip through scalar registers is needed.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move_rows(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_total_last(double v)
{
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    v += dpp_move_rows<0x142, 0xA>(v);  // row_bcast:15
    v += dpp_move_rows<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// v plus its partner 16 (32) lanes away, the lower lane's value first, by
// the gfx950 row swaps (both operands the same value: each output holds the
// partner's value in one half of the rows and the lane's own in the other).
__device__ __forceinline__ double swap16_sum(double v)
{
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// The 16-lane row swap on a pair of values: lanes l with bit 4 set take b
// of lane l ^ 16 into a, lanes with it clear hand their a to lane l ^ 16's
// b.  On the register pair x[i], x[i | M] (register bit M clear / set) this
// exchanges register bit M with thread bit 4.
__device__ __forceinline__ void row_swap16(double &a, double &b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ void row_swap16(double2 &a, double2 &b)
{
    row_swap16(a.x, b.x);
    row_swap16(a.y, b.y);
}

__device__ __forceinline__ double swap32_sum(double v)
{
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// Wave sums of three values a, b, c at once, fixed order: the total of a
// ends in every lane whose index is 0 mod 4, of b in lanes 1 mod 4, of c in
// lanes 2 mod 4.  The first two exchange steps (partners lane ^ 1, lane ^ 2)
// also sort the values by lane class, so the remaining four (row rotations
// by 4 and 8, then the 16- and 32-lane swaps, all class-preserving) carry
// one value instead of three.  Every lane must be active.
__device__ __forceinline__ double wave_total3(double a, double b, double c)
{
    const int lane = (int)threadIdx.x & 63;
    const bool o1 = lane & 1, o2 = lane & 2;
    // partner lane ^ 1: even lanes keep a and c, odd lanes b and nothing
    double k1 = o1 ? b : a, k2 = o1 ? 0.0 : c;
    const double s1 = o1 ? a : b, s2 = o1 ? c : 0.0;
    k1 += dpp_move<0xB1>(s1);  // quad_perm [1, 0, 3, 2]
    k2 += dpp_move<0xB1>(s2);
    // partner lane ^ 2: lanes 0, 1 of a quad keep k1 (a, b), lanes 2, 3 keep k2 (c, 0)
    double k = o2 ? k2 : k1;
    const double s = o2 ? k1 : k2;
    k += dpp_move<0x4E>(s);  // quad_perm [2, 3, 0, 1]
    k += dpp_move<0x124>(k);  // row_ror:4
    k += dpp_move<0x128>(k);  // row_ror:8
    return swap32_sum(swap16_sum(k));
}

// sum of v over the workgroup (kThreads threads), fixed order; result in
// thread 0.  red must hold kThreads/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
__global__ void k_prepare(double2 *__restrict__ psi, uint64_t dim_mask, uint64_t total,
                          uint64_t ref)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        psi[i] = make_double2((i & dim_mask) == ref ? 1.0 : 0.0, 0.0);
}

// 2x2 matrix of a gate on its pair (first, second) at angle a
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

// matrices of gate g of instance b
__global__ void k_gate_mats(const GateDev *__restrict__ gates, int n_gates,
                            const double *__restrict__ theta, int n_params, int64_t batch,
                            double2 *__restrict__ mats)
{
    const int64_t total = batch * n_gates;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / n_gates;
        const int g = (int)(i - b * n_gates);
        const GateDev gd = gates[g];
        gate_matrix(gd.kind, gd.pidx >= 0 ? theta[b * n_params + gd.pidx] : gd.fixed, mats + i * 4);
    }
}

// parameter-shift rows: row (b, r) evaluates instance b with gate rows[r].gate shifted
__global__ void k_shift_mats(const GateDev *__restrict__ gates, int n_gates, const double *__restrict__ theta,
                             int n_params, int64_t batch, const ShiftRow *__restrict__ rows, int rows_per_inst,
                             double2 *__restrict__ mats)
{
    const int64_t total = batch * rows_per_inst * n_gates;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / n_gates;
        const int g = (int)(i - row * n_gates);
        const int64_t b = row / rows_per_inst;
        const int r = (int)(row - b * rows_per_inst);
        const GateDev gd = gates[g];
        double a = gd.pidx >= 0 ? theta[b * n_params + gd.pidx] : gd.fixed;
        if (rows[r].gate == g) a += rows[r].shift;
        gate_matrix(gd.kind, a, mats + i * 4);
    }
}

// energy[b] = E[b][0]; grad[b][p] = sum_k coef[k] E[b][row[k]] over p's entries
__global__ void k_shift_combine(const double *__restrict__ erows, int rows_per_inst, const int32_t *__restrict__ off,
                                const int32_t *__restrict__ row, const double *__restrict__ coef, int n_params,
                                int64_t batch, double *__restrict__ energy, double *__restrict__ grad)
{
    const int64_t total = batch * (int64_t)(n_params + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / (n_params + 1);
        const int p = (int)(i - b * (n_params + 1));
        const double *e = erows + b * rows_per_inst;
        if (p == n_params) {
            energy[b] = e[0];
        } else {
            double s = 0.0;
            for (int k = off[p]; k < off[p + 1]; ++k) s += coef[k] * e[row[k]];
            grad[b * n_params + p] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// forward pass: apply the pass's ops in order to every tile
__global__ __launch_bounds__(kThreads) void k_forward_pass(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const OpDesc *__restrict__ ops,
    int nops, const double2 *__restrict__ mats, int n_gates, double2 *__restrict__ psi, int64_t tiles)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tile = reinterpret_cast<double2 *>(smem);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (16u << k));
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    double2 *st = psi + (uint64_t)blockIdx.y * dim;
    const double2 *M = mats + (size_t)blockIdx.y * n_gates * 4;
    const int T = 1 << k;
    const uint32_t lowm = (1u << c) - 1u;
    fill_hoff(gp, k, c, hoff);
    __syncthreads();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        tile_in<8, false>(tile, st, base, hoff, T, c);
        __syncthreads();
        for (int q = 0; q < nops; ++q) {
            const OpDesc o = ops[q];
            if ((base & o.cmask_out) != o.cval_out) continue;
            const uint64_t pk = fix_pack(o);
            const double2 u00 = M[o.gate * 4 + 0], u01 = M[o.gate * 4 + 1];
            const double2 u10 = M[o.gate * 4 + 2], u11 = M[o.gate * 4 + 3];
            const int np = 1 << (k - o.nfix);
            for (int j = tid; j < np; j += kThreads) {
                const uint32_t p0 = insert_zeros((uint32_t)j, pk, o.nfix) | o.fixed_bits;
                const uint32_t p1 = p0 ^ o.m;
                const double2 a = tile[p0], b = tile[p1];
                if (o.cls == CLS_SWAP) {
                    tile[p0] = b;
                    tile[p1] = a;
                } else if (o.cls == CLS_DIAG) {
                    tile[p0] = cmul(u00, a);
                    tile[p1] = cmul(u11, b);
                } else {
                    tile[p0] = cmac(u00, a, u01, b);
                    tile[p1] = cmac(u10, a, u11, b);
                }
            }
            __syncthreads();
        }
        tile_out<8, false>(tile, st, base, hoff, T, c);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// reverse (adjoint) pass: for each op, in the plan's (reversed) order,
//   g_l += Im <lam|G_l|psi> over the tile's active pairs, then
//   psi <- U_l^dag psi, lam <- U_l^dag lam.
// Per-op sums are reduced per wave into LDS slots red[slot][wave] (summed
// across this workgroup's tiles), then written as one partial per
// (instance, parametric gate, workgroup).
__global__ __launch_bounds__(kThreads) void k_reverse_pass(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const OpDesc *__restrict__ ops,
    int nops, int n_param_ops, const double2 *__restrict__ mats, int n_gates,
    double2 *__restrict__ psi, double2 *__restrict__ lam, int64_t tiles,
    double *__restrict__ partials, int n_pgates)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tp = reinterpret_cast<double2 *>(smem);
    double2 *tl = tp + (1u << k);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (32u << k));
    double *red = reinterpret_cast<double *>(hoff + (1u << (k - c)));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t dim = 1ull << n;
    double2 *sp = psi + (uint64_t)blockIdx.y * dim;
    double2 *sl = lam + (uint64_t)blockIdx.y * dim;
    const double2 *M = mats + (size_t)blockIdx.y * n_gates * 4;
    const int T = 1 << k;
    const uint32_t lowm = (1u << c) - 1u;
    fill_hoff(gp, k, c, hoff);
    for (int i = tid; i < n_param_ops * 4; i += kThreads) red[i] = 0.0;
    __syncthreads();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        tile_in2<8, false>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
        int slot = 0;
        for (int q = 0; q < nops; ++q) {
            const OpDesc o = ops[q];
            const bool param = o.pgate >= 0;
            const int my_slot = slot;
            if (param) ++slot;
            if ((base & o.cmask_out) != o.cval_out) continue;
            // U^dagger
            const double2 v00 = cconj(M[o.gate * 4 + 0]), v01 = cconj(M[o.gate * 4 + 2]);
            const double2 v10 = cconj(M[o.gate * 4 + 1]), v11 = cconj(M[o.gate * 4 + 3]);
            const int np = 1 << (k - o.nfix);
            const uint64_t pk = fix_pack(o);
            double acc = 0.0;
            for (int j = tid; j < np; j += kThreads) {
                const uint32_t p0 = insert_zeros((uint32_t)j, pk, o.nfix) | o.fixed_bits;
                const uint32_t p1 = p0 ^ o.m;
                const double2 a = tp[p0], b = tp[p1];
                const double2 la = tl[p0], lb = tl[p1];
                if (param) {
                    if (o.gen == GEN_Y)  // Im(<la|-i b> + <lb|i a>)
                        acc += -(la.x * b.x + la.y * b.y) + (lb.x * a.x + lb.y * a.y);
                    else if (o.gen == GEN_X)  // Im(<la|b> + <lb|a>)
                        acc += (la.x * b.y - la.y * b.x) + (lb.x * a.y - lb.y * a.x);
                    else  // GEN_Z: Im(<la|a> - <lb|b>)
                        acc += (la.x * a.y - la.y * a.x) - (lb.x * b.y - lb.y * b.x);
                }
                if (o.cls == CLS_SWAP) {
                    tp[p0] = b;
                    tp[p1] = a;
                    tl[p0] = lb;
                    tl[p1] = la;
                } else if (o.cls == CLS_DIAG) {
                    tp[p0] = cmul(v00, a);
                    tp[p1] = cmul(v11, b);
                    tl[p0] = cmul(v00, la);
                    tl[p1] = cmul(v11, lb);
                } else {
                    tp[p0] = cmac(v00, a, v01, b);
                    tp[p1] = cmac(v10, a, v11, b);
                    tl[p0] = cmac(v00, la, v01, lb);
                    tl[p1] = cmac(v10, la, v11, lb);
                }
            }
            if (param) {
                acc = wave_sum(acc);
                if (lane == 0) red[my_slot * 4 + wave] += acc;
            }
            __syncthreads();
        }
        tile_out2<8, false>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
    }
    // one partial per parametric op of this pass
    if (tid == 0) {
        int slot = 0;
        const int W = gridDim.x;
        for (int q = 0; q < nops; ++q) {
            const int pg = ops[q].pgate;
            if (pg < 0) continue;
            const double v = red[slot * 4 + 0] + red[slot * 4 + 1] + red[slot * 4 + 2] + red[slot * 4 + 3];
            partials[((size_t)blockIdx.y * n_pgates + pg) * W + blockIdx.x] = v;
            ++slot;
        }
    }
}

// ---------------------------------------------------------------------------
// Register-staged passes (tiles with k >= 8).  The tile sits in LDS under an
// XOR swizzle (bits 4..7 folded into bits 0..3) so that sub-cubes strided in
// any four bits spread over all banks.  Per stage each thread loads its
// 16-amplitude sub-cube into registers, applies the stage's ops there (the
// pair partner i ^ M is resolved at compile time for every mask M), and
// stores the sub-cube back: one LDS round trip per stage instead of per op.

struct Mat2 {
    double2 a, b, c, d;  // [[a, b], [c, d]] acting on (lower, upper) register index
};

__device__ __forceinline__ Mat2 stage_matrix(const double2 *__restrict__ M, int gate, int swap)
{
    const double2 u00 = M[gate * 4 + 0], u01 = M[gate * 4 + 1], u10 = M[gate * 4 + 2], u11 = M[gate * 4 + 3];
    Mat2 v;
    if (swap) {
        v.a = u11; v.b = u10; v.c = u01; v.d = u00;
    } else {
        v.a = u00; v.b = u01; v.c = u10; v.d = u11;
    }
    return v;
}

__device__ __forceinline__ Mat2 dagger(const Mat2 &v)
{
    Mat2 w;
    w.a = cconj(v.a);
    w.b = cconj(v.c);
    w.c = cconj(v.b);
    w.d = cconj(v.d);
    return w;
}

template <int RB, int M>
__device__ __forceinline__ void stage_fwd(double2 (&x)[1 << RB], const Mat2 &v, int cls, int lo, int cmr, int cvr,
                                          bool tpred)
{
    constexpr int HB = M >= 8 ? 8 : (M >= 4 ? 4 : (M >= 2 ? 2 : 1));
    if (cls == CLS_SWAP) {
#pragma unroll
        for (int i = 0; i < (1 << RB); ++i) {
            if (i & HB) continue;
            if (((i & M) == lo) && ((i & cmr) == cvr) && tpred) {
                const double2 t = x[i];
                x[i] = x[i ^ M];
                x[i ^ M] = t;
            }
        }
    } else if (cls == CLS_DIAG) {
#pragma unroll
        for (int i = 0; i < (1 << RB); ++i) {
            if (i & HB) continue;
            if (((i & M) == lo) && ((i & cmr) == cvr) && tpred) {
                x[i] = cmul(v.a, x[i]);
                x[i ^ M] = cmul(v.d, x[i ^ M]);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < (1 << RB); ++i) {
            if (i & HB) continue;
            if (((i & M) == lo) && ((i & cmr) == cvr) && tpred) {
                const double2 p = x[i], q = x[i ^ M];
                x[i] = cmac(v.a, p, v.b, q);
                x[i ^ M] = cmac(v.c, p, v.d, q);
            }
        }
    }
}

// reverse: gradient term over the pair (in (lower, upper) orientation; sgn
// restores the op's (first, second) orientation for the antisymmetric
// generators), then U^dagger on both states
template <int RB, int M>
__device__ __forceinline__ double stage_rev(double2 (&x)[1 << RB], double2 (&l)[1 << RB], const Mat2 &w, int cls,
                                            int gen, int lo, int cmr, int cvr, bool tpred, double sgn)
{
    constexpr int HB = M >= 8 ? 8 : (M >= 4 ? 4 : (M >= 2 ? 2 : 1));
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        if (i & HB) continue;
        if (((i & M) == lo) && ((i & cmr) == cvr) && tpred) {
            const double2 a = x[i], b = x[i ^ M], la = l[i], lb = l[i ^ M];
            if (gen == GEN_Y)
                acc += sgn * (-(la.x * b.x + la.y * b.y) + (lb.x * a.x + lb.y * a.y));
            else if (gen == GEN_X)
                acc += (la.x * b.y - la.y * b.x) + (lb.x * a.y - lb.y * a.x);
            else if (gen == GEN_Z)
                acc += sgn * ((la.x * a.y - la.y * a.x) - (lb.x * b.y - lb.y * b.x));
            if (cls == CLS_SWAP) {
                x[i] = b;
                x[i ^ M] = a;
                l[i] = lb;
                l[i ^ M] = la;
            } else if (cls == CLS_DIAG) {
                x[i] = cmul(w.a, a);
                x[i ^ M] = cmul(w.d, b);
                l[i] = cmul(w.a, la);
                l[i ^ M] = cmul(w.d, lb);
            } else {
                x[i] = cmac(w.a, a, w.b, b);
                x[i ^ M] = cmac(w.c, a, w.d, b);
                l[i] = cmac(w.a, la, w.b, lb);
                l[i ^ M] = cmac(w.c, la, w.d, lb);
            }
        }
    }
    return acc;
}

// A stage op with every field wave-uniform (scalar registers), so that the
// per-op branches below are scalar branches, not exec-masked ones.
struct UStageOp {
    uint64_t cmo, cvo;
    uint32_t cmt, cvt, M, lo, cmr, cvr, swap, cls, gen, amask;
    int32_t pgate;
};

__device__ __forceinline__ uint32_t ufirst32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ UStageOp uniform_sop(const StageOp &o)
{
    UStageOp u;
    u.cmo = ((uint64_t)ufirst32((uint32_t)(o.cmo >> 32)) << 32) | ufirst32((uint32_t)o.cmo);
    u.cvo = ((uint64_t)ufirst32((uint32_t)(o.cvo >> 32)) << 32) | ufirst32((uint32_t)o.cvo);
    u.cmt = ufirst32(o.cmt);
    u.cvt = ufirst32(o.cvt);
    const uint32_t w0 = ufirst32((uint32_t)o.M | ((uint32_t)o.lo << 8) | ((uint32_t)o.cmr << 16) | ((uint32_t)o.cvr << 24));
    const uint32_t w1 = ufirst32((uint32_t)o.swap | ((uint32_t)o.cls << 8) | ((uint32_t)o.gen << 16));
    u.M = w0 & 255u;
    u.lo = (w0 >> 8) & 255u;
    u.cmr = (w0 >> 16) & 255u;
    u.cvr = w0 >> 24;
    u.swap = w1 & 255u;
    u.cls = (w1 >> 8) & 255u;
    u.gen = (w1 >> 16) & 255u;
    u.pgate = (int32_t)ufirst32((uint32_t)o.pgate);
    u.amask = ufirst32((uint32_t)o.amask);
    return u;
}

// register flip masks of more than one bit (excitations): the generic,
// predicated path; one-bit masks take the fast paths below
#define VQE_MASK_CASES(X) X(3) X(5) X(6) X(7) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

template <int RB>
__device__ __forceinline__ void dispatch_fwd(int M, double2 (&x)[1 << RB], const Mat2 &v, int cls, int lo, int cmr,
                                             int cvr, bool tpred)
{
    switch (M) {
#define VQE_CASE(m)                                                                                    \
    case m:                                                                                            \
        if constexpr (m < (1 << RB)) stage_fwd<RB, m>(x, v, cls, lo, cmr, cvr, tpred);                \
        break;
        VQE_MASK_CASES(VQE_CASE)
#undef VQE_CASE
    default: break;
    }
}

template <int RB>
__device__ __forceinline__ double dispatch_rev(int M, double2 (&x)[1 << RB], double2 (&l)[1 << RB], const Mat2 &w,
                                               int cls, int gen, int lo, int cmr, int cvr, bool tpred, double sgn)
{
    switch (M) {
#define VQE_CASE(m)                                                                                    \
    case m:                                                                                            \
        if constexpr (m < (1 << RB)) return stage_rev<RB, m>(x, l, w, cls, gen, lo, cmr, cvr, tpred, sgn); \
        break;
        VQE_MASK_CASES(VQE_CASE)
#undef VQE_CASE
    default: break;
    }
    return 0.0;
}

// ---- one-bit register masks: every one-qubit gate and the targets of CNOT
// and CZ.  The pairs (i, i ^ M) to update come as a host-computed bit mask
// (register controls folded in); ALL marks the mask with every pair set, so
// the common uncontrolled gate runs with no per-pair test.
template <int RB, int M>
__host__ __device__ constexpr uint32_t full_pairs()
{
    uint32_t f = 0;
    for (int i = 0; i < (1 << RB); ++i)
        if (!(i & M)) f |= 1u << i;
    return f;
}

template <int CLS>
__device__ __forceinline__ void pair_fwd(double2 &a, double2 &b, const Mat2 &v)
{
    const double2 p = a, q = b;
    if (CLS == CLS_SWAP) {
        a = q;
        b = p;
    } else if (CLS == CLS_DIAG) {
        a = cmul(v.a, p);
        b = cmul(v.d, q);
    } else if (CLS == CLS_REAL) {
        a = make_double2(fma(v.a.x, p.x, v.b.x * q.x), fma(v.a.x, p.y, v.b.x * q.y));
        b = make_double2(fma(v.c.x, p.x, v.d.x * q.x), fma(v.c.x, p.y, v.d.x * q.y));
    } else {
        a = cmac(v.a, p, v.b, q);
        b = cmac(v.c, p, v.d, q);
    }
}

template <int RB, int M, int CLS, bool ALL>
__device__ __forceinline__ void pairs1_fwd(double2 (&x)[1 << RB], const Mat2 &v, uint32_t amask)
{
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        if (i & M) continue;
        if (!ALL && !((amask >> i) & 1u)) continue;
        pair_fwd<CLS>(x[i], x[i ^ M], v);
    }
}

template <int RB, int CLS>
__device__ __forceinline__ void apply1_fwd(uint32_t M, double2 (&x)[1 << RB], const Mat2 &v, uint32_t amask)
{
#define VQE_ONE(m)                                                                  \
    if (M == m) {                                                                   \
        if (amask == full_pairs<RB, m>())                                           \
            pairs1_fwd<RB, m, CLS, true>(x, v, amask);                              \
        else                                                                        \
            pairs1_fwd<RB, m, CLS, false>(x, v, amask);                             \
        return;                                                                     \
    }
    VQE_ONE(1)
    VQE_ONE(2)
    VQE_ONE(4)
    if constexpr (RB > 3) {
        VQE_ONE(8)
    }
#undef VQE_ONE
}

// gradient term Im<la|G|a> + ... of one pair in the op's (first, second)
// orientation (sgn = -1 when the lower register holds the second element)
template <int GEN>
__device__ __forceinline__ double pair_grad(const double2 &a, const double2 &b, const double2 &la, const double2 &lb,
                                            double sgn)
{
    if (GEN == GEN_Y) return sgn * ((lb.x * a.x + lb.y * a.y) - (la.x * b.x + la.y * b.y));
    if (GEN == GEN_X) return (la.x * b.y - la.y * b.x) + (lb.x * a.y - lb.y * a.x);
    if (GEN == GEN_Z) return sgn * ((la.x * a.y - la.y * a.x) - (lb.x * b.y - lb.y * b.x));
    return 0.0;
}

// gradient term of one pair for a runtime generator (three forms, selected)
__device__ __forceinline__ double pair_grad_rt(int gen, const double2 &a, const double2 &b, const double2 &la,
                                               const double2 &lb, double sgn)
{
    const double gy = sgn * ((lb.x * a.x + lb.y * a.y) - (la.x * b.x + la.y * b.y));
    const double gx = (la.x * b.y - la.y * b.x) + (lb.x * a.y - lb.y * a.x);
    const double gz = sgn * ((la.x * a.y - la.y * a.x) - (lb.x * b.y - lb.y * b.x));
    return gen == GEN_Y ? gy : (gen == GEN_X ? gx : (gen == GEN_Z ? gz : 0.0));
}

template <int RB, int M, int CLS>
__device__ __forceinline__ double pairs1_rev(double2 (&x)[1 << RB], double2 (&l)[1 << RB], const Mat2 &w,
                                             uint32_t amask, int gen, double sgn)
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        if (i & M) continue;
        if (!((amask >> i) & 1u)) continue;
        acc += pair_grad_rt(gen, x[i], x[i ^ M], l[i], l[i ^ M], sgn);
        pair_fwd<CLS>(x[i], x[i ^ M], w);
        pair_fwd<CLS>(l[i], l[i ^ M], w);
    }
    return acc;
}

template <int RB, int CLS>
__device__ __forceinline__ double apply1_rev(uint32_t M, double2 (&x)[1 << RB], double2 (&l)[1 << RB],
                                             const Mat2 &w, uint32_t amask, int gen, double sgn)
{
    if (M == 1) return pairs1_rev<RB, 1, CLS>(x, l, w, amask, gen, sgn);
    if (M == 2) return pairs1_rev<RB, 2, CLS>(x, l, w, amask, gen, sgn);
    if (M == 4) return pairs1_rev<RB, 4, CLS>(x, l, w, amask, gen, sgn);
    if constexpr (RB > 3)
        if (M == 8) return pairs1_rev<RB, 8, CLS>(x, l, w, amask, gen, sgn);
    return 0.0;
}

// one forward op on a thread's sub-cube (o wave-uniform)
template <int RB>
__device__ __forceinline__ void apply_fwd(const UStageOp &o, double2 (&x)[1 << RB], const Mat2 &v, uint32_t bl)
{
    const bool tpred = o.cmt == 0 || (bl & o.cmt) == o.cvt;  // control on a sub-cube bit
    if ((o.M & (o.M - 1)) == 0) {
        if (!tpred) return;
        switch (o.cls) {
        case CLS_SWAP: apply1_fwd<RB, CLS_SWAP>(o.M, x, v, o.amask); break;
        case CLS_DIAG: apply1_fwd<RB, CLS_DIAG>(o.M, x, v, o.amask); break;
        case CLS_REAL: apply1_fwd<RB, CLS_REAL>(o.M, x, v, o.amask); break;
        default: apply1_fwd<RB, CLS_GENERAL>(o.M, x, v, o.amask); break;
        }
    } else {
        dispatch_fwd<RB>((int)o.M, x, v, (int)o.cls, (int)o.lo, (int)o.cmr, (int)o.cvr, tpred);
    }
}

// one reverse op: returns this thread's gradient partial (0 for fixed gates)
template <int RB>
__device__ __forceinline__ double apply_rev(const UStageOp &o, double2 (&x)[1 << RB], double2 (&l)[1 << RB],
                                            const Mat2 &w, uint32_t bl, bool have)
{
    const bool tpred = have && (o.cmt == 0 || (bl & o.cmt) == o.cvt);
    const double sgn = o.swap ? -1.0 : 1.0;
    const int gen = o.pgate >= 0 ? (int)o.gen : GEN_NONE;
    if ((o.M & (o.M - 1)) == 0) {
        if (!tpred) return 0.0;
        switch (o.cls) {
        case CLS_REAL: return apply1_rev<RB, CLS_REAL>(o.M, x, l, w, o.amask, gen, sgn);
        case CLS_DIAG: return apply1_rev<RB, CLS_DIAG>(o.M, x, l, w, o.amask, gen, sgn);
        case CLS_SWAP: return apply1_rev<RB, CLS_SWAP>(o.M, x, l, w, o.amask, gen, sgn);
        default: return apply1_rev<RB, CLS_GENERAL>(o.M, x, l, w, o.amask, gen, sgn);
        }
    }
    return dispatch_rev<RB>((int)o.M, x, l, w, (int)o.cls, gen, (int)o.lo, (int)o.cmr, (int)o.cvr, tpred, sgn);
}

template <int RB>
__device__ __forceinline__ void stage_offsets(uint32_t rpack, uint32_t (&roff)[1 << RB])
{
    uint32_t r[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) r[b] = 1u << ((rpack >> (4 * b)) & 15u);
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b) o |= ((i >> b) & 1) ? r[b] : 0u;
        roff[i] = o;
    }
}

__device__ __forceinline__ uint32_t subcube_base(uint64_t cpack, int nc, uint32_t u)
{
    uint32_t b = 0;
    for (int i = 0; i < nc; ++i)
        if ((u >> i) & 1u) b |= 1u << ((uint32_t)(cpack >> (4 * i)) & 15u);
    return b;
}

// Per-workgroup copy of a pass's control data: stage descriptors, stage ops
// and each op's matrix for this instance, so the inner loops read LDS
// (broadcast) instead of chains of dependent global loads.
struct StageCtl {
    uint64_t cpack;
    uint32_t rpack;
    int32_t op_begin, op_count, n_param_ops;
};

__device__ __forceinline__ void load_stage_ctl(const StageDesc *__restrict__ stages, int nstages,
                                               const StageOp *__restrict__ sops, const double2 *__restrict__ Mx,
                                               StageCtl *sctl, StageOp *sop_l, Mat2 *mat_l, int reverse)
{
    const int ob0 = nstages ? stages[0].op_begin : 0;
    for (int s = threadIdx.x; s < nstages; s += blockDim.x) {
        sctl[s].cpack = stages[s].cpack;
        sctl[s].rpack = stages[s].rpack;
        sctl[s].op_begin = stages[s].op_begin - ob0;
        sctl[s].op_count = stages[s].op_count;
        sctl[s].n_param_ops = stages[s].n_param_ops;
    }
    const int nops = nstages ? stages[nstages - 1].op_begin + stages[nstages - 1].op_count - ob0 : 0;
    for (int q = threadIdx.x; q <= nops; q += blockDim.x) {
        if (q == nops) {  // padding entry: the op loop reads one op ahead
            StageOp z = {};
            z.M = 1;
            sop_l[q] = z;
            mat_l[q] = Mat2{};
            continue;
        }
        const StageOp o = sops[ob0 + q];
        sop_l[q] = o;
        const Mat2 v = stage_matrix(Mx, o.gate, o.swap);
        mat_l[q] = reverse ? dagger(v) : v;
    }
}

__host__ __device__ inline size_t stage_ctl_bytes(int nstages, int nops)
{
    return (size_t)nstages * sizeof(StageCtl) + (size_t)(nops + 1) * (sizeof(StageOp) + sizeof(Mat2));
}

template <int RB>
__global__ __launch_bounds__(kThreads) void k_forward_staged(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const StageDesc *__restrict__ stages,
    int nstages, int nops, const StageOp *__restrict__ sops, const double2 *__restrict__ mats, int n_gates,
    double2 *__restrict__ psi, int64_t tiles)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tile = reinterpret_cast<double2 *>(smem);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (16u << k));
    Mat2 *mat_l = reinterpret_cast<Mat2 *>(hoff + (1u << (k - c)));
    StageOp *sop_l = reinterpret_cast<StageOp *>(mat_l + nops + 1);  // + one padding op
    StageCtl *sctl = reinterpret_cast<StageCtl *>(sop_l + nops + 1);
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    double2 *st = psi + (uint64_t)blockIdx.y * dim;
    const double2 *Mx = mats + (size_t)blockIdx.y * n_gates * 4;
    const int T = 1 << k;
    const int nsub = 1 << (k - RB);
    const uint32_t lowm = (1u << c) - 1u;
    fill_hoff(gp, k, c, hoff);
    load_stage_ctl(stages, nstages, sops, Mx, sctl, sop_l, mat_l, 0);
    __syncthreads();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        tile_in<16, true>(tile, st, base, hoff, T, c);
        __syncthreads();
        for (int s = 0; s < nstages; ++s) {
            const StageCtl sc = sctl[s];
            uint32_t roff[1 << RB];
            stage_offsets<RB>(sc.rpack, roff);
            for (int u = tid; u < nsub; u += kThreads) {
                const uint32_t bl = subcube_base(sc.cpack, k - RB, (uint32_t)u);
                double2 x[1 << RB];
#pragma unroll
                for (int i = 0; i < (1 << RB); ++i) x[i] = tile[swz(bl | roff[i])];
                StageOp nop = sop_l[sc.op_begin];
                Mat2 nmat = mat_l[sc.op_begin];
                for (int q = sc.op_begin; q < sc.op_begin + sc.op_count; ++q) {
                    const UStageOp o = uniform_sop(nop);
                    const Mat2 v = nmat;
                    nop = sop_l[q + 1];  // the next op's record, read while this op runs
                    nmat = mat_l[q + 1];
                    if ((base & o.cmo) != o.cvo) continue;
                    apply_fwd<RB>(o, x, v, bl);
                }
#pragma unroll
                for (int i = 0; i < (1 << RB); ++i) tile[swz(bl | roff[i])] = x[i];
            }
            __syncthreads();
        }
        tile_out<16, true>(tile, st, base, hoff, T, c);
        __syncthreads();
    }
}

template <int RB>
__global__ __launch_bounds__(kThreads) void k_reverse_staged(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const StageDesc *__restrict__ stages,
    int nstages, int nops, const StageOp *__restrict__ sops, int n_param_ops, const double2 *__restrict__ mats,
    int n_gates, double2 *__restrict__ psi, double2 *__restrict__ lam, int64_t tiles,
    double *__restrict__ partials, int n_pgates)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tp = reinterpret_cast<double2 *>(smem);
    double2 *tl = tp + (1u << k);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (32u << k));
    double *red = reinterpret_cast<double *>(hoff + (1u << (k - c)));
    Mat2 *mat_l = reinterpret_cast<Mat2 *>(red + 4 * (size_t)(n_param_ops > 0 ? n_param_ops : 1));
    StageOp *sop_l = reinterpret_cast<StageOp *>(mat_l + nops + 1);  // + one padding op
    StageCtl *sctl = reinterpret_cast<StageCtl *>(sop_l + nops + 1);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t dim = 1ull << n;
    double2 *sp = psi + (uint64_t)blockIdx.y * dim;
    double2 *sl = lam + (uint64_t)blockIdx.y * dim;
    const double2 *Mx = mats + (size_t)blockIdx.y * n_gates * 4;
    const int T = 1 << k;
    const int nsub = 1 << (k - RB);
    const uint32_t lowm = (1u << c) - 1u;
    fill_hoff(gp, k, c, hoff);
    load_stage_ctl(stages, nstages, sops, Mx, sctl, sop_l, mat_l, 1);
    for (int i = tid; i < n_param_ops * 4; i += kThreads) red[i] = 0.0;
    __syncthreads();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        tile_in2<8, true>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
        int slot0 = 0;
        for (int s = 0; s < nstages; ++s) {
            const StageCtl sc = sctl[s];
            uint32_t roff[1 << RB];
            stage_offsets<RB>(sc.rpack, roff);
            // every thread walks the ops (a thread with no sub-cube contributes 0)
            for (int u0 = 0; u0 < nsub; u0 += kThreads) {
                const int u = u0 + tid;
                const bool have = u < nsub;
                const uint32_t bl = have ? subcube_base(sc.cpack, k - RB, (uint32_t)u) : 0u;
                double2 x[1 << RB], l[1 << RB];
#pragma unroll
                for (int i = 0; i < (1 << RB); ++i) {
                    x[i] = have ? tp[swz(bl | roff[i])] : make_double2(0.0, 0.0);
                    l[i] = have ? tl[swz(bl | roff[i])] : make_double2(0.0, 0.0);
                }
                int slot = slot0;
                StageOp nop = sop_l[sc.op_begin];
                Mat2 nmat = mat_l[sc.op_begin];
                for (int q = sc.op_begin; q < sc.op_begin + sc.op_count; ++q) {
                    const UStageOp o = uniform_sop(nop);
                    const Mat2 w = nmat;
                    nop = sop_l[q + 1];  // the next op's record, read while this op runs
                    nmat = mat_l[q + 1];
                    const int my_slot = slot;
                    if (o.pgate >= 0) ++slot;
                    if ((base & o.cmo) != o.cvo) continue;
                    double acc = apply_rev<RB>(o, x, l, w, bl, have);
                    if (o.pgate >= 0) {
                        acc = wave_sum(acc);
                        if (lane == 0) red[my_slot * 4 + wave] += acc;
                    }
                }
                if (have) {
#pragma unroll
                    for (int i = 0; i < (1 << RB); ++i) {
                        tp[swz(bl | roff[i])] = x[i];
                        tl[swz(bl | roff[i])] = l[i];
                    }
                }
            }
            slot0 += sc.n_param_ops;
            __syncthreads();
        }
        tile_out2<8, true>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
    }
    if (tid == 0) {
        const int W = gridDim.x;
        int slot = 0;
        for (int q = 0; q < nops; ++q) {
            const int pg = sop_l[q].pgate;
            if (pg < 0) continue;
            const double v = red[slot * 4 + 0] + red[slot * 4 + 1] + red[slot * 4 + 2] + red[slot * 4 + 3];
            partials[((size_t)blockIdx.y * n_pgates + pg) * W + blockIdx.x] = v;
            ++slot;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused stages (forward passes of one-qubit gates, X and CNOT).
//
// fused[inst][slot] = product of the slot's gate matrices in application
// order (identity for an empty slot).
__global__ void k_fuse_mats(const int32_t *__restrict__ slot_off, const int32_t *__restrict__ slot_gate, int n_slots,
                            const double2 *__restrict__ mats, int n_gates, int64_t batch, double2 *__restrict__ fused)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= batch * n_slots) return;
    const int64_t inst = w / n_slots;
    const int slot = (int)(w - inst * n_slots);
    double2 a = make_double2(1.0, 0.0), b = make_double2(0.0, 0.0), c = b, d = a;  // [[a, b], [c, d]]
    for (int e = slot_off[slot]; e < slot_off[slot + 1]; ++e) {
        const double2 *U = mats + ((size_t)inst * n_gates + slot_gate[e]) * 4;
        const double2 u00 = U[0], u01 = U[1], u10 = U[2], u11 = U[3];
        const double2 na = cadd(cmul(u00, a), cmul(u01, c)), nb = cadd(cmul(u00, b), cmul(u01, d));
        const double2 nc = cadd(cmul(u10, a), cmul(u11, c)), nd = cadd(cmul(u10, b), cmul(u11, d));
        a = na;
        b = nb;
        c = nc;
        d = nd;
    }
    double2 *o = fused + (size_t)w * 4;
    o[0] = a;
    o[1] = b;
    o[2] = c;
    o[3] = d;
}

// The tile index of sub-cube u's first amplitude: u with zero bits inserted
// at the stage's register positions (the other tile bits, ascending, carry
// the bits of u).  The positions are wave-uniform, so their sort runs on the
// scalar unit; four or three insertions replace a loop over every tile bit.
__device__ __forceinline__ void cswap_u(uint32_t &a, uint32_t &b)
{
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

template <int RB>
__device__ __forceinline__ uint32_t subcube_base_of(uint32_t u, const FusedStage &fs)
{
    uint32_t p[4] = {fs.rpos[0], fs.rpos[1], fs.rpos[2], RB > 3 ? fs.rpos[3] : 0u};
    if (RB > 3) {
        cswap_u(p[0], p[1]);
        cswap_u(p[2], p[3]);
        cswap_u(p[0], p[2]);
        cswap_u(p[1], p[3]);
        cswap_u(p[1], p[2]);
    } else {
        cswap_u(p[0], p[1]);
        cswap_u(p[1], p[2]);
        cswap_u(p[0], p[1]);
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) u = ((u >> p[i]) << (p[i] + 1)) | (u & ((1u << p[i]) - 1u));
    return u;
}

// general 2x2 on register bit B (compile time) of a 16-amplitude sub-cube
template <int B>
__device__ __forceinline__ void fused_bit(double2 (&x)[16], const Mat2 &v)
{
    constexpr int M = 1 << B;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & M) continue;
        const double2 p = x[i], q = x[i | M];
        x[i] = cmac(v.a, p, v.b, q);
        x[i | M] = cmac(v.c, p, v.d, q);
    }
}

// A parity phase of a stage as staged in LDS: the two diagonal entries of
// its gate for this instance (forward U, adjoint U^dagger) and, in adjoint
// passes, the gradient slot of a parametric one (-1 otherwise).
struct PhaseL {
    uint32_t mask, cbit;
    int32_t pslot, pg;
    double2 d0, d1;
};

// the stage's parity phases on a sub-cube of N amplitudes at tile indices
// bl | roff[i]: the parity splits into the thread's part (bl) and a
// wave-uniform part (roff[i])
template <int N>
__device__ __forceinline__ void apply_phases(double2 (&x)[N], const PhaseL *phl, int count, uint32_t bl,
                                             const uint32_t (&roff)[N])
{
    for (int p = 0; p < count; ++p) {
        const PhaseL &ph = phl[p];
        const uint32_t mask = __builtin_amdgcn_readfirstlane(ph.mask);
        const uint32_t sb = ((uint32_t)__popc(mask & bl) ^ __builtin_amdgcn_readfirstlane(ph.cbit)) & 1u;
        const double2 e0 = sb ? ph.d1 : ph.d0, e1 = sb ? ph.d0 : ph.d1;
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = cmul((__popc(mask & roff[i]) & 1) ? e1 : e0, x[i]);
    }
}

// one fused stage for this thread's sub-cube u (na active register bits;
// PERM: the CNOT / X network moves the amplitudes on the way back to LDS).
// sub = the plan's entry for (stage, u): swz(bl) | swz(lbl) << 16 (see
// build_fsub); the swizzle is linear over xor, so every address is one of
// them xor a wave-uniform term.
// A pass whose first stage holds no gates and no phases only permutes the
// tile by its network (the amplitude at tile index v moves to L v ^ c, c
// depending on the tile through X gates conditioned on bits outside it).
// That map is applied while the tile is read in, instead of by a round trip
// through LDS: mcol[b] = L e_b for every tile bit b (threads 0 .. k-1 fill
// it), and element j = tid + 256 u of the tile goes to swz(L tid ^ L (256 u)
// ^ c).
__device__ __forceinline__ bool network_only(const FusedStage &fs)
{
    return __builtin_amdgcn_readfirstlane((uint32_t)fs.na) == 0 &&
           __builtin_amdgcn_readfirstlane((uint32_t)fs.phase_count) == 0 &&
           __builtin_amdgcn_readfirstlane((uint32_t)fs.xbit) == 0;
}

__device__ __forceinline__ void network_columns(const FusedStage &fs, int k, uint32_t *mcol)
{
    const int b = (int)threadIdx.x, nb = fs.nb;
    if (b < nb)
        mcol[fs.rpos[b]] = fs.lr[1 << b];
    else if (b < k)
        mcol[fs.cpos[b - nb]] = fs.lc[b - nb];
}

// L tid (bits 0-7 of the tile index) and L e_{8+i} (i < 4) from the columns
struct NetMap {
    uint32_t lt, m[4];
};

__device__ __forceinline__ NetMap network_map(const uint32_t *mcol, int k)
{
    NetMap nm;
    nm.lt = 0;
    for (int b = 0; b < 8 && b < k; ++b)
        if ((threadIdx.x >> b) & 1u) nm.lt ^= mcol[b];
#pragma unroll
    for (int i = 0; i < 4; ++i) nm.m[i] = 8 + i < k ? mcol[8 + i] : 0u;
    return nm;
}

// the constant of a stage's network for the tile at `base`
__device__ __forceinline__ uint32_t stage_const(const FusedStage &fs, const FusedCond *__restrict__ fconds,
                                                uint64_t base)
{
    uint32_t ctile = fs.c0;
    for (int q = 0; q < fs.cond_count; ++q) {
        const FusedCond fc = fconds[fs.cond_begin + q];
        if ((base & fc.cmo) == fc.cvo) ctile ^= fc.xmask;
    }
    return ctile;
}

// LDS index of tile element tid + 256 u under the network (u compile-time)
__device__ __forceinline__ uint32_t net_index(const NetMap &nm, uint32_t cn, int u)
{
    return swz(nm.lt ^ cn ^ ((u & 1) ? nm.m[0] : 0u) ^ ((u & 2) ? nm.m[1] : 0u) ^ ((u & 4) ? nm.m[2] : 0u) ^
               ((u & 8) ? nm.m[3] : 0u));
}

// tile_in (one state / two states) with the network folded in; the tile has
// at most NB * kThreads amplitudes
template <int NB>
__device__ __forceinline__ void tile_in_net(double2 *tile, const double2 *__restrict__ src, uint64_t base,
                                            const uint64_t *hoff, int T, int c, const NetMap &nm, uint32_t cn)
{
    const uint32_t lowm = (1u << c) - 1u;
    double rx[NB], ry[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j0 = (int)threadIdx.x + u * kThreads;
        const int j = j0 < T ? j0 : (int)threadIdx.x;
        const double2 v = src[base + hoff[j >> c] + (j & lowm)];
        rx[u] = v.x;
        ry[u] = v.y;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
        if ((int)threadIdx.x + u * kThreads < T) tile[net_index(nm, cn, u)] = make_double2(rx[u], ry[u]);
}

template <int NB>
__device__ __forceinline__ void tile_in2_net(double2 *ta, double2 *tb, const double2 *__restrict__ a,
                                             const double2 *__restrict__ b, uint64_t base, const uint64_t *hoff,
                                             int T, int c, const NetMap &nm, uint32_t cn)
{
    const uint32_t lowm = (1u << c) - 1u;
    double ax[NB], ay[NB], bx[NB], by[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j0 = (int)threadIdx.x + u * kThreads;
        const int j = j0 < T ? j0 : (int)threadIdx.x;
        const uint64_t gi = base + hoff[j >> c] + (j & lowm);
        const double2 va = a[gi], vb = b[gi];
        ax[u] = va.x;
        ay[u] = va.y;
        bx[u] = vb.x;
        by[u] = vb.y;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
        if ((int)threadIdx.x + u * kThreads < T) {
            const uint32_t d = net_index(nm, cn, u);
            ta[d] = make_double2(ax[u], ay[u]);
            tb[d] = make_double2(bx[u], by[u]);
        }
}

// XB: the stage's qubit on thread bit 4 (tile bit cpos[4]) is exchanged
// into register bit 3 after the register chains and takes its chain there
// (fm[4]); the store then follows the exchanged layout (PERM).
template <int NA, bool PERM, bool PH, bool XB = false>
__device__ __forceinline__ void fused_stage(double2 *tile, const FusedStage &fs, const Mat2 *fm, int nsub,
                                            uint32_t ctile, const PhaseL *phl, int nph, uint32_t sub)
{
    static_assert(!XB || (NA == 4 && PERM), "the exchange follows four register chains and stores through the map");
    const bool have = (int)threadIdx.x < nsub;
    const uint32_t sbl = sub & 0xFFFFu, slbl = sub >> 16;
    uint32_t roff[16], sro[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        roff[i] = ((i & 1) ? 1u << fs.rpos[0] : 0u) | ((i & 2) ? 1u << fs.rpos[1] : 0u) |
                  ((i & 4) ? 1u << fs.rpos[2] : 0u) | ((i & 8) ? 1u << fs.rpos[3] : 0u);
        sro[i] = swz(roff[i]);  // uniform
    }
    // every thread loads (one without a sub-cube reads sub-cube 0's
    // addresses, which the caller passes it); only owners compute and store
    double2 x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = lds_get(tile + (sbl ^ sro[i]));
    if (have) {
        if (NA > 0) fused_bit<0>(x, fm[0]);
        if (NA > 1) fused_bit<1>(x, fm[1]);
        if (NA > 2) fused_bit<2>(x, fm[2]);
        if (NA > 3) fused_bit<3>(x, fm[3]);
    }
    uint32_t bl = swz(sbl);  // swz is its own inverse
    if (XB) {
        // every lane takes part (threads with and without sub-cubes pair
        // among themselves: the sub-cube count is a multiple of 32)
#pragma unroll
        for (int i = 0; i < 8; ++i) row_swap16(x[i], x[i + 8]);
        if (have) fused_bit<3>(x, fm[4]);
        const uint32_t d = (1u << fs.rpos[3]) ^ (1u << fs.cpos[kXLane]);  // the exchanged tile bits
        if ((threadIdx.x >> kXLane) & 1u) bl ^= d;
#pragma unroll
        for (int i = 8; i < 16; ++i) roff[i] ^= d;
    }
    if (PH && have) apply_phases<16>(x, phl, nph, bl, roff);
    if (PERM) {
        lds_barrier();  // every sub-cube is read before any amplitude moves
        if (have) {
#pragma unroll
            for (int i = 0; i < 16; ++i) tile[slbl ^ swz(fs.lr[i] ^ ctile)] = x[i];
        }
    } else if (have) {
#pragma unroll
        for (int i = 0; i < 16; ++i) tile[sbl ^ sro[i]] = x[i];
    }
}

template <bool PH>
__global__ __launch_bounds__(kThreads) void k_forward_fused(const TileGeom *__restrict__ gp, int n, int k, int c,
                                                            int nout, const FusedStage *__restrict__ fstages,
                                                            int nstages, const FusedCond *__restrict__ fconds,
                                                            const double2 *__restrict__ fused, int n_slots,
                                                            const FusedPhase *__restrict__ fphases, int ph0,
                                                            int nph, const double2 *__restrict__ mats,
                                                            int n_gates, double2 *__restrict__ psi, int64_t tiles,
                                                            const uint32_t *__restrict__ fsub)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tile = reinterpret_cast<double2 *>(smem);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (16u << k));
    Mat2 *fm = reinterpret_cast<Mat2 *>(hoff + (1u << (k - c)));  // 4 per stage
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    double2 *st = psi + (uint64_t)blockIdx.y * dim;
    const int T = 1 << k;
    const int nsub = 1 << (k - 4);
    fill_hoff(gp, k, c, hoff);
    const int slot0 = nstages ? fstages[0].slot : 0;
    const double2 *F = fused + ((size_t)blockIdx.y * n_slots + slot0) * 4;
    double2 *fmd = reinterpret_cast<double2 *>(fm);
    for (int i = tid; i < 20 * nstages; i += kThreads) fmd[i] = F[i];  // 5 slots per stage, 4 double2 each
    PhaseL *phl = reinterpret_cast<PhaseL *>(fm + 5 * nstages);
    const double2 *Mx = mats + (size_t)blockIdx.y * n_gates * 4;
    for (int i = tid; PH && i < nph; i += kThreads) {
        const FusedPhase f = fphases[ph0 + i];
        PhaseL &q = phl[i];  // field by field (a whole-struct copy into LDS goes through scratch)
        q.mask = f.mask;
        q.cbit = f.cbit;
        q.pslot = -1;
        q.pg = -1;
        q.d0 = Mx[f.gate * 4 + 0];
        q.d1 = Mx[f.gate * 4 + 3];
    }
    uint32_t *mcol = reinterpret_cast<uint32_t *>(phl + nph);  // 16
    const bool fold = nstages > 0 && T <= 16 * kThreads && network_only(fstages[0]);
    if (fold) network_columns(fstages[0], k, mcol);
    __syncthreads();
    const NetMap nm = fold ? network_map(mcol, k) : NetMap{};
    const int s0 = fold ? 1 : 0;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        if (fold)
            tile_in_net<16>(tile, st, base, hoff, T, c, nm, stage_const(fstages[0], fconds, base));
        else
            tile_in<16, true>(tile, st, base, hoff, T, c);
        lds_barrier();
        const uint32_t *fsu = fsub + (tid < nsub ? tid : 0);
        uint32_t sub_next = fsu[(size_t)s0 * nsub];
        for (int s = s0; s < nstages; ++s) {
            const uint32_t sub = sub_next;
            if (s + 1 < nstages) sub_next = fsu[(size_t)(s + 1) * nsub];  // in flight during this stage
            const FusedStage fs = fstages[s];  // uniform: scalar loads
            const int na = (int)__builtin_amdgcn_readfirstlane((uint32_t)fs.na);
            const int perm = (int)__builtin_amdgcn_readfirstlane((uint32_t)fs.perm);
            uint32_t ctile = fs.c0;
            for (int q = 0; q < fs.cond_count; ++q) {
                const FusedCond fc = fconds[fs.cond_begin + q];
                if ((base & fc.cmo) == fc.cvo) ctile ^= fc.xmask;
            }
            const Mat2 *m4 = fm + 5 * s;
            const PhaseL *sp = phl + (fs.phase_begin - ph0);
            const int np = fs.phase_count;
            if (__builtin_amdgcn_readfirstlane((uint32_t)fs.xbit)) {
                fused_stage<4, true, PH, true>(tile, fs, m4, nsub, ctile, sp, np, sub);
                lds_barrier();
                continue;
            }
            switch (na * 2 + perm) {
            case 0: fused_stage<0, false, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 1: fused_stage<0, true, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 2: fused_stage<1, false, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 3: fused_stage<1, true, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 4: fused_stage<2, false, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 5: fused_stage<2, true, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 6: fused_stage<3, false, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 7: fused_stage<3, true, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            case 8: fused_stage<4, false, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            default: fused_stage<4, true, PH>(tile, fs, m4, nsub, ctile, sp, np, sub); break;
            }
            lds_barrier();
        }
        tile_out<16, true>(tile, st, base, hoff, T, c);
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// Fused adjoint stages (reverse passes of one-qubit gates, X and CNOT; three
// register bits per sub-cube, both states).
//
// The gates of one register bit j (one slot, listed in the order they are
// undone, W_i = U_i^dagger) act on psi and lam as one product W = W_m ... W_1,
// and every gradient term of the slot follows from the states before it:
// with V_i = W_{i-1} ... W_1 and the generator G_i of a parametric entry,
//   Im <lam_i| G_i |psi_i> = Im <lam| K_i |psi>,   K_i = V_i^dagger G_i V_i,
// K_i Hermitian and traceless, so per pair (a, b) of psi and (la, lb) of lam
//   Im <.|K_i|.> = k00 Q0 + Re k01 Q1 + Im k01 Q2,
//   Q0 = Im(conj(la) a) - Im(conj(lb) b),  Q1 = Im(conj(la) b + conj(lb) a),
//   Q2 = Re(conj(la) b - conj(lb) a).
// Gates on the other bits of the stage commute with G_i and cancel in the
// inner product, so their order does not matter.  The kernels sum Q over
// the state (per slot, three numbers), and the per-instance coefficients
// turn the sums into the slot's gradient partials; the state update is one
// general 2x2 per bit.
//
// k_adjoint_coefs: per (instance, slot) the product W and per entry the
// coefficients (k00, Re k01, Im k01, 0) (zeros for fixed gates).
__global__ void k_adjoint_coefs(const int32_t *__restrict__ slot_off, const int32_t *__restrict__ slot_gate,
                                const int32_t *__restrict__ slot_info, int n_slots, int n_entries,
                                const double2 *__restrict__ mats, int n_gates, int64_t batch,
                                double2 *__restrict__ wout, double *__restrict__ coef)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= batch * n_slots) return;
    const int64_t inst = w / n_slots;
    const int slot = (int)(w - inst * n_slots);
    double2 v00 = make_double2(1.0, 0.0), v01 = make_double2(0.0, 0.0), v10 = v01, v11 = v00;  // V
    for (int e = slot_off[slot]; e < slot_off[slot + 1]; ++e) {
        const int info = slot_info[e];
        double *ce = coef + ((size_t)inst * n_entries + e) * 4;
        double k00 = 0.0, k01r = 0.0, k01i = 0.0;
        if (info >= 16) {
            // G V for the Pauli generator, then the first row of V^dagger (G V)
            double2 g00, g01, g10, g11;
            const int gen = info & 3;
            if (gen == GEN_X) {
                g00 = v10; g01 = v11; g10 = v00; g11 = v01;
            } else if (gen == GEN_Y) {  // [[0, -i], [i, 0]]
                g00 = make_double2(v10.y, -v10.x); g01 = make_double2(v11.y, -v11.x);
                g10 = make_double2(-v00.y, v00.x); g11 = make_double2(-v01.y, v01.x);
            } else {  // GEN_Z
                g00 = v00; g01 = v01; g10 = make_double2(-v10.x, -v10.y); g11 = make_double2(-v11.x, -v11.y);
            }
            const double2 K00 = cadd(cmul(cconj(v00), g00), cmul(cconj(v10), g10));
            const double2 K01 = cadd(cmul(cconj(v00), g01), cmul(cconj(v10), g11));
            k00 = K00.x;
            k01r = K01.x;
            k01i = K01.y;
        }
        ce[0] = k00;
        ce[1] = k01r;
        ce[2] = k01i;
        ce[3] = 0.0;
        // V <- U^dagger V
        const double2 *U = mats + ((size_t)inst * n_gates + slot_gate[e]) * 4;
        const double2 w00 = cconj(U[0]), w01 = cconj(U[2]), w10 = cconj(U[1]), w11 = cconj(U[3]);
        const double2 n00 = cadd(cmul(w00, v00), cmul(w01, v10)), n01 = cadd(cmul(w00, v01), cmul(w01, v11));
        const double2 n10 = cadd(cmul(w10, v00), cmul(w11, v10)), n11 = cadd(cmul(w10, v01), cmul(w11, v11));
        v00 = n00;
        v01 = n01;
        v10 = n10;
        v11 = n11;
    }
    double2 *o = wout + (size_t)w * 4;
    o[0] = v00;
    o[1] = v01;
    o[2] = v10;
    o[3] = v11;
}

// the three pair sums Q over this thread's sub-cube for register bit B
template <int B>
__device__ __forceinline__ void rbit_q(const double2 (&x)[8], const double2 (&l)[8], double &q0, double &q1,
                                       double &q2)
{
    constexpr int M = 1 << B;
    // FMA chains into two interleaved accumulator sets (pairs alternate)
    double s[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    int k = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (i & M) continue;
        const double2 a = x[i], b = x[i | M], la = l[i], lb = l[i | M];
        double *t = s[k++ & 1];
        t[0] = fma(lb.y, b.x, fma(-lb.x, b.y, fma(-la.y, a.x, fma(la.x, a.y, t[0]))));
        t[1] = fma(-lb.y, a.x, fma(lb.x, a.y, fma(-la.y, b.x, fma(la.x, b.y, t[1]))));
        t[2] = fma(-lb.y, a.y, fma(-lb.x, a.x, fma(la.y, b.y, fma(la.x, b.x, t[2]))));
    }
    q0 = s[0][0] + s[1][0];
    q1 = s[0][1] + s[1][1];
    q2 = s[0][2] + s[1][2];
}

template <int B>
__device__ __forceinline__ void rbit_step(double2 (&x)[8], double2 (&l)[8], const Mat2 &w, int qs, double *red,
                                          bool have)
{
    constexpr int M = 1 << B;
    if (qs >= 0) {  // the slot holds parametric gates (uniform)
        double q0, q1, q2;
        rbit_q<B>(x, l, q0, q1, q2);
        if (!have) q0 = q1 = q2 = 0.0;  // a thread without a sub-cube adds zeros
        const double t = wave_total3(q0, q1, q2);
        const int lane = (int)threadIdx.x & 63;
        if (lane < 3)  // lane j holds Q_j's wave total; LDS adds without a return value: no wait
            atomicAdd(red + (size_t)qs * 12 + 4 * lane + (threadIdx.x >> 6), t);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (i & M) continue;
        pair_fwd<CLS_GENERAL>(x[i], x[i | M], w);
        pair_fwd<CLS_GENERAL>(l[i], l[i | M], w);
    }
}

// XB as in fused_stage: the qubit on thread bit 4 is exchanged into register
// bit 2 of both states and undone there (wm[3], sums under qidx[3]).
template <int NA, bool PERM, bool PH, bool XB = false>
__device__ __forceinline__ void rev_fused_stage(double2 *tp, double2 *tl, const FusedStage &fs, const Mat2 *wm,
                                                const int32_t *qidx, int nsub, uint32_t ctile, double *red,
                                                const PhaseL *phl, int nph, double *phred, uint32_t sub)
{
    static_assert(!XB || (NA == 3 && PERM), "the exchange follows three register chains and stores through the map");
    const bool have = (int)threadIdx.x < nsub;
    // sub = swz(bl) | swz(lbl) << 16 (build_fsub); addresses are these xor a uniform term
    const uint32_t sbl = sub & 0xFFFFu, slbl = sub >> 16;
    uint32_t bl = PH ? swz(sbl) : 0u;  // swz is its own inverse
    uint32_t roff[8], sro[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        roff[i] = ((i & 1) ? 1u << fs.rpos[0] : 0u) | ((i & 2) ? 1u << fs.rpos[1] : 0u) |
                  ((i & 4) ? 1u << fs.rpos[2] : 0u);
        sro[i] = swz(roff[i]);  // uniform
    }
    // every thread loads a sub-cube (one without its own reads sub-cube 0's
    // addresses, which the caller passes it) and takes part in the sums,
    // adding zeros; only owners store
    double2 x[8], l[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        x[i] = lds_get(tp + (sbl ^ sro[i]));
        l[i] = lds_get(tl + (sbl ^ sro[i]));
    }
    if (NA > 0) rbit_step<0>(x, l, wm[0], (int)__builtin_amdgcn_readfirstlane((uint32_t)qidx[0]), red, have);
    if (NA > 1) rbit_step<1>(x, l, wm[1], (int)__builtin_amdgcn_readfirstlane((uint32_t)qidx[1]), red, have);
    if (NA > 2) rbit_step<2>(x, l, wm[2], (int)__builtin_amdgcn_readfirstlane((uint32_t)qidx[2]), red, have);
    if (XB) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            row_swap16(x[i], x[i + 4]);
            row_swap16(l[i], l[i + 4]);
        }
        rbit_step<2>(x, l, wm[3], (int)__builtin_amdgcn_readfirstlane((uint32_t)qidx[3]), red, have);
        const uint32_t d = (1u << fs.rpos[2]) ^ (1u << fs.cpos[kXLane]);  // the exchanged tile bits
        if (PH && ((threadIdx.x >> kXLane) & 1u)) bl ^= d;
#pragma unroll
        for (int i = 4; i < 8; ++i) roff[i] ^= d;
    }
    if (PH) {
        // parity phases: every gradient term is (-1)^{parity} Im(conj(lam) psi)
        // summed over the sub-cube (diagonal phases leave Im(conj(lam) psi)
        // unchanged, so one set of products serves all), then U^dagger on both
        double e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = fma(l[i].x, x[i].y, -l[i].y * x[i].x);
        for (int p = 0; p < nph; ++p) {
            const PhaseL &ph = phl[p];
            const uint32_t mask = __builtin_amdgcn_readfirstlane(ph.mask);
            const uint32_t sb = ((uint32_t)__popc(mask & bl) ^ __builtin_amdgcn_readfirstlane(ph.cbit)) & 1u;
            const int ps = (int)__builtin_amdgcn_readfirstlane((uint32_t)ph.pslot);
            if (ps >= 0) {
                double g = 0.0;
#pragma unroll
                for (int i = 0; i < 8; ++i) g += ((__popc(mask & roff[i]) & 1) ^ sb) ? -e[i] : e[i];
                if (!have) g = 0.0;
                g = wave_total_last(g);
                if ((threadIdx.x & 63) == 63) atomicAdd(phred + ps * 4 + (threadIdx.x >> 6), g);
            }
            const double2 e0 = sb ? ph.d1 : ph.d0, e1 = sb ? ph.d0 : ph.d1;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double2 d = (__popc(mask & roff[i]) & 1) ? e1 : e0;
                x[i] = cmul(d, x[i]);
                l[i] = cmul(d, l[i]);
            }
        }
    }
    if (PERM) {
        lds_barrier();  // every sub-cube is read before any amplitude moves
        if (have) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t d = slbl ^ swz(fs.lr[i] ^ ctile);
                tp[d] = x[i];
                tl[d] = l[i];
            }
        }
    } else if (have) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            tp[sbl ^ sro[i]] = x[i];
            tl[sbl ^ sro[i]] = l[i];
        }
    }
}

// One partial per (instance, parametric gate, workgroup), as the staged
// adjoint writes them.  The pass owns slots [slot0, slot0 + 3 * nstages) and
// their entries [e0, e0 + ne); wadj / coef hold the per-instance products
// and coefficients of every slot / entry of the plan (n_slots / n_entries).
template <bool PH>
__global__ __launch_bounds__(kThreads) void k_reverse_fused(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const FusedStage *__restrict__ fstages,
    int nstages, const FusedCond *__restrict__ fconds, const int32_t *__restrict__ slot_off,
    const int32_t *__restrict__ slot_info, const int32_t *__restrict__ slot_q, const int32_t *__restrict__ phase_q,
    int nq, int slot0, int n_slots, int n_entries, const double2 *__restrict__ wadj,
    const double *__restrict__ coef, const FusedPhase *__restrict__ fphases, int ph0, int nph,
    const double2 *__restrict__ mats, int n_gates, double2 *__restrict__ psi, double2 *__restrict__ lam,
    int64_t tiles, double *__restrict__ partials, int n_pgates, const uint32_t *__restrict__ fsub)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tp = reinterpret_cast<double2 *>(smem);
    double2 *tl = tp + (1u << k);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (32u << k));
    const int ns = 4 * nstages;  // slots: three register bits and the exchanged qubit per stage
    Mat2 *wm = reinterpret_cast<Mat2 *>(hoff + (1u << (k - c)));
    PhaseL *phl = reinterpret_cast<PhaseL *>(wm + ns);
    double *phred = reinterpret_cast<double *>(phl + nph);  // 4 per phase
    int32_t *qidx = reinterpret_cast<int32_t *>(phred + 4 * (size_t)nph);
    double *red = reinterpret_cast<double *>(qidx + ((ns + 1) & ~1));
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    double2 *sp = psi + (uint64_t)blockIdx.y * dim;
    double2 *sl = lam + (uint64_t)blockIdx.y * dim;
    const int T = 1 << k;
    const int nsub = 1 << (k - 3);  // at most kThreads (k <= 11)
    fill_hoff(gp, k, c, hoff);
    const double2 *Wg = wadj + ((size_t)blockIdx.y * n_slots + slot0) * 4;
    double2 *wmd = reinterpret_cast<double2 *>(wm);
    for (int i = tid; i < 4 * ns; i += kThreads) wmd[i] = Wg[i];
    // slots (phases) with parametric gates carry their index among this
    // pass's, numbered by the plan
    for (int i = tid; i < ns; i += kThreads) qidx[i] = slot_q[slot0 + i];
    for (int i = tid; i < 12 * nq; i += kThreads) red[i] = 0.0;
    {
        const double2 *Mx = mats + (size_t)blockIdx.y * n_gates * 4;
        for (int i = tid; PH && i < nph; i += kThreads) {
            const FusedPhase f = fphases[ph0 + i];
            PhaseL &q = phl[i];  // field by field (a whole-struct copy into LDS goes through scratch)
            q.mask = f.mask;
            q.cbit = f.cbit;
            q.pslot = phase_q[ph0 + i];
            q.pg = (f.info >> 4) - 1;
            q.d0 = cconj(Mx[f.gate * 4 + 0]);
            q.d1 = cconj(Mx[f.gate * 4 + 3]);
        }
        for (int i = tid; i < 4 * nph; i += kThreads) phred[i] = 0.0;
    }
    uint32_t *mcol = reinterpret_cast<uint32_t *>(red + 12 * (size_t)nq);  // 16
    const bool fold = nstages > 0 && network_only(fstages[0]);  // k <= 11: T <= 8 * kThreads
    if (fold) network_columns(fstages[0], k, mcol);
    __syncthreads();
    const NetMap nm = fold ? network_map(mcol, k) : NetMap{};
    const int s0 = fold ? 1 : 0;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        if (fold)
            tile_in2_net<8>(tp, tl, sp, sl, base, hoff, T, c, nm, stage_const(fstages[0], fconds, base));
        else
            tile_in2<8, true>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
        const uint32_t *fsu = fsub + (tid < nsub ? tid : 0);
        uint32_t sub_next = fsu[(size_t)s0 * nsub];
        for (int s = s0; s < nstages; ++s) {
            const uint32_t sub = sub_next;
            if (s + 1 < nstages) sub_next = fsu[(size_t)(s + 1) * nsub];  // in flight during this stage
            const FusedStage fs = fstages[s];  // uniform: scalar loads
            const int na = (int)__builtin_amdgcn_readfirstlane((uint32_t)fs.na);
            const int perm = (int)__builtin_amdgcn_readfirstlane((uint32_t)fs.perm);
            uint32_t ctile = fs.c0;
            for (int q = 0; q < fs.cond_count; ++q) {
                const FusedCond fc = fconds[fs.cond_begin + q];
                if ((base & fc.cmo) == fc.cvo) ctile ^= fc.xmask;
            }
            const Mat2 *w3 = wm + 4 * s;
            const int32_t *q3 = qidx + 4 * s;
            const PhaseL *sp = phl + (fs.phase_begin - ph0);
            const int np = fs.phase_count;
            if (__builtin_amdgcn_readfirstlane((uint32_t)fs.xbit)) {
                rev_fused_stage<3, true, PH, true>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub);
                lds_barrier();
                continue;
            }
            switch (na * 2 + perm) {
            case 0: rev_fused_stage<0, false, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 1: rev_fused_stage<0, true, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 2: rev_fused_stage<1, false, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 3: rev_fused_stage<1, true, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 4: rev_fused_stage<2, false, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 5: rev_fused_stage<2, true, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            case 6: rev_fused_stage<3, false, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            default: rev_fused_stage<3, true, PH>(tp, tl, fs, w3, q3, nsub, ctile, red, sp, np, phred, sub); break;
            }
            lds_barrier();
        }
        tile_out2<8, true>(tp, tl, sp, sl, base, hoff, T, c);
        __syncthreads();
    }
    // partial of entry e = coef(e) . (the slot's three sums over the four
    // waves); one thread per slot (phase)
    {
        const int W = gridDim.x;
        const double *cf = coef + (size_t)blockIdx.y * n_entries * 4;
        for (int i = tid; i < ns; i += kThreads) {
            const int qs = qidx[i];
            if (qs < 0) continue;
            const double *r = red + (size_t)qs * 12;
            const double Q0 = ((r[0] + r[1]) + r[2]) + r[3];
            const double Q1 = ((r[4] + r[5]) + r[6]) + r[7];
            const double Q2 = ((r[8] + r[9]) + r[10]) + r[11];
            for (int e = slot_off[slot0 + i]; e < slot_off[slot0 + i + 1]; ++e) {
                const int info = slot_info[e];
                if (info < 16) continue;
                const double v = cf[e * 4 + 0] * Q0 + cf[e * 4 + 1] * Q1 + cf[e * 4 + 2] * Q2;
                partials[((size_t)blockIdx.y * n_pgates + ((info >> 4) - 1)) * W + blockIdx.x] = v;
            }
        }
        for (int i = tid; PH && i < nph; i += kThreads) {
            const PhaseL &q = phl[i];
            if (q.pslot < 0) continue;
            const double *r = phred + (size_t)q.pslot * 4;
            partials[((size_t)blockIdx.y * n_pgates + q.pg) * W + blockIdx.x] = ((r[0] + r[1]) + r[2]) + r[3];
        }
    }
}

// ---------------------------------------------------------------------------
// Pauli sweep over the groups of one sweep.
//
// Expectation (lam == nullptr), paired over (b, b ^ f) with b's pivot bit 0,
// w = conj(psi[b ^ f]) psi[b], sigma_t(b) = (-1)^{z_t . b}:
//   f != 0:  2 * (Re w * sum_{real t} w_t sigma_t(b) - Im w * sum_{imag t} w_t sigma_t(b))
//   f == 0:  |psi_b|^2 * sum_t w_t sigma_t(b)
// H psi (lam != nullptr): with A = sum_real w sigma(b), B = sum_imag w sigma(b),
//   lam[b ^ f] += (A + iB) psi[b],   lam[b] += (A - iB) psi[b ^ f]
// (kappa_t = w_t or i w_t, sigma_t(b ^ f) = sigma_t(b) (-1)^{ny_t}).
// The sign from index bits outside the tile, (-1)^{z_t . base}, is folded
// into w_t per tile.
// sign flip of a double by the parity of popcount(z & b): the parity bit is
// moved to the sign position of the high word (integer ops only)
__device__ __forceinline__ double signed_by_parity(double w, uint32_t zb)
{
    const uint32_t flip = (uint32_t)__popc(zb) << 31;
    return __hiloint2double(__double2hiint(w) ^ (int)flip, __double2loint(w));
}

// Expectation of a flip group with a single term (most groups of a random
// Pauli sum): MODE 0 diagonal (sum of |psi_b|^2 sigma(b)), 1 a real phase
// (Re conj(psi[b ^ f]) psi[b]), 2 an imaginary one (-Im of the same), each
// with the term's sign sigma(b) = (-1)^{z . b}; the caller scales by the
// weight (and by 2 for the pair form).  No per-pair weight sums to clear.
template <int RP, int MODE>
__device__ __forceinline__ double single_term_sum(const double2 *tp, int npos, uint32_t pv, uint32_t f, uint32_t z)
{
    double s0 = 0.0, s1 = 0.0;
    for (int j0 = 0; j0 < npos; j0 += RP * kThreads) {
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const int j = j0 + r * kThreads + (int)threadIdx.x;
            const bool ok = j < npos;
            const uint32_t jj = ok ? (uint32_t)j : 0u;
            const uint32_t b = MODE == 0 ? jj : (((jj >> pv) << (pv + 1)) | (jj & ((1u << pv) - 1u)));
            const double2 x0 = tp[b];
            double v;
            if (MODE == 0) {
                v = fma(x0.x, x0.x, x0.y * x0.y);
            } else {
                const double2 x1 = tp[b ^ f];
                v = MODE == 1 ? fma(x1.x, x0.x, x1.y * x0.y) : fma(x1.y, x0.x, -x1.x * x0.y);
            }
            v = ok ? v : 0.0;
            if (r & 1)
                s1 += signed_by_parity(v, z & b);
            else
                s0 += signed_by_parity(v, z & b);
        }
    }
    return s0 + s1;
}

// Expectation of a flip group with many terms on a 12-bit tile, through a
// Walsh-Hadamard transform of each thread's own positions.  The thread's
// pair elements are b_r = b_0 ^ e(r), r < R (e(r) = the bits of r placed at
// tile bits 8.. with the pivot bit skipped, b_0 from the thread id), so a
// term's sign splits as sigma(b_r) = (-1)^{z . b_0} (-1)^{zr . r} with zr the
// bits of z at those places.  With v_r the pair products,
//   sum_r sigma(b_r) v_r = (-1)^{z . b_0} V[zr],  V = WHT(v),
// so after one transform (R log R additions per part) every term costs a
// lookup, a sign and an FMA instead of R sign evaluations.
template <int R, bool DIAG>
__device__ __forceinline__ double walsh_group(const double2 *tp, uint32_t pv, uint32_t f, const uint32_t *zl,
                                              const double *wl, int ib, int im, int ie)
{
    constexpr int LR = R == 16 ? 4 : (R == 8 ? 3 : (R == 4 ? 2 : (R == 2 ? 1 : 0)));
    const uint32_t tid = threadIdx.x;
    const uint32_t lowp = (1u << pv) - 1u;
    auto ins = [&](uint32_t j) { return DIAG ? j : (((j >> pv) << (pv + 1)) | (j & lowp)); };
    double vr[R], vi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t b = ins(tid + 256u * (uint32_t)r);
        const double2 x0 = tp[b];
        if (DIAG) {
            vr[r] = fma(x0.x, x0.x, x0.y * x0.y);
            vi[r] = 0.0;
        } else {
            const double2 x1 = tp[b ^ f];
            vr[r] = fma(x1.x, x0.x, x1.y * x0.y);
            vi[r] = fma(x1.y, x0.x, -x1.x * x0.y);
        }
    }
#pragma unroll
    for (int st = 0; st < LR; ++st)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & (1 << st)) continue;
            const double a = vr[r], b = vr[r | (1 << st)];
            vr[r] = a + b;
            vr[r | (1 << st)] = a - b;
            if (!DIAG) {
                const double c = vi[r], d = vi[r | (1 << st)];
                vi[r] = c + d;
                vi[r | (1 << st)] = c - d;
            }
        }
    const uint32_t b0 = ins(tid);
    double sum = 0.0;
    for (int i = ib; i < ie; ++i) {
        const uint32_t z = __builtin_amdgcn_readfirstlane(zl[i]);
        uint32_t zr = 0;  // bit q of zr = bit of z where bit q of r lands
#pragma unroll
        for (int q = 0; q < LR; ++q) {
            const uint32_t pos = DIAG ? 8u + q : (8u + q >= pv ? 9u + q : 8u + q);
            zr |= ((z >> pos) & 1u) << q;
        }
        // uniform index: a scalar branch picks the register (no per-lane selects)
        const bool re = i < im;
        double v;
        switch (zr) {
#define VQE_PICK(m)                                  \
    case m:                                          \
        if constexpr (m < R) v = re ? vr[m] : vi[m]; \
        break;
            VQE_PICK(0) VQE_PICK(1) VQE_PICK(2) VQE_PICK(3) VQE_PICK(4) VQE_PICK(5) VQE_PICK(6) VQE_PICK(7)
            VQE_PICK(8) VQE_PICK(9) VQE_PICK(10) VQE_PICK(11) VQE_PICK(12) VQE_PICK(13) VQE_PICK(14)
#undef VQE_PICK
        default:
            if constexpr (R > 15) v = re ? vr[15] : vi[15];
            break;
        }
        sum = fma(wl[i], signed_by_parity(v, z & b0), sum);
    }
    return DIAG ? sum : 2.0 * sum;
}

// RP pairs per thread at a time share each term read
template <bool HPSI, int RP>
__global__ __launch_bounds__(kThreads) void k_pauli_sweep(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout,
    const GroupDev *__restrict__ groups, int ngroups,
    const int32_t *__restrict__ toff, int n_ugroups, const TermDev *__restrict__ terms,
    int ham_div, const double2 *__restrict__ psi, double2 *__restrict__ lam, int64_t tiles,
    int first, int last, double *__restrict__ partials, int n_slots, int slot, int tcap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tp = reinterpret_cast<double2 *>(smem);
    double2 *tl = tp + (1u << k);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + ((HPSI ? 32u : 16u) << k));
    double *red = reinterpret_cast<double *>(hoff + (1u << (k - c)));
    uint64_t *zf = reinterpret_cast<uint64_t *>(red + 4);
    double *w0 = reinterpret_cast<double *>(zf + tcap);
    double *wl = w0 + tcap;
    uint32_t *zl = reinterpret_cast<uint32_t *>(wl + tcap);
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    const int inst = blockIdx.y;
    const double2 *sp = psi + (uint64_t)inst * dim;
    double2 *sl = HPSI ? lam + (uint64_t)inst * dim : nullptr;
    // ham_div 0: one Hamiltonian for every row; else rows [i*ham_div, (i+1)*ham_div) use table i
    const int32_t *to = toff + (size_t)(ham_div == 0 ? 0 : inst / ham_div) * n_ugroups * 3;
    const int T = 1 << k;
    const uint32_t lowm = (1u << c) - 1u;
    // this sweep's terms for this instance are one contiguous range
    const int tstart = to[groups[0].ugroup * 3];
    const int nt = to[groups[ngroups - 1].ugroup * 3 + 2] - tstart;
    const bool staged = nt <= tcap;
    fill_hoff(gp, k, c, hoff);
    if (staged)
        for (int i = tid; i < nt; i += kThreads) {
            const TermDev d = terms[tstart + i];
            zf[i] = d.zfull;
            zl[i] = d.zloc;
            w0[i] = d.w;
        }
    __syncthreads();
    double acc = 0.0;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base(gp, nout, t);
        tile_in<8, false>(tp, sp, base, hoff, T, c);
        if (HPSI)
            for (int j = tid; j < T; j += kThreads) tl[j] = make_double2(0.0, 0.0);
        if (staged)  // fold the sign of the bits outside the tile into the weights
            for (int i = tid; i < nt; i += kThreads)
                wl[i] = signed_by_parity(w0[i], (uint32_t)(__popcll(zf[i] & base) & 1));
        __syncthreads();
        for (int q = 0; q < ngroups; ++q) {
            const GroupDev gd = groups[q];
            const int tb = to[gd.ugroup * 3 + 0], tm = to[gd.ugroup * 3 + 1], te = to[gd.ugroup * 3 + 2];
            if (te == tb) continue;
            const bool diag = gd.floc == 0;
            const int npos = diag ? T : (T >> 1);
            const uint32_t pv = gd.pivot;
            if (!HPSI && staged && k == 12 && te - tb >= 4) {  // many terms: one transform per thread
                acc += diag ? walsh_group<16, true>(tp, pv, gd.floc, zl, wl, tb - tstart, tm - tstart, te - tstart)
                            : walsh_group<8, false>(tp, pv, gd.floc, zl, wl, tb - tstart, tm - tstart, te - tstart);
                continue;
            }
            if (!HPSI && staged && te - tb == 1) {  // a single term: no weight sums per pair
                const int i = tb - tstart;
                const uint32_t z = __builtin_amdgcn_readfirstlane(zl[i]);
                const double w = wl[i];
                double sum;
                if (diag)
                    sum = single_term_sum<RP, 0>(tp, npos, pv, gd.floc, z);
                else if (tm > tb)
                    sum = 2.0 * single_term_sum<RP, 1>(tp, npos, pv, gd.floc, z);
                else
                    sum = 2.0 * single_term_sum<RP, 2>(tp, npos, pv, gd.floc, z);
                acc = fma(w, sum, acc);
                continue;
            }
            for (int j0 = 0; j0 < npos; j0 += RP * kThreads) {
                uint32_t b[RP];
                double A[RP], B[RP];
                bool ok[RP];
#pragma unroll
                for (int r = 0; r < RP; ++r) {
                    const int j = j0 + r * kThreads + tid;
                    ok[r] = j < npos;
                    const uint32_t jj = ok[r] ? (uint32_t)j : 0u;
                    b[r] = diag ? jj : (((jj >> pv) << (pv + 1)) | (jj & ((1u << pv) - 1u)));
                    A[r] = 0.0;
                    B[r] = 0.0;
                }
                if (staged) {
                    for (int i = tb - tstart; i < tm - tstart; ++i) {
                        const uint32_t z = zl[i];
                        const double w = wl[i];
#pragma unroll
                        for (int r = 0; r < RP; ++r) A[r] += signed_by_parity(w, z & b[r]);
                    }
                    for (int i = tm - tstart; i < te - tstart; ++i) {
                        const uint32_t z = zl[i];
                        const double w = wl[i];
#pragma unroll
                        for (int r = 0; r < RP; ++r) B[r] += signed_by_parity(w, z & b[r]);
                    }
                } else {
                    for (int i = tb; i < te; ++i) {
                        const TermDev d = terms[i];
                        const double w = signed_by_parity(d.w, (uint32_t)(__popcll(d.zfull & base) & 1));
#pragma unroll
                        for (int r = 0; r < RP; ++r) {
                            const double v = signed_by_parity(w, d.zloc & b[r]);
                            if (i < tm)
                                A[r] += v;
                            else
                                B[r] += v;
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < RP; ++r) {
                    if (!ok[r]) continue;
                    if (diag) {
                        const double2 a = tp[b[r]];
                        if (HPSI)
                            tl[b[r]] = cadd(tl[b[r]], make_double2(A[r] * a.x, A[r] * a.y));
                        else
                            acc += (a.x * a.x + a.y * a.y) * A[r];
                    } else {
                        const uint32_t bf = b[r] ^ gd.floc;
                        const double2 x0 = tp[b[r]], x1 = tp[bf];
                        if (HPSI) {
                            // lam[bf] += (A + iB) x0 ; lam[b] += (A - iB) x1
                            tl[bf] = cadd(tl[bf], make_double2(A[r] * x0.x - B[r] * x0.y, A[r] * x0.y + B[r] * x0.x));
                            tl[b[r]] = cadd(tl[b[r]], make_double2(A[r] * x1.x + B[r] * x1.y, A[r] * x1.y - B[r] * x1.x));
                        } else {
                            // w = conj(x1) x0
                            const double wr = x1.x * x0.x + x1.y * x0.y;
                            const double wi = x1.x * x0.y - x1.y * x0.x;
                            acc += 2.0 * (wr * A[r] - wi * B[r]);
                        }
                    }
                }
            }
            if (HPSI) __syncthreads();  // the next group updates other threads' lam entries
        }
        if (!HPSI) __syncthreads();  // expectation: psi is read-only until the next tile
        if (HPSI) {
            // lam += the tile's H psi, all reads of a batch in flight together
            constexpr int NB = 8;
            for (int j0 = tid; j0 < T; j0 += NB * kThreads) {
                double px[NB], py[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int j = j0 + u * kThreads < T ? j0 + u * kThreads : j0;
                    px[u] = 0.0;
                    py[u] = 0.0;
                    if (!first) {
                        const double2 v = sl[base + hoff[j >> c] + (j & lowm)];
                        px[u] = v.x;
                        py[u] = v.y;
                    }
                }
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int j = j0 + u * kThreads;
                    if (j >= T) continue;
                    const double2 v = first ? tl[j] : cadd(tl[j], make_double2(px[u], py[u]));
                    sl[base + hoff[j >> c] + (j & lowm)] = v;
                    if (last) {
                        const double2 a = tp[j];
                        acc += a.x * v.x + a.y * v.y;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (!HPSI || last) {
        const double s = block_sum(acc, red);
        if (tid == 0) partials[((size_t)inst * n_slots + slot) * gridDim.x + blockIdx.x] = s;
    }
}

// A wide flip group f over the whole state: every pair (b, b ^ f) with bit
// `pivot` of b clear, b anywhere in the index space (no tile holds the
// pair).  A(b) and B(b) are the group's real- and imaginary-phase weights
// signed by (-1)^{|z & b|} over the full z masks; the expectation term is
// 2 (Re w A - Im w B) with w = conj(psi[b ^ f]) psi[b] (the same pair form
// as the tile sweeps), and H psi adds (A + iB) psi[b] to lambda[b ^ f] and
// (A - iB) psi[b ^ f] to lambda[b] (each element belongs to one pair, so no
// two threads update it) and accumulates the same energy term.
template <bool HPSI>
__global__ __launch_bounds__(kThreads) void k_pauli_wide(int n, uint64_t f, int pivot, int ug,
                                                        const int32_t *__restrict__ toff, int n_ugroups,
                                                        const TermDev *__restrict__ terms, int ham_div,
                                                        const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                                        double *__restrict__ partials, int n_slots, int slot)
{
    __shared__ double red[4];
    const int inst = blockIdx.y;
    const uint64_t dim = 1ull << n, half = dim >> 1;
    const double2 *sp = psi + (uint64_t)inst * dim;
    double2 *sl = HPSI ? lam + (uint64_t)inst * dim : nullptr;
    const int32_t *to = toff + (size_t)(ham_div == 0 ? 0 : inst / ham_div) * n_ugroups * 3;
    const int tb = to[ug * 3 + 0], tm = to[ug * 3 + 1], te = to[ug * 3 + 2];
    const uint64_t lowm = (1ull << pivot) - 1ull;
    double acc = 0.0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < half;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = ((j >> pivot) << (pivot + 1)) | (j & lowm);
        const uint64_t bf = b ^ f;
        const double2 x0 = sp[b], x1 = sp[bf];
        double A = 0.0, B = 0.0;
        for (int i = tb; i < tm; ++i) {
            const TermDev d = terms[i];
            A += signed_by_parity(d.w, (uint32_t)(__popcll(d.zfull & b) & 1));
        }
        for (int i = tm; i < te; ++i) {
            const TermDev d = terms[i];
            B += signed_by_parity(d.w, (uint32_t)(__popcll(d.zfull & b) & 1));
        }
        const double wr = x1.x * x0.x + x1.y * x0.y;
        const double wi = x1.x * x0.y - x1.y * x0.x;
        acc += 2.0 * (wr * A - wi * B);
        if (HPSI) {
            const double2 l1 = sl[bf], l0 = sl[b];
            sl[bf] = cadd(l1, make_double2(A * x0.x - B * x0.y, A * x0.y + B * x0.x));
            sl[b] = cadd(l0, make_double2(A * x1.x + B * x1.y, A * x1.y - B * x1.x));
        }
    }
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) partials[((size_t)inst * n_slots + slot) * gridDim.x + blockIdx.x] = sum;
}

// H psi of one sweep by gathering.  Every thread owns NO amplitudes
// o = tid + r * kThreads of the tile and accumulates (H psi)[o] in registers
// over the sweep's groups.  For a flip group f with pivot bit v, let
// p = o when bit v of o is 0 and p = o ^ f otherwise (the pair's element with
// the pivot bit clear, where the pair form above evaluates A and B); then
//   (H psi)[o] += (A(p) + i s B(p)) psi[o ^ f],   s = +1 if bit v of o is 1, else -1,
// and the diagonal group adds A(o) psi[o].  psi is only read from LDS, so the
// groups need no barrier between them, and lambda never passes through LDS:
// each thread reads its running lambda from HBM after the groups, adds and
// writes the sum back.  The last sweep also
// accumulates Re <psi|lambda> (the energy) over its amplitudes.
template <int NO>
__global__ __launch_bounds__(kThreads) void k_hpsi_gather(
    const TileGeom *__restrict__ gp, int n, int k, int c, int nout, const GroupDev *__restrict__ groups,
    int ngroups, const int32_t *__restrict__ toff, int n_ugroups, const TermDev *__restrict__ terms, int ham_div,
    const double2 *__restrict__ psi, double2 *__restrict__ lam, int64_t tiles, int first, int last,
    double *__restrict__ partials, int n_slots, int tcap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tp = reinterpret_cast<double2 *>(smem);
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (16u << k));
    double *red = reinterpret_cast<double *>(hoff + (1u << (k - c)));
    uint64_t *zf = reinterpret_cast<uint64_t *>(red + 4);
    double *w0 = reinterpret_cast<double *>(zf + tcap);
    double *wl = w0 + tcap;
    uint32_t *zl = reinterpret_cast<uint32_t *>(wl + tcap);
    __shared__ uint64_t obit[64];
    const int tid = threadIdx.x;
    const uint64_t dim = 1ull << n;
    const int inst = blockIdx.y;
    const double2 *sp = psi + (uint64_t)inst * dim;
    double2 *sl = lam + (uint64_t)inst * dim;
    const int32_t *to = toff + (size_t)(ham_div == 0 ? 0 : inst / ham_div) * n_ugroups * 3;
    const uint32_t lowm = (1u << c) - 1u;
    const int tstart = to[groups[0].ugroup * 3];
    const int nt = to[groups[ngroups - 1].ugroup * 3 + 2] - tstart;
    const bool staged = nt <= tcap;
    fill_hoff(gp, k, c, hoff);
    fill_obit(gp, nout, obit);
    if (staged)
        for (int i = tid; i < nt; i += kThreads) {
            const TermDev d = terms[tstart + i];
            zf[i] = d.zfull;
            zl[i] = d.zloc;
            w0[i] = d.w;
        }
    __syncthreads();
    double eacc = 0.0;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t base = tile_base_l(obit, nout, t);
        {
            double2 own[NO];
#pragma unroll
            for (int r = 0; r < NO; ++r) {
                const uint32_t o = (uint32_t)(tid + r * kThreads);
                own[r] = sp[base + hoff[o >> c] + (o & lowm)];
            }
#pragma unroll
            for (int r = 0; r < NO; ++r) tp[tid + r * kThreads] = own[r];
        }
        if (staged)  // fold the sign of the bits outside the tile into the weights
            for (int i = tid; i < nt; i += kThreads)
                wl[i] = signed_by_parity(w0[i], (uint32_t)(__popcll(zf[i] & base) & 1));
        lds_barrier();
        double2 acc[NO];
#pragma unroll
        for (int r = 0; r < NO; ++r) acc[r] = make_double2(0.0, 0.0);
        for (int q = 0; q < ngroups; ++q) {
            const GroupDev gd = groups[q];
            const int tb = to[gd.ugroup * 3 + 0], tm = to[gd.ugroup * 3 + 1], te = to[gd.ugroup * 3 + 2];
            if (te == tb) continue;
            const uint32_t f = gd.floc, pv = gd.pivot;
            if (staged && f != 0 && te - tb == 1) {
                // a single term (most flip groups of a random Pauli sum): its
                // signed weight times the partner, no weight sums
                const int i = tb - tstart;
                const uint32_t z = __builtin_amdgcn_readfirstlane(zl[i]);
                const double w = wl[i];
                const bool re = tm > tb;  // real: A = +-w; imaginary: B = +-w
#pragma unroll
                for (int r = 0; r < NO; ++r) {
                    const uint32_t o = (uint32_t)(tid + r * kThreads);
                    const uint32_t piv = (o >> pv) & 1u;
                    const double2 x = tp[o ^ f];
                    const double v = signed_by_parity(w, z & (piv ? o ^ f : o));
                    if (re) {
                        acc[r].x = fma(v, x.x, acc[r].x);
                        acc[r].y = fma(v, x.y, acc[r].y);
                    } else {
                        const double b = signed_by_parity(v, piv ^ 1u);  // -B below the pivot
                        acc[r].x = fma(-b, x.y, acc[r].x);
                        acc[r].y = fma(b, x.x, acc[r].y);
                    }
                }
                continue;
            }
            uint32_t pr[NO];
            double A[NO], B[NO];
#pragma unroll
            for (int r = 0; r < NO; ++r) {
                const uint32_t o = (uint32_t)(tid + r * kThreads);
                pr[r] = ((o >> pv) & 1u) ? o ^ f : o;
                A[r] = 0.0;
                B[r] = 0.0;
            }
            if (staged) {
                for (int i = tb - tstart; i < tm - tstart; ++i) {
                    const uint32_t z = zl[i];
                    const double w = wl[i];
#pragma unroll
                    for (int r = 0; r < NO; ++r) A[r] += signed_by_parity(w, z & pr[r]);
                }
                for (int i = tm - tstart; i < te - tstart; ++i) {
                    const uint32_t z = zl[i];
                    const double w = wl[i];
#pragma unroll
                    for (int r = 0; r < NO; ++r) B[r] += signed_by_parity(w, z & pr[r]);
                }
            } else {
                for (int i = tb; i < te; ++i) {
                    const TermDev d = terms[i];
                    const double w = signed_by_parity(d.w, (uint32_t)(__popcll(d.zfull & base) & 1));
#pragma unroll
                    for (int r = 0; r < NO; ++r) {
                        const double v = signed_by_parity(w, d.zloc & pr[r]);
                        if (i < tm)
                            A[r] += v;
                        else
                            B[r] += v;
                    }
                }
            }
            if (f == 0) {
#pragma unroll
                for (int r = 0; r < NO; ++r) {
                    const double2 x = tp[tid + r * kThreads];
                    acc[r].x = fma(A[r], x.x, acc[r].x);
                    acc[r].y = fma(A[r], x.y, acc[r].y);
                }
            } else {
#pragma unroll
                for (int r = 0; r < NO; ++r) {
                    const uint32_t o = (uint32_t)(tid + r * kThreads);
                    const double2 x = tp[o ^ f];
                    const double b = ((o >> pv) & 1u) ? B[r] : -B[r];
                    acc[r].x += A[r] * x.x - b * x.y;
                    acc[r].y += A[r] * x.y + b * x.x;
                }
            }
        }
        // lambda += the tile's H psi, all reads of the running sum in flight
        // together (read here rather than at the start of the tile: held
        // across the groups they cost registers, and occupancy, that the
        // overlap does not repay)
        uint64_t gi[NO];
        double2 run[NO];
#pragma unroll
        for (int r = 0; r < NO; ++r) {
            const uint32_t o = (uint32_t)(tid + r * kThreads);
            gi[r] = base + hoff[o >> c] + (o & lowm);
            run[r] = first ? make_double2(0.0, 0.0) : sl[gi[r]];
        }
#pragma unroll
        for (int r = 0; r < NO; ++r) {
            const double2 v = cadd(acc[r], run[r]);
            sl[gi[r]] = v;
            if (last) {
                const double2 a = tp[tid + r * kThreads];
                eacc += a.x * v.x + a.y * v.y;
            }
        }
        lds_barrier();  // every read of this tile is done before the next tile's writes
    }
    if (last) {
        const double e = block_sum(eacc, red);
        if (tid == 0) partials[(size_t)inst * n_slots * gridDim.x + blockIdx.x] = e;
    }
}

// out[inst * stride] = scale * sum_{slot, wg} partials[inst][slot][wg], fixed order
__global__ __launch_bounds__(kThreads) void k_reduce_slots(const double *__restrict__ partials,
                                                           int n, double *__restrict__ out,
                                                           int64_t stride, double scale)
{
    __shared__ double red[kThreads / 64];
    const double *p = partials + (size_t)blockIdx.x * n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += p[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * stride] = scale * s;
}

// grad[inst][p] = sum over the parametric gates using p (ascending) of
// sum_wg partials[inst][pgate][wg]
__global__ __launch_bounds__(kThreads) void k_grad_reduce(const double *__restrict__ partials,
                                                          int n_pgates, int W,
                                                          const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ idx,
                                                          int n_params, double *__restrict__ grad)
{
    __shared__ double red[kThreads / 64];
    const int p = blockIdx.x, inst = blockIdx.y;
    double s = 0.0;
    for (int e = off[p]; e < off[p + 1]; ++e) {
        const double *q = partials + ((size_t)inst * n_pgates + idx[e]) * W;
        for (int i = threadIdx.x; i < W; i += kThreads) s += q[i];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) grad[(size_t)inst * n_params + p] = s;
}

__global__ void k_adam(int64_t count, double *__restrict__ theta, double *__restrict__ m,
                       double *__restrict__ v, const double *__restrict__ g, double lr, double b1,
                       double b2, double eps, double c1, double c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double gi = g[i];
        const double mi = b1 * m[i] + (1.0 - b1) * gi;
        const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
    }
}

__global__ void k_gd(int64_t count, double *__restrict__ theta, const double *__restrict__ g,
                     double lr)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        theta[i] -= lr * g[i];
}

// One optimiser step of a loop whose launches are replayed unchanged (a
// captured graph): the step index t - 1 comes from device memory, so the
// bias corrections 1 - b^t are formed here; the first `batch` threads also
// file the step's energies into column *step of energies[batch][stride].
__global__ void k_opt_step(int opt, int64_t batch, int64_t count, double *__restrict__ theta, double *__restrict__ m,
                           double *__restrict__ v, const double *__restrict__ g, const double *__restrict__ e,
                           double *__restrict__ energies, int64_t e_stride, const int64_t *__restrict__ step,
                           double lr, double b1, double b2, double eps)
{
    const int64_t it = *step;
    const double t = (double)(it + 1);
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    const int64_t total = count > batch ? count : batch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < batch) energies[i * e_stride + it] = e[i];
        if (i >= count) continue;
        const double gi = g[i];
        if (opt == 0) {
            const double mi = b1 * m[i] + (1.0 - b1) * gi;
            const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
            m[i] = mi;
            v[i] = vi;
            theta[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
        } else {
            theta[i] -= lr * gi;
        }
    }
}

__global__ void k_step_set(int64_t *step, int64_t value, int64_t add)
{
    if (threadIdx.x == 0) *step = add ? *step + 1 : value;
}

__global__ void k_fill(double *__restrict__ p, int64_t count, double value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Eq. (3) through the Jordan-Wigner map, on the device: for each member i and
// string t, coef[i][t] = sum_k val[k] * ints[i][col[k]] over row t.
__global__ void k_family_coeffs(const int64_t *__restrict__ row_off, const int32_t *__restrict__ col,
                                const double *__restrict__ val, int64_t n_terms, const double *__restrict__ ints,
                                int64_t n_inputs, int64_t count, double *__restrict__ coef)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count * n_terms;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / n_terms, t = i - m * n_terms;
        const double *v = ints + m * n_inputs;
        double s = 0.0;
        for (int64_t k = row_off[t]; k < row_off[t + 1]; ++k) s += val[k] * v[col[k]];
        coef[i] = s;
    }
}

__global__ void k_refresh_weights(const WeightSrc *__restrict__ src, const double *__restrict__ coef,
                                  TermDev *__restrict__ terms, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        terms[i].w = src[i].sgn * coef[src[i].idx];
}

inline int grid_for(int64_t n, int block) { return (int)std::min<int64_t>((n + block - 1) / block, 1 << 20); }

template <typename K>
hipError_t ensure_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_prepare(double2 *psi, int n, int64_t batch, uint64_t ref, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const uint64_t total = dim * (uint64_t)batch;
    const int blocks = (int)std::min<uint64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, psi, dim - 1, total, ref);
    return hipGetLastError();
}

hipError_t launch_gate_mats(const GateDev *gates, int n_gates, const double *theta, int n_params,
                            int64_t batch, double2 *mats, hipStream_t s)
{
    const int64_t total = batch * n_gates;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gate_mats, dim3(grid_for(total, 128)), dim3(128), 0, s, gates, n_gates,
                       theta, n_params, batch, mats);
    return hipGetLastError();
}

static size_t fwd_lds(const TileGeom &g) { return (16u << g.k) + (8u << (g.k - g.c)); }
static size_t rev_lds(const TileGeom &g, int nparam)
{
    return (32u << g.k) + (8u << (g.k - g.c)) + 32u * (size_t)std::max(nparam, 1);
}

hipError_t launch_forward_pass(const PassPlan &pp, const TileGeom *geom_dev, const OpDesc *ops,
                               const double2 *mats, int n_gates, double2 *psi, int64_t batch,
                               int wg_max, hipStream_t s)
{
    const TileGeom &g = pp.geom;
    const int64_t tiles = 1ll << g.nout;
    const int W = pass_workgroups(tiles, wg_max);
    const size_t lds = fwd_lds(g);
    hipError_t e = ensure_lds(k_forward_pass, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_forward_pass, dim3(W, (unsigned)batch), dim3(kThreads), lds, s, geom_dev, g.n, g.k,
                       g.c, g.nout, ops + pp.op_begin, pp.op_count, mats, n_gates, psi, tiles);
    return hipGetLastError();
}

hipError_t launch_reverse_pass(const PassPlan &pp, const TileGeom *geom_dev, const OpDesc *ops,
                               const double2 *mats, int n_gates, double2 *psi, double2 *lam,
                               int64_t batch, int wg_per_inst, double *partials, int n_pgates,
                               hipStream_t s)
{
    const TileGeom &g = pp.geom;
    const int64_t tiles = 1ll << g.nout;
    const size_t lds = rev_lds(g, pp.n_param_ops);
    hipError_t e = ensure_lds(k_reverse_pass, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reverse_pass, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), lds, s, geom_dev,
                       g.n, g.k, g.c, g.nout, ops + pp.op_begin, pp.op_count, pp.n_param_ops, mats, n_gates,
                       psi, lam, tiles, partials, n_pgates);
    return hipGetLastError();
}

hipError_t launch_fuse_mats(const int32_t *slot_off, const int32_t *slot_gate, int n_slots, const double2 *mats,
                            int n_gates, int64_t batch, double2 *fused, hipStream_t s)
{
    const int64_t total = batch * n_slots;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fuse_mats, dim3(grid_for(total, 128)), dim3(128), 0, s, slot_off, slot_gate, n_slots, mats,
                       n_gates, batch, fused);
    return hipGetLastError();
}

hipError_t launch_forward_fused(const PassPlan &pp, const TileGeom *geom_dev, const FusedStage *fstages,
                                const FusedCond *fconds, const double2 *fused, int n_slots,
                                const FusedPhase *fphases, const double2 *mats, int n_gates, double2 *psi,
                                int64_t batch, int wg_max, const uint32_t *fsub, int fsub_n, hipStream_t s)
{
    const TileGeom &g = pp.geom;
    if (g.k < 8 || g.k > 12 || !fsub || fsub_n != (1 << (g.k - 4))) return hipErrorInvalidValue;
    const int64_t tiles = 1ll << g.nout;
    const int W = pass_workgroups(tiles, wg_max);
    const size_t lds = forward_fused_lds(g.k, g.c, pp.fstage_count, pp.fphase_count);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto kern = pp.fphase_count > 0 ? k_forward_fused<true> : k_forward_fused<false>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(W, (unsigned)batch), dim3(kThreads), lds, s, geom_dev, g.n, g.k, g.c,
                       g.nout, fstages + pp.fstage_begin, pp.fstage_count, fconds, fused, n_slots, fphases,
                       pp.fphase_begin, pp.fphase_count, mats, n_gates, psi, tiles,
                       fsub + (size_t)pp.fstage_begin * fsub_n);
    return hipGetLastError();
}

hipError_t launch_adjoint_coefs(const int32_t *slot_off, const int32_t *slot_gate, const int32_t *slot_info,
                                int n_slots, int n_entries, const double2 *mats, int n_gates, int64_t batch,
                                double2 *wadj, double *coef, hipStream_t s)
{
    const int64_t total = batch * n_slots;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_coefs, dim3(grid_for(total, 128)), dim3(128), 0, s, slot_off, slot_gate, slot_info,
                       n_slots, n_entries, mats, n_gates, batch, wadj, coef);
    return hipGetLastError();
}

size_t reverse_fused_lds(int k, int c, int nstages, int n_qslots, int n_phases)
{
    const size_t ns = 4 * (size_t)nstages;
    return (32u << k) + (8u << (k - c)) + ns * sizeof(Mat2) + (size_t)n_phases * (sizeof(PhaseL) + 32) +
           4 * ((ns + 1) & ~(size_t)1) + 96 * (size_t)n_qslots + 64;  // + network columns
}

size_t forward_fused_lds(int k, int c, int nstages, int n_phases)
{
    return (16u << k) + (8u << (k - c)) + (size_t)nstages * 5 * sizeof(Mat2) + (size_t)n_phases * sizeof(PhaseL) +
           64;  // + network columns
}

hipError_t launch_reverse_fused(const PassPlan &pp, const TileGeom *geom_dev, const FusedStage *fstages,
                                const FusedCond *fconds, const int32_t *slot_off, const int32_t *slot_info,
                                const int32_t *slot_q, const int32_t *phase_q, int slot0, int n_slots,
                                int n_entries, int n_qslots, const double2 *wadj,
                                const double *coef, const FusedPhase *fphases, const double2 *mats, int n_gates,
                                double2 *psi, double2 *lam, int64_t batch, int wg_per_inst, double *partials,
                                int n_pgates, const uint32_t *fsub, int fsub_n, hipStream_t s)
{
    const TileGeom &g = pp.geom;
    if (g.k < 8 || g.k > 11 || slot0 < 0 || slot0 + 4 * pp.fstage_count > n_slots) return hipErrorInvalidValue;
    if (!fsub || fsub_n != (1 << (g.k - 3))) return hipErrorInvalidValue;
    if (!slot_q || (pp.fphase_count > 0 && !phase_q)) return hipErrorInvalidValue;
    const int64_t tiles = 1ll << g.nout;
    const size_t lds = reverse_fused_lds(g.k, g.c, pp.fstage_count, n_qslots, pp.fphase_count);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto kern = pp.fphase_count > 0 ? k_reverse_fused<true> : k_reverse_fused<false>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), lds, s, geom_dev, g.n,
                       g.k, g.c, g.nout, fstages + pp.fstage_begin, pp.fstage_count, fconds, slot_off, slot_info,
                       slot_q, phase_q, n_qslots, slot0, n_slots, n_entries, wadj, coef, fphases, pp.fphase_begin, pp.fphase_count, mats,
                       n_gates, psi, lam, tiles, partials, n_pgates, fsub + (size_t)pp.fstage_begin * fsub_n);
    return hipGetLastError();
}

hipError_t launch_forward_staged(const PassPlan &pp, int stage_bits, const TileGeom *geom_dev,
                                 const StageDesc *stages, const StageOp *sops, const double2 *mats,
                                 int n_gates, double2 *psi, int64_t batch, int wg_max, hipStream_t s)
{
    const TileGeom &g = pp.geom;
    const int64_t tiles = 1ll << g.nout;
    const int W = pass_workgroups(tiles, wg_max);
    const size_t lds = fwd_lds(g) + stage_ctl_bytes(pp.stage_count, pp.op_count);
    if (stage_bits != 3 && stage_bits != 4) return hipErrorInvalidValue;
    auto kern = stage_bits == 4 ? k_forward_staged<4> : k_forward_staged<3>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(W, (unsigned)batch), dim3(kThreads), lds, s, geom_dev, g.n, g.k, g.c, g.nout,
                       stages + pp.stage_begin, pp.stage_count, pp.op_count, sops, mats, n_gates, psi, tiles);
    return hipGetLastError();
}

hipError_t launch_reverse_staged(const PassPlan &pp, int stage_bits, const TileGeom *geom_dev,
                                 const StageDesc *stages, const StageOp *sops, const double2 *mats,
                                 int n_gates, double2 *psi, double2 *lam, int64_t batch,
                                 int wg_per_inst, double *partials, int n_pgates, hipStream_t s)
{
    const TileGeom &g = pp.geom;
    const int64_t tiles = 1ll << g.nout;
    const size_t lds = rev_lds(g, pp.n_param_ops) + stage_ctl_bytes(pp.stage_count, pp.op_count);
    if (stage_bits != 3 && stage_bits != 4) return hipErrorInvalidValue;
    auto kern = stage_bits == 4 ? k_reverse_staged<4> : k_reverse_staged<3>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), lds, s, geom_dev, g.n, g.k, g.c,
                       g.nout, stages + pp.stage_begin, pp.stage_count, pp.op_count, sops, pp.n_param_ops, mats,
                       n_gates, psi, lam, tiles, partials, n_pgates);
    return hipGetLastError();
}

static constexpr size_t kLdsLimit = 160 * 1024;
static constexpr size_t kTermBytes = 28;  // zfull + w + folded w + zloc

hipError_t launch_pauli_sweep(const SweepPlan &sp, const PauliPlan &pp, int sweep_idx,
                              const double2 *psi, double2 *lam, int64_t batch, int ham_div,
                              int wg_per_inst, double *partials, int n_slots, bool write_lambda,
                              bool first, bool last, hipStream_t s)
{
    const TileGeom &g = sp.geom;
    const int64_t tiles = 1ll << g.nout;
    // tiles, hoff, the reduction slots and alignment slack; then kTermBytes per staged term
    const size_t base = ((write_lambda ? 32u : 16u) << g.k) + (8u << (g.k - g.c)) + 64 + 16;
    // stage up to tcap terms; keep two workgroups per CU when the tile allows it
    const size_t budget = base + 64 * kTermBytes <= kLdsLimit / 2 ? kLdsLimit / 2 : kLdsLimit;
    const int tcap = (int)std::min<size_t>(2048, (budget - std::min(budget, base)) / kTermBytes);
    const size_t lds = base + (size_t)tcap * kTermBytes;
    if (lds > kLdsLimit) return hipErrorInvalidValue;
    const bool big = g.k >= 11;
    void (*kern)(const TileGeom *, int, int, int, int, const GroupDev *, int, const int32_t *, int,
                 const TermDev *, int, const double2 *, double2 *, int64_t, int, int, double *, int, int, int);
    if (write_lambda)
        kern = big ? k_pauli_sweep<true, 4> : k_pauli_sweep<true, 1>;
    else  // expectation: eight pairs per thread per term read on 12-bit tiles
        kern = g.k >= 12 ? k_pauli_sweep<false, 8> : (big ? k_pauli_sweep<false, 4> : k_pauli_sweep<false, 1>);
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), lds, s,
                       reinterpret_cast<const TileGeom *>(pp.geoms.p) + sweep_idx, g.n, g.k, g.c, g.nout,
                       reinterpret_cast<const GroupDev *>(pp.groups.p) + sp.grp_begin, sp.grp_count,
                       reinterpret_cast<const int32_t *>(pp.toff.p), pp.n_ugroups,
                       reinterpret_cast<const TermDev *>(pp.terms.p), ham_div, psi,
                       write_lambda ? lam : nullptr, tiles, (int)first, (int)last, partials,
                       write_lambda ? 1 + (int)pp.wide.size() : n_slots, write_lambda ? 0 : sweep_idx, tcap);
    return hipGetLastError();
}

hipError_t launch_pauli_wide(const WideGroup &w, const PauliPlan &pp, const double2 *psi, double2 *lam,
                             int64_t batch, int ham_div, int wg_per_inst, double *partials, int n_slots, int slot,
                             hipStream_t s)
{
    if (lam)
        hipLaunchKernelGGL(k_pauli_wide<true>, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), 0, s, pp.n, w.f,
                           w.pivot, w.ugroup, reinterpret_cast<const int32_t *>(pp.toff.p), pp.n_ugroups,
                           reinterpret_cast<const TermDev *>(pp.terms.p), ham_div, psi, lam, partials, n_slots, slot);
    else
        hipLaunchKernelGGL(k_pauli_wide<false>, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), 0, s, pp.n, w.f,
                           w.pivot, w.ugroup, reinterpret_cast<const int32_t *>(pp.toff.p), pp.n_ugroups,
                           reinterpret_cast<const TermDev *>(pp.terms.p), ham_div, psi, lam, partials, n_slots, slot);
    return hipGetLastError();
}

hipError_t launch_hpsi_gather(const SweepPlan &sp, const PauliPlan &pp, int sweep_idx, const double2 *psi,
                              double2 *lam, int64_t batch, int ham_div, int wg_per_inst, double *partials,
                              bool first, bool last, hipStream_t s)
{
    const TileGeom &g = sp.geom;
    if (g.k < 8 || g.k > 11) return hipErrorInvalidValue;
    const int64_t tiles = 1ll << g.nout;
    // the psi tile, hoff, the reduction slots and alignment slack; then
    // kTermBytes per staged term, within a quarter, half or all of the LDS
    const size_t base = (16u << g.k) + (8u << (g.k - g.c)) + 64 + 16 + 512;
    size_t budget = kLdsLimit / 4;
    if (base + 64 * kTermBytes > budget) budget = kLdsLimit / 2;
    if (base + 64 * kTermBytes > budget) budget = kLdsLimit;
    const int tcap = (int)std::min<size_t>(2048, (budget - std::min(budget, base)) / kTermBytes);
    const size_t lds = base - 512 + (size_t)tcap * kTermBytes;  // obit is static LDS
    if (lds + 512 > kLdsLimit) return hipErrorInvalidValue;
    void (*kern)(const TileGeom *, int, int, int, int, const GroupDev *, int, const int32_t *, int, const TermDev *,
                 int, const double2 *, double2 *, int64_t, int, int, double *, int, int);
    switch (g.k) {
    case 8: kern = k_hpsi_gather<1>; break;
    case 9: kern = k_hpsi_gather<2>; break;
    case 10: kern = k_hpsi_gather<4>; break;
    default: kern = k_hpsi_gather<8>; break;
    }
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(wg_per_inst, (unsigned)batch), dim3(kThreads), lds, s,
                       reinterpret_cast<const TileGeom *>(pp.geoms.p) + sweep_idx, g.n, g.k, g.c, g.nout,
                       reinterpret_cast<const GroupDev *>(pp.groups.p) + sp.grp_begin, sp.grp_count,
                       reinterpret_cast<const int32_t *>(pp.toff.p), pp.n_ugroups,
                       reinterpret_cast<const TermDev *>(pp.terms.p), ham_div, psi, lam, tiles, (int)first,
                       (int)last, partials, 1 + (int)pp.wide.size(), tcap);
    return hipGetLastError();
}

hipError_t launch_reduce_slots(const double *partials, int n_slots, int wg_per_inst, int64_t batch,
                               double *out, int64_t out_stride, double scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_slots, dim3((unsigned)batch), dim3(kThreads), 0, s, partials,
                       n_slots * wg_per_inst, out, out_stride, scale);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double *partials, int n_pgates, int wg_per_inst,
                              const int32_t *pmap_off, const int32_t *pmap_idx, int n_params,
                              int64_t batch, double *grad, hipStream_t s)
{
    if (n_params == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_reduce, dim3(n_params, (unsigned)batch), dim3(kThreads), 0, s,
                       partials, n_pgates, wg_per_inst, pmap_off, pmap_idx, n_params, grad);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t count, double *theta, double *m, double *v, const double *g, int t,
                       double lr, double b1, double b2, double eps, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(count, 256)), dim3(256), 0, s, count, theta, m, v, g,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_gd(int64_t count, double *theta, const double *g, double lr, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gd, dim3(grid_for(count, 256)), dim3(256), 0, s, count, theta, g, lr);
    return hipGetLastError();
}

hipError_t launch_opt_step(int opt, int64_t batch, int32_t n_params, double *theta, double *m, double *v,
                           const double *g, const double *e, double *energies, int64_t e_stride,
                           const int64_t *step, double lr, double b1, double b2, double eps, hipStream_t s)
{
    const int64_t count = batch * n_params;
    const int64_t total = std::max(count, batch);
    hipLaunchKernelGGL(k_opt_step, dim3(grid_for(total, 256)), dim3(256), 0, s, opt, batch, count, theta, m, v, g,
                       e, energies, e_stride, step, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_step_set(int64_t *step, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, s, step, value, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_step_advance(int64_t *step, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, s, step, (int64_t)0, (int64_t)1);
    return hipGetLastError();
}

hipError_t launch_family_coeffs(const int64_t *row_off, const int32_t *col, const double *val, int64_t n_terms,
                                const double *ints, int64_t n_inputs, int64_t count, double *coef, hipStream_t s)
{
    if (count * n_terms == 0) return hipSuccess;
    hipLaunchKernelGGL(k_family_coeffs, dim3(grid_for(count * n_terms, 256)), dim3(256), 0, s, row_off, col, val,
                       n_terms, ints, n_inputs, count, coef);
    return hipGetLastError();
}

hipError_t launch_refresh_weights(const WeightSrc *src, const double *coef, TermDev *terms, int64_t n,
                                  hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_refresh_weights, dim3(grid_for(n, 256)), dim3(256), 0, s, src, coef, terms, n);
    return hipGetLastError();
}

hipError_t launch_shift_mats(const GateDev *gates, int n_gates, const double *theta, int n_params,
                             int64_t batch, const ShiftRow *rows, int rows_per_inst, double2 *mats,
                             hipStream_t s)
{
    const int64_t total = batch * rows_per_inst * n_gates;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shift_mats, dim3(grid_for(total, 128)), dim3(128), 0, s, gates, n_gates, theta, n_params,
                       batch, rows, rows_per_inst, mats);
    return hipGetLastError();
}

hipError_t launch_shift_combine(const double *erows, int rows_per_inst, const int32_t *off, const int32_t *row,
                                const double *coef, int n_params, int64_t batch, double *energy, double *grad,
                                hipStream_t s)
{
    const int64_t total = batch * (int64_t)(n_params + 1);
    hipLaunchKernelGGL(k_shift_combine, dim3(grid_for(total, 256)), dim3(256), 0, s, erows, rows_per_inst, off, row,
                       coef, n_params, batch, energy, grad);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t count, double value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

}  // namespace vqe
