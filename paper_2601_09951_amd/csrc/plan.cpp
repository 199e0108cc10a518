// plan.cpp -- host-side compilers of libvqe.
//
// * Circuits: every gate of the ansatz (Eqs. 4-5 of arXiv 2601.09951 and the
//   hardware-efficient ansatz of the scaling study, Section 5.2.5) is a 2x2
//   update of amplitude pairs (b, b ^ m) selected by a bit pattern.  The
//   circuit compiler packs gates into passes: a pass holds a tile of 2^k
//   amplitudes (all index bits of the tile set S) in LDS and applies every
//   gate whose flip bits lie in S, so one HBM round trip serves many gates.
//   Gates on disjoint qubits commute, so a gate may join a pass ahead of an
//   earlier gate that is blocked, provided it touches none of the blocked
//   gates' qubits.
// * Pauli sums (Eq. 2, Section 3.2): terms are grouped by flip mask
//   f = xmask.  A sweep walks tiles over a bit set S and serves every group
//   whose flip bits lie in S; sweeps are chosen greedily to cover all groups.
#include <algorithm>
#include <cstring>
#include <map>
#include <set>
#include <sstream>

#include "internal.h"

namespace vqe {

namespace {

// bounds that keep a pass's control data plus a two-state 2^12 tile inside 160 KiB of LDS
constexpr int kMaxParamOpsPerPass = 128;
constexpr int kMaxOpsPerPass = 128;
// bit exchanges tried per sweep tile: a plan of one Hamiltonian is built once
// and serves every step of a loop; plans over a batch of request
// Hamiltonians are built per batch, so they keep the plain cover
constexpr int kSweepSwapRounds = 16;

inline int popc(uint64_t v) { return __builtin_popcountll(v); }
inline int bit_of_wire(int n, int w) { return n - 1 - w; }

// compress the bits of v at positions S (ascending) into local bits 0..|S|-1
uint32_t compress(uint64_t v, const std::vector<int> &S)
{
    uint32_t out = 0;
    for (size_t i = 0; i < S.size(); ++i)
        if ((v >> S[i]) & 1) out |= 1u << i;
    return out;
}

uint64_t mask_of(const std::vector<int> &S)
{
    uint64_t m = 0;
    for (int b : S) m |= 1ull << b;
    return m;
}

std::vector<int> bits_of(uint64_t m)
{
    std::vector<int> v;
    for (int b = 0; b < 64; ++b)
        if ((m >> b) & 1) v.push_back(b);
    return v;
}

// Fill a tile set up to exactly k bits: keep `must`, then add the lowest
// unused bits.
std::vector<int> complete_tile(uint64_t must, int n, int k)
{
    uint64_t S = must;
    for (int b = 0; b < n && popc(S) < k; ++b) S |= 1ull << b;
    return bits_of(S);
}

}  // namespace

TileGeom make_geom(int n, int k, int c, const std::vector<int> &tile_bits)
{
    TileGeom g;
    std::memset(&g, 0, sizeof(g));
    g.n = n;
    g.k = k;
    g.c = c;
    g.nout = n - k;
    for (int i = 0; i < k; ++i) g.tpos[i] = (uint8_t)tile_bits[i];
    uint64_t tm = mask_of(tile_bits);
    int j = 0;
    for (int b = 0; b < n; ++b)
        if (!((tm >> b) & 1)) g.opos[j++] = (uint8_t)b;
    return g;
}

// ---------------------------------------------------------------------------
// circuits
// ---------------------------------------------------------------------------
int build_circuit_gates(Circ *C, int64_t n_gates, const int32_t *kind, const int32_t *wires,
                        const int32_t *pidx, const double *fixed, std::string &err)
{
    const int n = C->n;
    C->gates.clear();
    C->pgate_of_gate.clear();
    int npg = 0;
    for (int64_t g = 0; g < n_gates; ++g) {
        GateHost h;
        std::memset(&h, 0, sizeof(h));
        h.kind = kind[g];
        int arity;
        bool parametric;
        switch (h.kind) {
        case VQE_GATE_RX: case VQE_GATE_RY: case VQE_GATE_RZ: arity = 1; parametric = true; break;
        case VQE_GATE_H: case VQE_GATE_X: arity = 1; parametric = false; break;
        case VQE_GATE_CNOT: case VQE_GATE_CZ: arity = 2; parametric = false; break;
        case VQE_GATE_SINGLE_EXC: arity = 2; parametric = true; break;
        case VQE_GATE_DOUBLE_EXC: arity = 4; parametric = true; break;
        default: {
            std::ostringstream os;
            os << "gate " << g << ": unknown kind " << h.kind;
            err = os.str();
            return VQE_EUNSUPPORTED;
        }
        }
        h.nw = arity;
        for (int j = 0; j < 4; ++j) {
            int w = wires[4 * g + j];
            if (j < arity) {
                if (w < 0 || w >= n) {
                    std::ostringstream os;
                    os << "gate " << g << ": wire " << w << " out of range [0, " << n << ")";
                    err = os.str();
                    return VQE_EINVAL;
                }
                for (int i = 0; i < j; ++i)
                    if (h.wires[i] == w) {
                        std::ostringstream os;
                        os << "gate " << g << ": repeated wire " << w;
                        err = os.str();
                        return VQE_EINVAL;
                    }
            }
            h.wires[j] = j < arity ? w : -1;
        }
        h.pidx = pidx ? pidx[g] : -1;
        h.fixed = fixed ? fixed[g] : 0.0;
        if (h.pidx >= C->n_params || h.pidx < -1) {
            std::ostringstream os;
            os << "gate " << g << ": parameter index " << h.pidx << " outside [-1, " << C->n_params << ")";
            err = os.str();
            return VQE_EINVAL;
        }
        if (h.pidx >= 0 && !parametric) {
            std::ostringstream os;
            os << "gate " << g << ": a fixed gate kind cannot take a parameter";
            err = os.str();
            return VQE_EINVAL;
        }
        if (h.pidx < 0 && !std::isfinite(h.fixed)) {
            err = "non-finite fixed angle";
            return VQE_EINVAL;
        }
        auto B = [&](int j) { return 1ull << bit_of_wire(n, h.wires[j]); };
        h.cls = CLS_GENERAL;
        h.gen = GEN_NONE;
        switch (h.kind) {
        case VQE_GATE_RX: h.m = B(0); h.gen = GEN_X; break;
        case VQE_GATE_RY: h.m = B(0); h.gen = GEN_Y; h.cls = CLS_REAL; break;
        case VQE_GATE_RZ: h.m = B(0); h.gen = GEN_Z; h.cls = CLS_DIAG; break;
        case VQE_GATE_H: h.m = B(0); h.cls = CLS_REAL; break;
        case VQE_GATE_X: h.m = B(0); h.cls = CLS_SWAP; break;
        case VQE_GATE_CNOT: h.m = B(1); h.cmask = h.cval = B(0); h.cls = CLS_SWAP; break;
        case VQE_GATE_CZ: h.m = B(1); h.cmask = h.cval = B(0); h.cls = CLS_DIAG; break;
        case VQE_GATE_SINGLE_EXC:  // first element |01> on (a, b)
            h.m = B(0) | B(1); h.first = B(1); h.gen = GEN_Y; h.cls = CLS_REAL; break;
        case VQE_GATE_DOUBLE_EXC:  // first element |0011> on (a, b, c, d)
            h.m = B(0) | B(1) | B(2) | B(3); h.first = B(2) | B(3); h.gen = GEN_Y; h.cls = CLS_REAL; break;
        }
        if (h.pidx < 0) h.gen = GEN_NONE;
        C->gates.push_back(h);
        C->pgate_of_gate.push_back(h.pidx >= 0 ? npg++ : -1);
    }
    C->n_pgates = npg;
    return VQE_OK;
}

// Number, within each pass, its slots and its phases that hold parametric
// gates (0, 1, ... in slot / phase order; -1 for the others): the adjoint
// kernel files each slot's three pair sums and each phase's sum under these
// indices.
static void number_param_slots(CircPlan *plan)
{
    plan->host_fslot_q.assign(plan->n_fslots(), -1);
    plan->host_fphase_q.assign(plan->host_fphases.size(), -1);
    for (const PassPlan &pp : plan->passes) {
        if (pp.fstage_count == 0) continue;
        const FusedStage &f0 = plan->host_fstages[pp.fstage_begin];
        int nq = 0;
        for (int i = 0; i < (f0.nb + 1) * pp.fstage_count; ++i) {
            const int sl = f0.slot + i;
            bool par = false;
            for (int e = plan->host_fslot_off[sl]; e < plan->host_fslot_off[sl + 1]; ++e)
                par = par || plan->host_fslot_info[e] >= 16;
            if (par) plan->host_fslot_q[sl] = nq++;
        }
        int np = 0;
        for (int i = 0; i < pp.fphase_count; ++i)
            if (plan->host_fphases[pp.fphase_begin + i].info >= 16) plan->host_fphase_q[pp.fphase_begin + i] = np++;
    }
}

static void free_plan(Context *ctx, CircPlan *p)
{
    if (p) {
        dev_free(ctx, p->ops);
        dev_free(ctx, p->geoms);
        dev_free(ctx, p->stages);
        dev_free(ctx, p->sops);
        dev_free(ctx, p->fstages);
        dev_free(ctx, p->fconds);
        dev_free(ctx, p->fslot_off);
        dev_free(ctx, p->fslot_gate);
        dev_free(ctx, p->fslot_info);
        dev_free(ctx, p->fphases);
        dev_free(ctx, p->fslot_q);
        dev_free(ctx, p->fphase_q);
        dev_free(ctx, p->fsub);
        ready_free(p->ready);
    }
}

void free_circ_plans(Context *ctx, Circ *C)
{
    for (auto *cache : {&C->fwd, &C->rev}) {
        for (auto &kv : *cache) free_plan(ctx, kv.second.get());
        cache->clear();
    }
}

// Per fused stage and sub-cube u the two LDS indices a thread needs (see
// FusedStage): the swizzled base of its sub-cube, swz(bl(u)) with bl(u) = u
// with zeros inserted at the register bits, and for stages whose store map
// moves amplitudes the swizzled image of u under that map, swz(lbl(u)) with
// lbl(u) = xor of lc[j] over the set bits j of u; packed as low | high << 16.
// The LDS swizzle is linear over xor, so every amplitude address is one of
// these xor a wave-uniform term.
static uint32_t lds_swz(uint32_t i) { return i ^ ((i >> 4) & 15u); }

static void build_fsub(CircPlan *plan, int keff)
{
    plan->fsub_n = 0;
    plan->host_fsub.clear();
    if (plan->host_fstages.empty()) return;
    const int nb = plan->host_fstages[0].nb;
    const int nsub = 1 << (keff - nb);
    plan->fsub_n = nsub;
    plan->host_fsub.resize(plan->host_fstages.size() * (size_t)nsub);
    for (size_t st = 0; st < plan->host_fstages.size(); ++st) {
        const FusedStage &fs = plan->host_fstages[st];
        for (int u = 0; u < nsub; ++u) {
            uint32_t bl = 0;  // thread bit j is tile bit cpos[j]
            for (int j = 0; j < keff - nb; ++j)
                if ((u >> j) & 1) bl |= 1u << fs.cpos[j];
            uint32_t lbl = 0;
            for (int j = 0; j < 12; ++j)
                if ((u >> j) & 1) lbl ^= fs.lc[j];
            plan->host_fsub[st * nsub + u] = lds_swz(bl) | (lds_swz(lbl) << 16);
        }
    }
}

// Fused stages of a forward pass (see FusedStage).  Accepts passes of
// uncontrolled one-qubit gates (RX, RY, RZ, H), X and CNOT (target in the
// tile, control anywhere); returns false otherwise.  The ops are walked in
// order: one-qubit gates gather per qubit until a gate meets a qubit that a
// pending CNOT / X already touched; then the gathered qubits are emitted in
// stages of four (one-qubit gates on different qubits commute) and the
// network goes to the last of them as its store map.
static bool build_fused(const Circ *C, const std::vector<int> &take, const std::vector<int> &tile, int keff,
                        int RB, CircPlan *plan, PassPlan &pp)
{
    // one sub-cube of 2^RB amplitudes per thread of a 256-thread workgroup
    if (keff < kStageMinK || keff > RB + 8) return false;
    const uint64_t tmask = mask_of(tile);
    struct Perm {
        int kind;          // 0: CNOT inside the tile, 1: X, 2: X under a control outside the tile
        int t, c;          // tile-local target, control
        uint64_t cmo, cvo;
    };
    for (int g : take) {
        const GateHost &h = C->gates[g];
        const bool one = h.kind == VQE_GATE_RX || h.kind == VQE_GATE_RY || h.kind == VQE_GATE_RZ ||
                         h.kind == VQE_GATE_H || h.kind == VQE_GATE_X;
        if (one && h.cmask == 0) continue;
        if (h.kind == VQE_GATE_CNOT && popc(h.m) == 1 && popc(h.cmask) == 1 && h.cval == h.cmask) continue;
        return false;
    }
    std::vector<std::vector<int>> oneq(keff);  // gates per tile bit, in order
    std::vector<int> order;                    // bits with gates, in order of appearance
    std::vector<Perm> perm;
    std::vector<FusedPhase> phases;            // RZ met after the network touched its qubit
    uint32_t touched = 0;
    const int st0 = (int)plan->host_fstages.size();

    auto flush = [&]() {
        if (order.empty() && perm.empty()) return;
        // the network as v -> L v ^ c0, plus conditional constants
        uint32_t col[16];
        for (int b = 0; b < 16; ++b) col[b] = b < keff ? 1u << b : 0u;
        uint32_t c0 = 0;
        std::vector<FusedCond> conds;
        auto cnot = [](uint32_t v, int c, int t) { return ((v >> c) & 1u) ? v ^ (1u << t) : v; };
        for (const Perm &q : perm) {
            if (q.kind == 0) {
                for (int b = 0; b < keff; ++b) col[b] = cnot(col[b], q.c, q.t);
                c0 = cnot(c0, q.c, q.t);
                for (FusedCond &f : conds) f.xmask = cnot(f.xmask, q.c, q.t);
            } else if (q.kind == 1) {
                c0 ^= 1u << q.t;
            } else {
                FusedCond f;
                std::memset(&f, 0, sizeof(f));
                f.cmo = q.cmo;
                f.cvo = q.cvo;
                f.xmask = 1u << q.t;
                conds.push_back(f);
            }
        }
        bool ident = c0 == 0 && conds.empty();
        for (int b = 0; b < keff; ++b) ident = ident && col[b] == (1u << b);
        // stages of up to RB gathered qubits in registers and, when the tile
        // has more than kXLane thread bits, one more exchanged into registers
        // by the row swap (thread bit kXLane); the network rides on the last
        const size_t cap = RB + (keff - RB > kXLane ? 1 : 0);
        const size_t ngroups = std::max<size_t>(1, (order.size() + cap - 1) / cap);
        for (size_t gi = 0; gi < ngroups; ++gi) {
            FusedStage fs;
            std::memset(&fs, 0, sizeof(fs));
            std::vector<int> act(order.begin() + std::min(order.size(), cap * gi),
                                 order.begin() + std::min(order.size(), cap * gi + cap));
            const int xq = act.size() > RB ? act[RB] : -1;
            if (xq >= 0) act.pop_back();
            uint32_t R = 0;
            for (int b : act) R |= 1u << b;
            std::vector<int> rb = act;
            for (int b = 0; b < keff && (int)rb.size() < RB; ++b)
                if (!((R >> b) & 1) && b != xq) {
                    R |= 1u << b;
                    rb.push_back(b);
                }
            std::vector<int> cb;
            for (int b = 0; b < keff; ++b)
                if (!((R >> b) & 1) && b != xq) cb.push_back(b);
            if (xq >= 0) cb.insert(cb.begin() + kXLane, xq);  // thread bit kXLane
            for (int i = 0; i < RB; ++i) fs.rpos[i] = (uint8_t)rb[i];
            fs.nb = RB;
            for (size_t j = 0; j < cb.size(); ++j) fs.cpos[j] = (uint8_t)cb[j];
            fs.na = (int)act.size();
            fs.xbit = xq >= 0;
            fs.slot = plan->n_fslots();
            for (int i = 0; i <= RB; ++i) {  // per register bit, then the exchanged qubit: its gates in order
                const int qb = i < RB ? (i < fs.na ? rb[i] : -1) : xq;
                if (qb >= 0)
                    for (int g : oneq[qb]) {
                        plan->host_fslot_gate.push_back(g);
                        const GateHost &h = C->gates[g];
                        plan->host_fslot_info.push_back(((C->pgate_of_gate[g] + 1) << 4) | (h.cls << 2) | h.gen);
                    }
                plan->host_fslot_off.push_back((int32_t)plan->host_fslot_gate.size());
            }
            // the tile bit of register bit j and of thread bit j as stored
            // (after the exchange when the stage has one)
            auto reg_bit = [&](int j) { return fs.xbit && j == RB - 1 ? xq : rb[j]; };
            auto thr_bit = [&](int j) { return fs.xbit && j == kXLane ? rb[RB - 1] : cb[j]; };
            const bool last = gi + 1 == ngroups;
            const bool net = last && !ident;
            fs.cond_begin = (int)plan->host_fconds.size();
            if (net || fs.xbit) {
                fs.perm = 1;
                for (int i = 0; i < (1 << RB); ++i) {
                    uint32_t v = 0;
                    for (int j = 0; j < RB; ++j)
                        if ((i >> j) & 1) v ^= net ? col[reg_bit(j)] : 1u << reg_bit(j);
                    fs.lr[i] = (uint16_t)v;
                }
                for (size_t j = 0; j < cb.size(); ++j) fs.lc[j] = (uint16_t)(net ? col[thr_bit((int)j)] : 1u << thr_bit((int)j));
                if (net) {
                    fs.c0 = (uint16_t)c0;
                    fs.cond_count = (int)conds.size();
                    for (const FusedCond &f : conds) plan->host_fconds.push_back(f);
                }
            } else {
                for (int i = 0; i < (1 << RB); ++i) {
                    uint32_t v = 0;
                    for (int j = 0; j < RB; ++j)
                        if ((i >> j) & 1) v |= 1u << rb[j];
                    fs.lr[i] = (uint16_t)v;
                }
                for (size_t j = 0; j < cb.size(); ++j) fs.lc[j] = (uint16_t)(1u << cb[j]);
            }
            plan->host_fstages.push_back(fs);
        }
        // the group's phases ride on its last stage
        FusedStage &last = plan->host_fstages.back();
        last.phase_begin = (int)plan->host_fphases.size();
        last.phase_count = (int)phases.size();
        for (const FusedPhase &f : phases) plan->host_fphases.push_back(f);
        for (int b : order) oneq[b].clear();
        order.clear();
        perm.clear();
        phases.clear();
        touched = 0;
    };

    // an RZ on touched bit t as a parity phase (only while the network has no
    // X conditioned on bits outside the tile); false: flush instead
    // A phase pays off only when it saves a flush: when the next gate of the
    // pass on tile bit t is a network gate (or there is none).  When a
    // non-diagonal one-qubit gate comes next, the group flushes there anyway
    // and the RZ is cheaper as part of that qubit's next 2x2.
    auto next_is_network = [&](size_t pos, int t) {
        for (size_t q = pos + 1; q < take.size(); ++q) {
            const GateHost &h = C->gates[take[q]];
            const uint32_t bits = compress(h.m | (h.cmask & tmask), tile);
            if (!((bits >> t) & 1u)) continue;
            return h.kind == VQE_GATE_CNOT || h.kind == VQE_GATE_X;
        }
        return true;
    };
    auto as_phase = [&](int g, int t) {
        if (C->gates[g].kind != VQE_GATE_RZ) return false;
        uint32_t col[16];
        for (int b = 0; b < 16; ++b) col[b] = b < keff ? 1u << b : 0u;
        uint32_t c0 = 0;
        auto cnot = [](uint32_t v, int c, int tt) { return ((v >> c) & 1u) ? v ^ (1u << tt) : v; };
        for (const Perm &q : perm) {
            if (q.kind == 2) return false;
            if (q.kind == 0) {
                for (int b = 0; b < keff; ++b) col[b] = cnot(col[b], q.c, q.t);
                c0 = cnot(c0, q.c, q.t);
            } else {
                c0 ^= 1u << q.t;
            }
        }
        FusedPhase f;
        std::memset(&f, 0, sizeof(f));
        for (int b = 0; b < keff; ++b)
            if ((col[b] >> t) & 1u) f.mask |= 1u << b;
        f.cbit = (c0 >> t) & 1u;
        f.gate = g;
        const GateHost &h = C->gates[g];
        f.info = ((C->pgate_of_gate[g] + 1) << 4) | (h.cls << 2) | h.gen;
        phases.push_back(f);
        return true;
    };

    for (size_t pos = 0; pos < take.size(); ++pos) {
        const int g = take[pos];
        const GateHost &h = C->gates[g];
        const int t = __builtin_ctz(compress(h.m, tile));
        if (h.kind == VQE_GATE_CNOT || h.kind == VQE_GATE_X) {
            Perm q;
            q.t = t;
            q.c = -1;
            q.cmo = q.cvo = 0;
            if (h.kind == VQE_GATE_X) {
                q.kind = 1;
            } else if (h.cmask & tmask) {
                q.kind = 0;
                q.c = __builtin_ctz(compress(h.cmask & tmask, tile));
                touched |= 1u << q.c;
            } else {
                q.kind = 2;
                q.cmo = h.cmask;
                q.cvo = h.cval;
            }
            touched |= 1u << t;
            perm.push_back(q);
            continue;
        }
        if ((touched >> t) & 1) {
            if (next_is_network(pos, t) && as_phase(g, t)) continue;
            flush();
        }
        if (oneq[t].empty()) order.push_back(t);
        oneq[t].push_back(g);
    }
    flush();
    pp.fstage_begin = st0;
    pp.fstage_count = (int)plan->host_fstages.size() - st0;
    return pp.fstage_count > 0;
}

// Split a pass's ops (tile-local, in order) into register stages of
// `nbits` bits.  An op needs its flip bits in registers; its controls may
// be anywhere (register, other tile bits or outside the tile).  An op may
// move ahead of skipped ops only if it shares no tile bit with them.
static bool build_stages(const Circ *C, const std::vector<int> &take, const std::vector<int> &tile,
                         int keff, int nbits, CircPlan *plan, PassPlan &pp)
{
    // the stage width must hold the widest gate of the pass
    for (int g : take) nbits = std::max(nbits, popc(C->gates[g].m));
    if (nbits > 4 || nbits > keff) return false;
    pp.stage_bits = nbits;
    const uint64_t tmask = mask_of(tile);
    struct Loc {
        uint32_t m, first, cin, cvin;
    };
    std::vector<Loc> loc(take.size());
    for (size_t q = 0; q < take.size(); ++q) {
        const GateHost &h = C->gates[take[q]];
        loc[q].m = compress(h.m, tile);
        loc[q].first = compress(h.first, tile);
        loc[q].cin = compress(h.cmask & tmask, tile);
        loc[q].cvin = compress(h.cval & tmask, tile);
    }
    std::vector<char> done(take.size(), 0);
    size_t remaining = take.size();
    pp.stage_begin = (int)plan->host_stages.size();
    while (remaining > 0) {
        uint32_t R = 0, blocked = 0;
        std::vector<size_t> st;
        for (size_t q = 0; q < take.size(); ++q) {
            if (done[q]) continue;
            const uint32_t touched = loc[q].m | loc[q].cin;
            if (touched & blocked) {
                blocked |= touched;
                continue;
            }
            const uint32_t need = loc[q].m & ~R;
            if (popc(R) + popc(need) <= nbits) {
                R |= need;
                st.push_back(q);
            } else {
                blocked |= touched;
            }
        }
        if (st.empty()) return false;  // cannot happen once nbits >= every gate's width
        // pad the register set to exactly nbits bits
        for (int b = 0; b < keff && popc(R) < nbits; ++b) R |= 1u << b;
        std::vector<int> rbits, cbits;
        for (int b = 0; b < keff; ++b) ((R >> b) & 1 ? rbits : cbits).push_back(b);
        StageDesc sd;
        std::memset(&sd, 0, sizeof(sd));
        sd.nbits = nbits;
        for (int i = 0; i < nbits; ++i) {
            sd.rpos[i] = (uint8_t)rbits[i];
            sd.rpack |= (uint32_t)rbits[i] << (4 * i);
        }
        for (size_t i = 0; i < cbits.size(); ++i) {
            sd.cpos[i] = (uint8_t)cbits[i];
            sd.cpack |= (uint64_t)cbits[i] << (4 * i);
        }
        sd.op_begin = (int)plan->host_sops.size();
        sd.op_count = (int)st.size();
        int nparam = 0;
        for (size_t q : st) {
            const GateHost &h = C->gates[take[q]];
            StageOp so;
            std::memset(&so, 0, sizeof(so));
            so.M = (uint8_t)compress(loc[q].m, rbits);
            const uint32_t q0 = compress(loc[q].first, rbits);
            const uint32_t hb = 1u << (31 - __builtin_clz((uint32_t)so.M));
            if (q0 & hb) {
                so.lo = (uint8_t)(q0 ^ so.M);
                so.swap = 1;
            } else {
                so.lo = (uint8_t)q0;
                so.swap = 0;
            }
            const uint32_t cin_r = loc[q].cin & R, cin_t = loc[q].cin & ~R;
            so.cmr = (uint8_t)compress(cin_r, rbits);
            so.cvr = (uint8_t)compress(loc[q].cvin & R, rbits);
            so.cmt = cin_t;
            so.cvt = loc[q].cvin & ~R;
            so.cmo = h.cmask & ~tmask;
            so.cvo = h.cval & ~tmask;
            so.gate = take[q];
            so.pgate = C->pgate_of_gate[take[q]];
            so.cls = (uint8_t)h.cls;
            so.gen = (uint8_t)h.gen;
            {
                const uint32_t hbm = 1u << (31 - __builtin_clz((uint32_t)so.M));
                for (uint32_t i = 0; i < (1u << sd.nbits); ++i)
                    if (!(i & hbm) && (i & so.M) == so.lo && (i & so.cmr) == so.cvr) so.amask |= (uint16_t)(1u << i);
            }
            if (so.pgate >= 0) ++nparam;
            plan->host_sops.push_back(so);
            done[q] = 1;
            --remaining;
        }
        sd.n_param_ops = nparam;
        plan->host_stages.push_back(sd);
    }
    pp.stage_count = (int)plan->host_stages.size() - pp.stage_begin;
    return true;
}

CircPlan *find_circ_plan(Circ *C, bool reverse, int k, int c, int *rc)
{
    const int n = C->n;
    const auto key = std::make_pair(n <= k ? n : k, n <= k ? n : std::min(c, k));
    auto &cache = reverse ? C->rev : C->fwd;
    auto it = cache.find(key);
    *rc = VQE_OK;
    if (it == cache.end()) return nullptr;
    *rc = ready_wait(C->ctx, it->second->ready);
    return *rc ? nullptr : it->second.get();
}

CircPlan *get_circ_plan(Circ *C, bool reverse, int k, int c, int *rc)
{
    const int n = C->n;
    int keff = n <= k ? n : k;
    int ceff = n <= k ? n : std::min(c, k);
    auto &cache = reverse ? C->rev : C->fwd;
    auto key = std::make_pair(keff, ceff);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *rc = ready_wait(C->ctx, it->second->ready);
        return *rc ? nullptr : it->second.get();
    }
    std::unique_ptr<CircPlan> plan(new CircPlan);
    plan->k = keff;
    plan->c = ceff;
    plan->reverse = reverse;
    plan->stage_bits = reverse ? kStageBitsRev : kStageBitsFwd;

    const int G = (int)C->gates.size();
    std::vector<int> order(G);
    for (int g = 0; g < G; ++g) order[g] = reverse ? G - 1 - g : g;
    std::vector<char> done(G, 0);
    int remaining = G;
    std::vector<OpDesc> ops;
    const uint64_t low = ceff >= 64 ? ~0ull : ((1ull << ceff) - 1);

    // One pass: walk the gates not yet applied in list order and take every
    // gate whose flip bits the tile can hold, unless a gate it must follow
    // (one touching a shared bit) was left out.  With fixed = 0 the walk
    // claims tile bits for gates first come, first served; otherwise the
    // tile's bits are `fixed` and only gates inside it are taken.
    auto walk = [&](uint64_t fixed, uint64_t &S, int &nparam) {
        std::vector<int> take;
        S = fixed ? fixed : low;
        nparam = 0;
        uint64_t blocked = 0;
        for (int oi = 0; oi < G; ++oi) {
            int g = order[oi];
            if (done[g]) continue;
            const GateHost &h = C->gates[g];
            uint64_t touched = h.m | h.cmask;
            if (touched & blocked) {
                blocked |= touched;
                continue;
            }
            uint64_t need = h.m & ~S;
            bool room = fixed ? need == 0 : popc(S) + popc(need) <= keff;
            bool param_room = (h.pidx < 0 || nparam < kMaxParamOpsPerPass) && (int)take.size() < kMaxOpsPerPass;
            if (room && param_room) {
                S |= need;
                take.push_back(g);
                if (h.pidx >= 0) ++nparam;
            } else {
                blocked |= touched;
            }
        }
        return take;
    };
    // Tile choice: the first-come walk fills the tile with the first free bits
    // it meets, which for circuits whose dependencies advance like a wavefront
    // (a CNOT ladder repeated over layers) leaves the front behind after the
    // first pass.  Every window of k - c consecutive index bits above the low
    // bits is scored too, by the gates a walk restricted to it takes; the
    // window that takes the most gates is used (ties keep the first-come
    // tile), so a pass never takes fewer gates than before.
    const int free_bits = keff - ceff;
    while (remaining > 0) {
        uint64_t S = low;
        int nparam = 0;
        std::vector<int> take = walk(0, S, nparam);
        for (int b = ceff; free_bits > 0 && b + free_bits <= n; ++b) {
            const uint64_t win = low | (((1ull << free_bits) - 1) << b);
            uint64_t Sw;
            int npw;
            std::vector<int> tw = walk(win, Sw, npw);
            if (tw.size() > take.size()) {
                take.swap(tw);
                S = Sw;
                nparam = npw;
            }
        }
        if (take.empty()) {  // cannot happen: a gate touches at most 4 bits
            *rc = VQE_EUNSUPPORTED;
            return nullptr;
        }
        std::vector<int> tile = complete_tile(S, n, keff);
        PassPlan pp;
        pp.geom = make_geom(n, keff, ceff, tile);
        pp.op_begin = (int)ops.size();
        pp.op_count = (int)take.size();
        pp.n_param_ops = nparam;
        plan->max_param_ops = std::max(plan->max_param_ops, nparam);
        const uint64_t tmask = mask_of(tile);
        for (int g : take) {
            const GateHost &h = C->gates[g];
            OpDesc o;
            std::memset(&o, 0, sizeof(o));
            o.m = compress(h.m, tile);
            uint64_t cin = h.cmask & tmask;
            uint32_t cin_loc = compress(cin, tile);
            o.fixed_bits = compress(h.first, tile) | compress(h.cval & tmask, tile);
            o.cmask_out = h.cmask & ~tmask;
            o.cval_out = h.cval & ~tmask;
            o.gate = g;
            o.pgate = C->pgate_of_gate[g];
            o.cls = h.cls;
            o.gen = h.gen;
            uint32_t fixm = o.m | cin_loc;
            o.nfix = (int8_t)popc(fixm);
            int j = 0;
            for (int b = 0; b < 32; ++b)
                if ((fixm >> b) & 1) o.fixpos[j++] = (uint8_t)b;
            ops.push_back(o);
            done[g] = 1;
            --remaining;
        }
        {
            const size_t f0 = plan->host_fstages.size(), c0 = plan->host_fconds.size();
            const size_t s0 = plan->host_fslot_off.size(), g0 = plan->host_fslot_gate.size();
            const size_t ph0 = plan->host_fphases.size();
            bool ok = build_fused(C, take, tile, keff, reverse ? 3 : 4, plan.get(), pp);
            if (ok && reverse) {
                // the adjoint kernel keeps both tiles, every slot's product and
                // three sums per slot with parametric gates in LDS
                int np = 0, nq = 0;
                for (int sl = (int)s0 - 1; sl < plan->n_fslots(); ++sl) {
                    int here = 0;
                    for (int e = plan->host_fslot_off[sl]; e < plan->host_fslot_off[sl + 1]; ++e)
                        here += plan->host_fslot_info[e] >= 16;
                    np += here;
                    nq += here > 0;
                }
                int nph = 0, npp = 0;
                for (size_t e = ph0; e < plan->host_fphases.size(); ++e) {
                    ++nph;
                    npp += plan->host_fphases[e].info >= 16;
                }
                np += npp;
                const int nst = (int)(plan->host_fstages.size() - f0);
                pp.fq_count = nq;
                ok = np == nparam && reverse_fused_lds(keff, ceff, nst, nq, nph) <= 160 * 1024;
            } else if (ok) {
                const size_t nph = plan->host_fphases.size() - ph0;
                ok = forward_fused_lds(keff, ceff, (int)(plan->host_fstages.size() - f0), (int)nph) <= 160 * 1024;
            }
            pp.fphase_begin = (int)ph0;
            pp.fphase_count = ok ? (int)(plan->host_fphases.size() - ph0) : 0;
            if (!ok) {
                plan->host_fstages.resize(f0);
                plan->host_fconds.resize(c0);
                plan->host_fslot_off.resize(s0);
                plan->host_fslot_gate.resize(g0);
                plan->host_fslot_info.resize(g0);
                plan->host_fphases.resize(ph0);
                pp.fstage_begin = (int)f0;
                pp.fstage_count = 0;
                pp.fq_count = 0;
            }
        }
        if (keff >= kStageMinK) {
            const size_t st0 = plan->host_stages.size(), so0 = plan->host_sops.size();
            if (!build_stages(C, take, tile, keff, plan->stage_bits, plan.get(), pp)) {
                // no register stages for this pass: the one-op-per-round-trip kernel runs it
                plan->host_stages.resize(st0);
                plan->host_sops.resize(so0);
                pp.stage_begin = (int)st0;
                pp.stage_count = 0;
                pp.stage_bits = 0;
            }
        }
        plan->passes.push_back(pp);
    }
    if (!ops.empty()) {
        int r = upload(C->ctx, plan->ops, ops.data(), ops.size() * sizeof(OpDesc));
        std::vector<TileGeom> geoms;
        for (const PassPlan &pp : plan->passes) geoms.push_back(pp.geom);
        if (!r) r = upload(C->ctx, plan->geoms, geoms.data(), geoms.size() * sizeof(TileGeom));
        if (!r && !plan->host_stages.empty())
            r = upload(C->ctx, plan->stages, plan->host_stages.data(), plan->host_stages.size() * sizeof(StageDesc));
        if (!r && !plan->host_sops.empty())
            r = upload(C->ctx, plan->sops, plan->host_sops.data(), plan->host_sops.size() * sizeof(StageOp));
        if (!r && !plan->host_fstages.empty())
            r = upload(C->ctx, plan->fstages, plan->host_fstages.data(),
                       plan->host_fstages.size() * sizeof(FusedStage));
        if (!r && !plan->host_fconds.empty())
            r = upload(C->ctx, plan->fconds, plan->host_fconds.data(), plan->host_fconds.size() * sizeof(FusedCond));
        if (!r && plan->n_fslots() > 0)
            r = upload(C->ctx, plan->fslot_off, plan->host_fslot_off.data(),
                       plan->host_fslot_off.size() * sizeof(int32_t));
        if (!r && !plan->host_fslot_gate.empty())
            r = upload(C->ctx, plan->fslot_gate, plan->host_fslot_gate.data(),
                       plan->host_fslot_gate.size() * sizeof(int32_t));
        if (!r && !plan->host_fslot_info.empty())
            r = upload(C->ctx, plan->fslot_info, plan->host_fslot_info.data(),
                       plan->host_fslot_info.size() * sizeof(int32_t));
        if (!r && !plan->host_fphases.empty())
            r = upload(C->ctx, plan->fphases, plan->host_fphases.data(),
                       plan->host_fphases.size() * sizeof(FusedPhase));
        if (!r && plan->n_fslots() > 0) {
            number_param_slots(plan.get());
            r = upload(C->ctx, plan->fslot_q, plan->host_fslot_q.data(), plan->host_fslot_q.size() * sizeof(int32_t));
            if (!r && !plan->host_fphase_q.empty())
                r = upload(C->ctx, plan->fphase_q, plan->host_fphase_q.data(),
                           plan->host_fphase_q.size() * sizeof(int32_t));
        }
        if (!r && !plan->host_fstages.empty()) {
            build_fsub(plan.get(), keff);
            r = upload(C->ctx, plan->fsub, plan->host_fsub.data(), plan->host_fsub.size() * sizeof(uint32_t));
        }
        if (r) {
            free_plan(C->ctx, plan.get());
            *rc = r;
            return nullptr;
        }
    }
    plan->host_ops = std::move(ops);
    ready_mark(C->ctx, plan->ready);
    CircPlan *out = plan.get();
    cache[key] = std::move(plan);
    *rc = VQE_OK;
    return out;
}

// ---------------------------------------------------------------------------
// Pauli sums
// ---------------------------------------------------------------------------
PauliPlan *get_pauli_plan(Context *ctx, int n_hams, Ham *const *hams, int n_inst, int k, int c,
                          int *rc)
{
    const int n = hams[0]->n;
    const int keff = n <= k ? n : k;
    const int ceff = n <= k ? n : std::min(c, k);
    std::ostringstream key;
    key << n << ':' << keff << ':' << ceff << ':' << n_inst;
    for (int i = 0; i < n_hams; ++i) key << ':' << hams[i]->id;
    auto it = ctx->pauli_cache.find(key.str());
    if (it != ctx->pauli_cache.end()) {
        *rc = ready_wait(ctx, it->second->ready);
        if (*rc) return nullptr;
        if (ctx->capture_plans) ctx->capture_plans->push_back(it->second.get());
        return it->second.get();
    }
    // bound the cache: plans are small, but a serving loop creates many
    if (ctx->pauli_cache.size() >= 256) {  // stream-ordered: no device synchronisation
        for (auto &kv : ctx->pauli_cache) retire_pauli_plan(ctx, kv.second.get());
        ctx->pauli_cache.clear();
    }

    std::unique_ptr<PauliPlan> plan(new PauliPlan);
    plan->n = n;
    plan->n_inst = n_inst;
    plan->k = keff;
    plan->c = ceff;

    // union of flip masks
    std::set<uint64_t> fset;
    for (int i = 0; i < n_hams; ++i)
        for (uint64_t x : hams[i]->x) fset.insert(x);
    std::vector<uint64_t> flips(fset.begin(), fset.end());  // ascending: 0 first if present
    std::map<uint64_t, int> ug;
    for (size_t g = 0; g < flips.size(); ++g) ug[flips[g]] = (int)g;
    plan->n_ugroups = (int)flips.size();

    // greedy sweep cover.  A group with more flip bits outside the low c bits
    // than a tile has free bits cannot pair inside any tile: it is a wide
    // group, evaluated by a whole-state pair sweep of its own (after the tile
    // sweeps), and the cover skips it (sweep_of = -2).
    const uint64_t low = ((1ull << ceff) - 1);
    std::vector<int> sweep_of(flips.size(), -1);
    std::vector<std::vector<int>> sweep_tiles;
    std::vector<std::vector<int>> sweep_groups;
    std::vector<int> wide_groups;
    size_t assigned = 0;
    for (size_t g = 0; g < flips.size(); ++g)
        if (popc(flips[g] & ~low) > keff - ceff) {
            sweep_of[g] = -2;
            wide_groups.push_back((int)g);
            ++assigned;
        }
    while (assigned < flips.size()) {
        uint64_t S = low;
        for (;;) {
            int best = -1, best_new = 1 << 30;
            for (size_t g = 0; g < flips.size(); ++g) {
                if (sweep_of[g] != -1) continue;
                uint64_t f = flips[g];
                int nw = popc(f & ~S);
                if (nw == 0) continue;
                if (popc(S) + nw <= keff && nw < best_new) {
                    best = (int)g;
                    best_new = nw;
                }
            }
            if (best < 0) break;
            S |= flips[best];
        }
        // Fill the tile's remaining bits with those that let the most
        // unassigned groups in, then exchange single bits (outside the low
        // ones) while that lets more groups in: fewer sweeps of the state.
        auto covered = [&](uint64_t T) {
            int cnt = 0;
            for (size_t g = 0; g < flips.size(); ++g) cnt += sweep_of[g] == -1 && (flips[g] & ~T) == 0;
            return cnt;
        };
        while (popc(S) < keff) {
            int best_b = -1, best_c = -1;
            for (int b = 0; b < n; ++b) {
                if ((S >> b) & 1) continue;
                const int cv = covered(S | (1ull << b));
                if (cv > best_c) {
                    best_c = cv;
                    best_b = b;
                }
            }
            S |= 1ull << best_b;
        }
        for (int it = 0, cur = covered(S); it < (n_hams == 1 ? kSweepSwapRounds : 0); ++it) {
            int best_c = cur;
            uint64_t best_S = S;
            for (int bo = ceff; bo < n; ++bo) {
                if (!((S >> bo) & 1)) continue;
                for (int bi = ceff; bi < n; ++bi) {
                    if ((S >> bi) & 1) continue;
                    const uint64_t T = S ^ (1ull << bo) ^ (1ull << bi);
                    const int cv = covered(T);
                    if (cv > best_c) {
                        best_c = cv;
                        best_S = T;
                    }
                }
            }
            if (best_c == cur) break;
            S = best_S;
            cur = best_c;
        }
        std::vector<int> tile = bits_of(S);
        uint64_t tmask = mask_of(tile);
        int s = (int)sweep_tiles.size();
        sweep_tiles.push_back(tile);
        sweep_groups.emplace_back();
        for (size_t g = 0; g < flips.size(); ++g) {
            if (sweep_of[g] != -1) continue;
            if ((flips[g] & ~tmask) == 0) {
                sweep_of[g] = s;
                sweep_groups[s].push_back((int)g);
                ++assigned;
            }
        }
        if (sweep_groups[s].empty()) {  // cannot happen: every group left fits the low bits plus k - c more
            *rc = VQE_EUNSUPPORTED;
            return nullptr;
        }
    }

    // renumber the union groups in sweep order, so that every sweep's terms
    // form one contiguous range per instance; the wide groups come last
    {
        std::vector<uint64_t> nf;
        std::vector<int> nsweep;
        for (size_t s = 0; s < sweep_tiles.size(); ++s)
            for (int &g : sweep_groups[s]) {
                nf.push_back(flips[g]);
                nsweep.push_back((int)s);
                g = (int)nf.size() - 1;
            }
        for (int g : wide_groups) {
            WideGroup w;
            w.f = flips[g];
            w.pivot = __builtin_ctzll(flips[g]);
            w.ugroup = (int32_t)nf.size();
            plan->wide.push_back(w);
            nf.push_back(flips[g]);
            nsweep.push_back(-2);
        }
        flips.swap(nf);
        sweep_of.assign(nsweep.begin(), nsweep.end());
    }

    std::vector<GroupDev> gdev;
    for (size_t s = 0; s < sweep_tiles.size(); ++s) {
        SweepPlan sp;
        sp.geom = make_geom(n, keff, ceff, sweep_tiles[s]);
        sp.grp_begin = (int)gdev.size();
        sp.grp_count = (int)sweep_groups[s].size();
        for (int g : sweep_groups[s]) {
            GroupDev d;
            std::memset(&d, 0, sizeof(d));
            d.floc = compress(flips[g], sweep_tiles[s]);
            d.pivot = d.floc ? (uint32_t)__builtin_ctz(d.floc) : 0u;
            d.ugroup = g;
            gdev.push_back(d);
        }
        plan->sweeps.push_back(sp);
    }

    // per-instance term tables, grouped by union group, real terms first
    const HamFamily *fam = hams[0]->fam;
    for (int i = 0; i < n_hams; ++i)
        if (hams[i]->fam != fam) {  // a plan draws device weights from one family at most
            *rc = VQE_EUNSUPPORTED;
            return nullptr;
        }
    std::vector<WeightSrc> wsrc;
    std::vector<int32_t> toff((size_t)n_inst * flips.size() * 3, 0);
    std::vector<TermDev> terms;
    for (int i = 0; i < n_inst; ++i) {
        const Ham *H = hams[n_hams == 1 ? 0 : i];
        // terms of this Hamiltonian by flip mask
        std::map<uint64_t, std::vector<size_t>> by_f;
        for (size_t t = 0; t < H->x.size(); ++t) by_f[H->x[t]].push_back(t);
        for (size_t g = 0; g < flips.size(); ++g) {
            int32_t *o = &toff[((size_t)i * flips.size() + g) * 3];
            static const std::vector<int> no_tile;  // wide groups: signs from the full z mask only
            const std::vector<int> &tile = sweep_of[g] >= 0 ? sweep_tiles[sweep_of[g]] : no_tile;
            o[0] = (int32_t)terms.size();
            auto itf = by_f.find(flips[g]);
            int cnt = 0;
            for (int pass = 0; pass < 2; ++pass) {
                if (pass == 1) o[1] = (int32_t)terms.size();
                if (itf == by_f.end()) continue;
                for (size_t t : itf->second) {
                    int ny = popc(H->x[t] & H->z[t]);
                    if ((ny & 1) != pass) continue;
                    TermDev d;
                    std::memset(&d, 0, sizeof(d));
                    d.zfull = H->z[t];
                    d.zloc = compress(H->z[t], tile);
                    // kappa = c i^ny: real part c (-1)^{ny/2} (ny even);
                    // kappa = i w with w = c (-1)^{(ny-1)/2} (ny odd)
                    int e = pass == 0 ? ny / 2 : (ny - 1) / 2;
                    d.w = (e & 1) ? -H->c[t] : H->c[t];
                    if (fam) wsrc.push_back({H->member * (int64_t)fam->x.size() + (int64_t)t, (e & 1) ? -1.0 : 1.0});
                    terms.push_back(d);
                    ++cnt;
                }
            }
            o[2] = (int32_t)terms.size();
            plan->max_terms_group = std::max(plan->max_terms_group, cnt);
        }
        if (n_hams == 1) break;
    }
    std::vector<TileGeom> sgeoms;
    for (const SweepPlan &sp : plan->sweeps) sgeoms.push_back(sp.geom);
    int r = upload(ctx, plan->groups, gdev.data(), gdev.size() * sizeof(GroupDev));
    if (!r) r = upload(ctx, plan->geoms, sgeoms.data(), sgeoms.size() * sizeof(TileGeom));
    if (!r) r = upload(ctx, plan->toff, toff.data(), toff.size() * sizeof(int32_t));
    if (!r && !terms.empty()) r = upload(ctx, plan->terms, terms.data(), terms.size() * sizeof(TermDev));
    if (!r && fam) {
        plan->fam = fam;
        r = upload(ctx, plan->wsrc, wsrc.data(), wsrc.size() * sizeof(WeightSrc));
    }
    if (r) {
        dev_free(ctx, plan->groups);
        dev_free(ctx, plan->geoms);
        dev_free(ctx, plan->wsrc);
        dev_free(ctx, plan->toff);
        dev_free(ctx, plan->terms);
        *rc = r;
        return nullptr;
    }
    plan->host_groups = std::move(gdev);
    plan->host_toff = std::move(toff);
    plan->host_terms = std::move(terms);
    ready_mark(ctx, plan->ready);
    PauliPlan *out = plan.get();
    if (ctx->capture_plans) ctx->capture_plans->push_back(out);
    ctx->pauli_cache[key.str()] = std::move(plan);
    *rc = VQE_OK;
    return out;
}

}  // namespace vqe
