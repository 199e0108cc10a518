// internal.h -- shared host/device declarations of libvqe (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vqe.h"

namespace vqe {

// ---------------------------------------------------------------------------
// Device-side descriptors (plain structs, copied to device memory or passed
// by value as kernel arguments).
// ---------------------------------------------------------------------------

constexpr int kMaxTileBits = 13;   // 2^13 complex128 = 128 KiB of LDS
constexpr int kPassWgMin = 512;    // two workgroups on each of the 256 compute units

// Workgroups per instance of a tile pass over `tiles` tiles: about four tiles
// per workgroup, so that workgroups end and their successors start at
// staggered times (two of these workgroups share a compute unit, and two
// that start together keep their LDS, arithmetic and HBM phases in step,
// which leaves each unit idle in turn), at least kPassWgMin, at most tiles
// and the cap wg_max.
inline int pass_workgroups(int64_t tiles, int wg_max)
{
    const int64_t w = tiles / 4 > kPassWgMin ? tiles / 4 : kPassWgMin;
    return (int)std::min<int64_t>(std::min<int64_t>(tiles, w), wg_max);
}
constexpr int kMaxOutBits = 40;
constexpr int kThreads = 256;      // workgroup size of the state passes

// Geometry of one tile pass: the tile holds the amplitudes whose index bits
// outside `tpos` equal the tile's base.  tpos[0..k) are ascending; the first
// c of them are 0..c-1 (contiguous runs of 2^c amplitudes).
struct TileGeom {
    int32_t n;           // qubits
    int32_t k;           // tile bits
    int32_t c;           // low contiguous bits (c <= k)
    int32_t nout;        // n - k
    uint8_t tpos[16];    // bit position of local bit i
    uint8_t opos[kMaxOutBits];  // bit position of tile-index bit i
};

// Gate classes on an amplitude pair (first, second).
// CLS_REAL: a general 2x2 whose entries are real for every angle (RY, H, the
// excitations); kernels may apply it with real arithmetic or as CLS_GENERAL.
enum : int16_t { CLS_GENERAL = 0, CLS_DIAG = 1, CLS_SWAP = 2, CLS_REAL = 3 };
// Generator classes for the adjoint gradient.
enum : int16_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3 };

// One gate in tile-local coordinates.  The active pairs are
// p0 = insert_zeros(j, fixpos) | fixed_bits, p1 = p0 ^ m, j in [0, 2^(k-nfix)),
// restricted to tiles with (base & cmask_out) == cval_out.
struct OpDesc {
    uint32_t m;          // local flip mask
    uint32_t fixed_bits; // local pattern of the first element and local controls
    uint64_t cmask_out;  // controls on index bits outside the tile
    uint64_t cval_out;
    int32_t gate;        // index in the circuit's gate list (matrix slot)
    int32_t pgate;       // index among parametric gates, -1 if none
    int16_t cls;         // CLS_*
    int16_t gen;         // GEN_*
    int8_t nfix;         // number of fixed local bits
    uint8_t fixpos[7];   // ascending local positions of the fixed bits
};
static_assert(sizeof(OpDesc) == 48, "OpDesc layout");
static_assert(sizeof(TileGeom) == 72, "TileGeom layout");

// Register stages of a pass (tiles with k >= kStageMinK).  A stage holds
// four tile bits (rpos) in registers: each thread owns 2^4 amplitudes that
// differ only in those bits and applies the stage's ops to them in
// registers; the other k - 4 tile bits (cpos) number the sub-cubes.
constexpr int kStageBitsFwd = 4;   // forward passes: 16 amplitudes per thread
constexpr int kStageBitsRev = 3;   // adjoint passes: 8 amplitudes of psi and of lambda per thread
constexpr int kStageMinK = 8;

struct StageDesc {
    uint8_t rpos[4];     // tile-local positions of the register bits (ascending)
    uint8_t cpos[12];    // tile-local positions of the sub-cube bits (ascending)
    int32_t op_begin, op_count;
    int32_t n_param_ops;
    int32_t nbits;       // register bits of this stage (rpos[0..nbits))
    uint64_t cpack;      // cpos packed 4 bits apiece (register-resident copy)
    uint32_t rpack;      // rpos packed 4 bits apiece
    uint32_t pad2;
};
static_assert(sizeof(StageDesc) == 48, "StageDesc layout");

// One op inside a stage.  Register index i (4 bits) pairs with i ^ M; the
// pair is active when (i & M) == lo, (i & cmr) == cvr, the sub-cube base
// satisfies (base_loc & cmt) == cvt and the tile base (base & cmo) == cvo.
// swap = 1: the lower register index holds the op's second element.
struct StageOp {
    uint64_t cmo, cvo;
    uint32_t cmt, cvt;
    int32_t gate, pgate;
    uint8_t M, lo, cmr, cvr;
    uint8_t swap, cls, gen, pad;
    uint16_t amask;      // bit i: register pair (i, i ^ M) passes the register predicates
    uint16_t pad2[3];
};
static_assert(sizeof(StageOp) == 48, "StageOp layout");

// Fused stages: forward passes of circuits made of one-qubit gates, X and
// CNOT.  A stage applies one fused 2x2 per active register bit (the product
// of that qubit's consecutive one-qubit gates) and then moves every amplitude
// of the tile by the affine map v -> L v ^ c of the CNOT / X network that
// follows, folded into the LDS store addresses (CNOTs cost no arithmetic).
// The register bits are rpos[0..na) (active) and rpos[na..nb) (padding).
// Adjoint plans use the same stages with three register bits: each active
// bit's gates are undone one by one (gradient term, then U^dagger on psi
// and lambda), after the network that precedes them in the reversed order
// has been applied by the previous stage's store map.
//
// A stage may also apply the chain of one more qubit, the tile bit
// cpos[4] (xbit = 1): the threads are ordered so that thread bit 4 is that
// tile bit, and after the register chains the 16-lane row swap of gfx950
// exchanges register bit nb-1 with it, so its pairs sit in registers.  The
// stage then stores through its map (perm = 1), and lr / lc describe the
// layout after the exchange: register bit nb-1 is the tile bit cpos[4], and
// thread bit 4 is rpos[nb-1].  Every stage owns nb + 1 slots (the last for
// the exchanged qubit's chain, empty without one).
struct FusedStage {
    uint8_t rpos[4];
    uint8_t cpos[12];    // the other tile bits, ascending (sub-cube index bits)
    uint16_t lr[16];     // L applied to register offset i
    uint16_t lc[12];     // L applied to sub-cube bit j (tile bit cpos[j])
    uint16_t c0;         // constant part of the map (X gates, transformed)
    uint16_t perm;       // 1 when the map is not the identity
    int32_t na;          // active register bits
    int32_t cond_begin, cond_count;  // X conditioned on index bits outside the tile
    int32_t slot;        // gate list of register bit j: slot + j
    int32_t nb;          // register bits: 4 (forward stages) or 3 (adjoint stages)
    int32_t phase_begin, phase_count;  // parity phases applied after the 2x2s, before the store
    int32_t xbit;        // 1: the chain of tile bit cpos[4] too, through the row swap
};
static_assert(sizeof(FusedStage) == 108, "FusedStage layout");
constexpr int kXLane = 4;  // the thread bit the row swap exchanges (lanes l and l ^ 16)

// An RZ met after the network had touched its qubit t: with the network so
// far as w = L v ^ c, RZ on w_t is, in the stage's own index frame v, the
// phase u00 or u11 of the gate chosen by parity(mask & v) ^ cbit (mask =
// row t of L, cbit = c_t).  It is diagonal, so it commutes with the group's
// other phases and with the one-qubit gates on qubits the network has not
// touched; the last stage of the group applies it after its 2x2s.
struct FusedPhase {
    uint32_t mask;       // tile bits whose parity selects the phase
    uint32_t cbit;
    int32_t gate;        // circuit gate (its matrix is diagonal)
    int32_t info;        // (parametric gate index + 1) << 4 | class << 2 | generator
};
static_assert(sizeof(FusedPhase) == 16, "FusedPhase layout");

struct FusedCond {
    uint64_t cmo, cvo;   // active when (tile base & cmo) == cvo
    uint32_t xmask;      // tile-local bits flipped (already transformed by the later CNOTs)
    uint32_t pad;
};
static_assert(sizeof(FusedCond) == 24, "FusedCond layout");

// Per-gate data for the matrix preparation kernel.
struct GateDev {
    int32_t kind;
    int32_t pidx;
    double fixed;
};

// A Pauli term inside a sweep: sign over the tile's outside bits comes from
// zfull, the in-tile sign from zloc; w is the real weight described in
// pauli.cpp (kappa = w for "real" terms, kappa = i*w for "imaginary" ones).
struct TermDev {
    uint64_t zfull;
    uint32_t zloc;
    uint32_t pad;
    double w;
};

// A flip group inside a sweep.
struct GroupDev {
    uint32_t floc;       // local flip mask (0 for the diagonal group)
    uint32_t pivot;      // local bit cleared to enumerate pairs (0 if floc == 0)
    int32_t ugroup;      // group index in the union ordering
    int32_t pad;
};

// ---------------------------------------------------------------------------
// Host objects behind the opaque handles.
// ---------------------------------------------------------------------------
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    int pool_cls = -1;   // >= 0: a block of the context's table pool (size class 2^pool_cls)
};

// Streams a plan's device tables were last read on, each with an event
// recorded after the reads (see note_use): the tables may be recycled once
// every event has completed, with no device-wide synchronisation.
struct StreamUse {
    hipStream_t stream;
    hipEvent_t event;
};

// Device tables uploaded during a call that enqueues work on a stream are
// copied on that stream (no host wait); `ev` is recorded there after the
// copies, and a call on another stream waits for it on the device before
// reading the tables.  Tables uploaded by calls without a stream go through
// the context's upload stream and are covered by Context::upload_ev.
struct Ready {
    hipEvent_t ev = nullptr;
    hipStream_t s = nullptr;
};

struct Context;

struct HamFamily;

struct Ham {
    Context *ctx = nullptr;
    int n = 0;
    uint64_t id = 0;
    std::vector<uint64_t> x, z;  // merged, sorted by (x, z)
    std::vector<double> c;       // host coefficients (zeros for family members)
    int64_t n_groups = 0;
    HamFamily *fam = nullptr;    // set for members whose coefficients live on the device
    int64_t member = -1;
};

// Jordan-Wigner image of Eq. (3) as a linear map integrals -> coefficients,
// with device storage for the coefficients of `capacity` members.
struct HamFamily {
    Context *ctx = nullptr;
    int n_orb = 0, n = 0;
    int64_t n_inputs = 0, capacity = 0;
    std::vector<uint64_t> x, z;
    std::vector<int64_t> row_off;
    std::vector<int32_t> col;
    std::vector<double> val;
    DevMem d_row, d_col, d_val, d_coef;  // coefficients: double [capacity][T]
};

// Source of a plan term's weight for family members: w = sgn * coef[idx].
struct WeightSrc {
    int64_t idx;
    double sgn;
};

struct GateHost {
    int kind;
    int wires[4];
    int nw;
    int pidx;
    double fixed;
    // index-bit view
    uint32_t mbits_pos[4];   // positions of flip bits
    int nm;
    uint64_t m;              // flip mask (global)
    uint64_t first;          // pattern of m-bits for the first element
    uint64_t cmask, cval;    // controls (global)
    int16_t cls, gen;
};

struct PassPlan {
    TileGeom geom;
    int op_begin = 0, op_count = 0;
    int n_param_ops = 0;     // parametric ops in this pass (reverse plans)
    int stage_begin = 0, stage_count = 0;  // register stages (k >= kStageMinK)
    int stage_bits = 0;                     // register bits of this pass's stages
    int fstage_begin = 0, fstage_count = 0; // fused stages (0: not fusable)
    int fq_count = 0;                       // adjoint fused stages: slots holding parametric gates
    int fphase_begin = 0, fphase_count = 0; // parity phases of the fused stages
};

struct CircPlan {
    int k = 0, c = 0;
    int stage_bits = 0;      // preferred register bits (a pass widens to its widest gate)
    bool reverse = false;
    std::vector<PassPlan> passes;
    DevMem ops;              // OpDesc[]
    DevMem geoms;            // TileGeom[passes] (read through a pointer by the kernels)
    DevMem stages, sops;     // StageDesc[], StageOp[]
    std::vector<OpDesc> host_ops;
    std::vector<StageDesc> host_stages;
    std::vector<StageOp> host_sops;
    int max_param_ops = 0;
    // fused stages: descriptors, conditional X, and per fused matrix (slot)
    // the CSR list of gates multiplied into it, in application order
    DevMem fstages, fconds, fslot_off, fslot_gate, fslot_info, fphases;
    std::vector<FusedStage> host_fstages;
    std::vector<FusedCond> host_fconds;
    std::vector<FusedPhase> host_fphases;
    std::vector<int32_t> host_fslot_off{0}, host_fslot_gate;
    std::vector<int32_t> host_fslot_info;  // per slot entry: (pgate + 1) << 4 | class << 2 | generator
    int n_fslots() const { return (int)host_fslot_off.size() - 1; }
    // per slot and per phase its index among the parametric slots (phases)
    // of its pass, -1 when it holds no parametric gate
    DevMem fslot_q, fphase_q;
    std::vector<int32_t> host_fslot_q, host_fphase_q;
    // per fused stage and sub-cube: swizzled sub-cube base | swizzled store-map image << 16
    DevMem fsub;
    std::vector<uint32_t> host_fsub;
    int fsub_n = 0;          // sub-cubes per stage
    Ready ready;             // where the device tables were uploaded
};

// Parameter-shift schedule of a circuit: row r of an instance evaluates the
// circuit with gate `gate` shifted by `shift` (row 0: unshifted); parameter p's
// derivative is sum_k coef[k] * E[row[k]] over its CSR entries.
struct ShiftRow {
    int32_t gate;
    int32_t pad;
    double shift;
};

struct Circ {
    Context *ctx = nullptr;
    int n = 0;
    int n_params = 0;
    int n_pgates = 0;
    std::vector<GateHost> gates;
    std::vector<int> pgate_of_gate;  // -1 or index among parametric gates
    DevMem gates_dev;                // GateDev[]
    DevMem pmap_off, pmap_idx;       // CSR param -> pgates
    std::map<std::pair<int, int>, std::unique_ptr<CircPlan>> fwd, rev;
    uint64_t id = 0;
    int shift_rows = 0;              // rows per instance of the parameter-shift schedule
    DevMem shift_tab;                // ShiftRow[shift_rows]
    DevMem shift_off, shift_row, shift_coef;  // CSR param -> (row, coefficient)
    Ready shift_ready;
};

// A flip group too wide for any tile (more flip bits outside the low c bits
// than a tile has free bits): evaluated by a whole-state pair sweep over
// b with bit `pivot` clear and its partner b ^ f.
struct WideGroup {
    uint64_t f;
    int32_t pivot;       // lowest set bit of f
    int32_t ugroup;      // union group index (after every tile sweep's groups)
};
static_assert(sizeof(WideGroup) == 16, "WideGroup layout");

// Union Pauli plan for a list of Hamiltonians on one tile geometry.
struct SweepPlan {
    TileGeom geom;
    int grp_begin = 0, grp_count = 0;
};

struct PauliPlan {
    int n = 0, n_inst = 0, k = 0, c = 0;
    int n_ugroups = 0;
    std::vector<SweepPlan> sweeps;
    std::vector<WideGroup> wide;     // whole-state pair sweeps, after the tile sweeps
    DevMem groups;   // GroupDev[total groups over sweeps]
    DevMem geoms;    // TileGeom[sweeps]
    DevMem toff;     // int32 [n_inst][n_ugroups][3] (begin_re, begin_im, end)
    DevMem terms;    // TermDev[] (per instance, grouped)
    std::vector<GroupDev> host_groups;
    std::vector<int32_t> host_toff;
    std::vector<TermDev> host_terms;
    int max_terms_group = 0;
    const HamFamily *fam = nullptr;  // weights refreshed from the family's device coefficients
    DevMem wsrc;                     // WeightSrc[terms] when fam is set
    std::vector<StreamUse> uses;     // where the tables were read (recycling is stream-ordered)
    Ready ready;                     // where the tables were uploaded
};

struct Context {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    int k_fwd = 12, k_rev = 11, c_low = 3;  // c_low 3: runs of 8 amplitudes = one 128-byte line
    int wg_max = 8192;          // cap on workgroups per instance in tile passes
    int force_generic = 0;      // route vqe_run through the per-step launches
    int no_stages = 0;          // use the one-op-per-LDS-round-trip pass kernels only
    int fuse = 1;               // forward and adjoint passes: fused stages where the plan has them
    std::string err;
    DevMem scratch;
    std::vector<StreamUse> scratch_uses;  // streams that read the scratch buffer (growth is stream-ordered)
    std::map<std::string, std::unique_ptr<PauliPlan>> pauli_cache;
    uint64_t next_id = 1;
    int cu_count = 256;
    void *noalloc_scratch = nullptr;  // this device's static array of vqe_apply_ansatz_noalloc
    // Table pool: device blocks of power-of-two size classes carved from
    // chunks that live until the context is destroyed, so freeing a table
    // never calls hipFree (which waits for the whole device).
    std::vector<std::vector<void *>> pool_free;
    std::vector<void *> pool_chunks;
    // tables dropped while kernels may still read them: recycled once every
    // event recorded after those reads has completed
    struct Retired {
        std::vector<DevMem> mem;
        std::vector<StreamUse> uses;
        std::vector<hipGraphExec_t> execs;
    };
    std::vector<Retired> retired;
    // The call in progress (set by StreamCall): uploads made inside a call
    // that enqueues work are copied on its stream, so a request never waits
    // on the host for another stream's work.
    bool in_call = false;
    hipStream_t cur_stream = nullptr;
    // Uploads made outside such a call (creating circuits and families) are
    // copied on the context's upload stream (a hardware queue of its own);
    // upload_ev follows the latest, and every call waits for it on the device
    // while it is pending.
    hipStream_t upload_stream = nullptr;
    hipEvent_t upload_ev = nullptr;
    // pinned staging for uploads: chunks reused once the copies from them completed
    struct StageChunk {
        void *p = nullptr;
        size_t bytes = 0, off = 0;
        std::vector<StreamUse> uses;
    };
    std::vector<StageChunk> stage_chunks;
    // kernel timing (vqe_ctx_set_profiling): an event pair around every
    // timed launch, on the launch's own stream, folded into totals when read
    int profile = 0;
    struct ProfRec {
        const char *name;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_events;
    struct ProfAcc {
        int64_t launches = 0;
        double ms = 0.0, bytes = 0.0;
    };
    std::map<std::string, ProfAcc> prof_acc;

    // Launch graphs (vqe_ctx_set_graphs): a launch sequence seen a second
    // time with identical arguments is captured into a hipGraph and replayed
    // from then on.  Arguments that change between launches of one sequence
    // (the optimiser step) live in device memory.  An entry is dropped when a
    // Pauli plan it reads is retired (plan_epoch) or its circuit destroyed.
    int graphs = 0;  // off by default: measured replays were no faster than eager launches here
    uint64_t plan_epoch = 0;
    hipStream_t capture_stream = nullptr;
    std::vector<PauliPlan *> *capture_plans = nullptr;  // Pauli plans read by the sequence being captured
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        bool failed = false;             // capture failed once: stays eager
        uint64_t epoch = 0;
        uint64_t circ_id = 0;
        std::vector<PauliPlan *> plans;
        std::vector<StreamUse> uses;     // streams the graph was launched on
    };
    std::map<std::string, GraphEntry> graph_cache;
    int64_t graph_launches = 0, graph_captures = 0;

    // Autotuned execution choices (vqe_autotune) per (circuit, batch, mode).
    struct Tuned {
        int k_fwd = 12, k_rev = 11, c_low = 3, wg_max = 8192;
        int64_t batch_tile = 0;          // instances per launch sequence (0: the whole batch)
    };
    std::map<std::string, Tuned> tuned;
    const Tuned *tune_override = nullptr;  // set while the tuner times a candidate
};

// Applies the tuned tiles of (circ, batch, mode) to the context for one call
// (calls on a context are single-threaded) and restores the defaults after.
struct TileScope {
    Context *ctx;
    int kf, kr, cl, wm;
    int64_t bt = 0;  // batch tile of the call (0: whole batch)
    TileScope(Context *c, const Circ *C, int64_t batch, int mode);
    ~TileScope();
};

// Times the launches enqueued during its lifetime on stream s under `name`
// (no-op unless profiling is on, or while s is being captured); `bytes` is
// the algorithmic HBM traffic of those launches.
struct ProfScope {
    Context *ctx;
    const char *name;
    hipStream_t s;
    double bytes;
    hipEvent_t e0 = nullptr;
    ProfScope(Context *c, const char *nm, hipStream_t st, double b);
    ~ProfScope();
};

// ---------------------------------------------------------------------------
// helpers implemented in api.cpp
// ---------------------------------------------------------------------------
int set_err(Context *ctx, int code, const std::string &msg);
int dev_alloc(Context *ctx, DevMem &m, size_t bytes);
void dev_free(Context *ctx, DevMem &m);
int upload(Context *ctx, DevMem &m, const void *src, size_t bytes);
int hip_check(Context *ctx, hipError_t e, const char *what);
int scratch_get(Context *ctx, size_t bytes, void **p);
// Held by every entry point that enqueues work on `s` (see Context::in_call);
// rc is the status of waiting for pending uploads.
struct StreamCall {
    Context *ctx;
    bool prev_in;
    hipStream_t prev;
    int rc = 0;
    StreamCall(Context *c, hipStream_t s);
    ~StreamCall();
};
// after a set of tables was uploaded / before reading them on ctx->cur_stream
void ready_mark(Context *ctx, Ready &r);
int ready_wait(Context *ctx, Ready &r);
void ready_free(Ready &r);
// a stream on a hardware queue of its own (all compute units, default priority)
int dedicated_stream(Context *ctx, hipStream_t *out);
// record on `s` that plan tables were read there (no-op while `s` is captured)
int note_use(Context *ctx, std::vector<StreamUse> &uses, hipStream_t s);
// drop device tables that queued kernels may still read (stream-ordered)
void retire(Context *ctx, std::vector<DevMem> mem, std::vector<StreamUse> uses);
void retire_pauli_plan(Context *ctx, PauliPlan *p);
// drop the graphs of a circuit (circ_id != 0) or every graph (circ_id == 0)
void drop_graphs(Context *ctx, uint64_t circ_id);
void poll_retired(Context *ctx, bool wait);

// jw.cpp
int jordan_wigner(int n_orb, const double *h1, const double *h2, double e_core,
                  std::vector<uint64_t> &x, std::vector<uint64_t> &z, std::vector<double> &c,
                  std::string &err);
void merge_terms(std::vector<uint64_t> &x, std::vector<uint64_t> &z, std::vector<double> &c,
                 double drop);
int jordan_wigner_linear(int n_orb, std::vector<uint64_t> &xo, std::vector<uint64_t> &zo,
                         std::vector<int64_t> &row_off, std::vector<int32_t> &col,
                         std::vector<double> &val, std::string &err);

// plan.cpp
int build_circuit_gates(Circ *C, int64_t n_gates, const int32_t *kind, const int32_t *wires,
                        const int32_t *pidx, const double *fixed, std::string &err);
CircPlan *get_circ_plan(Circ *C, bool reverse, int k, int c, int *rc);
void free_circ_plans(Context *ctx, Circ *C);  // immediate: the caller has synchronised
CircPlan *find_circ_plan(Circ *C, bool reverse, int k, int c, int *rc);  // cached plan or nullptr; never builds
PauliPlan *get_pauli_plan(Context *ctx, int n_hams, Ham *const *hams, int n_inst, int k, int c,
                          int *rc);
TileGeom make_geom(int n, int k, int c, const std::vector<int> &tile_bits);

// kernels.hip -- launchers (return hipError_t of the launch)
hipError_t launch_prepare(double2 *psi, int n, int64_t batch, uint64_t ref, hipStream_t s);
hipError_t launch_gate_mats(const GateDev *gates, int n_gates, const double *theta,
                            int n_params, int64_t batch, double2 *mats, hipStream_t s);
hipError_t launch_forward_pass(const PassPlan &pp, const TileGeom *geom_dev, const OpDesc *ops,
                               const double2 *mats, int n_gates, double2 *psi, int64_t batch,
                               int wg_max, hipStream_t s);
hipError_t launch_fuse_mats(const int32_t *slot_off, const int32_t *slot_gate, int n_slots, const double2 *mats,
                            int n_gates, int64_t batch, double2 *fused, hipStream_t s);
hipError_t launch_adjoint_coefs(const int32_t *slot_off, const int32_t *slot_gate, const int32_t *slot_info,
                                int n_slots, int n_entries, const double2 *mats, int n_gates, int64_t batch,
                                double2 *wadj, double *coef, hipStream_t s);
size_t reverse_fused_lds(int k, int c, int nstages, int n_qslots, int n_phases);
size_t forward_fused_lds(int k, int c, int nstages, int n_phases);
hipError_t launch_reverse_fused(const PassPlan &pp, const TileGeom *geom_dev, const FusedStage *fstages,
                                const FusedCond *fconds, const int32_t *slot_off, const int32_t *slot_info,
                                const int32_t *slot_q, const int32_t *phase_q, int slot0, int n_slots,
                                int n_entries, int n_qslots, const double2 *wadj,
                                const double *coef, const FusedPhase *fphases, const double2 *mats, int n_gates,
                                double2 *psi, double2 *lam, int64_t batch, int wg_per_inst, double *partials,
                                int n_pgates, const uint32_t *fsub, int fsub_n, hipStream_t s);
hipError_t launch_forward_fused(const PassPlan &pp, const TileGeom *geom_dev, const FusedStage *fstages,
                                const FusedCond *fconds, const double2 *fused, int n_slots,
                                const FusedPhase *fphases, const double2 *mats, int n_gates, double2 *psi,
                                int64_t batch, int wg_max, const uint32_t *fsub, int fsub_n, hipStream_t s);
hipError_t launch_forward_staged(const PassPlan &pp, int stage_bits, const TileGeom *geom_dev,
                                 const StageDesc *stages, const StageOp *sops, const double2 *mats,
                                 int n_gates, double2 *psi, int64_t batch, int wg_max, hipStream_t s);
hipError_t launch_reverse_staged(const PassPlan &pp, int stage_bits, const TileGeom *geom_dev,
                                 const StageDesc *stages, const StageOp *sops, const double2 *mats,
                                 int n_gates, double2 *psi, double2 *lam, int64_t batch,
                                 int wg_per_inst, double *partials, int n_pgates, hipStream_t s);
hipError_t launch_reverse_pass(const PassPlan &pp, const TileGeom *geom_dev, const OpDesc *ops,
                               const double2 *mats,
                               int n_gates, double2 *psi, double2 *lam, int64_t batch,
                               int wg_per_inst, double *partials, int n_pgates,
                               hipStream_t s);
hipError_t launch_pauli_sweep(const SweepPlan &sp, const PauliPlan &pp, int sweep_idx,
                              const double2 *psi, double2 *lam, int64_t batch,
                              int ham_div, int wg_per_inst, double *partials,
                              int n_slots, bool write_lambda, bool first, bool last,
                              hipStream_t s);
// a wide group's whole-state pair sweep: lam NULL = expectation into slot
// `slot` of partials [batch][n_slots][wg]; else H psi added into lam and its
// energy term into that slot
hipError_t launch_pauli_wide(const WideGroup &w, const PauliPlan &pp, const double2 *psi, double2 *lam,
                             int64_t batch, int ham_div, int wg_per_inst, double *partials, int n_slots, int slot,
                             hipStream_t s);
hipError_t launch_hpsi_gather(const SweepPlan &sp, const PauliPlan &pp, int sweep_idx, const double2 *psi,
                              double2 *lam, int64_t batch, int ham_div, int wg_per_inst, double *partials,
                              bool first, bool last, hipStream_t s);
hipError_t launch_reduce_slots(const double *partials, int n_slots, int wg_per_inst,
                               int64_t batch, double *out, int64_t out_stride, double scale,
                               hipStream_t s);
hipError_t launch_grad_reduce(const double *partials, int n_pgates, int wg_per_inst,
                              const int32_t *pmap_off, const int32_t *pmap_idx, int n_params,
                              int64_t batch, double *grad, hipStream_t s);
hipError_t launch_adam(int64_t count, double *theta, double *m, double *v, const double *g,
                       int t, double lr, double b1, double b2, double eps, hipStream_t s);
hipError_t launch_gd(int64_t count, double *theta, const double *g, double lr, hipStream_t s);
// one optimiser step of a replayable loop: the step index lives in *step
// (read, not advanced); energies[b * stride + *step] = e[b] for b < batch
hipError_t launch_opt_step(int opt, int64_t batch, int32_t n_params, double *theta, double *m, double *v,
                           const double *g, const double *e, double *energies, int64_t e_stride,
                           const int64_t *step, double lr, double b1, double b2, double eps, hipStream_t s);
hipError_t launch_step_set(int64_t *step, int64_t value, hipStream_t s);   // *step = value
hipError_t launch_step_advance(int64_t *step, hipStream_t s);             // *step += 1
hipError_t launch_fill(double *p, int64_t count, double value, hipStream_t s);
hipError_t launch_shift_mats(const GateDev *gates, int n_gates, const double *theta, int n_params,
                             int64_t batch, const ShiftRow *rows, int rows_per_inst, double2 *mats,
                             hipStream_t s);
hipError_t launch_shift_combine(const double *erows, int rows_per_inst, const int32_t *off,
                                const int32_t *row, const double *coef, int n_params, int64_t batch,
                                double *energy, double *grad, hipStream_t s);
hipError_t launch_family_coeffs(const int64_t *row_off, const int32_t *col, const double *val, int64_t n_terms,
                                const double *ints, int64_t n_inputs, int64_t count, double *coef,
                                hipStream_t s);
hipError_t launch_refresh_weights(const WeightSrc *src, const double *coef, TermDev *terms, int64_t n,
                                  hipStream_t s);

// small-state persistent loop (kernels_small.hip)
struct SmallRunArgs {
    int n, n_gates, n_params, iters, opt, n_inst;
    uint64_t ref;
    double lr, b1, b2, eps;
    const GateDev *gates;          // [n_gates]
    const OpDesc *ops;             // [n_gates] (single-tile forward plan, gate order)
    const GroupDev *groups;        // union groups (single sweep)
    int n_groups;
    const int32_t *toff;           // [n_inst or 1][n_groups][3]
    const TermDev *terms;
    int shared_ham;
    double *theta;                 // [B][P]
    double *energies;              // [B][iters+1]
    double2 *hist;                 // [B][n_gates + 1][slots][64][2] pair values after each gate (fast loop;
                                   // a real state packs real values at the same indices)
};
hipError_t launch_small_run(const SmallRunArgs &a, const OpDesc *rops, const int32_t *pmap_off,
                            const int32_t *pmap_idx, int n_pgates, int mode, int max_inst_terms, int max_pairs,
                            int64_t batch, hipStream_t s);
// real_gates: every gate matrix is real for every angle (no RX, RZ), so with a
// real Hamiltonian the state stays real and the loop runs on real amplitudes
int small_run_plan(int n, int n_gates, int n_params, int n_pgates, int n_groups, int max_inst_terms,
                   int has_imag, int real_gates, int max_pairs, int *mode_out, size_t *lds_out);
// name of the persistent kernel variant that launch_small_run runs (profiling records it)
const char *small_run_variant(const SmallRunArgs &a, int mode, int max_pairs);
size_t small_fast_hist_bytes(int n, int n_gates);  // per instance
}  // namespace vqe

struct vqe_ctx : vqe::Context {};
struct vqe_ham : vqe::Ham {};
struct vqe_circ : vqe::Circ {};
struct vqe_hfam : vqe::HamFamily {};
