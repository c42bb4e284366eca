// Context state shared by the host sources of the library (the C ABI in
// runtime.hip, the batched step, the adjoint window).
#pragma once

#include "rzpic.h"

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace rz {

constexpr double kPi = 3.141592653589793;

// External circuit of the powered electrode (device resident): electrode
// potential V, electrode charge Q, capacitor charge Q_c, and of the last
// solve the charge arrived Q_conv and the electrode charges Q_P of the
// charge solution and Q_L of the unit Laplace solution; the z = 0 tallies
// (fixed point) the last solve counted up to.
struct CircuitState {
    double V, Q, Qc, Qconv, Qp, Ql;
    unsigned long long prev[2];
};

struct CircuitArgs {
    int nr, rule;
    double hr, hz, C, Vs;
    const double *eps, *rho, *vol, *phiP, *phiL;
    const unsigned long long *tally;  // [2][3], z = 0 first
    double q[2], quantum[2];
    CircuitState *st;
};

hipError_t launch_circuit(const CircuitArgs &a, hipStream_t st);
hipError_t launch_combine(int nn, const double *phiP, const double *phiL, const CircuitState *cs,
                          double *phi, hipStream_t st);
hipError_t launch_circuit_set(CircuitState *cs, double V, double Q, double Qc, hipStream_t st);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct SpeciesState {
    bool bound = false;
    rzpic_species_view v{};
    int64_t cap = 0;
    Chunks ch{};
    int64_t nchunks_max = 0;
    // staging of the new particles of ionizations (electron species only):
    // [0] new electrons, [1] new ions, slots indexed like electron particles
    void *stage[2][9] = {};  // 9th: a_theta (global X-Y-Z push only)
    bool has_xsec = false;
    Xsec xs{};
    double nu_max = 0.0, p_null = 0.0;
    DevBuf sigma;
    // tile sort: sorted-copy staging (8 real arrays + identities), per-segment
    // tile counts/offsets, scan partials, and the window plan of the pass
    void *sort_buf[10] = {};  // 10th: a_theta (global X-Y-Z push only)
    int64_t *sort_off = nullptr, *sort_part = nullptr, *tile_pb = nullptr;
    int4 *tile_win = nullptr;
    int64_t sort_seg = 0, sort_nseg = 0;
    int tile_nb = 0;  // pass blocks the plan is made for
};

}  // namespace rz

struct rzpic_ctx {
    rzpic_config c{};
    hipStream_t st = nullptr;
    int device = 0, cus = 0;
    size_t lds_block = 0, lds_cu = 0;
    int mixed = 0;
    int pass_threads = 512;
    int tile_per_cu = 1;  // resident blocks per CU of the tiled merged pass
    int64_t parts_per_block = 8192;  // particles of capacity per pass block
    double hr = 0, hz = 0;
    int L = 0;
    int nn = 0;
    double quantum[2] = {1.0, 1.0};
    std::vector<void *> allocs;
    int ntr = 1, nt = 1, kbits = 0;  // tiles in r, tiles, bits of a tile key

    // grids
    double *phi, *rho, *chi, *er, *ez, *dens[2], *vol, *f, *eps;
    double *phi_alt;  // FP64 cycles sweep the finest level from one phi buffer into the other
    // external circuit (config.circuit_C > 0): the charge and unit Laplace
    // solutions with their partner buffers, a zero right-hand side, the state
    double *phiP = nullptr, *phiP_alt = nullptr, *phiL = nullptr, *phiL_alt = nullptr;
    double *fzero = nullptr;
    rz::CircuitState *circ = nullptr;
    void *E2;
    unsigned long long *acc[2];
    unsigned long long *slices = nullptr;
    int slice_blocks = 0;
    bool lds_ok = false;    // the whole deposit grid fits one block's LDS (slices allocated)
    bool lds_form = false;  // the fused pass uses that form (else the tiled windows)
    int lds_resident = 0;   // blocks of that form resident at once for the current thread
                            //    count (at most slice_blocks): the merged pass's block count
    rz::MgLevels mg{};
    // device scalars
    rz::Counts *cnt;
    rz::FixRec *fix;
    rz::ChildRec *crec;
    rz::CloneRec *clrec;
    unsigned long long *tally;   // [2][3]
    unsigned long long *mcstat;  // [2][1 + kMaxProc]
    unsigned long long *norm;    // [2]
    int32_t *status;
    // host-side bookkeeping
    rz::SpeciesState sp[2];
    bool children_pending[2] = {false, false};  // staged children not yet appended
    bool children_scanned = false;
    int last_cycles = 0;
    double last_relres = 0.0;
    // Tolerance-mode solves run their cycles in batches with one
    // synchronisation per batch: the finest-level solution is kept before
    // each cycle of a batch (ring_slots copies of nn doubles; 0 on meshes
    // too large for them, which check after every cycle), the residual norm
    // before the batch and after each of its cycles goes to normk, then to a
    // pinned host copy.  cyc_hint: cycles of the last solve per solution
    // buffer (phi, phi_P, phi_L, the adjoint's), the next first batch.
    static constexpr int kRingMax = 8;
    double *ring = nullptr;
    int ring_slots = 0;
    unsigned long long *normk = nullptr;       // [kRingMax + 1]
    unsigned long long *normk_host = nullptr;  // pinned, [kRingMax + 2]
    int cyc_hint[4] = {1, 1, 1, 1};
    unsigned long long *psteps;  // [2]
    // timing: per recorded step 10 events (see mark())
    bool timing = false;
    static constexpr int kEvPerStep = 10, kPool = 128;
    std::vector<hipEvent_t> evpool;
    int ev_used = 0;        // steps recorded in the pool
    double acc_ms[8] = {};  // accumulated phase times (see flush_timing)
    double acc_cycles = 0, acc_n[2] = {0, 0};
    int acc_steps = 0;
    std::vector<double> step_n0, step_n1;  // per recorded step, from the pass counts
    // graph replay of rzpic_step (rzpic_set_step_graph): the step's launches
    // are captured and replayed; one executable graph per step variant
    // (ions moving, weight split, tile sort), updated in place with each
    // step's arguments
    bool step_graph = false;
    hipGraphExec_t gexec[8] = {};
    // step pipelining (rzpic_set_step_pipeline): a directly launched step
    // also prepares the grid of step `prepared` (-1: none) in the launches
    // of its list maintenance; prep_ready tells the next solve that the
    // line tables and the first way down are in place (consumed by it)
    bool pipeline = false;
    int64_t prepared = -1;
    bool prep_ready = false;
    // a pipelined step's hole filling and appending, launched beside the
    // next step's way-down launches (or on their own before anything else
    // reads the particles: flush_tail)
    rz::ListTail tail;
};
