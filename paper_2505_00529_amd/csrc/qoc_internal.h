// Internal declarations shared by the kernel and API translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace qoc {

constexpr int kMaxN = 288;       // largest supported system dimension (complex 144 embedded)
constexpr int kBatchMaxN = 128;  // largest dimension of a problem in a batch
constexpr int kMaxP = 4096;      // largest supported parameter count
constexpr int kThreads = 256;    // threads per workgroup of every kernel
constexpr int kMaxPg = 32;       // tangent / second-adjoint columns carried per workgroup

// Longest chain of warm-started eigendecompositions (an eigen chunk).  Along a chain, the warm
// start diag(lambda_{j-1}) + (f_j - f_{j-1}) Mt_{j-1} leaves out each step's rounding residue
// and the rotated eigenvector matrix loses orthogonality by unbiased rounding, both growing with
// the chain (about 4e-15 relative per step in the backward error ||V diag(l) V^T - H_j|| at
// n = 36).  Chunks therefore restart cold at least every 32 steps.
constexpr int kMaxWarmChain = 32;

// Pad n to an even count of Jacobi "players" (a dummy index when n is odd).
inline int pad_even(int n) { return (n + 1) & ~1; }

// Device status word bits.
constexpr int kStatusNoConv = 1;

// Pointers into one evaluation workspace; every per-theta array is laid out
// [theta][step][...] with theta-major strides given by nt and n.
struct Work {
  int n = 0, np = 0, nt = 0, P = 0, nb = 0;
  int nchunks = 0, chunk = 0;
  // Step range of the current launches and layout of the eigen-data arrays (lam, mt, sm, ov):
  // [nb][eig_stride] indexed by j - seg_begin.  Without checkpointing seg_begin = 0,
  // seg_len = eig_stride = nt; with checkpointing they describe one segment.
  int seg_begin = 0, seg_len = 0, eig_stride = 0;
  // Checkpointed evaluation: O across segment boundaries, the previous segment's last V,
  // the initial-state override, and the backward carry.
  double* obound = nullptr;     // [nb][nseg][n][n]  O_{j0-1} at the start of segment s (s >= 1)
  double* vsave = nullptr;      // [nb][n][n]        last V of the previous segment
  double2* bcarry = nullptr;    // [nb][n][2]        backward state carried between segments
  double2* bcarry2 = nullptr;   // [nb][n][2]        (ping-pong partner)
  double2* xf2 = nullptr;       // [nb][n][1+P]      forward carry ping-pong partner of xf
  int nseg = 1;
  // per-launch wiring of the sweeps (set by the caller before each launch)
  const double* o_in = nullptr;     // [nb][n][n] O_{seg_begin-1}
  const double2* x_in = nullptr;    // forward carry in
  double2* x_out = nullptr;         // forward carry out (xf for the last range)
  const double2* b_in = nullptr;    // backward state in (binit for the last range)
  double2* b_out = nullptr;         // backward state out
  const double* v_last_step = nullptr;  // [nb] x n x n at stride v_last_stride: V_{J-1}
  size_t v_last_stride = 0;
  double* f = nullptr;        // [nb][nt]          control samples f_j
  double* u = nullptr;        // [nb][nt]          u = B v (HVP forcing)
  double* lam = nullptr;      // [nb][nt][n]       eigenvalues of H_j
  double* mt = nullptr;       // [nb][nt][n][n]    Mt_j = V_j^T M V_j
  double* sm = nullptr;       // [nb][nt][n][n]    S_j = sinc(dt (l_p - l_q)/2) o Mt_j
  double* ov = nullptr;       // [nb][nt][n][n]    O_j = V_{j+1}^T V_j   (j < nt-1)
  double* vfirst = nullptr;   // [nb][nchunks][n][n]  V at the first step of each chunk
  double* vlast = nullptr;    // [nb][nchunks][n][n]  V at the last step of each chunk
                              // (chunk indices are local to the launch's step range)
  double* gscratch = nullptr; // eigen-kernel matrices when they do not fit in LDS
  double2* at = nullptr;      // [nb][nt][n]  state a_j in basis j
  double2* yt = nullptr;      // [nb][nt][n]  y_j = U'_j a_j in basis j
  double2* mu = nullptr;      // [nb][nt][n]  costate lambda_{j+1} in basis j
  double2* ah = nullptr;      // [nb][nt][n]  HVP tangent a'_j in basis j
  double* s = nullptr;        // [nb][nt]     s_j = Re(lambda_{j+1}^H U''_j a_j)
  double* q = nullptr;        // [nb][nt]     q_j = Re(lambda_{j+1}^H U'_j a_j)
  double* e = nullptr;        // [nb][nt]     HVP per-step terms
  double* K = nullptr;        // [nb][nt][P]  K_j = Re(xi_j^H y_j)
  double2* xf = nullptr;      // [nb][n][1+P] final X (a_J and A'_J in basis nt-1)
  double2* binit = nullptr;   // [nb][n][2]   backward-sweep initial columns
  double* rr = nullptr;       // [nb]         |a_J - beta|^2
  double* aa = nullptr;       // [nb][P][P]   rho Re(A'_J^H A'_J)
  int* status = nullptr;
  unsigned long long* stats = nullptr;   // [0] eigen steps, [1] Jacobi sweeps
};

struct SysDev {
  int n = 0;
  const double* h0 = nullptr;     // [n][n]
  const double* m = nullptr;      // [n][n]
  const double* psi0 = nullptr;   // [n] complex
  const double* psit = nullptr;   // [n] complex, or [nb][n] complex when psit_bstride != 0
  size_t psit_bstride = 0;        // doubles between consecutive thetas' targets (0: shared target)
};

struct BasisDev {
  int nt = 0, P = 0;
  double dt = 0.0;
  const double* B = nullptr;      // [nt][P]
};

enum class Mode { Cost = 0, Grad = 1, Hess = 2, Hvp = 3 };

// ---------------------------------------------------------------- kernel arguments
// Each kernel is a device body over (argument block, block coordinates).  The single-problem
// kernels take their block coordinates from the grid; the multi-problem kernels pull work
// items (argument index, block coordinates) from a queue, so one launch covers many problems.

struct CtlArgs {
  int nt, P;
  const double* B;
  const double* theta;
  double* f;
};

struct EigArgs {
  int n, np, nt, chunk, nchunks;
  int j_base, nsteps;      // this launch covers global steps [j_base, j_base + nsteps)
  int eig_stride;          // steps per theta in the eigen-data arrays (indexed by j - j_base)
  double dt, tol_rel;
  int max_sweeps, store_derivs, lds_mats;
  const double* h0;
  const double* m;
  const double* f;
  double* lam;
  double* mt;
  double* sm;
  double* ov;
  double* vfirst;
  double* vlast;
  double* gscratch;
  int* status;
  unsigned long long* stats;
};

struct BndArgs {
  int n, nsteps, chunk, nchunks, eig_stride;
  const double* vfirst;
  const double* vlast;
  double* ov;
};

struct SweepArgs {
  int n, nt, P, pg, ngroups, hvp, need_y;
  int j_begin, j_end;     // step range of this launch
  int eig_j0;             // eigen-data arrays are indexed by j - eig_j0 ...
  size_t eig_stride;      // ... with this many steps per theta
  double dt;
  const double* ov;
  const double* sm;
  const double* lam;
  const double* F;        // forcing: [nt][fcols] (shared) or [nb][nt] (HVP)
  int fcols;
  size_t f_bstride;
  const double* vfirst;
  int nchunks;
  const double* psi0;     // complex n
  double2* at;
  double2* yt;
  double2* ah;
  double2* mu;
  double* q;
  double* e;
  double* K;
  const double* o_in;     // [nb][n][n] O_{j_begin-1} joining the previous segment (j_begin > 0)
  const double2* xin;     // forward state entering the range ([nb][n][1+P], j_begin > 0)
  double2* xout;          // forward: X after the range's last step ([nb][n][1+P])
  const double2* binit;   // backward state entering the range ([nb][n][2])
  double2* bout;          // backward state leaving the range in basis j_begin-1 ([nb][n][2])
};

struct TermArgs {
  int n, P, mode;
  double rho;
  const double2* xf;
  const double* vlast_step;
  size_t v_bstride;
  const double* psit;
  size_t psit_bstride;
  double2* binit;
  double* rr;
  double* aa;
};

struct StermArgs {
  int n, nt, ntasks;
  int j_begin, nsteps, eig_j0;   // tasks cover steps [j_begin, j_begin + nsteps) of every theta
  size_t eig_stride;
  double dt, tau;
  const double* mt;
  const double* sm;
  const double* lam;
  const double2* mu;
  const double2* at;
  double* s;
};

struct AsmArgs {
  int nt, P, mode, gx;   // gx: blocks sharing one theta's P x P outputs
  double gamma, rho;
  const double* B;
  const double* f;
  const double* u;
  const double* q;
  const double* s;
  const double* e;
  const double* K;
  const double* rr;
  const double* aa;
  double* cost;
  double* grad;
  double* out;
};

// One queue entry of a multi-problem launch.
struct Item {
  int arg;      // index into the launch's argument array
  int bx, by;   // block coordinates within that problem's grid
  int pad;
};

// Launchers (all enqueue on `stream`; return hipSuccess or the first launch error).
hipError_t launch_fourier_basis(double* B, int nt, int K, hipStream_t stream);
hipError_t launch_controls(const BasisDev& bs, const double* theta, double* f, int nb, hipStream_t stream);
hipError_t launch_eig(const SysDev& sy, const BasisDev& bs, Work& w, bool store_derivs,
                      double tol_rel, int max_sweeps, hipStream_t stream);
hipError_t launch_boundary(Work& w, hipStream_t stream);
// Segment join for checkpointed sweeps: obound_s = V_first^T vsave (if do_overlap), vsave = V_last.
hipError_t launch_seg_join(Work& w, double* obound_s, bool do_overlap, hipStream_t stream);
int eig_chunk_len(int seg_len, int nb, int np);
hipError_t launch_forward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream);
hipError_t launch_terminal(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, double rho,
                           hipStream_t stream);
hipError_t launch_backward(const SysDev& sy, const BasisDev& bs, Work& w, Mode mode, hipStream_t stream);
hipError_t launch_sterm(const SysDev& sy, const BasisDev& bs, Work& w, hipStream_t stream);
hipError_t launch_assemble(const BasisDev& bs, Work& w, Mode mode, double gamma, double rho,
                           double* cost, double* grad, double* hess_or_hv, hipStream_t stream);
hipError_t launch_identity_basis(double* B, int nt, hipStream_t stream);
// U_j, U'_j, U''_j for control value fj from a cold eigendecomposition (inspection aid).
// gs: device scratch of step_props_scratch_doubles(n) doubles.
hipError_t launch_step_props(const SysDev& sy, double fj, double dt, double* gs, double* u, double* u1,
                             double* u2, int* status, hipStream_t stream);
size_t step_props_scratch_doubles(int n);
// Batched symmetric eigendecomposition (parallel-order Jacobi, one workgroup per matrix):
// h: count x P x P (symmetrised on the fly), evals: count x P, evecs: count x P x P (column i
// is eigenvector i).  gs: device scratch of sym_eig_scratch_doubles(P, count) doubles.
hipError_t launch_sym_eig(const double* h, int P, int count, double* evals, double* evecs, double* gs,
                          int* status, hipStream_t stream);
size_t sym_eig_scratch_doubles(int P, int count);

// Argument blocks of the kernels (the single-problem launchers build theirs the same way).
CtlArgs controls_args(const BasisDev& bs, const double* theta, double* f);
EigArgs eig_args(const SysDev& sy, const BasisDev& bs, const Work& w, bool store_derivs, double tol_rel,
                 int max_sweeps);
BndArgs boundary_args(const Work& w);
// pg > 0 overrides the tangent columns per workgroup of the Hessian sweeps (clamped to P).
SweepArgs sweep_args(const SysDev& sy, const BasisDev& bs, const Work& w, Mode mode, int pg);
TermArgs terminal_args(const SysDev& sy, const Work& w, Mode mode, double rho);
StermArgs sterm_args(const BasisDev& bs, const Work& w);
AsmArgs assemble_args(const BasisDev& bs, const Work& w, Mode mode, double gamma, double rho, double* cost,
                      double* grad, double* out);

// Multi-problem (queue) launches: one launch per kernel variant covers many problems.
enum class MultiKind {
  Controls, EigWave4, EigWave8, EigWave16, EigWg36, EigWg64, EigChunk, EigBig, EigSlot, Boundary, ForwardStaged, ForwardSmall,
  ForwardGlobal, Terminal, BackwardStaged, BackwardSmall, BackwardGlobal, Sterm, Assemble, Count
};
MultiKind eig_kind(int np);
MultiKind forward_kind(int n);
MultiKind backward_kind(int n);
int multi_threads(MultiKind k);
size_t eig_launch_lds(int np);
size_t sweep_launch_lds(int n, int pg);
hipError_t configure_multi_kernels();
// Sweep launches from prepared arguments (grid: column groups x nb thetas).
hipError_t launch_forward_args(const SweepArgs& a, int nb, hipStream_t stream);
hipError_t launch_backward_args(const SweepArgs& a, int nb, hipStream_t stream);
int multi_grid(MultiKind k, size_t lds, int nitems, int num_cus);
hipError_t launch_multi(MultiKind k, const void* d_args, const Item* d_items, int nitems, int* d_counter,
                        size_t lds, int grid, hipStream_t stream);
hipError_t launch_fill_int(int* p, int count, int v, hipStream_t stream);
// Workspace layout for nb thetas, checkpoint segment seg (0: whole horizon) and eigen chunk length
// chunk (0: default); assigns w's pointers inside base (may be null to size only) and returns
// the bytes needed.
size_t layout_work(Work& w, int n, int nt, int P, int nb, int seg, int chunk, void* base);

// Largest dynamic LDS request of any kernel; set once per device.
hipError_t configure_kernels();
// The same for the kernels of the several-direction path.
hipError_t configure_mc_kernels();
size_t eig_scratch_doubles(int n, int nb, int nchunks);
int choose_pg(int P, int nb);

}  // namespace qoc
