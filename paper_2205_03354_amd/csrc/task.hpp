// A Krylov solve as a resumable state machine.
//
// A SolveTask owns the device state of one biharmonic BVP or Cahn-Hilliard
// step (workspace vectors, scalars, partial sums) and advances it in chunks:
// every call enqueues the next chunk of work on the task's stream (a block of
// CG iterations, replayed from a captured hipGraph, or a true-residual
// sweep) followed by a copy of the scalar block to pinned host memory, and
// returns. Once that copy has landed the owner calls advance() again. The
// blocking entry points loop start/advance with a stream synchronisation;
// the request server interleaves many tasks on separate streams.
#pragma once

#include "internal.hpp"

namespace sc {

// TASK_BVP: ring-mode biharmonic BVP (b from f and the ring values);
// TASK_CH: periodic Cahn-Hilliard step (b from u); TASK_LIN: periodic
// solve of A x = b for a given b (the stages of an IMEX step).
enum TaskKind : int { TASK_BVP = 0, TASK_CH = 1, TASK_LIN = 2 };

// A read-only FP64 grid view: `p` addresses interior element (0,0,0).
struct GridView {
  const double* p = nullptr;
  int64_t pitch = 0;
  int64_t zpitch = 0;
};

struct TaskSpec {
  int kind = TASK_BVP;
  int dim = 2;
  int64_t n[3] = {1, 1, 1};
  KStencil ksA;        // the operator A (weights scaled by h^-p)
  KStencil ksL;        // TASK_CH: the Laplacian (scaled by h^-2)
  double dt = 0.0;     // TASK_CH
  double S = 0.0;      // TASK_CH
  double h = 0.0;      // grid spacing (the fast-Poisson preconditioner's eigenvalues)
  sc_solve_opts o{};
};

// Device bytes a task of this shape holds while it is alive.
size_t task_footprint(const TaskSpec& spec);
// The task is a small 2D FP64 BVP without preconditioner that the options
// allow on chip and that fits one workgroup.
bool task_onchip(const TaskSpec& spec);

// Fast-Poisson preconditioner z = L_D^-2 r (see precond.cpp).
class FastPoisson {
 public:
  FastPoisson() = default;
  FastPoisson(const FastPoisson&) = delete;
  FastPoisson& operator=(const FastPoisson&) = delete;
  ~FastPoisson();
  // Tables for the n unknowns per axis with spacing h (enqueued on st).
  sc_status init(int dim, const int64_t* n, double h, int dtype, hipStream_t st);
  // z = M^-1 r on the interiors of r, z, tmp (all of layout lay); the
  // scaling kernel is skipped once s->done is set.
  sc_status apply(const void* r, void* z, void* tmp, const Layout& lay, const DevScalars* s, hipStream_t st) const;

 private:
  // One sine transform along the rows of `in` (m rows of n, row pitch pin),
  // written transposed into `out` (n rows of m, row pitch pout), by a real
  // FFT of the odd extension (2D grids of side >= kFftMinSide with n + 1 a
  // power of two).
  struct Dst {
    int64_t n = 0, m = 0;
    void* plan = nullptr;  // rocfft_plan
    void* info = nullptr;  // rocfft_execution_info
    void* work = nullptr;
    size_t work_bytes = 0;
  };
  sc_status dst_init(Dst* d, int64_t n, int64_t m, hipStream_t st);
  sc_status dst_rows(const Dst& d, const void* in, int64_t pin, void* out, int64_t pout, hipStream_t st) const;
  bool fft_ = false;
  Dst dx_, dy_;          // along x (n0, batch n1) and along y (n1, batch n0)
  void* ext_ = nullptr;  // odd extensions, max m (2n + 2) reals
  void* spec_ = nullptr; // their half spectra, max m (n + 2) complex
  void* tr_ = nullptr;   // the x-transformed field, transposed (n0 rows of n1)
  int dim_ = 2;
  int dtype_ = SC_F64;
  bool split_ = false;  // GEMM transforms split by the sine matrix's even/odd symmetry
  int64_t n_[3] = {1, 1, 1};
  void* S_[3] = {nullptr, nullptr, nullptr};
  double* lam_[3] = {nullptr, nullptr, nullptr};
  std::vector<void*> allocs_;
};
size_t fastpoisson_bytes(int dim, const int64_t* n, int dtype);
constexpr int64_t kFftMinSide = 200;  // 2D sides from which the transforms may use FFTs
constexpr int64_t kSplitMinSide = 768;  // 2D GEMM-transform sides from which the transforms are split

class SolveTask {
 public:
  SolveTask() = default;
  SolveTask(const SolveTask&) = delete;
  SolveTask& operator=(const SolveTask&) = delete;
  ~SolveTask();

  // Allocate and clear the workspace (enqueued on `st`).
  sc_status init(const TaskSpec& spec, hipStream_t st);
  // x0 := u0; right-hand side (BVP: f - A g_ring, g may be null; CH: from
  // x0); first true residual; scalars to the host.
  sc_status start(const GridView& u0, const GridView& f, const GridView* g);
  // TASK_LIN: solve again with a new x0 and right-hand side f, reusing the
  // workspace and the captured graphs (the previous solve has finished).
  sc_status restart(const GridView& u0, const GridView& f);
  // The previously enqueued chunk has completed: decide, enqueue the next
  // chunk. *done = true when the solve has finished (see status()).
  sc_status advance(bool* done);
  // x -> dst (device FP64 view).
  sc_status enqueue_copy_out(double* dst, int64_t pitch, int64_t zpitch);

  sc_status status() const { return status_; }
  const sc_solve_stats& stats() const { return stats_; }
  hipStream_t stream() const { return st_; }
  size_t footprint() const { return bytes_; }

 private:
  enum Phase { P_NONE, P_CHECK64, P_ITER64, P_FINAL, P_OUTER, P_INNER, P_ONCHIP, P_DONE };
  struct Vec {
    void* alloc = nullptr;
    void* base = nullptr;
    Layout lay;
  };
  sc_status make(Vec* v, int dtype);
  sc_status enqueue_block(bool f32);
  sc_status enqueue_residual(int flag, double c = 0.0);
  sc_status enqueue_read(bool both);
  sc_status fall_back_to_f64();
  sc_status make_pc(bool f32);
  sc_status precondition(bool f32, int start);
  void finish(sc_status s);
  sc_status sweep(int kind, int dtype, const KStencil& ks, const void* in, const Layout* lin, const void* in2,
                  const void* aux, void* out, void* out2, const Layout& lout, int flag, double c0, double c1,
                  double c2, DevScalars* sc, const GridView* in_view = nullptr, const GridView* aux_view = nullptr,
                  const double* fold = nullptr);

  TaskSpec spec_;
  bool periodic_ = false;
  bool f32_ = false;   // FP32 inner iterations (refinement or reliable updates)
  bool ru_ = false;    // reliable updates: keep the FP32 direction across replacements
  bool restart_ = true;  // next FP32 stretch starts from p = r
  int halo_ = 0;
  hipStream_t st_ = nullptr;
  Vec x_, b_, r64_, r32_, d32_, p_[2], q_;
  DevScalars* d64_ = nullptr;
  DevScalars* d32s_ = nullptr;
  DevScalars* h64_ = nullptr;
  DevScalars* h32_ = nullptr;
  double* partials_ = nullptr;
  double* upd_partials_ = nullptr;  // the CG update's partials (the sweep's stay readable)
  void* dev_block_ = nullptr;
  std::vector<void*> allocs_;
  size_t bytes_ = 0;
  int cur_ = 0;          // p_[cur_] holds the latest search direction
  int block_cur0_ = 0;    // cur_ and the device iteration count when the
  long long block_iter0_ = 0;  // last block was enqueued
  hipGraphExec_t graph_[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [FP32][parity]
  Phase phase_ = P_NONE;
  sc_status pending_ = SC_OK;
  sc_status status_ = SC_OK;
  int outer_ = 0;
  int stalled_ = 0;
  double best_ = 0.0;
  long long inner_start_ = 0;
  int inner_keep_ = 0;    // the running FP32 stretch continued the previous direction
  double stretch_best_ = 0.0;  // smallest FP32 recursive rr seen in the running stretch
  int stretch_idle_ = 0;       // blocks since it last halved
  bool fell_back_ = false;     // a mixed-precision solve that continued in FP64
  bool pc_ = false;            // preconditioned CG (BVP, fast-Poisson)
  TapTable taps_;              // the operator's taps (double-double residual)
  bool onchip_ = false;        // one-kernel solve of a small 2D BVP (see small.hip)
  SmallDesc sdesc_{};
  SmallTaps staps_{};
  SmallDesc* sdesc_dev_ = nullptr;
  SmallResult* sres_dev_ = nullptr;
  FastPoisson pc64_, pc32_;
  Vec z64_, t64_, z32_, t32_;  // z = M^-1 r and its scratch, per precision
  sc_solve_stats stats_{};
};

// A grid's interior as a view; the stream a blocking call runs on (a
// library stream ordered after the NULL stream when the caller passes it);
// drive a started task to completion on its stream.
GridView view_of(const sc_grid* g);
sc_status blocking_stream(hipStream_t caller, hipStream_t* out);
sc_status run_blocking(SolveTask& t);
// cI I + cLL (L o L) + cL L with L = lap's weights as given (no h scaling).
sc_status lap_operator(const sc_stencil* lap, long double cI, long double cLL, long double cL, KStencil* out);
size_t vec_bytes(int dim, const int64_t* n, int halo, int dtype);
// A sweep descriptor for n with no buffers yet; launch one after deriving
// its alignment flags (SC_EUNSUPPORTED when no kernel instance fits).
SweepLaunch sweep_on(int kind, const KStencil& ks, bool periodic, int dtype, const int64_t* n);
sc_status launch(SweepLaunch L, hipStream_t st);
Layout make_layout(int dim, const int64_t* n, int halo, int dtype);

// Pinned host slots for scalar read-back (one pair per live task).
DevScalars* pinned_pair_alloc();
void pinned_pair_free(DevScalars* p);

}  // namespace sc
