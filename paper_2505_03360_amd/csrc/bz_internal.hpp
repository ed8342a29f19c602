// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "bz.h"
#include "kinetic.hpp"

namespace bz {

// Thread-local last-error text; every failing entry point sets it.
bz_status fail(bz_status code, const char* fmt, ...);
void clear_error();

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Every workspace starts with a status region: int32 word 0 is set by the
// output epilogues when they write a non-finite value.
constexpr size_t kStatusBytes = 256;
// Directions per launch pair of the chunked plain path: each keeps one
// stage-A volume per cell in the workspace, so n = 48 (0.9 MB per volume in
// FP32, 1.8 MB in FP64) takes four, except FP32 plans of at most 1024 cells,
// which take eight (7.3 GB of volumes at 1024 cells; 6 % faster).
inline int plain_chunk(int n, bool fp32, int max_cells) {
  if (n <= 32) return 8;
  return (fp32 && max_cells <= 1024) ? 8 : 4;
}
constexpr int kPlainChunkMax = 17;  // 33 passes of a 32-direction plan: two launch pairs
// Two-dimensional plans keep a cell's spectrum in the workspace from n = 32
// up (the LDS then holds one transpose buffer per cell: twice the waves per
// CU); at n = 16 it stays in the LDS, which does not limit occupancy there.
constexpr bool spectrum2d_in_workspace(int n) { return n >= 32; }

// Workspace regions of a bound plan, each [capacity][...].
struct WsLayout {
  size_t status_off = 0;                  // byte offset of the status word
  size_t fh_off, y_off, acc_off, par_off;  // byte offsets into ws_dev
  size_t fh_cell, y_cell, acc_cell, par_cell;  // bytes per cell of each region
  // dealiased plans: padded f, padded raw Q, padded spectrum, the padded plan's workspace
  size_t fp_off = 0, qp_off = 0, gp_off = 0, pad_off = 0;
  size_t fp_cell = 0, qp_cell = 0, gp_cell = 0, pad_cell = 0;
};

// Device memory one evaluation runs on: the plan's uploaded tables and a
// workspace holding `capacity` cells.
struct Binding {
  const void* tables = nullptr;
  void* ws = nullptr;
  int capacity = 0;
  WsLayout lay{};
};

}  // namespace bz

struct bz_plan {
  bz_plan_desc d{};  // copy of the descriptor (dirs/weights pointers cleared)
  int n = 0;         // points per axis
  int dim = 3;       // velocity dimensions (2: Maxwell molecules in two dimensions)
  size_t npts = 0;   // n^dim grid points per cell
  int m = 0;         // directions
  int m1 = 0;        // m + 1: the loss term is evaluated as one more pass
  double L = 0, R = 0, gamma = 1, C = 4, dv = 0;
  int fp32 = 1;      // plan precision
  int project = 1;
  int transform = BZ_XF_PLAIN;  // resolved strategy
  int chunks = 1;               // direction chunks per cell (fused path)
  int slices = 2;               // j3 slices of the fused kernel's transposes
  int pchunk = 0;               // plain path: directions per chunk (stage-A volumes per cell)
  int plain_k = 0;              // plain path: directions per chunk asked for (desc.chunks), 0 = by size
  bz_plan* pad = nullptr;       // dealiased plans: the same operator on the 3n/2 grid (raw Q)
  std::vector<double> dirs;     // [m][3]
  std::vector<double> w;        // [m]
  int rule_t = 0;               // antipodal design degree reached by a BZ_DIRS_DESIGN rule (0: not a DESIGN rule)
  // FP64 host tables in device layout [p][k2][k3][k1] x (a, a'), p < m1;
  // pass p = m carries (Bhat_M, 1) with weight -1.
  std::vector<double> mult;
  std::vector<double> wext;     // [m1] device weights: w_p, then the loss scale
  std::vector<double> pscale;   // [m1] per-pass balance factor of the packed transform
  double ginv[25] = {};         // (C C^T)^-1 of the five invariants (dim = 2: 4x4 of four)
  size_t table_mult_bytes = 0, table_w_off = 0, tables_bytes = 0;
  size_t table_dft_off = 0;     // DFT-as-GEMM plans: matrix-core fragments of the inverse DFT
  size_t ws_fixed = 0, ws_per_cell = 0;
  // binding
  void* tables_dev = nullptr;
  void* ws_dev = nullptr;
  size_t ws_bytes = 0;
  int capacity = 0;
  bz::WsLayout ws{};  // per-cell region sizes; offsets of the plan's own binding
  // timing: a ring of event quadruples, one per timed call
  static constexpr int kTimingSlots = 512;
  bool timing = false;
  bool events_ready = false;
  std::vector<hipEvent_t> evs;  // 4 per slot
  int timed_calls = 0;          // calls recorded since the last summary
  hipEvent_t* ev = nullptr;     // quadruple of the current call
};

namespace bz {
// kernel launchers (collide.hip); `timed` records the plan's timing events
bz_status launch_collide(const bz_plan* p, const Binding& b, const void* f, int f_fp32,
                         const int32_t* idx, int ncells, const int32_t* ncells_dev, void* q,
                         int scatter, hipStream_t s, bool timed, const bzk::ImexDev* imex = nullptr);
// two velocity dimensions (collide2d.hip)
bz_status launch_collide2d(const bz_plan* p, const Binding& b, const void* f, int f_fp32, const int32_t* idx,
                           int ncells, const int32_t* ncells_dev, void* q, int scatter, hipStream_t s, bool timed);
// clears a status word with a vector store (collide.hip)
void launch_clear_status(void* ws, const WsLayout& lay, hipStream_t s);
// per-cell IMEX parameters (kinetic.hip)
bool kinetic_n_supported(int n);
bz_status launch_imex_params(int n, double dv, const int32_t* idx, int ncells, const int32_t* ncells_dev,
                             const double* f, const double* tr, double dt, double* par, hipStream_t s);
// direction rules (plan.cpp, design.cpp)
void rule_spiral(int m, std::vector<double>& d, std::vector<double>& w);
constexpr int kDesignMaxM = 256;
int design_terms(int m);
void rule_design(int m, std::vector<double>& d, std::vector<double>& w, int* t);
int rule_degree(const std::vector<double>& d, const std::vector<double>& w);
// plan helpers (plan.cpp)
Binding make_binding(const bz_plan* p, const void* tables, void* ws, size_t ws_bytes);
bz_status upload_tables(const bz_plan* p, void* tables_dev, hipStream_t s);
void fill_tables_host(const bz_plan* p, unsigned char* host);  // the device image of the tables (tables_bytes)
bool fused_supported(int n, int fp32);
bool dft_gemm_supported(int n, int fp32);
bool fused_slices_supported(int n, int slices);
int fused_default_chunks(int n, int max_cells);
// evaluation strategy a three-dimensional descriptor resolves to at a capacity (plan.cpp)
struct Strategy {
  int transform = BZ_XF_PLAIN, chunks = 1, slices = 2, plain_k = 8;
  bool operator==(const Strategy& o) const {
    return transform == o.transform && chunks == o.chunks && slices == o.slices && plain_k == o.plain_k;
  }
};
Strategy resolve_strategy(const bz_plan_desc& d, int max_cells, size_t ws_budget = ~size_t(0));
size_t plain_ws_per_cell(int n, bool fp32, int K);
}  // namespace bz
