// Internal definition of the op handle and Leja plans, shared by the host
// translation units of libadl (host.cpp, batch.hip).
#pragma once

#include "internal.h"
#include "adl.h"

#include <cmath>
#include <vector>

namespace adl {

constexpr int kMaxDegreeDefault = 500;
constexpr double kRhoMaxDefault = 1600.0;
constexpr int kMaxDoublings = 6;

struct Plan {
  int l = -1;
  double alpha = 0.0, h = 0.0;
  int M = 0;
  std::vector<double> d;      // d_0 .. d_{M-1}
  std::vector<double> shift;  // c + gamma xi_k
  std::vector<double> s;      // augmented scalars s_k
  double invg = 0.0;
  int last_degree = -1;
};


// Plan for phi_l on [alpha, 0] with step h and M coefficients.
void build_plan(Plan& P, int l, double alpha, double h, int M);

}  // namespace adl

// --------------------------------------------------------------------------
// opaque handle
// --------------------------------------------------------------------------
using adl::FieldView;
using adl::Tiling;
using adl::Ctl;
using adl::Plan;
using adl::kMaxDegreeDefault;
using adl::kRhoMaxDefault;

struct adl_op {
  FieldView f{};
  Tiling t{};   // preferred tiling (two columns per lane when nx is even)
  Tiling t1{};  // one column per lane: used when a caller's vector is not 16-byte aligned
  Tiling t2{};  // two-term Newton-Leja kernel (two columns per lane when nx is even)
  Tiling t21{}; // two-term kernel, one column per lane
  Tiling t3{};  // three-term kernel: the two-term tiling with fewer, longer runs (kMaxGrid3)
  Tiling t4s{}; // four-term staged kernel: strips of 60*VEC output columns, kMaxGrid3 blocks
  Tiling t4{};  // four-term Newton-Leja kernel (two columns per lane when nx is even)
  Tiling t41{}; // four-term kernel, one column per lane
  int fuse_terms = 1;  // 0 one Newton term per launch, 1 two (kernel by tiling), 2 two (LDS-staged), 3 two (frames),
                       // 4 four (grids below 2^20 points)
  int streaming = -1;  // non-temporal hints on Newton vectors: -1 auto, 0 off, 1 on
  int nx = 0, ny = 0, bc = 0, storage = 0;
  double hx = 0, hy = 0;
  long n = 0;
  int ws_max_degree = kMaxDegreeDefault;
  int max_degree = kMaxDegreeDefault;
  double rho_max = kRhoMaxDefault;
  int quad2_mode = ADL_QUAD2_AUGMENTED;
  bool has_bound = false;
  double alpha = 0.0;
  // learned bound: the interval came from the predictor; sweeps are capped at
  // `budget` terms and a failure falls back to power iteration
  double last_lambda = NAN;  // last power-iteration estimate of the spectral radius
  bool learned = false;
  int budget = 0;
  int substeps_hint = 0;
  double gersh = NAN;  // cached Gershgorin bound
  // workspace slices
  void* ybuf[2] = {nullptr, nullptr};
  double* p = nullptr;
  double* w1 = nullptr;
  double* w2 = nullptr;
  double* yacc = nullptr;
  double* tmp = nullptr;
  double* tmp2 = nullptr;
  double* p2 = nullptr;     // a sweep's third y buffer and its p buffers (with p and the caller's p_out)
  double* p3 = nullptr;
  double* p4 = nullptr;
  long slot_stride = 0;     // doubles per partials slot
  double* partials = nullptr;
  Ctl* ctl = nullptr;
  Ctl* host_ctl = nullptr;  // pinned
  adl::HostCtl* hctl = nullptr;  // sweep outcome mirror (coherent pinned host memory; null: copy back instead)
  adl::HostCtl* hctl_dev = nullptr;  // its device address
  int hseq = 0;             // sequence number of the pending publication
  int mirror_dev = 0;       // device whose pool holds the slot
  int host_wait = 1;        // 1: spin on the mirror when there is one; 0: copy back + synchronise
  std::vector<Plan> plans;  // small cache
  int plan_next = 0;
  // kernel profiling of the Newton-Leja iteration kernel: totals, and per
  // launch kind (ADL_LAUNCH_FIRST, _ONE, _TWO, _FOUR, _THREE)
  bool prof = false;
  double prof_ms = 0.0, prof_bytes = 0.0;
  long long prof_launches = 0;
  double kind_ms[5] = {0, 0, 0, 0, 0}, kind_bytes[5] = {0, 0, 0, 0, 0};
  long long kind_launches[5] = {0, 0, 0, 0, 0}, kind_terms[5] = {0, 0, 0, 0, 0};
  std::vector<hipEvent_t> evs;
};


namespace adl {
// Records the message of a failing entry point (returned by adl_last_error)
// and returns code.
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// cached plan of the op (l, alpha, h)
Plan& get_plan(adl_op* op, int l, double alpha, double h);
int substeps_for(double alpha, double dt, double rho_max);
}  // namespace adl
