// Lippmann-Schwinger Nystrom solver (Section 3.3, eq. descretls) on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "plan.hpp"

namespace ws {

// Solves of one plan run together by ls_run (one GMRES instance each).
constexpr int kMaxLsBatch = 64;

size_t ls_work_bytes(const Plan& p, int restart, bool mixed, int count = 1);

// Solve (I + kappa^2 A_n M_s) u_s = u_inc_s for s < count (contrasts, incident
// fields and solutions stacked [count][n][n]); info holds count entries.
// Returns the largest status over the solves: WS_OK, 1 (max_matvecs reached),
// 2 (breakdown: non-finite values), or a negative WS_E* code with *err set.
int ls_run(const Plan& p, int count, const double* contrast, const cx<double>* u_inc, double tol, int restart,
           int max_matvecs, bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s,
           std::string* err);

// Cache of captured GMRES step graphs kept by a Helmholtz plan (created with
// the plan, destroyed with it).
void* ls_graph_cache_create();
void ls_graph_cache_destroy(void* cache);

}  // namespace ws
