// The host-only part of the C ABI: plan creation, description and release,
// and the thread-local error text every entry point sets.  It runs no GPU
// code, so this file and the planner also build on their own (for instance
// under a host address sanitizer) into a library that plans without a GPU.
#include <algorithm>
#include <cstring>
#include <exception>
#include <string>

#include "engine.hpp"
#include "lmfao.h"

namespace lmfao {

static thread_local std::string g_last_error;

void record_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

}  // namespace lmfao

using namespace lmfao;

static lmfao_status plan_err(lmfao_status st, const std::string& m) {
  record_error(m);
  return st;
}

extern "C" {

void lmfao_default_options(lmfao_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = LMFAO_PREC_F64;
  o->form = LMFAO_FORM_FUSED;
  o->root_policy = LMFAO_ROOT_GROUPBY;
  o->n_order = nullptr;
  o->order = nullptr;
  o->min_segment = 0;
}

lmfao_status lmfao_plan(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                        const lmfao_options* opts, lmfao_plan_t* out) {
  clear_error();
  if (!out) return plan_err(LMFAO_EINVAL, "null output handle");
  *out = nullptr;
  try {
    Plan* P = build_plan(schema, tree, batch, opts);
    if (!P->supported) {
      std::string why = P->unsupported_reason;
      delete P;
      return plan_err(LMFAO_EUNSUPPORTED, why);
    }
    lmfao_plan_s* h = new lmfao_plan_s;
    h->P = P;
    *out = h;
    return LMFAO_OK;
  } catch (const PlanError& e) {
    return plan_err(e.status, e.msg);
  } catch (const std::exception& e) {
    return plan_err(LMFAO_EINVAL, e.what());
  }
}

lmfao_status lmfao_plan_describe(lmfao_plan_t plan, char* buf, size_t cap, size_t* need) {
  if (!plan) return plan_err(LMFAO_EINVAL, "null plan");
  const std::string& j = plan->P->json;
  if (need) *need = j.size() + 1;
  if (buf && cap) {
    size_t n = std::min(cap - 1, j.size());
    std::memcpy(buf, j.data(), n);
    buf[n] = 0;
  }
  return LMFAO_OK;
}

void lmfao_plan_free(lmfao_plan_t plan) {
  if (!plan) return;
  delete plan->P;
  delete plan;
}

const char* lmfao_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
