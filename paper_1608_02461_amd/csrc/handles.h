// Handle types and the exception guard shared by the extern "C" entry points.
#pragma once

#include <memory>
#include <new>
#include <string>

#include "fmm3.h"
#include "solver3.h"
#include "solver.h"

struct hfmm_tree_s {
  std::unique_ptr<hfmm::Tree> t;
};
struct hfmm_solver_s {
  std::unique_ptr<hfmm::Solver> s;
};
struct hfmm3_tree_s {
  std::unique_ptr<hfmm::Tree3> t;
};
struct hfmm3_solver_s {
  std::unique_ptr<hfmm::Solver3> s;
};

#define HFMM_GUARD_BEGIN try {
#define HFMM_GUARD_END                                              \
  }                                                                 \
  catch (const hfmm::Error& e) {                                    \
    hfmm::set_last_error(e.what());                                 \
    return e.code;                                                  \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    hfmm::set_last_error("host allocation failed");                 \
    return HFMM_ERR_OOM;                                            \
  }                                                                 \
  catch (const std::exception& e) {                                 \
    hfmm::set_last_error(std::string("internal: ") + e.what());     \
    return HFMM_ERR_INTERNAL;                                       \
  }                                                                 \
  catch (...) {                                                     \
    hfmm::set_last_error("internal: unknown exception");            \
    return HFMM_ERR_INTERNAL;                                       \
  }
