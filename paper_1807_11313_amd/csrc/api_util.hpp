// Helpers of the C-ABI layer shared by its source files: error reporting
// and parameter validation (defined in ebsd_api.hip).
#pragma once

#include "../../include/ebsd_tm.h"
#include "ebsd_internal.hpp"

#include <string>

namespace ebsd {
namespace api {

extern thread_local std::string g_last_error;
int fail(int code, const char* msg);
int fail_hip(hipError_t e, const char* where);
int resolve_params(const ebsd_params* in, int n, ebsd_params* out);
FilterParams filter_of(const ebsd_params& p, int n);
int check_master(const ebsd_master* mp);
int check_geometry(const ebsd_geometry* geo);
int64_t spec_complex(int n);
int f32_images_only(const ebsd_params& p);

}  // namespace api
}  // namespace ebsd
