// Runtime services the library's translation units share (context access,
// error reporting, argument validation, pass buffer planning).
#pragma once
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/reach.h"

namespace reach {
namespace rt {

int ctx_device(const reach_ctx* c);
int ctx_cus(const reach_ctx* c);
unsigned int* ctx_status(reach_ctx* c);
int64_t option(const reach_ctx* c, const char* key);
// Records `msg` as the context's last error and returns `st`.
reach_status set_error(reach_ctx* c, reach_status st, const std::string& msg);
// The checks every entry point applies to a system and dtype, for a
// REACH_USER system (the only kind the user entry points take).
reach_status validate_user(reach_ctx* c, const reach_system* s, reach_dtype dtype);
// Per pass (source, destination) buffer ids, 0 = x, 1 = r, 2 = workspace,
// such that no pass reads what it writes and the last pass writes r (else
// final_copy: copy the workspace into r).
void pass_buffers(int64_t passes, bool inplace_ok, bool alias,
                  std::vector<std::pair<int, int>>* io, bool* final_copy);

}  // namespace rt
}  // namespace reach
