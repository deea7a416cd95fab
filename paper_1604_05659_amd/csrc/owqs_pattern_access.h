// owqs_pattern_access.h -- host-side access to a loaded pattern for library
// code outside owqs_host.cpp (the reordering).  Not part of the public C ABI.
#pragma once

#include <string>
#include <vector>

#include "../../include/owqs.h"

namespace owqs {

// The pattern's commands in the public form: the caller's qubit ids, the
// current angles of the M commands, domains as ranges of `dom`.
void pattern_export(const owqs_pattern *pat, std::vector<owqs_cmd> &cmds, std::vector<int32_t> &dom,
                    std::vector<int32_t> &inputs, std::vector<int32_t> &outputs);
owqs_ctx *pattern_ctx(const owqs_pattern *pat);
// Records `msg` as the context's last error and returns `st`.
owqs_status pattern_fail(const owqs_pattern *pat, owqs_status st, const std::string &msg);

}  // namespace owqs
