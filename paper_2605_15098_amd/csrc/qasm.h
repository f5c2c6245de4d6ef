// OpenQASM 2.0 reader (host only).
#pragma once
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace svq {
// Parse a program into extended gate records (no SV_UK records: every gate
// of the language is one target with controls, or a swap). On failure
// returns the status and sets err to a message naming the line.
sv_status parse(const char *text, std::vector<sv_gate_ex> &out, int &nqubits, std::string &err);
}  // namespace svq
