// Host-side compiled circuit (internal to the library).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pbit.h"

namespace pbit {

struct CompiledCircuit {
    std::vector<uint32_t> blob;  // device image, layout in blob.h
    uint32_t n = 0, d = 0, K = 0, W = 0, WS = 0, L = 0, h = 0, ncol = 0, n_gates = 0, nqd = 0;
    uint32_t circuit_id = 0;
    uint32_t ny = 0;  // derived AND variables (three-qubit permutation gates)
    bool uniform = true;
    bool has_z = false;
    double Z = 0.0;
};

pbit_status compile_one(const pbit_circuit_desc &desc, CompiledCircuit &out, std::string &err);

}  // namespace pbit
