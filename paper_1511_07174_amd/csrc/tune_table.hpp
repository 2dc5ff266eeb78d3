// Reader of the autotuner's JSON table (host code only).
#pragma once
#include <stdint.h>
#include <string>
#include <vector>

namespace cds {

struct TuneRecord {
  int key;        // 0 getrf_nb, 1 potrf_nb, 2 vbatch_tile (the cds_tune_key_t values)
  int dtype;      // 0 f64, 1 f32 (the cds_dtype_t values)
  int64_t n_max;
  int64_t value;
};

// Parses the table at path into out; arch receives the table's "arch" string ("" when absent).
// Returns 0, or 1 with a message in err (out is then empty).
int read_tune_table(const char* path, std::vector<TuneRecord>& out, std::string& arch, std::string& err);

}  // namespace cds
