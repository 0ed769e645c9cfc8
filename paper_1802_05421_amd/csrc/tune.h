// Table of measured launch choices (tune.hip): one entry per (GPU
// architecture, kernel family, element type, shape) holding the time of every
// candidate configuration and the index of the fastest.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace cdl {

// Architecture name of a device ("none" without one), cached per device.
std::string tune_arch(int device);
// "square/bf16/ld16384", "apply/fp16/ld16384/k256", "residual/fp64/ld16384/k256".
std::string tune_key(const char *family, int prec, int64_t ld, int64_t kpad);
// Chosen candidate, its time in ms and the candidate count of an entry.
bool tune_get(const std::string &arch, const std::string &key, int *choice, double *ms,
              int *ncand);
// Stores the candidates' times (ms <= 0: not measured) and returns the index
// of the fastest; rewrites the file named by CDL_AUTOTUNE_CACHE, if any.
int tune_put(const std::string &arch, const std::string &key, const std::vector<double> &ms);
bool tune_load(const char *path, std::string *err);
bool tune_save(const char *path, std::string *err);
void tune_clear();
int tune_entries();

}  // namespace cdl
