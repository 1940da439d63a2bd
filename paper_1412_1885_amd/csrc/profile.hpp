// RAII bracket of a stage with HIP events when profiling is enabled.
#pragma once

#include <hip/hip_runtime.h>

namespace rt {

enum ProfStage {
  kStageFirstPass = 0,
  kStageSweepPass = 1,
  kStageCorePass = 2,
  kStageContract = 3,
  kStageQr = 4,
  kStageTruncate = 5,
  kStageFfcp = 6,
  kStageStats = 7,
  kStageConvert = 8
};

bool prof_enabled();

class ProfScope {
 public:
  ProfScope(int stage, hipStream_t s);
  ~ProfScope();

 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace rt
