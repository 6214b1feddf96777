// qedx_batch.cpp -- mixed-process batches (placeholder until the persistent
// kernel lands: every entry point reports QED_ERR_UNSUPPORTED).
#include <string>

#include "../../include/qedx.h"

extern "C" qed_status qed_batch_plan_create(const qed_segment*, int, int, qed_batch_plan** out) {
  if (out) *out = nullptr;
  return QED_ERR_UNSUPPORTED;
}
extern "C" qed_status qed_batch_launch(qed_batch_plan*, void*) { return QED_ERR_UNSUPPORTED; }
extern "C" qed_status qed_batch_plan_destroy(qed_batch_plan*) { return QED_OK; }
