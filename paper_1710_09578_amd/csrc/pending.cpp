// Entry points whose implementation is pending.
#include "runtime.h"
using namespace fm;
extern "C" {
fm_status fm_circulant_grad_generator(int64_t, int64_t, fm_dir, const void*, int64_t, const void*, int64_t, void*, int32_t, fm_dtype, void*) { set_error("not implemented"); return FM_E_UNSUPPORTED; }
}
