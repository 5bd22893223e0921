// capi.cpp -- option defaults and status strings of the C ABI.
#include <string.h>

#include "nnm.h"

extern "C" void nnm_default_options(nnm_options* opt)
{
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->precision = NNM_PREC_AUTO;
    opt->knn_k = 0;
}

extern "C" const char* nnm_strerror(int32_t status)
{
    switch (status) {
    case NNM_OK: return "ok";
    case NNM_EINVAL: return "invalid argument";
    case NNM_ENOMEM: return "out of memory";
    case NNM_EDEVICE: return "device error";
    case NNM_ENONFINITE: return "non-finite feature value";
    case NNM_EUNSUPPORTED: return "precision not supported for these inputs";
    case NNM_ETOOLARGE: return "input larger than the fixed scratch of mst_build_noalloc";
    default: return "unknown status";
    }
}
