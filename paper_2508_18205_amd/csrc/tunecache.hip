// Cache of tuned launch variants: the autotuner's choice kept in a text file
// across processes, keyed by everything the choice depends on (the plan's
// shape and the device), so that a caller who builds the same plan again
// sets the variant without timing the candidates.
#include <stdio.h>
#include <string.h>

#include <string>

#include "common.h"

namespace {

// The device (architecture without its feature suffix, compute-unit count)
// and the plan's shape: dimension, node counts, stencil sizes, field count,
// precisions, mode, polarisation, boundary and the longest halo list (which
// the node distribution sets).  No spaces, so one token of a cache line.
std::string tune_key(const rbffd_plan* p) {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    char arch[64];
    size_t k = 0;
    for (; k + 1 < sizeof arch && prop.gcnArchName[k] && prop.gcnArchName[k] != ':' && prop.gcnArchName[k] != ' ';
         ++k)
        arch[k] = prop.gcnArchName[k];
    arch[k] = '\0';
    char buf[512];
    snprintf(buf, sizeof buf, "%s/cu%d/d%d/N%lld/Nh%lld/n%d/nh%d/K%d/f%d/w%d/mode%d/pol%d/bc%d/hmax%d", arch,
             prop.multiProcessorCount, p->dim, (long long)p->E.N, (long long)p->H.N, p->n, p->nh, p->K,
             p->p.fdtype, p->p.wdtype, p->p.mode, p->p.pol, p->p.bc, p->opH.hmax);
    return buf;
}

}  // namespace

extern "C" int rbffd_autotune_cached(rbffd_plan* p, rbffd_fields* f, int32_t reps, const char* cache_path,
                                     int32_t* hit, void* stream) {
    if (hit) *hit = 0;
    if (!p) return RBFFD_EINVAL;
    if (!f || !cache_path || !cache_path[0]) return set_err(p, RBFFD_EINVAL, "rbffd_autotune_cached: null argument");
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    const std::string key = tune_key(p);
    if (key.empty()) return set_err(p, RBFFD_EHIP, "rbffd_autotune_cached: no current HIP device");
    if (FILE* fp = fopen(cache_path, "r")) {
        char line[1024];
        bool found = false;
        int v[4] = {0, 0, 0, 0};
        while (fgets(line, sizeof line, fp)) {
            char k[600];
            int b, x, l, pe;
            if (sscanf(line, "rbffd-variant %599s %d %d %d %d", k, &b, &x, &l, &pe) == 5 && key == k) {
                v[0] = b, v[1] = x, v[2] = l, v[3] = pe;   // the last entry for the key wins
                found = true;
            }
        }
        fclose(fp);
        if (found && rbffd_set_variant(p, v[0], v[1], v[2], v[3]) == RBFFD_OK) {
            if (hit) *hit = 1;
            return RBFFD_OK;
        }
    }
    int rc = rbffd_autotune(p, f, reps, stream);
    if (rc) return rc;
    FILE* fp = fopen(cache_path, "a");
    if (!fp) return set_err(p, RBFFD_EINVAL, std::string("rbffd_autotune_cached: cannot append to ") + cache_path);
    fprintf(fp, "rbffd-variant %s %d %d %d %d\n", key.c_str(), p->var.block, p->var.xcd, p->var.lds, p->var.persist);
    const bool bad = fclose(fp) != 0;
    if (bad) return set_err(p, RBFFD_EINVAL, std::string("rbffd_autotune_cached: cannot write ") + cache_path);
    return RBFFD_OK;
}
