// Batches of independent instances (placeholder until the persistent kernel).
#include "../../include/ace.h"

extern "C" {
int ace_batch_create(int, const ace_instance_desc *, ace_batch **out, int *)
{
    if (out) *out = nullptr;
    return ACE_E_STATE;
}
int ace_batch_destroy(ace_batch *) { return ACE_E_STATE; }
int ace_batch_shape(const ace_batch *, int, int64_t *, int64_t *, int64_t *) { return ACE_E_STATE; }
int ace_batch_set_stream(ace_batch *, void *) { return ACE_E_STATE; }
int ace_batch_set_phi0(ace_batch *, int, const double *, int) { return ACE_E_STATE; }
int ace_batch_set_all(ace_batch *, const double *, int) { return ACE_E_STATE; }
int ace_batch_step(ace_batch *, int64_t) { return ACE_E_STATE; }
int ace_batch_monitor(ace_batch *, double *, double *) { return ACE_E_STATE; }
int ace_batch_get_phi(ace_batch *, int, double *, int) { return ACE_E_STATE; }
int ace_batch_get_all(ace_batch *, double *, int) { return ACE_E_STATE; }
int ace_autotune(ace_solver *, int64_t, char *, size_t) { return ACE_E_STATE; }
}
