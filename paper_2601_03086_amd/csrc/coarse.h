// Coarse space of the two-level preconditioner (see coarse.cpp).
#pragma once

#include <memory>
#include <vector>

#include "mesh.h"

namespace pfem {

// Owner blocks per aggregate for this mesh.
int coarse_group(const pfem_mesh* m);
// Builds m->coarse on the host (once; thread-safe).
void coarse_build(pfem_mesh* m);
// Builds if needed and uploads the device arrays (once per upload of the mesh).
void coarse_upload(pfem_mesh* m, Ctx* ctx);
// Device bytes of the coarse arrays (for admission charges).
int64_t coarse_device_bytes(const pfem_mesh* m);

}  // namespace pfem
