/* A plain C99 caller of the library: the header must compile as C, and the
 * host-side calls (a mesh without a device context) must work from C.
 * Built and run by tests/test_abi_cpu.py; exits 0 on success. */
#include <stdio.h>
#include <string.h>

#include "pfem.h"

#define EXPECT(cond)                                                 \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond,         \
              pfem_last_error());                                    \
      return 1;                                                      \
    }                                                                \
  } while (0)

int main(void) {
  /* unit square, two triangles, left edge clamped, traction on the right */
  const double coords[] = {0, 0, 1, 0, 0, 1, 1, 1};
  const int32_t conn[] = {0, 1, 2, 1, 3, 2};
  const double E[] = {1.0, 1.0}, nu[] = {0.3, 0.3};
  const int32_t dnode[] = {0, 0, 2, 2};
  const int8_t dcomp[] = {0, 1, 0, 1};
  const double dval[] = {0, 0, 0, 0};
  const int32_t facet[] = {1, 3};
  const double traction[] = {0.01, 0.0};
  pfem_mesh* m = NULL;
  pfem_mesh_info info;
  int32_t perm[4];
  int64_t n = 0;

  EXPECT(strstr(pfem_version(), "gfx950") != NULL);
  EXPECT(pfem_mesh_finalize(NULL, 0) == PFEM_E_INVALID_ARG);
  EXPECT(pfem_mesh_create(NULL, 2, 4, coords, 2, conn, &m) == PFEM_OK && m != NULL);
  EXPECT(pfem_mesh_set_material(m, PFEM_LIN_PLANE_STRESS, PFEM_PARAM_E_NU, E, nu) == PFEM_OK);
  EXPECT(pfem_mesh_set_dirichlet(m, 4, dnode, dcomp, dval) == PFEM_OK);
  EXPECT(pfem_mesh_set_neumann(m, 1, facet, traction) == PFEM_OK);
  EXPECT(pfem_mesh_set_node_order(m, PFEM_ORDER_RCM) == PFEM_OK);
  EXPECT(pfem_mesh_finalize(m, 0) == PFEM_OK);
  EXPECT(pfem_mesh_get_info(m, &info) == PFEM_OK);
  EXPECT(info.dim == 2 && info.n_nodes == 4 && info.n_elems == 2);
  EXPECT(info.n_free == 4);
  EXPECT(pfem_mesh_query_int(m, PFEM_Q_PERM, NULL, 0, &n) == PFEM_OK && n == 4);
  EXPECT(pfem_mesh_query_int(m, PFEM_Q_PERM, perm, 4, &n) == PFEM_OK);
  EXPECT(perm[0] + perm[1] + perm[2] + perm[3] == 6);
  /* device calls on a host-only mesh are a state error, not a crash */
  EXPECT(pfem_force(m, PFEM_FP64, PFEM_LAYOUT_USER, PFEM_MASK_NONE, NULL, NULL) ==
         PFEM_E_STATE);
  pfem_mesh_destroy(m);
  printf("c abi ok\n");
  return 0;
}
