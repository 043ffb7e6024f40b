/* A plain C program against the C ABI: the header compiles as C99 and the library's
   host-side entry points (version, size queries, validation) answer without a GPU. */
#include <stdio.h>
#include <string.h>

#include "rbos.h"

int main(void) {
  if (rbos_version() != RBOS_ABI_VERSION) return 1;
  /* 8 corner values of 4 B per record, records for cells -1 .. n-1 on each axis */
  if (rbos_field_bytes(128, 128, 128, RBOS_F32) != (size_t)32 * 129 * 129 * 129) return 2;
  if (rbos_field_bytes(128, 128, 128, RBOS_BF16) != (size_t)16 * 129 * 129 * 129) return 3;
  if (rbos_field_bytes(1, 128, 128, RBOS_F32) != 0) return 4;
  /* validation happens on the host, before anything is enqueued */
  if (rbos_trace_forward(NULL, 1, NULL, NULL, NULL, 0, NULL) != RBOS_E_NULL) return 5;
  if (strlen(rbos_last_error()) == 0) return 6;
  rbos_scene s;
  memset(&s, 0, sizeof s);
  if (rbos_trace_forward(&s, 0, NULL, NULL, NULL, 0, NULL) != RBOS_OK) return 7; /* empty batch */
  if (rbos_mlp_param_count(64, 4) != (size_t)(3 * 64 + 64 + 3 * (64 * 64 + 64) + 64 * 5 + 5)) return 8;
  printf("c abi ok\n");
  return 0;
}
