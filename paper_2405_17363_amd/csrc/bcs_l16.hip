// Kernel variants with 16 lanes per cell.
#define BCS_LANES 16
#include "bcs_variants.h"

namespace bcs {
const Variant* variants_l16(int* count) {
  static const Variant table[] = {BCS_RPL_KMAX_LIST(BCS_VARIANT_ENTRY)};
  *count = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}
}  // namespace bcs
