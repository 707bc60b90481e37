// Count and batch kernels of genus 4: the explicit instantiation of
// CountEntry<4> (count_entry.h), in a translation unit of its own so that
// the genera compile in parallel.
#include "count_launch.h"

namespace hwc {
template struct CountEntry<4>;
}  // namespace hwc
