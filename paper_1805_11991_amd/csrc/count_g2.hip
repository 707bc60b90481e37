// Count and batch kernels of genus 2: the explicit instantiation of
// CountEntry<2> (count_entry.h), in a translation unit of its own so that
// the genera compile in parallel.
#include "count_launch.h"

namespace hwc {
template struct CountEntry<2>;
}  // namespace hwc
