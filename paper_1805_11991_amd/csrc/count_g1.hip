// Count and batch kernels of genus 1: the explicit instantiation of
// CountEntry<1> (count_entry.h), in a translation unit of its own so that
// the genera compile in parallel.
#include "count_launch.h"

namespace hwc {
template struct CountEntry<1>;
}  // namespace hwc
