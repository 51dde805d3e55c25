// extent.hpp -- how many entries of a column-major matrix a BLAS routine may
// touch: rows x cols with leading dimension ld reaches entry
// (rows-1) + (cols-1)*ld, so a tightly sized array holds ld*(cols-1) + rows
// entries (nothing when rows or cols is 0).  Host code only; no HIP types.
#ifndef MPDD_EXTENT_HPP
#define MPDD_EXTENT_HPP

#include <cstddef>
#include <cstdint>

namespace mpdd {

inline size_t blas_extent(int64_t ld, int64_t rows, int64_t cols) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)ld * (size_t)(cols - 1) + (size_t)rows;
}

}  // namespace mpdd

#endif  // MPDD_EXTENT_HPP
