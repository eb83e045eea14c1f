// Pointer into device global memory, for the tile bodies' global accesses.
//
// Operand pointers that reach a tile from a descriptor (the grouped launches)
// are generic pointers, and accesses through them compile to flat
// instructions.  Flat accesses also count against the LDS wait counter, so
// each LDS wait would also wait for the global prefetch in flight, and their
// addresses take extra registers.  Every operand lives in device global
// memory, so the tiles convert their pointers to this type once and make
// every global load and store through it.
#pragma once

namespace mm {

template <typename T> using gptr = __attribute__((address_space(1))) T *;

}  // namespace mm
