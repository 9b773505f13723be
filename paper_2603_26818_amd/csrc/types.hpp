// types.hpp -- plain data types shared by the kernels and the host runtime.
#pragma once

#include <stdint.h>

namespace pfc {

// interleaved complex value (re, im)
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

// Model parameters in the kernel's precision.  fk[a] = 2 pi / (n_a dx_a): the wavenumber of index
// m on axis a is fk[a] * m (m signed; x indices are 0..M).  Axis 0 is the last-axis pass's axis,
// axis 1 the rows (3D y), axis 2 x.
template <typename T>
struct ModelParams {
    T r, dt, q1sq, R1;
    T fk[3];
    T nl;  // 1: cubic term on; 0: linear PDE only
    int model;
};

}  // namespace pfc
