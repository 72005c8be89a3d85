// sizes.hpp - grid extents (points along one axis of the lifted grid) for
// which a register-resident pencil transform is compiled.  The plan rejects
// any other extent with IWFPM_ERR_UNSUPPORTED.
#pragma once

#define IWFPM_EXTENTS(X)                                                                     \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30)     \
    X(31) X(32) X(36) X(40) X(48) X(60) X(64)
