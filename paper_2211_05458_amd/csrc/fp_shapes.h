// (n, ng) = (N+1, Ngeo+1) pairs with compiled kernels
#pragma once
#define FP_FOR_EACH_SHAPE(X) X(2, 2) X(4, 2) X(4, 5) X(6, 5) X(8, 5) X(6, 7)
