// amgs_batched.h -- batched persistent solver (internal interface).
#pragma once
