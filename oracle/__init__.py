"""TEST INFRASTRUCTURE: FP64 CPU oracle (see oracle/oracle.py).  Not part of the product."""
