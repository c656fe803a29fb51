"""CPU oracle for GFD validation -- test infrastructure only (tests, smoke
check, benchmark CPU baseline).  Never imported by the product package."""
